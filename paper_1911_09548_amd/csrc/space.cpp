// Host-side spatial setup: topology, Whitney element matrices, assembly,
// transfers and Galerkin products (section 3; coarse-grid correction of
// section 2.2).
#include "space.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

namespace stmg {

double wall_time() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ sparse
Csr csr_transpose(const Csr &A) {
  Csr T;
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  T.ptr.assign(T.n_rows + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k) T.ptr[A.col[k] + 1]++;
  for (int32_t i = 0; i < T.n_rows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int64_t> next(T.ptr.begin(), T.ptr.end() - 1);
  for (int32_t i = 0; i < A.n_rows; ++i)
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int64_t p = next[A.col[k]]++;
      T.col[p] = i;
      T.val[p] = A.val[k];
    }
  return T;
}

Csr csr_multiply(const Csr &A, const Csr &B) {
  alloc_point("sparse product");
  STMG_REQUIRE(A.n_cols == B.n_rows, STMG_EINVAL, "csr_multiply: shape mismatch");
  Csr C;
  C.n_rows = A.n_rows;
  C.n_cols = B.n_cols;
  C.ptr.assign(C.n_rows + 1, 0);
  std::vector<int32_t> mark(B.n_cols, -1);
  std::vector<double> acc(B.n_cols, 0.0);
  std::vector<int32_t> cols;
  for (int32_t i = 0; i < A.n_rows; ++i) {
    cols.clear();
    for (int64_t ka = A.ptr[i]; ka < A.ptr[i + 1]; ++ka) {
      int32_t k = A.col[ka];
      double a = A.val[ka];
      for (int64_t kb = B.ptr[k]; kb < B.ptr[k + 1]; ++kb) {
        int32_t j = B.col[kb];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += a * B.val[kb];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      C.col.push_back(j);
      C.val.push_back(acc[j]);
    }
    C.ptr[i + 1] = (int64_t)C.col.size();
  }
  return C;
}

void csr_galerkin_pair(const Csr &P, const Csr &A, const Csr &B, Csr &Ac, Csr &Bc) {
  // Both products share the sparsity of A's and B's patterns (identical here),
  // so compute the pattern union explicitly: pattern(P^T (A+B) P).
  Csr Pt = csr_transpose(P);
  Csr AP = csr_multiply(A, P), BP = csr_multiply(B, P);
  Csr a = csr_multiply(Pt, AP), b = csr_multiply(Pt, BP);
  // merge to a common pattern
  Ac.n_rows = Bc.n_rows = a.n_rows;
  Ac.n_cols = Bc.n_cols = a.n_cols;
  Ac.ptr.assign(a.n_rows + 1, 0);
  Ac.col.clear();
  Ac.val.clear();
  Bc.val.clear();
  for (int32_t i = 0; i < a.n_rows; ++i) {
    int64_t p = a.ptr[i], q = b.ptr[i];
    while (p < a.ptr[i + 1] || q < b.ptr[i + 1]) {
      int32_t ca = p < a.ptr[i + 1] ? a.col[p] : INT32_MAX;
      int32_t cb = q < b.ptr[i + 1] ? b.col[q] : INT32_MAX;
      int32_t c = std::min(ca, cb);
      Ac.col.push_back(c);
      Ac.val.push_back(ca == c ? a.val[p++] : 0.0);
      Bc.val.push_back(cb == c ? b.val[q++] : 0.0);
    }
    Ac.ptr[i + 1] = (int64_t)Ac.col.size();
  }
  Bc.ptr = Ac.ptr;
  Bc.col = Ac.col;
}

Csr csr_permute_sym(const Csr &A, const std::vector<int32_t> &p) {
  int32_t n = A.n_rows;
  std::vector<int32_t> ip(n);
  for (int32_t i = 0; i < n; ++i) ip[p[i]] = i;
  Csr B;
  B.n_rows = B.n_cols = n;
  B.ptr.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) B.ptr[i + 1] = B.ptr[i] + (A.ptr[p[i] + 1] - A.ptr[p[i]]);
  B.col.resize(A.nnz());
  B.val.resize(A.nnz());
  std::vector<std::pair<int32_t, double>> row;
  for (int32_t i = 0; i < n; ++i) {
    row.clear();
    int32_t o = p[i];
    for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k) row.push_back({ip[A.col[k]], A.val[k]});
    std::sort(row.begin(), row.end());
    int64_t b = B.ptr[i];
    for (size_t k = 0; k < row.size(); ++k) {
      B.col[b + k] = row[k].first;
      B.val[b + k] = row[k].second;
    }
  }
  return B;
}

double csr_get(const Csr &A, int32_t i, int32_t j) {
  auto b = A.col.begin() + A.ptr[i], e = A.col.begin() + A.ptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  return (it != e && *it == j) ? A.val[it - A.col.begin()] : 0.0;
}

// ---------------------------------------------------------------- topology
void Topo::build(int32_t n_vertices, const double *xyz, int32_t n_tets, const int32_t *t, int32_t bc) {
  alloc_point("mesh topology");
  nv = n_vertices;
  nt = n_tets;
  STMG_REQUIRE(nv > 0 && nt > 0 && xyz && t, STMG_EINVAL, "empty mesh");
  coords.assign(xyz, xyz + 3 * (size_t)nv);
  tets.resize(4 * (size_t)nt);
  for (int32_t e = 0; e < nt; ++e) {
    int32_t v[4] = {t[4 * e], t[4 * e + 1], t[4 * e + 2], t[4 * e + 3]};
    for (int a = 0; a < 4; ++a)
      STMG_REQUIRE(v[a] >= 0 && v[a] < nv, STMG_EINVAL, "tet vertex id out of range");
    std::sort(v, v + 4);
    STMG_REQUIRE(v[0] != v[1] && v[1] != v[2] && v[2] != v[3], STMG_EINVAL, "degenerate tet");
    std::copy(v, v + 4, &tets[4 * (size_t)e]);
  }
  static const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  std::vector<int64_t> keys(6 * (size_t)nt);
  for (int32_t e = 0; e < nt; ++e)
    for (int l = 0; l < 6; ++l)
      keys[6 * (size_t)e + l] =
          (int64_t)tets[4 * (size_t)e + LE[l][0]] * nv + tets[4 * (size_t)e + LE[l][1]];
  edge_key = keys;
  std::sort(edge_key.begin(), edge_key.end());
  edge_key.erase(std::unique(edge_key.begin(), edge_key.end()), edge_key.end());
  ne = (int32_t)edge_key.size();
  edges.resize(2 * (size_t)ne);
  for (int32_t i = 0; i < ne; ++i) {
    edges[2 * i] = (int32_t)(edge_key[i] / nv);
    edges[2 * i + 1] = (int32_t)(edge_key[i] % nv);
  }
  tet_edges.resize(6 * (size_t)nt);
  for (size_t k = 0; k < keys.size(); ++k)
    tet_edges[k] = (int32_t)(std::lower_bound(edge_key.begin(), edge_key.end(), keys[k]) -
                             edge_key.begin());
  // faces: boundary faces belong to exactly one tet
  static const int LF[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
  std::vector<int64_t> fk(4 * (size_t)nt);
  for (int32_t e = 0; e < nt; ++e)
    for (int f = 0; f < 4; ++f) {
      const int32_t *v = &tets[4 * (size_t)e];
      fk[4 * (size_t)e + f] =
          ((int64_t)v[LF[f][0]] * nv + v[LF[f][1]]) * nv + v[LF[f][2]];
    }
  std::sort(fk.begin(), fk.end());
  bnd_vert.assign(nv, 0);
  bnd_edge.assign(ne, 0);
  for (size_t i = 0; i < fk.size();) {
    size_t j = i;
    while (j < fk.size() && fk[j] == fk[i]) ++j;
    STMG_REQUIRE(j - i <= 2, STMG_EINVAL, "non-manifold mesh: face shared by >2 tets");
    if (j - i == 1) {
      int64_t k = fk[i];
      int32_t c = (int32_t)(k % nv), b = (int32_t)((k / nv) % nv), a = (int32_t)(k / nv / nv);
      bnd_vert[a] = bnd_vert[b] = bnd_vert[c] = 1;
      bnd_edge[find_edge(a, b)] = 1;
      bnd_edge[find_edge(b, c)] = 1;
      bnd_edge[find_edge(a, c)] = 1;
    }
    i = j;
  }
  int_edges.clear();
  int_verts.clear();
  edge_to_int.assign(ne, -1);
  vert_to_int.assign(nv, -1);
  const bool neumann = bc == STMG_BC_NEUMANN;
  for (int32_t i = 0; i < ne; ++i)
    if (neumann || !bnd_edge[i]) {
      edge_to_int[i] = (int32_t)int_edges.size();
      int_edges.push_back(i);
    }
  for (int32_t i = 0; i < nv; ++i)
    if (neumann ? i > 0 : !bnd_vert[i]) {
      vert_to_int[i] = (int32_t)int_verts.size();
      int_verts.push_back(i);
    }
}

int32_t Topo::find_edge(int32_t a, int32_t b) const {
  if (a > b) std::swap(a, b);
  int64_t k = (int64_t)a * nv + b;
  auto it = std::lower_bound(edge_key.begin(), edge_key.end(), k);
  return (it != edge_key.end() && *it == k) ? (int32_t)(it - edge_key.begin()) : -1;
}

// --------------------------------------------------------------- assembly
namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }

// Barycentric gradients g[0..3] and volume of a tetrahedron.
void tet_geometry(const double *c, const int32_t *v, V3 g[4], double &vol) {
  V3 x[4];
  for (int a = 0; a < 4; ++a) x[a] = {c[3 * v[a]], c[3 * v[a] + 1], c[3 * v[a] + 2]};
  V3 a = sub(x[1], x[0]), b = sub(x[2], x[0]), d = sub(x[3], x[0]);
  double det = dot(a, cross(b, d));
  // rows of the inverse of [a b d] (columns): (b x d, d x a, a x b) / det
  g[1] = scale(cross(b, d), 1.0 / det);
  g[2] = scale(cross(d, a), 1.0 / det);
  g[3] = scale(cross(a, b), 1.0 / det);
  g[0] = scale({g[1].x + g[2].x + g[3].x, g[1].y + g[2].y + g[3].y, g[1].z + g[2].z + g[3].z}, -1.0);
  vol = std::fabs(det) / 6.0;
}

const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// Whitney element matrices: phi_ij = l_i g_j - l_j g_i,
// int l_a l_b = vol (1 + d_ab) / 20, curl phi_ij = 2 g_i x g_j.
void whitney_element(const V3 g[4], double vol, double sigma, double nu, double Me[36], double Ke[36]) {
  double gg[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) gg[a][b] = dot(g[a], g[b]);
  auto ll = [](int a, int b) { return (a == b ? 2.0 : 1.0) / 20.0; };
  V3 cu[6];
  for (int p = 0; p < 6; ++p) cu[p] = scale(cross(g[LE[p][0]], g[LE[p][1]]), 2.0);
  for (int p = 0; p < 6; ++p)
    for (int q = 0; q < 6; ++q) {
      int i = LE[p][0], j = LE[p][1], k = LE[q][0], l = LE[q][1];
      double m = ll(i, k) * gg[j][l] - ll(i, l) * gg[j][k] - ll(j, k) * gg[i][l] + ll(j, l) * gg[i][k];
      Me[6 * p + q] = sigma * vol * m;
      Ke[6 * p + q] = nu * vol * dot(cu[p], cu[q]);
    }
}

// Interior-edge adjacency pattern (edges sharing a tetrahedron).
Csr edge_pattern(const Topo &T) {
  int32_t n = T.n_int_edges();
  std::vector<std::vector<int32_t>> rows(n);
  for (int32_t e = 0; e < T.nt; ++e) {
    const int32_t *te = &T.tet_edges[6 * (size_t)e];
    for (int p = 0; p < 6; ++p) {
      int32_t i = T.edge_to_int[te[p]];
      if (i < 0) continue;
      for (int q = 0; q < 6; ++q) {
        int32_t j = T.edge_to_int[te[q]];
        if (j >= 0) rows[i].push_back(j);
      }
    }
  }
  Csr A;
  A.n_rows = A.n_cols = n;
  A.ptr.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    auto &r = rows[i];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    A.ptr[i + 1] = A.ptr[i] + (int64_t)r.size();
  }
  A.col.reserve(A.ptr[n]);
  for (int32_t i = 0; i < n; ++i) A.col.insert(A.col.end(), rows[i].begin(), rows[i].end());
  A.val.assign(A.col.size(), 0.0);
  return A;
}

inline int64_t csr_find(const Csr &A, int32_t i, int32_t j) {
  auto b = A.col.begin() + A.ptr[i], e = A.col.begin() + A.ptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  return (it != e && *it == j) ? (int64_t)(it - A.col.begin()) : -1;
}

void assemble_fine(const Topo &T, const double *sigma, const double *nu, Csr &M, Csr &K) {
  alloc_point("edge matrices");
  M = edge_pattern(T);
  K = M;
  for (int32_t e = 0; e < T.nt; ++e) {
    STMG_REQUIRE(sigma[e] > 0 && std::isfinite(sigma[e]), STMG_EINVAL, "sigma must be > 0");
    STMG_REQUIRE(nu[e] >= 0 && std::isfinite(nu[e]), STMG_EINVAL, "nu must be >= 0");
    V3 g[4];
    double vol;
    tet_geometry(T.coords.data(), &T.tets[4 * (size_t)e], g, vol);
    STMG_REQUIRE(vol > 0, STMG_EINVAL, "degenerate tetrahedron (zero volume)");
    double Me[36], Ke[36];
    whitney_element(g, vol, sigma[e], nu[e], Me, Ke);
    const int32_t *te = &T.tet_edges[6 * (size_t)e];
    for (int p = 0; p < 6; ++p) {
      int32_t i = T.edge_to_int[te[p]];
      if (i < 0) continue;
      for (int q = 0; q < 6; ++q) {
        int32_t j = T.edge_to_int[te[q]];
        if (j < 0) continue;
        int64_t k = csr_find(M, i, j);
        M.val[k] += Me[6 * p + q];
        K.val[k] += Ke[6 * p + q];
      }
    }
  }
}

Csr interior_gradient(const Topo &T) {
  Csr G;
  int32_t n = T.n_int_edges();
  G.n_rows = n;
  G.n_cols = T.n_int_verts();
  G.ptr.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    int32_t e = T.int_edges[i];
    int32_t tail = T.vert_to_int[T.edges[2 * e]], head = T.vert_to_int[T.edges[2 * e + 1]];
    // columns ascending: tail < head in global ids and vert_to_int is monotone
    if (tail >= 0) {
      G.col.push_back(tail);
      G.val.push_back(-1.0);
    }
    if (head >= 0) {
      G.col.push_back(head);
      G.val.push_back(1.0);
    }
    G.ptr[i + 1] = (int64_t)G.col.size();
  }
  return G;
}

// Whitney prolongation from coarse interior edges to fine interior edges:
// fine edge p->q takes l_i(p) l_j(q) - l_i(q) l_j(p) from coarse edge i->j,
// with l = 1 at a coinciding coarse vertex and 1/2 at both ends of the coarse
// edge whose midpoint the fine vertex is.
Csr edge_prolongation(const Topo &F, const Topo &C, const int32_t *vparent) {
  alloc_point("edge prolongation");
  Csr P;
  P.n_rows = F.n_int_edges();
  P.n_cols = C.n_int_edges();
  P.ptr.assign(P.n_rows + 1, 0);
  std::vector<std::pair<int32_t, double>> row;
  for (int32_t r = 0; r < P.n_rows; ++r) {
    int32_t e = F.int_edges[r];
    int32_t p = F.edges[2 * e], q = F.edges[2 * e + 1];
    int32_t sp[2] = {vparent[2 * p], vparent[2 * p + 1]};
    int32_t sq[2] = {vparent[2 * q], vparent[2 * q + 1]};
    auto lam = [](const int32_t s[2], int32_t v) {
      return (s[0] == v ? 0.5 : 0.0) + (s[1] == v ? 0.5 : 0.0);
    };
    int32_t sup[4] = {sp[0], sp[1], sq[0], sq[1]};
    std::sort(sup, sup + 4);
    int ns = (int)(std::unique(sup, sup + 4) - sup);
    row.clear();
    for (int a = 0; a < ns; ++a)
      for (int b = a + 1; b < ns; ++b) {
        int32_t i = sup[a], j = sup[b];
        double c = lam(sp, i) * lam(sq, j) - lam(sq, i) * lam(sp, j);
        if (c == 0.0) continue;
        int32_t ce = C.find_edge(i, j);
        STMG_REQUIRE(ce >= 0, STMG_EINVAL, "vertex_parent does not describe a nested refinement");
        int32_t ci = C.edge_to_int[ce];
        if (ci >= 0) row.push_back({ci, c});
      }
    std::sort(row.begin(), row.end());
    for (auto &x : row) {
      P.col.push_back(x.first);
      P.val.push_back(x.second);
    }
    P.ptr[r + 1] = (int64_t)P.col.size();
  }
  return P;
}

Csr vertex_prolongation(const Topo &F, const Topo &C, const int32_t *vparent) {
  Csr P;
  P.n_rows = F.n_int_verts();
  P.n_cols = C.n_int_verts();
  P.ptr.assign(P.n_rows + 1, 0);
  for (int32_t r = 0; r < P.n_rows; ++r) {
    int32_t v = F.int_verts[r];
    int32_t a = vparent[2 * v], b = vparent[2 * v + 1];
    STMG_REQUIRE(a >= 0 && a < C.nv && b >= 0 && b < C.nv, STMG_EINVAL, "vertex_parent out of range");
    std::pair<int32_t, double> ent[2];
    int k = 0;
    if (a == b) {
      ent[k++] = {C.vert_to_int[a], 1.0};
    } else {
      ent[k++] = {C.vert_to_int[a], 0.5};
      ent[k++] = {C.vert_to_int[b], 0.5};
    }
    std::sort(ent, ent + k);
    for (int i = 0; i < k; ++i)
      if (ent[i].first >= 0) {
        P.col.push_back(ent[i].first);
        P.val.push_back(ent[i].second);
      }
    P.ptr[r + 1] = (int64_t)P.col.size();
  }
  return P;
}

void tet_longest_edges(const Topo &T, std::vector<double> &h) {
  h.assign(T.nt, 0.0);
  for (int32_t e = 0; e < T.nt; ++e) {
    const int32_t *v = &T.tets[4 * (size_t)e];
    for (int p = 0; p < 6; ++p) {
      const double *a = &T.coords[3 * (size_t)v[LE[p][0]]], *b = &T.coords[3 * (size_t)v[LE[p][1]]];
      double d = std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) +
                           (a[2] - b[2]) * (a[2] - b[2]));
      h[e] = std::max(h[e], d);
    }
  }
}

}  // namespace

double SpaceLevel::anisotropy(double tau) const {
  double lam = INFINITY;
  for (size_t e = 0; e < h.size(); ++e) lam = std::min(lam, ratio[e] * tau / (h[e] * h[e]));
  return lam;
}

std::vector<SpaceLevel> build_space_levels(const stmg_problem &prob) {
  STMG_REQUIRE(prob.n_meshes >= 1 && prob.meshes, STMG_EINVAL, "no meshes");
  std::vector<SpaceLevel> L(prob.n_meshes);
  for (int32_t j = 0; j < prob.n_meshes; ++j) {
    const stmg_mesh &m = prob.meshes[j];
    SpaceLevel &S = L[j];
    S.topo.build(m.n_vertices, m.coords, m.n_tets, m.tets, prob.bc);
    tet_longest_edges(S.topo, S.h);
    if (j == 0) {
      STMG_REQUIRE(prob.sigma && prob.nu, STMG_EINVAL, "sigma/nu missing");
      assemble_fine(S.topo, prob.sigma, prob.nu, S.M, S.K);
      S.ratio.resize(S.topo.nt);
      for (int32_t e = 0; e < S.topo.nt; ++e) S.ratio[e] = prob.nu[e] / prob.sigma[e];
    } else {
      const SpaceLevel &F = L[j - 1];
      STMG_REQUIRE(m.vertex_parent && m.tet_parent, STMG_EINVAL, "coarse mesh without parent maps");
      S.Pe = edge_prolongation(F.topo, S.topo, m.vertex_parent);
      S.Pn = vertex_prolongation(F.topo, S.topo, m.vertex_parent);
      csr_galerkin_pair(S.Pe, F.M, F.K, S.M, S.K);
      S.ratio.assign(S.topo.nt, INFINITY);
      for (int32_t e = 0; e < F.topo.nt; ++e) {
        int32_t c = m.tet_parent[e];
        STMG_REQUIRE(c >= 0 && c < S.topo.nt, STMG_EINVAL, "tet_parent out of range");
        S.ratio[c] = std::min(S.ratio[c], F.ratio[e]);
      }
    }
    S.G = interior_gradient(S.topo);
    Csr Gt = csr_transpose(S.G);
    S.Kn = csr_multiply(Gt, csr_multiply(S.M, S.G));
    STMG_REQUIRE(S.topo.n_int_edges() > 0, STMG_EINVAL, "mesh has no interior edges");
  }
  return L;
}

}  // namespace stmg
