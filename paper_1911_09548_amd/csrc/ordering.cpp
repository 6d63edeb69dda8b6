// Geometric nested dissection and supernodal symbolic factorisation.
#include "ordering.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace stmg {

NdTree nested_dissection(const Topo &T, int32_t leaf_size) {
  alloc_point("nested-dissection tree");
  if (leaf_size < 1) leaf_size = 8;
  const int32_t nv = T.nv;
  // vertex adjacency from the edge list
  std::vector<int64_t> aptr(nv + 1, 0);
  for (int32_t e = 0; e < T.ne; ++e) {
    aptr[T.edges[2 * e] + 1]++;
    aptr[T.edges[2 * e + 1] + 1]++;
  }
  for (int32_t v = 0; v < nv; ++v) aptr[v + 1] += aptr[v];
  std::vector<int32_t> adj(aptr[nv]);
  {
    std::vector<int64_t> nx(aptr.begin(), aptr.end() - 1);
    for (int32_t e = 0; e < T.ne; ++e) {
      int32_t a = T.edges[2 * e], b = T.edges[2 * e + 1];
      adj[nx[a]++] = b;
      adj[nx[b]++] = a;
    }
  }
  NdTree nd;
  nd.node_of_vertex.assign(nv, -1);
  std::vector<int32_t> stamp(nv, -1);
  int32_t stamp_id = 0;

  struct Task {
    std::vector<int32_t> verts;
    int32_t parent, depth;
  };
  std::vector<Task> stack;
  std::vector<int32_t> all(nv);
  std::iota(all.begin(), all.end(), 0);
  stack.push_back({std::move(all), -1, 0});
  std::vector<std::vector<int32_t>> children;
  while (!stack.empty()) {
    Task t = std::move(stack.back());
    stack.pop_back();
    int32_t id = (int32_t)nd.parent.size();
    nd.parent.push_back(t.parent);
    nd.depth.push_back(t.depth);
    children.emplace_back();
    if (t.parent >= 0) children[t.parent].push_back(id);
    std::vector<int32_t> &V = t.verts;
    if ((int32_t)V.size() <= leaf_size) {
      for (int32_t v : V) nd.node_of_vertex[v] = id;
      continue;
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t v : V)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], T.coords[3 * (size_t)v + d]);
        hi[d] = std::max(hi[d], T.coords[3 * (size_t)v + d]);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    std::vector<int32_t> sorted = V;
    std::sort(sorted.begin(), sorted.end(), [&](int32_t a, int32_t b) {
      double ca = T.coords[3 * (size_t)a + ax], cb = T.coords[3 * (size_t)b + ax];
      return ca < cb || (ca == cb && a < b);
    });
    double c = T.coords[3 * (size_t)sorted[sorted.size() / 2] + ax];
    size_t split = (size_t)(std::lower_bound(sorted.begin(), sorted.end(), c,
                                             [&](int32_t a, double val) {
                                               return T.coords[3 * (size_t)a + ax] < val;
                                             }) -
                            sorted.begin());
    if (split == 0) split = sorted.size() / 2;  // all coordinates equal: split by position
    ++stamp_id;
    for (size_t i = split; i < sorted.size(); ++i) stamp[sorted[i]] = stamp_id;  // upper side
    std::vector<int32_t> Lrest, R(sorted.begin() + split, sorted.end());
    for (size_t i = 0; i < split; ++i) {
      int32_t v = sorted[i];
      bool touches = false;
      for (int64_t k = aptr[v]; k < aptr[v + 1] && !touches; ++k) touches = stamp[adj[k]] == stamp_id;
      if (touches)
        nd.node_of_vertex[v] = id;  // separator vertex
      else
        Lrest.push_back(v);
    }
    if (!R.empty()) stack.push_back({std::move(R), id, t.depth + 1});
    if (!Lrest.empty()) stack.push_back({std::move(Lrest), id, t.depth + 1});
  }
  // post-order (children in creation order, then the node)
  int32_t nn = (int32_t)nd.parent.size();
  nd.postorder.reserve(nn);
  std::vector<std::pair<int32_t, size_t>> st;
  for (int32_t r = 0; r < nn; ++r) {
    if (nd.parent[r] != -1) continue;
    st.push_back({r, 0});
    while (!st.empty()) {
      auto &top = st.back();
      if (top.second < children[top.first].size()) {
        int32_t ch = children[top.first][top.second++];
        st.push_back({ch, 0});
      } else {
        nd.postorder.push_back(top.first);
        st.pop_back();
      }
    }
  }
  return nd;
}

std::vector<int32_t> edge_nodes(const Topo &T, const NdTree &nd) {
  std::vector<int32_t> out(T.n_int_edges());
  for (int32_t i = 0; i < T.n_int_edges(); ++i) {
    int32_t e = T.int_edges[i];
    int32_t a = nd.node_of_vertex[T.edges[2 * e]], b = nd.node_of_vertex[T.edges[2 * e + 1]];
    out[i] = nd.depth[a] >= nd.depth[b] ? a : b;
  }
  return out;
}

std::vector<int32_t> vertex_nodes(const Topo &T, const NdTree &nd) {
  std::vector<int32_t> out(T.n_int_verts());
  for (int32_t i = 0; i < T.n_int_verts(); ++i) out[i] = nd.node_of_vertex[T.int_verts[i]];
  return out;
}

// Structural nonzeros per column of the Cholesky factor of A(perm, perm)
// (diagonal included), without the zeros that dense supernode blocks hold:
// the elimination tree (Liu's algorithm with path compression), then the
// row subtrees: L(i, j) != 0 exactly for the etree nodes j on the paths from
// the nonzeros A(i, k), k < i, up to i.
static std::vector<int64_t> column_counts(const Symbolic &S, const Csr &A) {
  const int32_t n = S.n;
  std::vector<int32_t> parent(n, -1), anc(n, -1);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t o = S.perm[i];
    for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k) {
      int32_t j = S.iperm[A.col[k]];
      while (j >= 0 && j < i) {
        const int32_t next = anc[j];
        anc[j] = i;
        if (next < 0) parent[j] = i;
        j = next;
      }
    }
  }
  std::vector<int64_t> cc(n, 1);
  std::vector<int32_t> mark(n, -1);
  for (int32_t i = 0; i < n; ++i) {
    mark[i] = i;
    const int32_t o = S.perm[i];
    for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k) {
      int32_t j = S.iperm[A.col[k]];
      if (j >= i) continue;
      while (mark[j] != i) {
        mark[j] = i;
        ++cc[j];
        j = parent[j];
      }
    }
  }
  return cc;
}

Symbolic symbolic_from_tree(const NdTree &nd, const std::vector<int32_t> &dof_node, const Csr &A) {
  alloc_point("symbolic factor");
  Symbolic S;
  const int32_t n = (int32_t)dof_node.size();
  S.n = n;
  const int32_t nn = (int32_t)nd.parent.size();
  // DOFs per node
  std::vector<std::vector<int32_t>> dofs(nn);
  for (int32_t i = 0; i < n; ++i) dofs[dof_node[i]].push_back(i);
  // supernodes: non-empty nodes in post-order
  std::vector<int32_t> sn_of_node(nn, -1);
  S.perm.reserve(n);
  S.col0.push_back(0);
  for (int32_t node : nd.postorder) {
    if (dofs[node].empty()) continue;
    sn_of_node[node] = S.ns++;
    for (int32_t i : dofs[node]) S.perm.push_back(i);
    S.col0.push_back((int32_t)S.perm.size());
  }
  STMG_REQUIRE((int32_t)S.perm.size() == n, STMG_EINVAL, "ordering lost DOFs");
  S.iperm.assign(n, 0);
  for (int32_t k = 0; k < n; ++k) S.iperm[S.perm[k]] = k;
  // supernode parent = nearest non-empty ancestor node
  S.parent.assign(S.ns, -1);
  for (int32_t node = 0; node < nn; ++node) {
    int32_t s = sn_of_node[node];
    if (s < 0) continue;
    int32_t a = nd.parent[node];
    while (a >= 0 && sn_of_node[a] < 0) a = nd.parent[a];
    S.parent[s] = a >= 0 ? sn_of_node[a] : -1;
  }
  // row structures in post-order
  std::vector<std::vector<int32_t>> kids(S.ns);
  for (int32_t s = 0; s < S.ns; ++s)
    if (S.parent[s] >= 0) kids[S.parent[s]].push_back(s);
  std::vector<std::vector<int32_t>> R(S.ns);
  std::vector<int32_t> mark(n, -1);
  S.height.assign(S.ns, 0);
  for (int32_t s = 0; s < S.ns; ++s) {
    int32_t c0 = S.col0[s], c1 = S.col0[s + 1];
    std::vector<int32_t> &r = R[s];
    for (int32_t j = c0; j < c1; ++j) {
      int32_t o = S.perm[j];
      for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k) {
        int32_t i = S.iperm[A.col[k]];
        if (i >= c1 && mark[i] != s) {
          mark[i] = s;
          r.push_back(i);
        }
      }
    }
    for (int32_t ch : kids[s]) {
      S.height[s] = std::max(S.height[s], S.height[ch] + 1);
      for (int32_t i : R[ch])
        if (i >= c1 && mark[i] != s) {
          mark[i] = s;
          r.push_back(i);
        }
    }
    std::sort(r.begin(), r.end());
  }
  // every row of R_s must be a column of an ancestor (multifrontal invariant)
  std::vector<int32_t> sn_of_col(n);
  for (int32_t s = 0; s < S.ns; ++s)
    for (int32_t j = S.col0[s]; j < S.col0[s + 1]; ++j) sn_of_col[j] = s;
  for (int32_t s = 0; s < S.ns; ++s)
    for (int32_t i : R[s]) {
      int32_t t = sn_of_col[i], a = S.parent[s];
      while (a >= 0 && a != t) a = S.parent[a];
      STMG_REQUIRE(a == t, STMG_EINVAL, "ordering is not an elimination tree of the pattern");
    }
  S.rptr.assign(S.ns + 1, 0);
  for (int32_t s = 0; s < S.ns; ++s) S.rptr[s + 1] = S.rptr[s] + (int64_t)R[s].size();
  S.rows.reserve(S.rptr[S.ns]);
  S.n_heights = 0;
  for (int32_t s = 0; s < S.ns; ++s) {
    S.rows.insert(S.rows.end(), R[s].begin(), R[s].end());
    int64_t w = S.width(s), rr = (int64_t)R[s].size();
    S.nnz_L += w * (w + 1) / 2 + rr * w;
    S.panel_entries += (w + rr) * w;
    S.max_front = std::max(S.max_front, (int32_t)(w + rr));
    S.n_heights = std::max(S.n_heights, S.height[s] + 1);
  }
  const std::vector<int64_t> cc = column_counts(S, A);
  S.sn_nnz.assign(S.ns, 0);
  for (int32_t s = 0; s < S.ns; ++s) {
    for (int32_t j = S.col0[s]; j < S.col0[s + 1]; ++j) S.sn_nnz[s] += cc[j];
    S.nnz_L_struct += S.sn_nnz[s];
  }
  return S;
}

}  // namespace stmg
