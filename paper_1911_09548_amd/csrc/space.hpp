// Spatial discretisation on the host: mesh topology, lowest-order Nedelec
// (Whitney) assembly, discrete gradient, nested-mesh transfers and Galerkin
// coarse operators (section 3 and the coarse-grid correction of section 2).
#pragma once

#include <vector>

#include "common.hpp"

namespace stmg {

struct Topo {
  int32_t nv = 0, nt = 0, ne = 0;
  std::vector<double> coords;      // [nv*3]
  std::vector<int32_t> tets;       // [nt*4], vertex ids ascending within a tet
  std::vector<int32_t> edges;      // [ne*2] (tail < head), lexicographic
  std::vector<int32_t> tet_edges;  // [nt*6] local order (01,02,03,12,13,23)
  std::vector<uint8_t> bnd_edge, bnd_vert;
  std::vector<int32_t> int_edges, int_verts;     // interior ids, ascending
  std::vector<int32_t> edge_to_int, vert_to_int; // -1 on the boundary
  std::vector<int64_t> edge_key;   // tail*nv + head, ascending (for lookup)

  // bc: STMG_BC_DIRICHLET eliminates boundary edges and vertices;
  // STMG_BC_NEUMANN keeps every edge and leaves vertex 0 out of the nodal
  // space (gauge of the constants, which G maps to zero).
  void build(int32_t n_vertices, const double *xyz, int32_t n_tets, const int32_t *t, int32_t bc);
  int32_t find_edge(int32_t a, int32_t b) const;  // -1 if absent
  int32_t n_int_edges() const { return (int32_t)int_edges.size(); }
  int32_t n_int_verts() const { return (int32_t)int_verts.size(); }
};

struct SpaceLevel {
  Topo topo;
  Csr M, K;        // interior edges, shared pattern
  Csr G;           // interior edges x interior vertices, entries +-1
  Csr Kn;          // G^T M G over interior vertices
  Csr Pe, Pn;      // from this mesh to the next finer one (empty on mesh 0)
  std::vector<double> ratio;  // nu/sigma per tet (min over contained finer tets)
  std::vector<double> h;      // longest edge per tet
  double anisotropy(double tau) const;  // min_T ratio_T tau / h_T^2, eq. (3)
};

// Build every mesh of the problem's hierarchy (finest first).
std::vector<SpaceLevel> build_space_levels(const stmg_problem &prob);

}  // namespace stmg
