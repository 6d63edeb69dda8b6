// Fill-reducing ordering and supernodal symbolic factorisation.
//
// Geometric nested dissection on the mesh's vertex graph: recursively split
// the vertex set at the median coordinate of its longest bounding-box axis,
// take as separator the vertices on the lower side that touch the upper side,
// and recurse on both remainders. A tree node owns its separator vertices
// (a leaf owns all of its vertices). Adjacent vertices always lie on one
// root-to-leaf path, so the tree is an elimination tree for
//   * the nodal matrix K_n (DOF = interior vertex, node = the vertex's node);
//   * the edge matrices M, K (DOF = interior edge, node = the deeper of its
//     two end vertices' nodes): two edges sharing a tetrahedron have all four
//     vertices pairwise adjacent, so their nodes are on one path.
// Numbering the DOFs of each tree node contiguously in post-order makes every
// node a supernode whose below-diagonal rows belong to its ancestors; the
// dense diagonal block of a separator is (nearly) full after elimination.
#pragma once

#include <vector>

#include "common.hpp"
#include "space.hpp"

namespace stmg {

struct Symbolic {
  int32_t n = 0;                 // matrix dimension
  std::vector<int32_t> perm;     // perm[new] = old (ascending interior index)
  std::vector<int32_t> iperm;    // iperm[old] = new
  int32_t ns = 0;                // supernodes, in post-order
  std::vector<int32_t> col0;     // [ns+1] first column of each supernode
  std::vector<int32_t> parent;   // [ns] parent supernode, -1 for a root
  std::vector<int64_t> rptr;     // [ns+1] offsets into rows
  std::vector<int32_t> rows;     // below-diagonal row structure R_s, ascending, new numbering
  std::vector<int32_t> height;   // [ns] 0 for leaves, 1 + max over children
  int32_t n_heights = 0;
  int64_t nnz_L = 0;             // sum w(w+1)/2 + r w (dense supernode blocks, as stored)
  int64_t nnz_L_struct = 0;      // structural nonzeros of L (column counts, diagonal included)
  std::vector<int64_t> sn_nnz;   // [ns] structural nonzeros of each supernode's columns
  int64_t panel_entries = 0;     // sum (w + r) w  (dense panels as stored)
  int32_t max_front = 0;         // max w + r

  int32_t width(int32_t s) const { return col0[s + 1] - col0[s]; }
  int32_t nrows(int32_t s) const { return (int32_t)(rptr[s + 1] - rptr[s]); }
};

struct NdTree {
  std::vector<int32_t> node_of_vertex;  // [nv]
  std::vector<int32_t> parent;          // [n_nodes]
  std::vector<int32_t> depth;           // [n_nodes]
  std::vector<int32_t> postorder;       // nodes in post-order
};

// Nested dissection of all vertices of a mesh (leaf_size: max vertices per leaf).
NdTree nested_dissection(const Topo &T, int32_t leaf_size);

// Symbolic factorisation of a symmetric pattern A (given in the ascending
// interior numbering) whose DOF i belongs to ND node dof_node[i].
Symbolic symbolic_from_tree(const NdTree &nd, const std::vector<int32_t> &dof_node, const Csr &A);

// DOF -> node maps for interior edges and interior vertices.
std::vector<int32_t> edge_nodes(const Topo &T, const NdTree &nd);
std::vector<int32_t> vertex_nodes(const Topo &T, const NdTree &nd);

}  // namespace stmg
