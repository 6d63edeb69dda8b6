// Numeric supernodal multifrontal factorisation A = L L^T (no conjugation)
// of the slab block and of the nodal matrix, in FP64.
//
// Real SPD (M + tau K for implicit Euler, K_n): Cholesky. Complex symmetric
// (mu M + tau K with mu = 2 + i sqrt(2), the diagonalised DG(1) slab block):
// L L^T with complex square roots and no pivoting; the real part 2M + tau K
// and imaginary part sqrt(2) M are SPD, so every leading principal minor is
// nonzero and the factorisation exists.
//
// Storage per supernode s (w columns, r below-diagonal rows, m = w + r): the
// supernode's elimination operator in inverted form (selective inversion),
//   P_s = [ inv(L_ss) ; -L_{R_s,s} inv(L_ss) ]     (m x w, column-major, ld = m),
// zero above the diagonal of the top block. The forward solve of the
// supernode is then one product P_s F (its columns' values and the update
// to its ancestors' rows), and the backward solve one product P_s^T [y; x_R].
#pragma once

#include <vector>

#include "common.hpp"
#include "ordering.hpp"

namespace stmg {

constexpr int NB = 64;  // column block of the dense partial factorisation

template <typename T>
struct HostFactor {
  const Symbolic *sym = nullptr;
  std::vector<T> panel;            // P_s of every supernode
  std::vector<int64_t> panel_off;  // [ns+1]
};

// Factor the matrix whose entries on the pattern of A (ascending interior
// numbering) are vals[k] (T per nonzero). Throws STMG_ENUMERIC on a zero or
// non-finite pivot.
template <typename T>
void factor_host(const Symbolic &S, const Csr &A, const std::vector<T> &vals, HostFactor<T> &F);

// Offsets of the panels for a symbolic structure.
void factor_layout(const Symbolic &S, std::vector<int64_t> &panel_off);

}  // namespace stmg
