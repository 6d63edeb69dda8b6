// Numeric supernodal multifrontal factorisation A = L L^T (no conjugation)
// of the slab block and of the nodal matrix, in FP64.
//
// Real SPD (M + tau K for implicit Euler, K_n): Cholesky. Complex symmetric
// (mu M + tau K with mu = 2 + i sqrt(2), the diagonalised DG(1) slab block):
// L L^T with complex square roots and no pivoting; the real part 2M + tau K
// and imaginary part sqrt(2) M are SPD, so every leading principal minor is
// nonzero and the factorisation exists.
//
// Storage per supernode s (w columns, r below-diagonal rows, m = w + r): a
// dense column-major panel of m rows x w columns (ld = m) whose top w x w
// block holds L_ss (lower triangle) and whose last r rows hold L_{R_s,s};
// and the inverses of its NB x NB diagonal sub-blocks (column-major, ld = NB,
// zero padded), used by the triangular solves.
#pragma once

#include <vector>

#include "common.hpp"
#include "ordering.hpp"

namespace stmg {

constexpr int NB = 64;  // diagonal sub-block size of the solves

template <typename T>
struct HostFactor {
  const Symbolic *sym = nullptr;
  std::vector<T> panel;
  std::vector<int64_t> panel_off;  // [ns+1]
  std::vector<T> dinv;
  std::vector<int64_t> dinv_off;   // [ns+1]
};

inline int64_t n_diag_blocks(int32_t w) { return (w + NB - 1) / NB; }

// Factor the matrix whose entries on the pattern of A (ascending interior
// numbering) are vals[k] (T per nonzero). Throws STMG_ENUMERIC on a zero or
// non-finite pivot.
template <typename T>
void factor_host(const Symbolic &S, const Csr &A, const std::vector<T> &vals, HostFactor<T> &F);

// Offsets of panels and diagonal inverses for a symbolic structure.
void factor_layout(const Symbolic &S, std::vector<int64_t> &panel_off, std::vector<int64_t> &dinv_off);

}  // namespace stmg
