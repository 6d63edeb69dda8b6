// Numeric multifrontal factorisation on the GPU (the same L L^T without
// pivoting and the same selective-inversion panels as the host version in
// factor.hpp), for setups that should not spend minutes on host dense
// algebra.
//
// Per supernode, in post-order on one stream:
//   1. front F (m x m, column-major, lower triangle) = entries of A in the
//      supernode's w columns + the update matrices of its children
//      (extend-add through precomputed positions);
//   2. blocked right-looking partial factorisation of the first w columns:
//      per 64-column block, L L^T of the diagonal block in LDS, the panel
//      below by a triangular solve (X L^T = B) and the trailing lower
//      triangle by a rank-64 symmetric update (C -= P P^T, no conjugation),
//      which leaves the Schur complement (the update matrix) in F22;
//   3. P_s = [inv(L11); -L21 inv(L11)]: inv(L11) from a triangular solve
//      against the identity, then a triangular product with L21.
// The dense triangular solves and symmetric updates are rocBLAS calls;
// assembly, the diagonal blocks and conversions are kernels here.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <vector>

#include "factor.hpp"
#include "kernels.hpp"

namespace stmg {

// Assembly plan of the fronts of one symbolic structure (per mesh).
struct FrontPlan {
  std::vector<int64_t> a_ptr;    // [ns+1] offsets into a_pos / a_k
  std::vector<int64_t> a_pos;    // entry of A -> position in its front (row + col * m)
  std::vector<int64_t> a_k;      // entry of A -> index of its value on A's pattern
  std::vector<int32_t> relpos;   // [rptr[ns]] update row of s -> row of its parent's front
  std::vector<int64_t> uoff;     // [ns+1] offsets of the r x r update matrices on the update stack
                                 // (post-order reuse); uoff[ns] = the stack's peak in entries
  std::vector<int32_t> kid_ptr;  // [ns+1] children of each supernode
  std::vector<int32_t> kids;
  int64_t max_m2 = 0;            // largest front, entries
};

// A is the matrix pattern in the ascending interior numbering (as for
// factor_host).
void build_front_plan(const Symbolic &S, const Csr &A, FrontPlan &fp);

// Device copies of the plan's index arrays.
struct FrontPlanDev {
  const int64_t *a_pos = nullptr, *a_k = nullptr;
  const int32_t *relpos = nullptr;
};

// Factor on `st` into `panel` (FP64 type T = double or cd; layout of
// factor_layout). vals: values on A's pattern (device). front: max_m2
// entries; arena: uoff[ns] entries (may be null when 0); flag: one int32 set
// to 1 on a zero or non-finite pivot (the caller clears and checks it).
// Throws StmgError (STMG_EHIP) when a rocBLAS call fails.
template <typename T>
void factor_device(const Symbolic &S, const FrontPlan &fp, const FrontPlanDev &fd,
                   const std::vector<int64_t> &panel_off, const T *vals, T *panel, T *front, T *arena,
                   int32_t *flag, rocblas_handle rb, hipStream_t st);

// out[e] = (TD) in[e] over all panel entries (may be null), and out_t = the
// per-supernode transposes P_s^T (w x m, column-major; may be null).
template <typename TS, typename TD>
void convert_panels(const TS *in, TD *out, TD *out_t, const int64_t *panel_off_dev, const int32_t *width_dev,
                    int32_t ns, int64_t n_entries, hipStream_t st);

}  // namespace stmg
