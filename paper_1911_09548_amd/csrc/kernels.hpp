// Device kernels of the space-time V-cycle (launch wrappers, host side).
//
// Internal vector layout: row-major [row][slab][component]; a row holds all
// N*q coefficients of one spatial DOF (an interior edge or vertex), numbered
// in the nested-dissection order of that level's factor. Slab-solve vectors
// hold one scalar per slab (complex for DG degree 1, real for degree 0).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stmg {

// Optional per-launch timing: when a Profiler is attached, launches are
// bracketed by events recorded on their own stream and tagged with their
// kernel name and algorithmic work (implemented by the handle).
struct Profiler {
  void begin(hipStream_t s);
  void end(hipStream_t s, const char *kernel, double flops, double bytes);
  void *impl = nullptr;
};

struct cd {  // complex double
  double re, im;
};
struct cf {  // complex float
  float re, im;
};
// Real scalar type of a (complex or real) scalar type.
template <typename T>
struct RealOf {
  using type = T;
};
template <>
struct RealOf<cd> {
  using type = double;
};
template <>
struct RealOf<cf> {
  using type = float;
};

// Space-time residual of one level (fused SpMM with M and K on their shared
// pattern + DG coupling to the previous slab in the same row).
template <typename R>
struct ResidualArgsT {
  int32_t n_rows;
  int32_t N, q;                 // slabs, components
  const int64_t *ptr;
  const int32_t *col;
  const R *mval, *kval;
  double tau;
  const R *x;                   // may be null: x = 0
  const R *b;
  R *out;
  double *partial;              // may be null: per-block sum of squares of r (FP64)
  int32_t mode;                 // 0: out = r; 1: out = slab-solve right-hand side
  int64_t nnz = 0;              // pattern nonzeros (work accounting only)
  Profiler *prof = nullptr;
  int32_t chunk = 0;            // max values per lane of a row segment (0: default)
  void *halo = nullptr;         // 2 * n_rows values of R: segment-to-segment end values
  const int32_t *sched = nullptr;  // visiting order of the rows (null: storage order)
  // LDS tiles (used when tile_cols is set and chunk == RES_CHUNK_TILES): tile t holds the
  // rows sched[t*RES_TILE ..], the sorted union of their neighbour rows
  // tile_cols[tile_ptr[t] .. tile_ptr[t+1]) and, per nonzero in CSR order,
  // the neighbour's position in that union (lcol)
  const int32_t *tile_ptr = nullptr, *tile_cols = nullptr;
  const uint16_t *lcol = nullptr;
  int32_t tile_union_max = 0, tile_nnz_max = 0;
  // Row groups (used for wide rows when gptr is set): group g holds the rows
  // sched[g*RES_GROUP .. +RES_GROUP) and the sorted union of their neighbour
  // rows, entries e in [gptr[g], gptr[g+1]): gent[2e] = neighbour row,
  // gent[2e+1] = bit mask of the group's rows coupled to it, and
  // gval[(e*RES_GROUP + j)*2 + {0, 1}] = the M and K entries of the group's
  // row j (0 where the mask bit is clear)
  const int32_t *gptr = nullptr, *gent = nullptr;
  const R *gval = nullptr;
};
using ResidualArgs = ResidualArgsT<double>;
constexpr int RES_GROUP = 4;      // rows per wave of the grouped residual
constexpr int RES_CHUNK_DEFAULT = 16;
constexpr int RES_CHUNK_TILES = 32;  // stream_chunk value selecting the LDS-tiled residual
constexpr int RES_TILE = 64;      // rows per LDS tile of the residual
constexpr int RES_TILE_SEG = 16;  // values per row segment staged in LDS
enum { RES_OUT_R = 0, RES_OUT_SLABRHS = 1 };
int residual_blocks(int32_t n_rows, int32_t W, int32_t q, int32_t chunk);
// LDS bytes of one residual tile (staged union segment + matrix entries).
int64_t residual_tile_lds(int32_t union_max, int32_t nnz_max, int32_t scalar_bytes);
// Returns the number of per-block norm partials written (when a.partial).
template <typename R>
int launch_residual(const ResidualArgsT<R> &a, hipStream_t s);

// Sum of `n` doubles in fixed order (deterministic), result at out[0].
void launch_sum(const double *partial, int32_t n, double *out, hipStream_t s);
// Sum of squares of v[0..n) into partial[blocks]; returns number of blocks.
int launch_sumsq(const double *v, int64_t n, double *partial, hipStream_t s);

// Jacobi update x += omega * (time back-transform of z) (eq. (2)).
// q = 2: x0 += omega 2 Re z, x1 += omega 2 (Re z - sqrt2 Im z); q = 1: x += omega z.
// assign != 0: x = (...) instead of +=.
template <typename R>
void launch_slab_update(int32_t n_rows, int32_t N, int32_t q, double omega, const R *z, R *x, int assign,
                        hipStream_t s);
// Slab-solve right-hand side from a residual-layout vector r (no SpMV).
template <typename R>
void launch_slab_rhs(int32_t n_rows, int32_t N, int32_t q, const R *r, R *w, hipStream_t s);

// Nodal correction pieces (eq. (8)).
template <typename R>
void launch_gradT(int32_t n_v, int32_t W, const int64_t *ptr, const int32_t *edge, const int8_t *sign,
                  const R *r, R *g, hipStream_t s);
template <typename R>
void launch_time_scan(int32_t n_v, int32_t N, int32_t q, R *g, hipStream_t s);
template <typename R>
void launch_grad_add(int32_t n_e, int32_t W, const int32_t *head, const int32_t *tail, const R *y, R *x,
                     hipStream_t s);

// One step of the Jacobi-preconditioned Chebyshev iteration for K y = g over
// all W columns of each row (K symmetric in CSR, dinv = 1 / diag K): with y
// null, d = b dinv g and y_out = d; otherwise d = a d + b dinv (g - K y) and
// y_out = y + d (y_out distinct from y).
template <typename R>
void launch_cheb_step(int32_t n, int32_t W, const int64_t *ptr, const int32_t *col, const R *val, const R *dinv,
                      const R *g, const R *y, R *d, R *y_out, double a, double b, hipStream_t s);

// Inexact slab solves (two-grid cycle), on slab-solve vectors of N scalars
// per row (T = cd or cf for DG degree 1, double or float for degree 0; M and
// K values in T's real type):
//   launch_tg_apply: mode 0: out = w - (mu M + tau K) z; mode 1: out = z +
//     omega dinv (w - (mu M + tau K) z) (out distinct from z, may be w);
//     mode 2: out = omega dinv w (z unused); rows visited in the order sched
//     (a permutation of 0..n-1);
//   launch_csr_slabs: y (+)= P x for a CSR matrix P (add != 0 accumulates);
//   launch_scale_slabs: y = diag(d) y.
template <typename T>
void launch_tg_apply(int32_t n, int32_t N, const int32_t *sched, const int64_t *ptr, const int32_t *col,
                     const typename RealOf<T>::type *mval, const typename RealOf<T>::type *kval, T mu, double tau,
                     const T *dinv, double omega, const T *w, const T *z, T *out, int mode, hipStream_t s);
template <typename T>
void launch_csr_slabs(int32_t n, int32_t N, const int64_t *ptr, const int32_t *col, const double *val, const T *x,
                      T *y, int add, hipStream_t s);
template <typename T>
void launch_scale_slabs(int32_t n, int32_t N, const T *d, T *y, hipStream_t s);
// y += x over n reals (R = double or float)
template <typename R>
void launch_tg_axpy(int64_t n, const R *x, R *y, hipStream_t s);

// Space-time transfers. P_s given as CSR (rows: coarse for restrict = P^T,
// fine for prolong = P); the identity when ptr == nullptr (same mesh).
template <typename R>
void launch_restrict(int32_t n_c, int32_t Nc, int32_t q, const int64_t *ptr, const int32_t *col,
                     const double *val, const R *r_f, R *r_c, hipStream_t s);
template <typename R>
void launch_prolong_add(int32_t n_f, int32_t Nc, int32_t q, const int64_t *ptr, const int32_t *col,
                        const double *val, const R *e_c, R *x_f, hipStream_t s);

// Layout changes between ABI vectors [N][q][ncols] and internal [row][N][q];
// map[row] = ABI column of the internal row.
void launch_abi_to_internal(int32_t n_rows, int32_t N, int32_t q, int32_t ncols, const int32_t *map,
                            const double *in, double *out, hipStream_t s);
void launch_internal_to_abi(int32_t n_rows, int32_t N, int32_t q, int32_t ncols, const int32_t *map,
                            const double *in, double *out, hipStream_t s);
// out[0][k][map[e]] += psi_k(0) * (M u0)[e] for the first slab; Mu0 computed
// from u0 given in ABI column order.
void launch_fold_initial(int32_t n_rows, int32_t N, int32_t q, const int64_t *ptr, const int32_t *col,
                         const double *mval, const int32_t *map, const double *u0_abi, double *b,
                         hipStream_t s);

template <typename R>
void launch_fill(R *p, int64_t n, double v, hipStream_t s);
void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s);
// refinement-loop conversions: out = (float) in; out = (double) in; y += (double) x
void launch_to_float(int64_t n, const double *in, float *out, hipStream_t s);
void launch_to_double(int64_t n, const float *in, double *out, hipStream_t s);
void launch_add_float(int64_t n, const float *x, double *y, hipStream_t s);

// ------------------------------------------------------------------ solves
// Multifrontal forward/backward solves with a supernodal L (L L^T = A) for
// `nc` right-hand sides stored as rows of X (one row per matrix row).
struct AsmTarget {
  int64_t dst;             // >= 0: X row; < 0: U row (-1 - index)
  int64_t src_begin;       // into asm_src
};
struct FactorDev {
  int32_t ns, n;
  const int32_t *col0;     // [ns+1]
  const int32_t *m;        // [ns] w + r
  const int64_t *rptr;     // [ns+1]
  const int32_t *rows;
  const int64_t *panel_off;
  const int64_t *uoff;     // [ns] first U row of each supernode
  const void *panel;       // P_s = [inv(L_ss); -L_{R,s} inv(L_ss)], column-major
  const void *panel_t;     // optional P_s^T (w x m, column-major) for the backward solve
  // forward assembly of update rows in the GEMM epilogue: supernode s's
  // update row i is target asm_tgt[uasm[s] + i], whose sources (children's
  // update rows) are asm_src[src_begin .. next target's src_begin)
  const int64_t *uasm;
  const AsmTarget *asm_tgt;
  const int64_t *asm_src;
};
struct SolveTask {          // one row tile of a GEMM launch
  int32_t s;               // supernode
  int32_t rt;              // row tile within the supernode
};
// Kernel launch plan of one factor (all arrays on device, built on the host).
struct SolvePlan {
  // forward assembly per height: targets [tgt_off[h], tgt_off[h+1]); each
  // target's sources [src_begin, next src_begin)
  int32_t n_heights;
  const int64_t *h_tgt_off;      // host [H+1]
  const int64_t *h_src_off;      // host [H+1] first source of each height
  const int64_t *h_xtgt_end;     // host [H] end of the column targets (update-row targets follow)
  const int64_t *h_xsrc_end;     // host [H] end of the column targets' sources
  const AsmTarget *tgt;          // device [n_tgt + 1] (sentinel)
  const int64_t *src;            // device U rows
  // one GEMM launch per height and direction: host descriptors, device tasks
  struct Launch {
    double nnz;                  // factor entries of its supernodes as stored (w(w+1)/2 + r w each)
    double nnz_struct;           // structural nonzeros of L in its supernodes' columns (work accounting)
    int32_t n_tasks;             // supernodes
    int32_t n_tiles, n_tiles32;  // 64-row and 32-row tiles
    int64_t rows;                // output rows over all supernodes
    int32_t kmax;                // longest K range (backward: max m)
    const SolveTask *tasks;      // device, one per 64-row tile
    const SolveTask *tasks32;    // device, one per 32-row tile
  };
  int32_t tile_rows;             // 0: choose per launch; 64 or 32: forced
  int32_t splitk;                // 0 auto, -1 never, >= 2 forced
  Profiler *prof;                // may be null
  void *splitk_ws;               // split-K partial sums (device), may be null
  int64_t splitk_bytes;
  const Launch *fwd;             // host [H]: row tiles over m = w + r
  const Launch *bwd;             // host [H]: row tiles over w
};

template <typename T>
void solve_forward(const FactorDev &f, const SolvePlan &p, int32_t nc, T *X, T *Z, T *U, hipStream_t s);
template <typename T>
void solve_backward(const FactorDev &f, const SolvePlan &p, int32_t nc, T *X, T *Z, hipStream_t s);

// Solves with several factors (one per member) at the same step, merged: one
// launch per tree height and tile shape for up to SOLVE_GROUP_MAX members
// (heights aligned at the leaves for the forward solve, at the roots for the
// backward solve). Bitwise the same results as separate solves; the plans'
// profilers are not used.
constexpr int SOLVE_GROUP_MAX = 8;
template <typename T>
struct SolveMember {
  const FactorDev *f;
  const SolvePlan *p;
  int32_t nc;
  T *X, *Z, *U;
};
template <typename T>
void solve_forward_group(const SolveMember<T> *m, int n, hipStream_t s);
template <typename T>
void solve_backward_group(const SolveMember<T> *m, int n, hipStream_t s);

}  // namespace stmg
