// HIP kernels for gfx950 of the inexact slab solves (two-grid Richardson
// steps, the inexact spatial solves of section 5). Every kernel streams slab
// vectors of the internal layout (one row per spatial DOF holding its N slab
// scalars: complex pairs for DG degree 1, reals for degree 0), a thread per
// (row, slab), so consecutive lanes read consecutive scalars of a row and the
// sparse rows' neighbours are N-scalar strided gathers.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace stmg {

namespace {

constexpr int BLOCK = 256;

// Blocks are dispatched round-robin over the 8 XCDs; each XCD takes a
// contiguous range of logical blocks, so the rows it has in flight (visited
// in a space-filling-curve order) form a compact patch of the mesh whose
// neighbour rows are gathered while still in its L2.
__device__ inline int64_t xcd_block(int64_t bid, int64_t nblocks) {
  const int64_t x = bid & 7, idx = bid >> 3;
  const int64_t per = nblocks >> 3, rem = nblocks & 7;
  return x * per + (x < rem ? x : rem) + idx;
}

// The spatial operator of a slab, A = mu M + tau K, on slab-solve vectors
// (one scalar per slab and row: complex for DG degree 1, real for degree 0),
// M and K on their shared pattern in the level's internal numbering. A
// thread per (row, slab):
//   mode 0: out = w - A z;
//   mode 1: out = z + omega dinv (w - A z)   (a damped Jacobi step; out != z,
//           out may be w: w is read at the thread's own entry only);
//   mode 2: out = omega dinv w               (the same step from z = 0; z unused).
__device__ inline double cmul(double a, double b) { return a * b; }
__device__ inline float cmul(float a, float b) { return a * b; }
__device__ inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cf cmul(cf a, cf b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline double cadd(double a, double b) { return a + b; }
__device__ inline float cadd(float a, float b) { return a + b; }
__device__ inline cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cf cadd(cf a, cf b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline double csub(double a, double b) { return a - b; }
__device__ inline float csub(float a, float b) { return a - b; }
__device__ inline cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cf csub(cf a, cf b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline double cscale(double a, double s) { return a * s; }
__device__ inline float cscale(float a, float s) { return a * s; }
__device__ inline cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }
__device__ inline cf cscale(cf a, float s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ inline T czero() {
  return T{};
}

// Rows are visited in the order sched[] (a permutation of the rows), four
// nonzeros per step with their loads issued before the first FMA. WIDE (N a
// multiple of 64): a wavefront lies within one row, whose index is then
// wave-uniform, so the pattern and matrix values are scalar loads. (Two slab
// scalars per thread measured 7% slower at N = 256.)
template <typename T, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_tg_apply(int32_t n, int32_t N, const int32_t *sched, const int64_t *ptr,
                                                    const int32_t *col, const typename RealOf<T>::type *mval,
                                                    const typename RealOf<T>::type *kval, T mu,
                                                    typename RealOf<T>::type tau, const T *dinv,
                                                    typename RealOf<T>::type omega, const T *w, const T *z, T *out,
                                                    int mode) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= (int64_t)n * N) return;
  const int32_t slot = (int32_t)(i / N), c = (int32_t)(i % N);
  int32_t row = sched[slot];
  if constexpr (WIDE) row = __builtin_amdgcn_readfirstlane(row);
  const int64_t off = (int64_t)row * N + c;
  if (mode == 2) {
    out[off] = cscale(cmul(dinv[row], w[off]), omega);
    return;
  }
  T mz = czero<T>(), kz = czero<T>();
  const int64_t k1 = ptr[row + 1];
  int64_t k = ptr[row];
  for (; k + 4 <= k1; k += 4) {
    const int32_t j0 = col[k], j1 = col[k + 1], j2 = col[k + 2], j3 = col[k + 3];
    const T z0 = z[(int64_t)j0 * N + c], z1 = z[(int64_t)j1 * N + c];
    const T z2 = z[(int64_t)j2 * N + c], z3 = z[(int64_t)j3 * N + c];
    mz = cadd(mz, cscale(z0, mval[k]));
    kz = cadd(kz, cscale(z0, kval[k]));
    mz = cadd(mz, cscale(z1, mval[k + 1]));
    kz = cadd(kz, cscale(z1, kval[k + 1]));
    mz = cadd(mz, cscale(z2, mval[k + 2]));
    kz = cadd(kz, cscale(z2, kval[k + 2]));
    mz = cadd(mz, cscale(z3, mval[k + 3]));
    kz = cadd(kz, cscale(z3, kval[k + 3]));
  }
  for (; k < k1; ++k) {
    const T zv = z[(int64_t)col[k] * N + c];
    mz = cadd(mz, cscale(zv, mval[k]));
    kz = cadd(kz, cscale(zv, kval[k]));
  }
  const T r = csub(w[off], cadd(cmul(mu, mz), cscale(kz, tau)));
  out[off] = mode == 0 ? r : cadd(z[off], cscale(cmul(dinv[row], r), omega));
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_tg_axpy(int64_t n, const R *x, R *y) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) y[i] += x[i];
}

// y[row] (+)= sum_k val[k] x[col[k]] for the N slab scalars of each row (a
// spatial transfer P or P^T in CSR), add != 0 accumulates into y.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_csr_slabs(int32_t n, int32_t N, const int64_t *ptr, const int32_t *col,
                                                     const double *val, const T *x, T *y, int add) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n * N) return;
  const int32_t row = (int32_t)(i / N), c = (int32_t)(i % N);
  using Rv = typename RealOf<T>::type;
  T acc = czero<T>();
  const int64_t k1 = ptr[row + 1];
  for (int64_t k = ptr[row]; k < k1; ++k) acc = cadd(acc, cscale(x[(int64_t)col[k] * N + c], (Rv)val[k]));
  const int64_t off = (int64_t)row * N + c;
  y[off] = add ? cadd(y[off], acc) : acc;
}

// y[row] = d[row] y[row] for the N slab scalars of each row.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_scale_slabs(int32_t n, int32_t N, const T *d, T *y) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n * N) return;
  y[i] = cmul(d[i / N], y[i]);
}

}  // namespace

template <typename T>
void launch_tg_apply(int32_t n, int32_t N, const int32_t *sched, const int64_t *ptr, const int32_t *col,
                     const typename RealOf<T>::type *mval, const typename RealOf<T>::type *kval, T mu, double tau,
                     const T *dinv, double omega, const T *w, const T *z, T *out, int mode, hipStream_t s) {
  using Rv = typename RealOf<T>::type;
  const int64_t nt = (int64_t)n * N;
  if (nt == 0) return;
  const dim3 grid((unsigned)((nt + BLOCK - 1) / BLOCK));
  if (N % 64 == 0)
    hipLaunchKernelGGL((k_tg_apply<T, true>), grid, dim3(BLOCK), 0, s, n, N, sched, ptr, col, mval, kval, mu, (Rv)tau,
                       dinv, (Rv)omega, w, z, out, mode);
  else
    hipLaunchKernelGGL((k_tg_apply<T, false>), grid, dim3(BLOCK), 0, s, n, N, sched, ptr, col, mval, kval, mu,
                       (Rv)tau, dinv, (Rv)omega, w, z, out, mode);
}
template <typename R>
void launch_tg_axpy(int64_t n, const R *x, R *y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_tg_axpy<R>), dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n, x, y);
}
template <typename T>
void launch_csr_slabs(int32_t n, int32_t N, const int64_t *ptr, const int32_t *col, const double *val, const T *x,
                      T *y, int add, hipStream_t s) {
  const int64_t nt = (int64_t)n * N;
  if (nt == 0) return;
  hipLaunchKernelGGL((k_csr_slabs<T>), dim3((unsigned)((nt + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n, N, ptr,
                     col, val, x, y, add);
}
template <typename T>
void launch_scale_slabs(int32_t n, int32_t N, const T *d, T *y, hipStream_t s) {
  const int64_t nt = (int64_t)n * N;
  if (nt == 0) return;
  hipLaunchKernelGGL((k_scale_slabs<T>), dim3((unsigned)((nt + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n, N, d, y);
}
#define TG_INST(T)                                                                                             \
  template void launch_tg_apply<T>(int32_t, int32_t, const int32_t *, const int64_t *, const int32_t *,        \
                                   const typename RealOf<T>::type *, const typename RealOf<T>::type *, T,      \
                                   double, const T *, double, const T *, const T *, T *, int, hipStream_t);    \
  template void launch_csr_slabs<T>(int32_t, int32_t, const int64_t *, const int32_t *, const double *,        \
                                    const T *, T *, int, hipStream_t);                                         \
  template void launch_scale_slabs<T>(int32_t, int32_t, const T *, T *, hipStream_t);
TG_INST(double)
TG_INST(cd)
TG_INST(float)
TG_INST(cf)
#undef TG_INST
template void launch_tg_axpy<double>(int64_t, const double *, double *, hipStream_t);
template void launch_tg_axpy<float>(int64_t, const float *, float *, hipStream_t);

}  // namespace stmg
