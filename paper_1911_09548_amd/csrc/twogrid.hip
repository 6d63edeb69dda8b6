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

// The spatial operator of a slab, A = mu M + tau K, on slab-solve vectors
// (one scalar per slab and row: complex for DG degree 1, real for degree 0),
// M and K on their shared pattern in the level's internal numbering. A
// thread per (row, slab):
//   mode 0: out = w - A z;
//   mode 1: out = z + omega dinv (w - A z)   (a damped Jacobi step; out != z,
//           out may be w: w is read at the thread's own entry only);
//   mode 2: out = omega dinv w               (the same step from z = 0; z unused).
template <typename T>
__device__ inline T cmul(T a, T b);
template <>
__device__ inline double cmul(double a, double b) { return a * b; }
template <>
__device__ inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline double cadd(double a, double b) { return a + b; }
__device__ inline cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline double csub(double a, double b) { return a - b; }
__device__ inline cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline double cscale(double a, double s) { return a * s; }
__device__ inline cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }
__device__ inline double czero(double) { return 0.0; }
__device__ inline cd czero(cd) { return {0.0, 0.0}; }

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_tg_apply(int32_t n, int32_t N, const int64_t *ptr, const int32_t *col,
                                                    const double *mval, const double *kval, T mu, double tau,
                                                    const T *dinv, double omega, const T *w, const T *z, T *out,
                                                    int mode) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n * N) return;
  const int32_t row = (int32_t)(i / N), c = (int32_t)(i % N);
  const int64_t off = (int64_t)row * N + c;
  if (mode == 2) {
    out[off] = cscale(cmul(dinv[row], w[off]), omega);
    return;
  }
  T mz = czero(T{}), kz = czero(T{});
  const int64_t k1 = ptr[row + 1];
  for (int64_t k = ptr[row]; k < k1; ++k) {
    const T zv = z[(int64_t)col[k] * N + c];
    mz = cadd(mz, cscale(zv, mval[k]));
    kz = cadd(kz, cscale(zv, kval[k]));
  }
  const T r = csub(w[off], cadd(cmul(mu, mz), cscale(kz, tau)));
  out[off] = mode == 0 ? r : cadd(z[off], cscale(cmul(dinv[row], r), omega));
}

// y[row] (+)= sum_k val[k] x[col[k]] for the N slab scalars of each row (a
// spatial transfer P or P^T in CSR), add != 0 accumulates into y.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_csr_slabs(int32_t n, int32_t N, const int64_t *ptr, const int32_t *col,
                                                     const double *val, const T *x, T *y, int add) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n * N) return;
  const int32_t row = (int32_t)(i / N), c = (int32_t)(i % N);
  T acc = czero(T{});
  const int64_t k1 = ptr[row + 1];
  for (int64_t k = ptr[row]; k < k1; ++k) acc = cadd(acc, cscale(x[(int64_t)col[k] * N + c], val[k]));
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
void launch_tg_apply(int32_t n, int32_t N, const int64_t *ptr, const int32_t *col, const double *mval,
                     const double *kval, T mu, double tau, const T *dinv, double omega, const T *w, const T *z,
                     T *out, int mode, hipStream_t s) {
  const int64_t nt = (int64_t)n * N;
  if (nt == 0) return;
  hipLaunchKernelGGL((k_tg_apply<T>), dim3((unsigned)((nt + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n, N, ptr,
                     col, mval, kval, mu, tau, dinv, omega, w, z, out, mode);
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
  template void launch_tg_apply<T>(int32_t, int32_t, const int64_t *, const int32_t *, const double *,         \
                                   const double *, T, double, const T *, double, const T *, const T *, T *, int, \
                                   hipStream_t);                                                               \
  template void launch_csr_slabs<T>(int32_t, int32_t, const int64_t *, const int32_t *, const double *,        \
                                    const T *, T *, int, hipStream_t);                                         \
  template void launch_scale_slabs<T>(int32_t, int32_t, const T *, T *, hipStream_t);
TG_INST(double)
TG_INST(cd)
#undef TG_INST

}  // namespace stmg
