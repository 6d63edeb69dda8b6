// Numeric multifrontal factorisation on the GPU (see factor_dev.hpp).
#include "factor_dev.hpp"

#include <algorithm>
#include <cmath>
#include <string>

namespace stmg {

// ------------------------------------------------------------- host plan
void build_front_plan(const Symbolic &S, const Csr &A, FrontPlan &fp) {
  const int32_t ns = S.ns;
  fp.a_ptr.assign(ns + 1, 0);
  fp.a_pos.clear();
  fp.a_k.clear();
  fp.uoff.assign(ns + 1, 0);
  fp.kid_ptr.assign(ns + 1, 0);
  fp.max_m2 = 1;
  std::vector<int32_t> pos(S.n, -1);
  for (int32_t s = 0; s < ns; ++s) {
    const int64_t w = S.width(s), r = S.nrows(s), m = w + r;
    const int32_t c0 = S.col0[s];
    for (int64_t j = 0; j < w; ++j) pos[c0 + j] = (int32_t)j;
    for (int64_t k = 0; k < r; ++k) pos[S.rows[S.rptr[s] + k]] = (int32_t)(w + k);
    for (int64_t j = 0; j < w; ++j) {
      const int32_t o = S.perm[c0 + j];
      for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k) {
        const int32_t i = S.iperm[A.col[k]];
        if (i < c0 + j) continue;  // lower triangle only
        fp.a_pos.push_back(pos[i] + j * m);
        fp.a_k.push_back(k);
      }
    }
    fp.a_ptr[s + 1] = (int64_t)fp.a_pos.size();
    fp.max_m2 = std::max(fp.max_m2, m * m);
    const bool keeps_update = S.parent[s] >= 0 && r > 0;
    fp.uoff[s + 1] = fp.uoff[s] + (keeps_update ? r * r : 0);
  }
  // children lists (post-order keeps children before parents)
  for (int32_t s = 0; s < ns; ++s)
    if (S.parent[s] >= 0) fp.kid_ptr[S.parent[s] + 1]++;
  for (int32_t s = 0; s < ns; ++s) fp.kid_ptr[s + 1] += fp.kid_ptr[s];
  fp.kids.assign(fp.kid_ptr[ns], 0);
  {
    std::vector<int32_t> nx(fp.kid_ptr.begin(), fp.kid_ptr.end() - 1);
    for (int32_t s = 0; s < ns; ++s)
      if (S.parent[s] >= 0) fp.kids[nx[S.parent[s]]++] = s;
  }
  // The update matrices live on a stack: in post-order the children of a
  // supernode are the top entries when it is assembled, so they are popped
  // and its own update is pushed in their place (the extend-adds read them
  // before the update is written, in stream order). uoff[ns] becomes the
  // stack's peak. A tree whose subtrees are not contiguous keeps one slot per
  // update.
  {
    std::vector<int64_t> off(ns, 0);
    int64_t top = 0, peak = 0;
    bool stack = true;
    for (int32_t s = 0; s < ns && stack; ++s) {
      int64_t base = top, kids_sz = 0;
      for (int32_t q = fp.kid_ptr[s]; q < fp.kid_ptr[s + 1]; ++q) {
        const int32_t ch = fp.kids[q];
        const int64_t rc = S.nrows(ch);
        if (rc == 0) continue;
        base = std::min(base, off[ch]);
        kids_sz += rc * rc;
      }
      stack = top - base == kids_sz;
      top = base;
      off[s] = top;
      const int64_t r = S.nrows(s);
      if (S.parent[s] >= 0 && r > 0) top += r * r;
      peak = std::max(peak, top);
    }
    if (stack) {
      for (int32_t s = 0; s < ns; ++s) fp.uoff[s] = off[s];
      fp.uoff[ns] = peak;
    }
  }
  // update row of s -> row of the parent's front
  fp.relpos.assign(S.rows.size(), 0);
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t p = S.parent[s];
    if (p < 0) continue;
    const int32_t pc0 = S.col0[p], pw = S.width(p);
    const int32_t *pr = S.rows.data() + S.rptr[p], *pe = S.rows.data() + S.rptr[p + 1];
    for (int64_t k = S.rptr[s]; k < S.rptr[s + 1]; ++k) {
      const int32_t g = S.rows[k];
      int32_t at;
      if (g >= pc0 && g < pc0 + pw) {
        at = g - pc0;
      } else {
        const int32_t *it = std::lower_bound(pr, pe, g);
        STMG_REQUIRE(it != pe && *it == g, STMG_EINVAL, "front plan: update row not in the parent's structure");
        at = pw + (int32_t)(it - pr);
      }
      fp.relpos[k] = at;
    }
  }
}

// --------------------------------------------------------------- kernels
namespace {

constexpr int FB = 256;  // threads per block

__device__ inline double f_zero(double) { return 0.0; }
__device__ inline cd f_zero(cd) { return {0.0, 0.0}; }
__device__ inline double f_one(double) { return 1.0; }
__device__ inline cd f_one(cd) { return {1.0, 0.0}; }
__device__ inline double f_add(double a, double b) { return a + b; }
__device__ inline cd f_add(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline double f_mul(double a, double b) { return a * b; }
__device__ inline cd f_mul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline double f_fms(double c, double a, double b) { return c - a * b; }  // c - a b
__device__ inline cd f_fms(cd c, cd a, cd b) {
  return {c.re - (a.re * b.re - a.im * b.im), c.im - (a.re * b.im + a.im * b.re)};
}
__device__ inline double f_recip(double a) { return 1.0 / a; }
__device__ inline cd f_recip(cd a) {
  const double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}
__device__ inline bool f_bad_pivot(double a) { return !(a > 0.0) || !isfinite(a); }
__device__ inline bool f_bad_pivot(cd a) {
  return !isfinite(a.re) || !isfinite(a.im) || (a.re == 0.0 && a.im == 0.0);
}
__device__ inline double f_sqrt(double a) { return sqrt(a); }
// principal square root: Re >= 0, and the sign of Im follows Im(a)
__device__ inline cd f_sqrt(cd a) {
  const double r = hypot(a.re, a.im);
  if (r == 0.0) return {0.0, 0.0};
  if (a.re >= 0.0) {
    const double t = sqrt(0.5 * (r + a.re));
    return {t, a.im / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (r - a.re));
  return {fabs(a.im) / (2.0 * t), copysign(t, a.im)};
}

template <typename T>
__global__ __launch_bounds__(FB) void k_front_zero(T *F, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * FB;
  for (int64_t i = (int64_t)blockIdx.x * FB + threadIdx.x; i < n; i += stride) F[i] = f_zero(T{});
}

// F[pos[e]] += vals[k[e]]; the positions of one front are distinct
template <typename T>
__global__ __launch_bounds__(FB) void k_front_assemble(T *F, const int64_t *pos, const int64_t *kidx, int64_t n,
                                                       const T *vals) {
  const int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (e < n) F[pos[e]] = f_add(F[pos[e]], vals[kidx[e]]);
}

// F[rel[a], rel[b]] += U[a, b] for a >= b (one child's update matrix)
template <typename T>
__global__ __launch_bounds__(FB) void k_extend_add(T *F, int64_t m, const T *U, int32_t r, const int32_t *rel) {
  const int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int32_t a = (int32_t)(e % r), b = (int32_t)(e / r);
  if (a < b) return;
  T *f = F + rel[a] + (int64_t)rel[b] * m;
  *f = f_add(*f, U[e]);
}

// Right-looking L L^T of the kb x kb lower triangle in LDS (leading
// dimension ld), kb <= 64, by the FB threads of a block: lane i (of each of
// the FB / 64 waves) owns row i; per column j every thread takes the pivot,
// wave 0 scales the column, then wave v updates the trailing columns
// c = j + 1 + v, j + 1 + v + FB / 64, ... of its lanes' rows. Every entry
// receives its updates in column order, two barriers per column. A zero or
// non-finite pivot sets *flag and is replaced by 1.
template <typename T>
__device__ void block_chol(T *Ls, int ld, int kb, int32_t *flag) {
  const int i = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < kb; ++j) {
    T p = Ls[j + j * ld];
    const bool bad = f_bad_pivot(p);
    if (bad) p = f_one(T{});
    const T d = f_sqrt(p), dinv = f_recip(d);
    if (wave == 0 && i > j && i < kb) Ls[i + j * ld] = f_mul(Ls[i + j * ld], dinv);
    __syncthreads();  // the scaled column is written and the pivot read by all
    if (wave == 0 && i == j) {
      Ls[j + j * ld] = d;
      if (bad) flag[0] = 1;
    }
    if (i > j && i < kb) {
      const T lij = Ls[i + j * ld];
      for (int c = j + 1 + wave; c <= i; c += FB / 64) Ls[i + c * ld] = f_fms(Ls[i + c * ld], lij, Ls[c + j * ld]);
    }
    __syncthreads();
  }
}

// In-place L L^T of the kb x kb diagonal block at A (ld), kb <= NB, in LDS.
template <typename T>
__global__ __launch_bounds__(FB) void k_diag_chol(T *A, int64_t ld, int kb, int32_t *flag) {
  __shared__ T Ls[NB * NB];
  const int i = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < kb; c += FB / 64)
    if (i < kb) Ls[i + c * kb] = i >= c ? A[i + c * ld] : f_zero(T{});
  __syncthreads();
  block_chol(Ls, kb, kb, flag);
  for (int c = wave; c < kb; c += FB / 64)
    if (i < kb && i >= c) A[i + c * ld] = Ls[i + c * kb];
}

// Fronts with w <= NB: the block factors the w x w diagonal block in LDS
// (block_chol), then inverts the lower triangle in place column by column
// from the last, Linv[i][j] = -(sum_{k=j+1..i} Linv[i][k] L[k][j]) / L[j][j],
// the sum split over the waves (k = j + 1 + v mod FB / 64) and added in a
// fixed order, and writes inv(L11) into the panel's top block (zeros above
// the diagonal).
template <typename T>
__global__ __launch_bounds__(FB) void k_chol_inv_small(const T *F, int64_t m, int w, T *P, int32_t *flag) {
  constexpr int NW = FB / 64;
  __shared__ T Ls[NB * NB];
  __shared__ T part[NW][64];
  const int i = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < w; c += NW)
    if (i < w) Ls[i + c * NB] = i >= c ? F[i + c * m] : f_zero(T{});
  __syncthreads();
  block_chol(Ls, NB, w, flag);
  for (int j = w - 1; j >= 0; --j) {
    T acc = f_zero(T{});
    if (i > j && i < w)
      for (int k = j + 1 + wave; k <= i; k += NW) acc = f_fms(acc, Ls[i + k * NB], Ls[k + j * NB]);
    part[wave][i] = acc;
    __syncthreads();
    if (wave == 0) {
      const T djinv = f_recip(Ls[j + j * NB]);
      T sum = part[0][i];
      for (int v = 1; v < NW; ++v) sum = f_add(sum, part[v][i]);
      if (i > j && i < w) Ls[i + j * NB] = f_mul(sum, djinv);
      if (i == j) Ls[j + j * NB] = djinv;
    }
    __syncthreads();
  }
  for (int c = wave; c < w; c += NW)
    if (i < w) P[i + c * m] = i >= c ? Ls[i + c * NB] : f_zero(T{});
}

// dst (r x w, ld) = src (r x w, ld)
template <typename T>
__global__ __launch_bounds__(FB) void k_copy_block(const T *src, T *dst, int64_t ld, int32_t r, int32_t w) {
  const int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (e >= (int64_t)r * w) return;
  const int32_t a = (int32_t)(e % r), c = (int32_t)(e / r);
  dst[a + c * ld] = src[a + c * ld];
}

// P (w x w, ld) = identity
template <typename T>
__global__ __launch_bounds__(FB) void k_set_identity(T *P, int64_t ld, int32_t w) {
  const int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (e >= (int64_t)w * w) return;
  const int32_t i = (int32_t)(e % w), c = (int32_t)(e / w);
  P[i + c * ld] = i == c ? f_one(T{}) : f_zero(T{});
}

// strict upper triangle of the w x w block at P (ld) = 0
template <typename T>
__global__ __launch_bounds__(FB) void k_zero_upper(T *P, int64_t ld, int32_t w) {
  const int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (e >= (int64_t)w * w) return;
  const int32_t i = (int32_t)(e % w), c = (int32_t)(e / w);
  if (i < c) P[i + c * ld] = f_zero(T{});
}

// U (r x r, lower, ld r) = F[w:, w:] (the update matrix)
template <typename T>
__global__ __launch_bounds__(FB) void k_take_update(const T *F, int64_t m, int32_t w, int32_t r, T *U) {
  const int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int32_t a = (int32_t)(e % r), b = (int32_t)(e / r);
  U[e] = a >= b ? F[(w + a) + (int64_t)(w + b) * m] : f_zero(T{});
}

__device__ inline void cvt(double a, double &b) { b = a; }
__device__ inline void cvt(double a, float &b) { b = (float)a; }
__device__ inline void cvt(cd a, cd &b) { b = a; }
__device__ inline void cvt(cd a, cf &b) { b = {(float)a.re, (float)a.im}; }

// Conversion / transposition of all panels: entry e lies in supernode s
// (binary search over panel_off); P_s is m x w column-major, P_s^T w x m.
template <typename TS, typename TD>
__global__ __launch_bounds__(FB) void k_convert_panels(const TS *in, TD *out, TD *out_t, const int64_t *off,
                                                       const int32_t *width, int32_t ns, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (e >= n) return;
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  TD v;
  cvt(in[e], v);
  if (out) out[e] = v;
  if (out_t) {
    const int64_t w = width[lo], m = (off[lo + 1] - off[lo]) / w, o = e - off[lo];
    const int64_t i = o % m, k = o / m;
    out_t[off[lo] + k + i * w] = v;
  }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + FB - 1) / FB); }

void rb_check(rocblas_status st, const char *what) {
  if (st != rocblas_status_success)
    fail(STMG_EHIP, std::string("rocBLAS ") + what + " failed: " + rocblas_status_to_string(st));
}

// Typed rocBLAS calls (column-major, host-side scalars).
void rb_trsm(rocblas_handle h, rocblas_side sd, rocblas_operation op, int m, int n, const double *A, int lda,
             double *B, int ldb) {
  const double one = 1.0;
  rb_check(rocblas_dtrsm(h, sd, rocblas_fill_lower, op, rocblas_diagonal_non_unit, m, n, &one, A, lda, B, ldb),
           "dtrsm");
}
void rb_trsm(rocblas_handle h, rocblas_side sd, rocblas_operation op, int m, int n, const cd *A, int lda, cd *B,
             int ldb) {
  const rocblas_double_complex one(1.0, 0.0);
  rb_check(rocblas_ztrsm(h, sd, rocblas_fill_lower, op, rocblas_diagonal_non_unit, m, n, &one,
                         reinterpret_cast<const rocblas_double_complex *>(A), lda,
                         reinterpret_cast<rocblas_double_complex *>(B), ldb),
           "ztrsm");
}
void rb_syrk_sub(rocblas_handle h, int n, int k, const double *A, int lda, double *C, int ldc) {
  const double alpha = -1.0, beta = 1.0;
  rb_check(rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, n, k, &alpha, A, lda, &beta, C, ldc),
           "dsyrk");
}
void rb_syrk_sub(rocblas_handle h, int n, int k, const cd *A, int lda, cd *C, int ldc) {
  const rocblas_double_complex alpha(-1.0, 0.0), beta(1.0, 0.0);
  rb_check(rocblas_zsyrk(h, rocblas_fill_lower, rocblas_operation_none, n, k, &alpha,
                         reinterpret_cast<const rocblas_double_complex *>(A), lda, &beta,
                         reinterpret_cast<rocblas_double_complex *>(C), ldc),
           "zsyrk");
}
// C = -B A with A lower triangular (right side)
void rb_trmm_neg(rocblas_handle h, int m, int n, const double *A, int lda, const double *B, int ldb, double *C,
                 int ldc) {
  const double alpha = -1.0;
  rb_check(rocblas_dtrmm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                         rocblas_diagonal_non_unit, m, n, &alpha, A, lda, B, ldb, C, ldc),
           "dtrmm");
}
void rb_trmm_neg(rocblas_handle h, int m, int n, const cd *A, int lda, const cd *B, int ldb, cd *C, int ldc) {
  const rocblas_double_complex alpha(-1.0, 0.0);
  rb_check(rocblas_ztrmm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                         rocblas_diagonal_non_unit, m, n, &alpha, reinterpret_cast<const rocblas_double_complex *>(A),
                         lda, reinterpret_cast<const rocblas_double_complex *>(B), ldb,
                         reinterpret_cast<rocblas_double_complex *>(C), ldc),
           "ztrmm");
}

// C = B A^T with A lower triangular (right side)
void rb_trmm_t(rocblas_handle h, int m, int n, const double *A, int lda, const double *B, int ldb, double *C,
               int ldc) {
  const double alpha = 1.0;
  rb_check(rocblas_dtrmm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                         rocblas_diagonal_non_unit, m, n, &alpha, A, lda, B, ldb, C, ldc),
           "dtrmm");
}
void rb_trmm_t(rocblas_handle h, int m, int n, const cd *A, int lda, const cd *B, int ldb, cd *C, int ldc) {
  const rocblas_double_complex alpha(1.0, 0.0);
  rb_check(rocblas_ztrmm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                         rocblas_diagonal_non_unit, m, n, &alpha, reinterpret_cast<const rocblas_double_complex *>(A),
                         lda, reinterpret_cast<const rocblas_double_complex *>(B), ldb,
                         reinterpret_cast<rocblas_double_complex *>(C), ldc),
           "ztrmm");
}

}  // namespace

template <typename T>
void factor_device(const Symbolic &S, const FrontPlan &fp, const FrontPlanDev &fd,
                   const std::vector<int64_t> &panel_off, const T *vals, T *panel, T *front, T *arena,
                   int32_t *flag, rocblas_handle rb, hipStream_t st) {
  rb_check(rocblas_set_stream(rb, st), "set_stream");
  for (int32_t s = 0; s < S.ns; ++s) {
    const int32_t w = S.width(s), r = S.nrows(s), m = w + r;
    T *F = front;
    // 1. assembly
    hipLaunchKernelGGL(k_front_zero<T>, dim3(std::min<unsigned>(4096, blocks_for((int64_t)m * m))), dim3(FB), 0,
                       st, F, (int64_t)m * m);
    const int64_t na = fp.a_ptr[s + 1] - fp.a_ptr[s];
    if (na > 0)
      hipLaunchKernelGGL(k_front_assemble<T>, dim3(blocks_for(na)), dim3(FB), 0, st, F, fd.a_pos + fp.a_ptr[s],
                         fd.a_k + fp.a_ptr[s], na, vals);
    for (int32_t q = fp.kid_ptr[s]; q < fp.kid_ptr[s + 1]; ++q) {
      const int32_t ch = fp.kids[q], rc = S.nrows(ch);
      if (rc == 0) continue;
      hipLaunchKernelGGL(k_extend_add<T>, dim3(blocks_for((int64_t)rc * rc)), dim3(FB), 0, st, F, (int64_t)m,
                         (const T *)(arena + fp.uoff[ch]), rc, fd.relpos + S.rptr[ch]);
    }
    T *P = panel + panel_off[s];
    if (w <= NB) {
      // small diagonal block: inv(L11) in one kernel, then
      // L21 = F21 inv(L11)^T (into the panel), F22 -= L21 L21^T,
      // W21 = -L21 inv(L11) (into F21's place, then the panel)
      hipLaunchKernelGGL(k_chol_inv_small<T>, dim3(1), dim3(FB), 0, st, (const T *)F, (int64_t)m, w, P, flag);
      if (r > 0) {
        rb_trmm_t(rb, r, w, P, m, F + w, m, P + w, m);
        rb_syrk_sub(rb, r, w, P + w, m, F + w + (int64_t)w * m, m);
        rb_trmm_neg(rb, r, w, P, m, P + w, m, F + w, m);
        hipLaunchKernelGGL(k_copy_block<T>, dim3(blocks_for((int64_t)r * w)), dim3(FB), 0, st, (const T *)(F + w),
                           P + w, (int64_t)m, r, w);
      }
      if (S.parent[s] >= 0 && r > 0)
        hipLaunchKernelGGL(k_take_update<T>, dim3(blocks_for((int64_t)r * r)), dim3(FB), 0, st, (const T *)F,
                           (int64_t)m, w, r, arena + fp.uoff[s]);
      continue;
    }
    // 2. partial factorisation of the first w columns
    for (int32_t k0 = 0; k0 < w; k0 += NB) {
      const int32_t kb = std::min(NB, w - k0), rest = m - k0 - kb;
      T *D = F + k0 + (int64_t)k0 * m;
      hipLaunchKernelGGL(k_diag_chol<T>, dim3(1), dim3(FB), 0, st, D, (int64_t)m, kb, flag);
      if (rest > 0) {
        T *B = F + (k0 + kb) + (int64_t)k0 * m;
        rb_trsm(rb, rocblas_side_right, rocblas_operation_transpose, rest, kb, D, m, B, m);
        rb_syrk_sub(rb, rest, kb, B, m, F + (k0 + kb) + (int64_t)(k0 + kb) * m, m);
      }
    }
    if (S.parent[s] >= 0 && r > 0)
      hipLaunchKernelGGL(k_take_update<T>, dim3(blocks_for((int64_t)r * r)), dim3(FB), 0, st, (const T *)F,
                         (int64_t)m, w, r, arena + fp.uoff[s]);
    // 3. selective inversion into the panel (ld = m)
    hipLaunchKernelGGL(k_set_identity<T>, dim3(blocks_for((int64_t)w * w)), dim3(FB), 0, st, P, (int64_t)m, w);
    rb_trsm(rb, rocblas_side_left, rocblas_operation_none, w, w, F, m, P, m);
    hipLaunchKernelGGL(k_zero_upper<T>, dim3(blocks_for((int64_t)w * w)), dim3(FB), 0, st, P, (int64_t)m, w);
    if (r > 0) rb_trmm_neg(rb, r, w, P, m, F + w, m, P + w, m);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(STMG_EHIP, std::string("factorisation kernels: ") + hipGetErrorString(e));
}

template <typename TS, typename TD>
void convert_panels(const TS *in, TD *out, TD *out_t, const int64_t *panel_off_dev, const int32_t *width_dev,
                    int32_t ns, int64_t n_entries, hipStream_t st) {
  if (n_entries == 0 || (!out && !out_t)) return;
  hipLaunchKernelGGL((k_convert_panels<TS, TD>), dim3(blocks_for(n_entries)), dim3(FB), 0, st, in, out, out_t,
                     panel_off_dev, width_dev, ns, n_entries);
}

template void factor_device<double>(const Symbolic &, const FrontPlan &, const FrontPlanDev &,
                                    const std::vector<int64_t> &, const double *, double *, double *, double *,
                                    int32_t *, rocblas_handle, hipStream_t);
template void factor_device<cd>(const Symbolic &, const FrontPlan &, const FrontPlanDev &,
                                const std::vector<int64_t> &, const cd *, cd *, cd *, cd *, int32_t *,
                                rocblas_handle, hipStream_t);
template void convert_panels<double, double>(const double *, double *, double *, const int64_t *, const int32_t *,
                                             int32_t, int64_t, hipStream_t);
template void convert_panels<double, float>(const double *, float *, float *, const int64_t *, const int32_t *,
                                            int32_t, int64_t, hipStream_t);
template void convert_panels<cd, cd>(const cd *, cd *, cd *, const int64_t *, const int32_t *, int32_t, int64_t,
                                     hipStream_t);
template void convert_panels<cd, cf>(const cd *, cf *, cf *, const int64_t *, const int32_t *, int32_t, int64_t,
                                     hipStream_t);

}  // namespace stmg
