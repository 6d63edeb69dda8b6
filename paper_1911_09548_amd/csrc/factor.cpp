// Host multifrontal L L^T factorisation (real SPD or complex symmetric).
#include "factor.hpp"

#include <algorithm>
#include <cmath>
#include <complex>

namespace stmg {

namespace {

inline double sq_root(double a) { return std::sqrt(a); }
inline cplx sq_root(cplx a) {
  std::complex<double> z = std::sqrt(std::complex<double>(a.re, a.im));
  return {z.real(), z.imag()};
}
inline bool bad_pivot(double a) { return !(a > 0.0) || !std::isfinite(a); }
inline bool bad_pivot(cplx a) {
  return !std::isfinite(a.re) || !std::isfinite(a.im) || (a.re == 0.0 && a.im == 0.0);
}
inline double zero(double) { return 0.0; }
inline cplx zero(cplx) { return {0.0, 0.0}; }
inline void add_to(double &a, double b) { a += b; }
inline void add_to(cplx &a, cplx b) {
  a.re += b.re;
  a.im += b.im;
}
inline double mul(double a, double b) { return a * b; }
inline cplx mul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline double recip(double a) { return 1.0 / a; }
inline cplx recip(cplx a) {
  double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}
inline double neg(double a) { return -a; }
inline cplx neg(cplx a) { return {-a.re, -a.im}; }

// y[i] -= x[i] * a for i in [0, n)
inline void axpy_sub(int64_t n, const double *x, double a, double *y) {
  for (int64_t i = 0; i < n; ++i) y[i] -= x[i] * a;
}
inline void axpy_sub(int64_t n, const cplx *x, cplx a, cplx *y) {
  for (int64_t i = 0; i < n; ++i) {
    double xr = x[i].re, xi = x[i].im;
    y[i].re -= xr * a.re - xi * a.im;
    y[i].im -= xr * a.im + xi * a.re;
  }
}
// y[i] -= x0[i] a0 + x1[i] a1 + x2[i] a2 + x3[i] a3
inline void axpy4_sub(int64_t n, const double *x0, const double *x1, const double *x2,
                      const double *x3, double a0, double a1, double a2, double a3, double *y) {
  for (int64_t i = 0; i < n; ++i) y[i] -= x0[i] * a0 + x1[i] * a1 + x2[i] * a2 + x3[i] * a3;
}
inline void axpy4_sub(int64_t n, const cplx *x0, const cplx *x1, const cplx *x2, const cplx *x3,
                      cplx a0, cplx a1, cplx a2, cplx a3, cplx *y) {
  for (int64_t i = 0; i < n; ++i) {
    double re = x0[i].re * a0.re - x0[i].im * a0.im + x1[i].re * a1.re - x1[i].im * a1.im +
                x2[i].re * a2.re - x2[i].im * a2.im + x3[i].re * a3.re - x3[i].im * a3.im;
    double im = x0[i].re * a0.im + x0[i].im * a0.re + x1[i].re * a1.im + x1[i].im * a1.re +
                x2[i].re * a2.im + x2[i].im * a2.re + x3[i].re * a3.im + x3[i].im * a3.re;
    y[i].re -= re;
    y[i].im -= im;
  }
}

// Partial factorisation of the first w columns of the m x m front F
// (column-major, ld = m, lower triangle). Columns >= w receive the Schur
// complement update.
template <typename T>
void partial_factor(int64_t m, int64_t w, T *F) {
  for (int64_t k0 = 0; k0 < w; k0 += NB) {
    int64_t kb = std::min<int64_t>(NB, w - k0);
    for (int64_t j = k0; j < k0 + kb; ++j) {
      T *cj = F + j * m;
      if (bad_pivot(cj[j])) fail(STMG_ENUMERIC, "zero or non-finite pivot in factorisation");
      T d = sq_root(cj[j]);
      cj[j] = d;
      T dinv = recip(d);
      for (int64_t i = j + 1; i < m; ++i) cj[i] = mul(cj[i], dinv);
      for (int64_t jj = j + 1; jj < k0 + kb; ++jj) axpy_sub(m - jj, cj + jj, cj[jj], F + jj * m + jj);
    }
    // trailing update of columns jj >= k0 + kb by the kb columns of this block
    int64_t ncol = m - (k0 + kb);
#pragma omp parallel for schedule(dynamic, 8) if (ncol * (m - k0) > 200000)
    for (int64_t jj = k0 + kb; jj < m; ++jj) {
      T *y = F + jj * m + jj;
      int64_t len = m - jj;
      int64_t t = k0;
      for (; t + 4 <= k0 + kb; t += 4) {
        const T *x0 = F + t * m + jj, *x1 = F + (t + 1) * m + jj, *x2 = F + (t + 2) * m + jj,
                *x3 = F + (t + 3) * m + jj;
        axpy4_sub(len, x0, x1, x2, x3, x0[0], x1[0], x2[0], x3[0], y);
      }
      for (; t < k0 + kb; ++t) {
        const T *x = F + t * m + jj;
        axpy_sub(len, x, x[0], y);
      }
    }
  }
}

// Replace the panel [L11; L21] (m x w, ld = m) by [inv(L11); -L21 inv(L11)].
// Column c of inv(L11) is L11^{-1} e_c (column-oriented forward
// substitution); then W21 = -L21 inv(L11) column by column:
// W21[:, j] = -sum_{k >= j} L21[:, k] inv(L11)[k, j].
template <typename T>
void invert_panel(int64_t m, int64_t w, T *P) {
  std::vector<T> Li(w * w, zero(T{}));
#pragma omp parallel for schedule(dynamic, 4) if (w > 96)
  for (int64_t c = 0; c < w; ++c) {
    T *x = Li.data() + c * w;
    x[c] = recip(P[c + c * m]);
    for (int64_t j = c; j < w; ++j) {
      if (j > c) x[j] = mul(x[j], recip(P[j + j * m]));
      // x[j+1:w] -= x_j * L[j+1:w, j]
      const T xj = x[j];
      axpy_sub(w - j - 1, P + j * m + j + 1, xj, x + j + 1);
    }
  }
  const int64_t r = m - w;
  std::vector<T> W(r * w, zero(T{}));
#pragma omp parallel for schedule(dynamic, 4) if (r * w > 4096)
  for (int64_t j = 0; j < w; ++j) {
    T *y = W.data() + j * r;
    for (int64_t k = j; k < w; ++k) axpy_sub(r, P + k * m + w, Li[k + j * w], y);  // y -= L21[:,k] Li[k,j]
  }
  for (int64_t j = 0; j < w; ++j) {
    std::copy(Li.begin() + j * w, Li.begin() + (j + 1) * w, P + j * m);
    std::copy(W.begin() + j * r, W.begin() + (j + 1) * r, P + j * m + w);
  }
}

}  // namespace

void factor_layout(const Symbolic &S, std::vector<int64_t> &panel_off) {
  panel_off.assign(S.ns + 1, 0);
  for (int32_t s = 0; s < S.ns; ++s) {
    int64_t w = S.width(s), m = w + S.nrows(s);
    panel_off[s + 1] = panel_off[s] + m * w;
  }
}

template <typename T>
void factor_host(const Symbolic &S, const Csr &A, const std::vector<T> &vals, HostFactor<T> &Fo) {
  alloc_point("host factor panels");
  STMG_REQUIRE((int64_t)vals.size() == A.nnz(), STMG_EINVAL, "factor: value count mismatch");
  Fo.sym = &S;
  factor_layout(S, Fo.panel_off);
  Fo.panel.assign(Fo.panel_off[S.ns], zero(T{}));
  std::vector<std::vector<T>> U(S.ns);   // update matrices waiting for their parent
  std::vector<std::vector<int32_t>> kids(S.ns);
  for (int32_t s = 0; s < S.ns; ++s)
    if (S.parent[s] >= 0) kids[S.parent[s]].push_back(s);
  std::vector<int32_t> pos(S.n, -1);
  std::vector<T> F;
  for (int32_t s = 0; s < S.ns; ++s) {
    const int64_t w = S.width(s), r = S.nrows(s), m = w + r;
    const int32_t c0 = S.col0[s];
    for (int64_t j = 0; j < w; ++j) pos[c0 + j] = (int32_t)j;
    for (int64_t k = 0; k < r; ++k) pos[S.rows[S.rptr[s] + k]] = (int32_t)(w + k);
    F.assign(m * m, zero(T{}));
    for (int64_t j = 0; j < w; ++j) {
      int32_t o = S.perm[c0 + j];
      for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k) {
        int32_t i = S.iperm[A.col[k]];
        if (i < c0 + j) continue;  // lower triangle only
        add_to(F[j * m + pos[i]], vals[k]);
      }
    }
    for (int32_t ch : kids[s]) {
      const int64_t rc = S.nrows(ch);
      const int32_t *Rc = &S.rows[S.rptr[ch]];
      const T *Uc = U[ch].data();
      for (int64_t b = 0; b < rc; ++b) {
        int64_t pb = pos[Rc[b]];
        for (int64_t a = b; a < rc; ++a) add_to(F[pb * m + pos[Rc[a]]], Uc[b * rc + a]);
      }
      std::vector<T>().swap(U[ch]);
    }
    partial_factor<T>(m, w, F.data());
    T *P = Fo.panel.data() + Fo.panel_off[s];
    std::copy(F.begin(), F.begin() + m * w, P);
    if (r > 0 && S.parent[s] >= 0) {
      U[s].resize(r * r);
      for (int64_t b = 0; b < r; ++b)
        std::copy(F.begin() + (w + b) * m + w, F.begin() + (w + b) * m + m, U[s].begin() + b * r);
    }
    invert_panel<T>(m, w, P);
  }
}

template void factor_host<double>(const Symbolic &, const Csr &, const std::vector<double> &,
                                  HostFactor<double> &);
template void factor_host<cplx>(const Symbolic &, const Csr &, const std::vector<cplx> &,
                                HostFactor<cplx> &);

}  // namespace stmg
