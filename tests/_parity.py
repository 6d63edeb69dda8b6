"""Comparison measures shared by the GPU parity suites (no test functions).

None of these bounds depends on a condition number:

* FWD64 = 1e-10: cap on the forward difference between the GPU's and the
  oracle's result of one step (S, A, SAS, a V-cycle, a slab solve), relative
  to the result, both norm-wise (2-norm) and entry-wise (largest entry
  difference over the largest entry). The two sides run different
  algorithms (complex diagonalised selective-inversion solves against real
  sparse LU), so the bound leaves room for rounding but not for a kernel
  error.
* SPARSE64 = 1e-13: the same for steps that apply sparse operators only
  (residual, transfers): every entry is one short sum in either code.
* Backward error of a solve A z = r (Rigal and Gaches; normwise, infinity
  norms, per right-hand side): max_n |A z_n - r_n| / (|A| |z_n| + |r_n|).
  A backward-stable solve gives a few units of roundoff whatever the
  conditioning of A; BWD64 = 1e-14 (about 45 u) and BWD32 = 1e-6 (about
  17 u in FP32, whose factors are the FP64 ones rounded).
* Smoother step as a solve: S sets x' = x + omega A^{-1}(b - L x), so
  A (x' - x) = omega (b - L x); its backward error takes perturbations of
  x and x' relative to their own size.
* Gradient orthogonality after the nodal correction (eq. (8)): A makes the
  new residual orthogonal to the space-time gradients,
  (I (x) G^T)(b - L x') = 0, measured relative to the same product with
  absolute values (the size of its rounding).
* Residual history: |h_k - h_ref_k| <= 1e-10 h_ref_k + u rho, where
  rho = || |b| + |L| |x| || / ||b|| is the roundoff level of the residual
  norm itself (u = 2^-53). At relative residuals above about 1e-5 the
  1e-10 relative term decides.
"""
import numpy as np
import scipy.sparse as sp

U64 = 2.0 ** -53
FWD64 = 1e-10
SPARSE64 = 1e-13
BWD64 = 1e-14
BWD32 = 1e-6


def rel(a, b):
    """Norm-wise relative difference ||a - b||_2 / ||b||_2."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_inf(a, b):
    """Entry-wise: max |a - b| / max |b|."""
    mb = float(np.abs(b).max()) if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if a.size else 0.0


def fwd(a, b):
    """The larger of the norm-wise and entry-wise relative differences."""
    return max(rel(a, b), rel_inf(a, b))


def slab_matrix(lev):
    """The real slab block K_t (x) M + M_t (x) K of an oracle level."""
    return sp.csr_matrix(sp.kron(lev.Kt, lev.space.M) + sp.kron(lev.Mt, lev.space.K))


def _norm_inf(A):
    return float(abs(A).sum(axis=1).max())


def slab_backward_error(lev, z, r):
    """Per slab n: |A z_n - r_n|_inf / (|A|_inf |z_n|_inf + |r_n|_inf); the max.
    z, r: (N, q, n_e)."""
    A = slab_matrix(lev)
    nA = _norm_inf(A)
    N = z.shape[0]
    zz, rr = z.reshape(N, -1), r.reshape(N, -1)
    res = (A @ zz.T).T - rr
    den = nA * np.abs(zz).max(axis=1) + np.abs(rr).max(axis=1)
    return float((np.abs(res).max(axis=1) / np.where(den > 0, den, 1.0)).max())


def smoother_backward_error(lev, x, b, out, omega=0.5):
    """S as a solve: A (out - x) = omega (b - L x), perturbations of x and out
    relative to their own size (per slab, infinity norms)."""
    A = slab_matrix(lev)
    nA = _norm_inf(A)
    N = x.shape[0]
    r = omega * lev.residual(x, b).reshape(N, -1)
    d = (out - x).reshape(N, -1)
    res = (A @ d.T).T - r
    den = nA * (np.abs(out.reshape(N, -1)).max(axis=1) + np.abs(x.reshape(N, -1)).max(axis=1)) \
        + np.abs(r).max(axis=1)
    return float((np.abs(res).max(axis=1) / np.where(den > 0, den, 1.0)).max())


def _abs_level_residual(lev, x, b):
    """|b| + |L| |x| for an oracle level (the entry-wise size of b - L x)."""
    M, K = abs(lev.space.M), abs(lev.space.K)
    q = lev.q
    ax = np.abs(x)
    Mx = np.stack([(M @ ax[:, k].T).T for k in range(q)], axis=1)
    Kx = np.stack([(K @ ax[:, k].T).T for k in range(q)], axis=1)
    y = np.einsum("lk,nkj->nlj", np.abs(lev.Kt), Mx) + np.einsum("lk,nkj->nlj", np.abs(lev.Mt), Kx)
    y[1:] += np.einsum("lk,nkj->nlj", np.abs(lev.Nt), Mx[:-1])
    return y + np.abs(b)


def gradient_orthogonality(lev, x, b):
    """||(I (x) G^T)(b - L x)|| / ||(I (x) |G|^T)(|b| + |L||x|)||."""
    G = lev.space.G
    r = lev.residual(x, b)
    s = _abs_level_residual(lev, x, b)
    q = lev.q
    g = np.stack([(G.T @ r[:, k].T).T for k in range(q)], axis=1)
    ga = np.stack([(abs(G).T @ s[:, k].T).T for k in range(q)], axis=1)
    den = np.linalg.norm(ga)
    return float(np.linalg.norm(g) / (den if den > 0 else 1.0))


def history_floor(lev, x, b):
    """u rho: roundoff level of ||b - L x|| / ||b|| (rho as in the module doc)."""
    return U64 * float(np.linalg.norm(_abs_level_residual(lev, x, b)) / np.linalg.norm(b))


def backward_error(A, X, B):
    """max over columns j of |A x_j - b_j|_inf / (|A|_inf |x_j|_inf + |b_j|_inf);
    X, B: (n, k) (or (n,)), real or complex."""
    X2 = X.reshape(X.shape[0], -1)
    B2 = B.reshape(B.shape[0], -1)
    res = A @ X2 - B2
    den = _norm_inf(A) * np.abs(X2).max(axis=0) + np.abs(B2).max(axis=0)
    return float((np.abs(res).max(axis=0) / np.where(den > 0, den, 1.0)).max())
