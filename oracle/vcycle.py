"""Space-time residual, smoothers, V-cycle and outer solve (oracle, test infrastructure).

Vectors are arrays of shape (N, q, n_e): slab, DG component, interior edge.

* All-at-once system (section 2.1): block lower-bidiagonal L with the slab
  block A = K_t (x) M + M_t (x) K on the diagonal and -N_t (x) M below it.
* Smoother S (eq. (2)): x <- x + omega (I (x) A^{-1}) (f - L x), omega = 0.5,
  with an exact sparse LU of the slab block (the real q*n_e block by default).
* Nodal auxiliary correction (eq. (8)): x <- x + G Sigma_t K_n^{-1} G^T (f - L x).
  Sigma_t is the inverse of the time operator L_t restricted to the gradient
  subspace (block bidiagonal, K_t on the diagonal, -N_t below); for implicit
  Euler it is the running sum over time steps of eq. (8). Here it is applied
  as forward substitution slab by slab.
* Hybrid smoother (section 4): SAS before and after the coarse-grid
  correction; the coarsest level (one slab) is solved exactly. The other
  orders of S and A that section 4 compares (SA, AS, SSA, ASS, SSAS, SSASS)
  are selected with the smoother argument. Section 4 reads a name like a
  product of matrices, right to left (SA = A first, then S), and smooths
  after the coarse-grid correction with the same steps in reversed order:
  the pre-smoother applies the name's letters from the last to the first,
  the post-smoother from the first to the last.
* Inexact slab solves (slab_solver="twogrid:k"): see SlabSolverTwoGrid.
* Inexact nodal solves (section 5 solves the spatial problems approximately,
  with a few preconditioned iterations): with nodal_cheb = k > 0 the K_n^{-1}
  of the nodal correction is replaced by k steps of the Chebyshev iteration
  with Jacobi preconditioning from a zero start (Saad, "Iterative Methods for
  Sparse Linear Systems", 2nd ed., Algorithm 12.1), on the interval
  [lmax / 30, lmax] with lmax the Gershgorin bound max_i sum_j |K_ij| / K_ii
  of D^{-1} K_n (the interval of Adams, Brezina, Hu and Tuminaro, 2003, for
  polynomial smoothers). It is a fixed polynomial in D^{-1} K_n, so the
  V-cycle stays a fixed linear iteration with the same fixed point.
* Power iteration for the convergence rate (section 5.1): zero right-hand side,
  random start in [0, 1], up to 200 cycles, maximum l2 reduction factor, stop
  once the total reduction is below 1e-100.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dgtime import time_matrices, time_prolongation, psi_at
from .hierarchy import build_space_levels, build_level_specs


class SlabSolverReal:
    """Exact solve with the real slab block K_t (x) M + M_t (x) K (sparse LU)."""

    def __init__(self, M, K, Kt, Mt):
        self.q, self.n = Kt.shape[0], M.shape[0]
        A = sp.kron(Kt, M) + sp.kron(Mt, K)
        self.lu = spla.splu(sp.csc_matrix(A))

    def solve(self, r):  # r: (N, q, n)
        N = r.shape[0]
        rhs = r.reshape(N, self.q * self.n).T
        return self.lu.solve(np.ascontiguousarray(rhs)).T.reshape(r.shape)


class SlabSolverComplex:
    """Exact degree-1 slab solve by diagonalising the 2x2 time block.

    M_t^{-1} K_t has eigenvalues mu/tau, conj(mu)/tau with mu = 2 + i sqrt(2),
    so one complex solve with mu M + tau K per slab replaces the real 2n block.
    """

    def __init__(self, M, K, tau):
        self.mu = 2.0 + 1j * np.sqrt(2.0)
        self.lu = spla.splu(sp.csc_matrix(self.mu * M + tau * K, dtype=np.complex128),
                            permc_spec="MMD_AT_PLUS_A")

    def solve(self, r):
        s2 = np.sqrt(2.0)
        w = (0.5 + 1j * s2 / 4) * r[:, 0] - (3j * s2 / 4) * r[:, 1]      # (N, n)
        z = self.lu.solve(np.ascontiguousarray(w.T)).T
        out = np.empty_like(r)
        out[:, 0] = 2.0 * z.real
        out[:, 1] = 2.0 * (z.real - s2 * z.imag)
        return out


def chebyshev_bounds(A):
    """(lmin, lmax) = (lmax / 30, max_i sum_j |A_ij| / A_ii): the Gershgorin
    bound of the spectrum of D^{-1} A and the lower end used for the
    Chebyshev iteration."""
    A = sp.csr_matrix(A)
    lmax = float(np.max(np.asarray(abs(A).sum(axis=1)).ravel() / A.diagonal()))
    return lmax / 30.0, lmax


def chebyshev_solve(A, g, k, bounds=None):
    """k steps of the Jacobi-preconditioned Chebyshev iteration for A y = g
    from y = 0 (Saad, Algorithm 12.1): theta, delta = centre and half-width of
    the interval, sigma = theta / delta; d_0 = D^{-1} g / theta, y_1 = d_0;
    then rho_i = 1 / (2 sigma - rho_{i-1}) (rho_0 = 1 / sigma),
    d_i = rho_i rho_{i-1} d_{i-1} + (2 rho_i / delta) D^{-1} (g - A y_i),
    y_{i+1} = y_i + d_i. The error after k steps is T_k((theta - D^{-1}A) /
    delta) / T_k(sigma) times the initial one. g may hold several right-hand
    sides as columns."""
    lmin, lmax = bounds if bounds is not None else chebyshev_bounds(A)
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta
    dinv = 1.0 / sp.csr_matrix(A).diagonal()
    dinv = dinv.reshape((-1,) + (1,) * (g.ndim - 1))
    rho = 1.0 / sigma
    d = dinv * g / theta
    y = d.copy()
    for _ in range(k - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * (g - A @ y)
        y = y + d
        rho = rho_new
    return y


class SlabSolverTwoGrid:
    """Inexact slab solve (section 5 solves the spatial problems with a few
    preconditioned iterations): k steps of preconditioned Richardson
    iteration from zero, z <- z + B (w - A z), for the spatial operator of
    the slab (A = mu M + tau K with mu = 2 + i sqrt(2) for degree 1, after the
    diagonalisation of the slab's time block; A = M + tau K for degree 0).
    B is one two-grid cycle on the nested meshes: `sweeps` sweeps of a hybrid
    smoother (a damped edge Jacobi step with diag(A), then a Jacobi step on
    the gradients of the nodal space, whose Galerkin operator is
    G^T A G = mu K_n because K G = 0), the correction with the exact solve of
    the Galerkin coarse operator P^T A P = mu M_c + tau K_c, and the same
    sweeps with their steps in reversed order.
    """

    def __init__(self, space, coarse, pt, tau, k, omega_e=0.5, sweeps=2):
        self.pt, self.k, self.omega, self.sweeps = pt, k, omega_e, sweeps
        self.mu = (2.0 + 1j * np.sqrt(2.0)) if pt == 1 else 1.0
        dt = np.complex128 if pt == 1 else np.float64
        self.A = sp.csr_matrix(self.mu * space.M + tau * space.K, dtype=dt)
        self.dinv = 1.0 / self.A.diagonal()
        self.G = sp.csr_matrix(space.G)
        self.dn = self.mu * space.Kn.diagonal()
        self.P = sp.csr_matrix(coarse.Pe)
        Ac = sp.csc_matrix(self.mu * coarse.M + tau * coarse.K, dtype=dt)
        self.lu_c = spla.splu(Ac)

    def _nodal(self, r, z):
        y = (self.G.T @ (r - self.A @ z)) / self.dn[:, None]
        return z + self.G @ y

    def _edge(self, r, z):
        return z + self.omega * self.dinv[:, None] * (r - self.A @ z)

    def precondition(self, r):
        """One two-grid cycle B r (columns of r are right-hand sides)."""
        z = np.zeros_like(r)
        for _ in range(self.sweeps):
            z = self._nodal(r, self._edge(r, z))
        z = z + self.P @ self.lu_c.solve(np.ascontiguousarray(self.P.T @ (r - self.A @ z)))
        for _ in range(self.sweeps):
            z = self._edge(r, self._nodal(r, z))
        return z

    def solve_spatial(self, w):
        z = np.zeros_like(w)
        for _ in range(self.k):
            z = z + self.precondition(w - self.A @ z)
        return z

    def solve(self, r):  # r: (N, q, n) real slab residuals
        s2 = np.sqrt(2.0)
        if self.pt == 1:
            w = (0.5 + 1j * s2 / 4) * r[:, 0] - (3j * s2 / 4) * r[:, 1]      # (N, n)
            z = self.solve_spatial(np.ascontiguousarray(w.T)).T
            out = np.empty_like(r)
            out[:, 0] = 2.0 * z.real
            out[:, 1] = 2.0 * (z.real - s2 * z.imag)
            return out
        z = self.solve_spatial(np.ascontiguousarray(r[:, 0].T)).T
        return z[:, None, :].copy()


class Level:
    def __init__(self, spec, space, pt, slab_solver="real", nodal_cheb=0, coarse_space=None):
        self.spec, self.space, self.pt = spec, space, pt
        self.q = pt + 1
        self.N, self.tau = spec.N, spec.tau
        self.Kt, self.Mt, self.Nt = time_matrices(pt, self.tau)
        M, K = space.M, space.K
        if slab_solver.startswith("twogrid:") and coarse_space is not None:
            self.slab = SlabSolverTwoGrid(space, coarse_space, pt, self.tau, int(slab_solver.split(":")[1]))
        elif slab_solver == "complex" and pt == 1:
            self.slab = SlabSolverComplex(M, K, self.tau)
        else:
            self.slab = SlabSolverReal(M, K, self.Kt, self.Mt)
        self._setup_nodal(nodal_cheb)

    def _setup_nodal(self, nodal_cheb):
        self.nodal_cheb = nodal_cheb
        if nodal_cheb > 0:
            self.Kn_bounds = chebyshev_bounds(self.space.Kn) if self.space.n_v > 0 else None
        else:
            self.Kn_lu = spla.splu(sp.csc_matrix(self.space.Kn))

    @classmethod
    def operator_only(cls, space, pt, N, tau, nodal=False):
        """A level that applies L and its residual but factorises no slab
        block (for checks at sizes where the exact slab factors are too
        costly for the oracle); with nodal=True it also applies the nodal
        correction A (the K_n factor is small)."""
        lev = cls.__new__(cls)
        lev.spec, lev.space, lev.pt = None, space, pt
        lev.q = pt + 1
        lev.N, lev.tau = N, tau
        lev.Kt, lev.Mt, lev.Nt = time_matrices(pt, tau)
        if nodal:
            lev._setup_nodal(0)
        return lev

    # -- operators -------------------------------------------------------
    def apply_L(self, x):
        """(L x)_n = A x_n - (N_t (x) M) x_{n-1}."""
        M, K = self.space.M, self.space.K
        Mx = np.stack([(M @ x[:, k].T).T for k in range(self.q)], axis=1)   # (N,q,n)
        Kx = np.stack([(K @ x[:, k].T).T for k in range(self.q)], axis=1)
        y = np.einsum("lk,nkj->nlj", self.Kt, Mx) + np.einsum("lk,nkj->nlj", self.Mt, Kx)
        y[1:] -= np.einsum("lk,nkj->nlj", self.Nt, Mx[:-1])
        return y

    def residual(self, x, b):
        return b - self.apply_L(x)

    def apply_slab(self, z):
        """(I (x) A) z, A = K_t (x) M + M_t (x) K: the slab block that the
        smoother of eq. (2) inverts, slab by slab."""
        M, K = self.space.M, self.space.K
        Mz = np.stack([(M @ z[:, k].T).T for k in range(self.q)], axis=1)
        Kz = np.stack([(K @ z[:, k].T).T for k in range(self.q)], axis=1)
        return np.einsum("lk,nkj->nlj", self.Kt, Mz) + np.einsum("lk,nkj->nlj", self.Mt, Kz)

    def smooth_S(self, x, b, omega=0.5):
        return x + omega * self.slab.solve(self.residual(x, b))

    def nodal_A(self, x, b):
        r = self.residual(x, b)
        G = self.space.G
        g = np.stack([(G.T @ r[:, k].T).T for k in range(self.q)], axis=1)   # (N,q,nv)
        N, q, nv = g.shape
        if self.nodal_cheb > 0:
            y = chebyshev_solve(self.space.Kn, np.ascontiguousarray(g.reshape(N * q, nv).T), self.nodal_cheb,
                                self.Kn_bounds).T.reshape(N, q, nv)
        else:
            y = self.Kn_lu.solve(np.ascontiguousarray(g.reshape(N * q, nv).T)).T.reshape(N, q, nv)
        # forward substitution with L_t: K_t y_n = y_n + N_t y_{n-1}
        z = np.empty_like(y)
        prev = np.zeros((q, nv))
        for n in range(N):
            z[n] = np.linalg.solve(self.Kt, y[n] + self.Nt @ prev)
            prev = z[n]
        corr = np.stack([(G @ z[:, k].T).T for k in range(q)], axis=1)
        return x + corr

    def smooth_SAS(self, x, b, omega=0.5, use_nodal=True):
        x = self.smooth_S(x, b, omega)
        if use_nodal:
            x = self.nodal_A(x, b)
        return self.smooth_S(x, b, omega)

    def smooth_sequence(self, x, b, seq, omega=0.5):
        """The steps of seq in the order given (first letter first): 'S' =
        damped block Jacobi (eq. (2)), 'A' = nodal auxiliary correction
        (eq. (8)). The V-cycle passes a smoother's name reversed before the
        coarse-grid correction and as written after it (section 4)."""
        for step in seq:
            if step == "S":
                x = self.smooth_S(x, b, omega)
            elif step == "A":
                x = self.nodal_A(x, b)
            else:
                raise ValueError(f"unknown smoother step {step!r}")
        return x

    def solve_exact_single_slab(self, b):
        assert self.N == 1
        return self.slab.solve(b)


class SpaceTimeMultigrid:
    """The oracle solver for one problem (see module docstring)."""

    def __init__(self, problem, lambda_crit=0.1, omega=0.5, slab_solver="real",
                 allow_space=True, use_nodal=True, space_levels=None, smoother=None, nodal_cheb=0):
        self.problem = problem
        self.pt, self.q = problem.pt, problem.pt + 1
        self.omega, self.use_nodal = omega, use_nodal
        # smoother sequence before and after the coarse-grid correction
        # (section 4); None: SAS, or SS without the nodal correction
        self.smoother = smoother
        self.space = space_levels if space_levels is not None else build_space_levels(problem)
        self.specs = build_level_specs(self.space, problem.T, problem.Nt, lambda_crit, allow_space)
        # inexact slab solves ("twogrid:k") use the next coarser mesh; a level
        # on the coarsest mesh, and the one-slab coarsest level, solve exactly
        def coarse_of(spec):
            if spec.N == 1 or spec.space + 1 >= len(self.space):
                return None
            return self.space[spec.space + 1]
        self.levels = [Level(s, self.space[s.space], problem.pt, slab_solver, nodal_cheb, coarse_of(s))
                       for s in self.specs]
        self.Pt = time_prolongation(problem.pt)
        self.fine = self.space[0]

    # -- transfers -------------------------------------------------------
    def restrict(self, l, r):
        """r_c = (P_t^T (x) P_s^T) r from level l to level l+1."""
        fine, coarse = self.levels[l], self.levels[l + 1]
        q = self.q
        if coarse.spec.space != fine.spec.space:
            Ps = self.space[coarse.spec.space].Pe
            r = np.stack([(Ps.T @ r[:, k].T).T for k in range(q)], axis=1)
        Nc = coarse.N
        rc = np.zeros((Nc, q, r.shape[2]))
        for h in range(2):
            blk = self.Pt[h * q:(h + 1) * q]          # [q_fine, q_coarse]
            rc += np.einsum("lk,nlj->nkj", blk, r[h::2])
        return rc

    def prolong(self, l, ec):
        """e = (P_t (x) P_s) e_c from level l+1 to level l."""
        fine, coarse = self.levels[l], self.levels[l + 1]
        q = self.q
        e = np.zeros((fine.N, q, ec.shape[2]))
        for h in range(2):
            blk = self.Pt[h * q:(h + 1) * q]
            e[h::2] = np.einsum("lk,nkj->nlj", blk, ec)
        if coarse.spec.space != fine.spec.space:
            Ps = self.space[coarse.spec.space].Pe
            e = np.stack([(Ps @ e[:, k].T).T for k in range(q)], axis=1)
        return e

    # -- cycle -------------------------------------------------------------
    def vcycle(self, l, x, b):
        lev = self.levels[l]
        if lev.N == 1:
            return lev.solve_exact_single_slab(b)
        x = self._smooth(lev, x, b, pre=True)
        r = lev.residual(x, b)
        rc = self.restrict(l, r)
        ec = self.vcycle(l + 1, np.zeros_like(rc), rc)
        x = x + self.prolong(l, ec)
        return self._smooth(lev, x, b, pre=False)

    def _smooth(self, lev, x, b, pre):
        """Pre-smoothing applies the smoother's name right to left (the
        product reading of section 4), post-smoothing the reversed order."""
        if self.smoother is None:
            return lev.smooth_SAS(x, b, self.omega, self.use_nodal)
        seq = self.smoother[::-1] if pre else self.smoother
        return lev.smooth_sequence(x, b, seq, self.omega)

    # -- ABI-shaped helpers ------------------------------------------------
    def to_interior(self, v_all):
        """(Nt, q, n_edges_all) -> (Nt, q, n_e) interior."""
        return np.ascontiguousarray(np.asarray(v_all)[..., self.fine.ie])

    def to_all(self, v_int):
        out = np.zeros(v_int.shape[:-1] + (self.fine.topo.n_edges,))
        out[..., self.fine.ie] = v_int
        return out

    def fold_initial(self, b, u0_all):
        """Add psi_k(0) M u0 to the first slab (the M u^0 term of eq. (1))."""
        b = b.copy()
        if u0_all is not None:
            Mu0 = self.fine.M @ np.asarray(u0_all)[self.fine.ie]
            b[0] += psi_at(self.pt, 0.0)[:, None] * Mu0[None, :]
        return b

    def residual_norm(self, x, b):
        return float(np.linalg.norm(self.levels[0].residual(x, b)))

    def solve(self, b, x0=None, rtol=1e-8, max_cycles=100):
        """V-cycles from x0 (default 0) until ||b - Lx|| <= rtol ||b||.

        Returns (x, history) with history[k] = ||b - L x_{k+1}|| / ||b||.
        """
        x = np.zeros_like(b) if x0 is None else x0.copy()
        nb = float(np.linalg.norm(b))
        hist = []
        if nb == 0.0:
            return np.zeros_like(b), hist
        for _ in range(max_cycles):
            x = self.vcycle(0, x, b)
            hist.append(self.residual_norm(x, b) / nb)
            if hist[-1] <= rtol:
                break
        return x, hist

    def power_rate(self, seed=0, max_cycles=200, underflow=1e-100):
        """Maximum l2 error-reduction factor over the power iteration."""
        rng = np.random.default_rng(seed)
        lev = self.levels[0]
        x = rng.uniform(0.0, 1.0, size=(lev.N, self.q, self.fine.n_e))
        b = np.zeros_like(x)
        n0 = prev = float(np.linalg.norm(x))
        rates = []
        for _ in range(max_cycles):
            x = self.vcycle(0, x, b)
            nx = float(np.linalg.norm(x))
            rates.append(nx / prev)
            prev = nx
            if nx / n0 < underflow:
                break
        return max(rates), rates


def assemble_global(solver):
    """The whole space-time matrix L of the finest level (for direct solves)."""
    lev = solver.levels[0]
    M, K = lev.space.M, lev.space.K
    A = sp.kron(lev.Kt, M) + sp.kron(lev.Mt, K)
    C = sp.kron(lev.Nt, M)
    N = lev.N
    sub = sp.diags([np.ones(N - 1)], [-1], shape=(N, N))
    return sp.csc_matrix(sp.kron(sp.identity(N), A) - sp.kron(sub, C))


def direct_solve(solver, b):
    """x = L^{-1} b by one sparse LU of the whole space-time system."""
    L = assemble_global(solver)
    x = spla.spsolve(L, b.reshape(-1))
    return x.reshape(b.shape)
