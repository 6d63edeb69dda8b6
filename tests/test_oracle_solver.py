"""Pins of the oracle's smoother, nodal correction and V-cycle.

* The V-cycle's fixed point is the solution of the whole space-time system,
  computed here by one sparse LU of L (brute force on tiny meshes).
* The complex diagonalised slab solve equals the real 2n block solve.
* On one slab the damped block-Jacobi smoother contracts the error by exactly
  1 - omega (eq. (2)).
* The nodal correction (eq. (8)) is a Galerkin projection on the space-time
  gradient subspace: it solves pure-gradient errors exactly and leaves a
  residual with G^T r = 0; its time solve equals the closed-form prefix sum.
* Rates: pure time coarsening with exact solves stays below 0.5 (section 3.1);
  spatial coarsening without the nodal correction is ineffective (section 3.1,
  rate near 1) and works again with it (section 3.4/4).
* Manufactured solution: the discretisation error falls under refinement.
* Smoother orders (section 4): SAS through the sequence path is the same
  arithmetic as the SAS smoother; every order's V-cycle converges to the
  direct solution and contracts the error; a name is applied right to left
  before the coarse-grid correction and in reversed order after it.
* Transfers: restriction after the fine operator after prolongation is the
  coarse operator (R L_f P = L_c), assembled column by column from unit
  vectors, on a level pair that coarsens in space and time and on one that
  coarsens in time only.
"""
import numpy as np
import pytest

from paper_1911_09548_amd import inputs
from oracle.vcycle import SpaceTimeMultigrid, direct_solve, SlabSolverReal, SlabSolverComplex
from oracle.manufactured import manufactured_problem, end_value
from oracle.dgtime import time_matrices


def _solver(n=4, Nt=16, pt=1, **kw):
    prob = inputs.config_block_random(n=n, Nt=Nt, pt=pt, seed=11, block_hexes=max(1, n // 2))
    return SpaceTimeMultigrid(prob, **kw)


@pytest.mark.parametrize("pt", [0, 1])
@pytest.mark.parametrize("n,Nt", [(2, 4), (4, 8), (4, 16)])
def test_vcycle_converges_to_direct_solution(n, Nt, pt):
    s = _solver(n, Nt, pt)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((Nt, pt + 1, s.fine.n_e))
    x, hist = s.solve(b, rtol=1e-12, max_cycles=60)
    xd = direct_solve(s, b)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_complex_slab_solve_equals_real_block():
    s = _solver(4, 2, 1)
    lev = s.levels[0]
    real = SlabSolverReal(lev.space.M, lev.space.K, lev.Kt, lev.Mt)
    cplx = SlabSolverComplex(lev.space.M, lev.space.K, lev.tau)
    r = np.random.default_rng(0).standard_normal((3, 2, s.fine.n_e))
    a, b = real.solve(r), cplx.solve(r)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


def test_single_slab_smoother_contracts_by_one_minus_omega():
    s = _solver(4, 1, 1)
    lev = s.levels[0]
    rng = np.random.default_rng(1)
    b = rng.standard_normal((1, 2, s.fine.n_e))
    xs = lev.solve_exact_single_slab(b)
    x = np.zeros_like(b)
    for k in range(3):
        x = lev.smooth_S(x, b, 0.5)
        assert np.allclose(xs - x, 0.5 ** (k + 1) * xs, atol=1e-12 * np.abs(xs).max())


@pytest.mark.parametrize("pt", [0, 1])
def test_nodal_correction_solves_gradient_errors(pt):
    s = _solver(4, 8, pt)
    lev = s.levels[0]
    rng = np.random.default_rng(2)
    phi = rng.standard_normal((lev.N, pt + 1, s.fine.n_v))
    u = np.stack([(s.fine.G @ phi[:, k].T).T for k in range(pt + 1)], axis=1)
    b = lev.apply_L(u)
    x = lev.nodal_A(np.zeros_like(b), b)
    assert np.linalg.norm(x - u) <= 1e-11 * np.linalg.norm(u)
    # after A on a general residual, G^T r = 0
    b = rng.standard_normal(b.shape)
    x0 = rng.standard_normal(b.shape)
    x = lev.nodal_A(x0, b)
    r = lev.residual(x, b)
    gr = np.stack([(s.fine.G.T @ r[:, k].T).T for k in range(pt + 1)], axis=1)
    assert np.linalg.norm(gr) <= 1e-11 * np.linalg.norm(b)


def test_time_solve_equals_prefix_sum_formula():
    """Forward substitution with L_t (K_t diagonal, -N_t below) against the
    closed form y_{n,0} = e_{n-1} + (g0 - g1)/2, y_{n,1} = (g0 + g1)/2 with
    e_n = sum_{m <= n} g_{m,0}; and against the plain running sum for degree 0."""
    rng = np.random.default_rng(4)
    N, nv = 7, 5
    for pt in (0, 1):
        q = pt + 1
        Kt, _, Nt = time_matrices(pt, 0.3)
        g = rng.standard_normal((N, q, nv))
        z = np.empty_like(g)
        prev = np.zeros((q, nv))
        for n in range(N):
            z[n] = np.linalg.solve(Kt, g[n] + Nt @ prev)
            prev = z[n]
        if pt == 0:
            ref = np.cumsum(g, axis=0)
        else:
            e = np.cumsum(g[:, 0], axis=0)
            ref = np.empty_like(g)
            ref[:, 0] = np.concatenate([np.zeros((1, nv)), e[:-1]]) + 0.5 * (g[:, 0] - g[:, 1])
            ref[:, 1] = 0.5 * (g[:, 0] + g[:, 1])
        assert np.allclose(z, ref, atol=1e-14)


def test_config1_hierarchy_follows_coarsening_rule():
    prob = inputs.config_unit_manufactured(4, 16, 1)
    s = SpaceTimeMultigrid(prob)
    ns = [prob.levels[sp_.space].n for sp_ in s.specs]
    assert list(zip(ns, [sp_.N for sp_ in s.specs])) == [(4, 16), (2, 8), (2, 4), (2, 2), (2, 1)]
    # lambda at the finest level: tau n^2 / 3 with h_T = sqrt(3)/n
    assert abs(s.space[0].anisotropy(1 / 16) - (1 / 16) * 16 / 3) < 1e-14


def test_semi_time_rate_below_half():
    s = _solver(4, 16, 1, allow_space=False)
    rate, _ = s.power_rate(seed=0, max_cycles=25)
    assert rate < 0.5


def test_spatial_coarsening_needs_nodal_correction():
    # 64 slabs of tau = 1/16 on the 4^3 mesh: lambda = 1/3, so space coarsens;
    # a long horizon makes the undamped gradient modes visible
    prob = inputs.config_unit_manufactured(4, 64, 1, T=4.0)
    without = SpaceTimeMultigrid(prob, use_nodal=False)
    with_a = SpaceTimeMultigrid(prob, use_nodal=True)
    assert without.specs[1].space == 1                    # space does coarsen here
    r_without, _ = without.power_rate(seed=0, max_cycles=25)
    r_with, _ = with_a.power_rate(seed=0, max_cycles=25)
    assert r_without > 0.95
    assert r_with < 0.2


def test_manufactured_error_decreases():
    errs = []
    for n, Nt in ((4, 16), (8, 64)):
        prob = inputs.config_unit_manufactured(n, Nt, 1)
        s = SpaceTimeMultigrid(prob)
        b_all, u0, uT = manufactured_problem(s)
        b = s.fold_initial(s.to_interior(b_all), u0)
        x, _ = s.solve(b, rtol=1e-11)
        e = end_value(x, 1) - uT[s.fine.ie]
        M = s.fine.M
        errs.append(np.sqrt(e @ M @ e) / np.sqrt(uT[s.fine.ie] @ M @ uT[s.fine.ie]))
    # at least first order in h (tau shrinks like h^2 here)
    assert errs[1] < 0.5 * errs[0]


def test_smoother_sequence_sas_is_the_sas_smoother():
    s = _solver(4, 8, 1)
    lev = s.levels[0]
    rng = np.random.default_rng(4)
    x, b = rng.standard_normal((2, 8, 2, s.fine.n_e))
    assert np.array_equal(lev.smooth_sequence(x, b, "SAS"), lev.smooth_SAS(x, b))
    assert np.array_equal(lev.smooth_sequence(x, b, "SS"), lev.smooth_SAS(x, b, use_nodal=False))


@pytest.mark.parametrize("seq", ["SA", "AS", "SSA", "ASS", "SSAS", "SSASS"])
def test_every_smoother_order_converges_to_direct_solution(seq):
    s = _solver(4, 8, 1, smoother=seq)
    rng = np.random.default_rng(6)
    b = rng.standard_normal((8, 2, s.fine.n_e))
    x, hist = s.solve(b, rtol=1e-12, max_cycles=80)
    xd = direct_solve(s, b)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    rate, _ = s.power_rate(seed=0, max_cycles=15)
    assert rate < 0.6, (seq, rate)


@pytest.mark.parametrize("pt", [0, 1])
def test_slab_operator_inverts_the_slab_solve(pt):
    """apply_slab is the block whose exact inverse the smoother applies: both
    slab solvers (the real 2n block LU, and for p_t = 1 the complex
    diagonalised one, checked against each other above) invert it."""
    s = _solver(4, 4, pt, slab_solver="complex") if pt == 1 else _solver(4, 4, pt)
    lev = s.levels[0]
    r = np.random.default_rng(8).standard_normal((4, pt + 1, s.fine.n_e))
    z = lev.slab.solve(r)
    assert np.linalg.norm(lev.apply_slab(z) - r) <= 1e-12 * np.linalg.norm(r)


def test_operator_only_level_matches_full_level():
    from oracle.hierarchy import finest_space
    from oracle.vcycle import Level
    prob = inputs.config_block_random(n=4, Nt=8, pt=1, seed=11, block_hexes=2)
    s = SpaceTimeMultigrid(prob)
    lev = Level.operator_only(finest_space(prob), 1, 8, prob.T / 8, nodal=True)
    rng = np.random.default_rng(9)
    x, b = rng.standard_normal((2, 8, 2, s.fine.n_e))
    assert np.array_equal(lev.residual(x, b), s.levels[0].residual(x, b))
    assert np.array_equal(lev.apply_slab(x), s.levels[0].apply_slab(x))
    assert np.array_equal(lev.nodal_A(x, b), s.levels[0].nodal_A(x, b))


def test_power_rate_of_a_single_slab_is_zero():
    """With one slab the V-cycle is the exact solve: from any start error the
    first cycle leaves exactly zero (b = 0), so the rate is 0 and the
    iteration stops at the underflow test after one cycle."""
    s = _solver(4, 1, 1)
    rate, rates = s.power_rate(seed=2, max_cycles=10)
    assert rates == [0.0] and rate == 0.0


@pytest.mark.parametrize("pt", [0, 1])
def test_restrict_fine_operator_prolong_is_coarse_operator(pt):
    """Galerkin identity of the hierarchy: the oracle's restriction and
    prolongation (P_t (x) P_s and its transpose) around the fine level's L
    give the coarse level's L (time operators rediscretised at 2 tau, spatial
    M and K Galerkin). Level 0 -> 1 of the 4^3 problem coarsens in space and
    time (eq. (3) holds), 1 -> 2 in time only."""
    s = SpaceTimeMultigrid(inputs.config_unit_manufactured(4, 8, pt))
    assert s.specs[1].space != s.specs[0].space and s.specs[2].space == s.specs[1].space
    for l in (0, 1):
        fine, coarse = s.levels[l], s.levels[l + 1]
        shape = (coarse.N, s.q, coarse.space.n_e)
        n = int(np.prod(shape))
        RLP = np.empty((n, n))
        Lc = np.empty((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            e = e.reshape(shape)
            RLP[:, j] = s.restrict(l, fine.apply_L(s.prolong(l, e))).reshape(-1)
            Lc[:, j] = coarse.apply_L(e).reshape(-1)
        assert np.abs(RLP - Lc).max() <= 1e-13 * np.abs(Lc).max(), (pt, l)
        assert np.abs(Lc).max() > 0


def test_smoother_names_read_right_to_left():
    """Section 4 writes smoothers as products (SA = A, then S) and uses the
    reversed order after the coarse-grid correction: one two-level cycle with
    SA is A, S, coarse correction, S, A; with AS the mirror image."""
    s_sa = _solver(4, 2, 1, smoother="SA")
    s_as = _solver(4, 2, 1, smoother="AS")
    lev = s_sa.levels[0]
    rng = np.random.default_rng(9)
    x = rng.standard_normal((2, 2, s_sa.fine.n_e))
    b = rng.standard_normal(x.shape)

    def two_level(s, first, second):
        y = second(first(x, b), b)
        rc = s.restrict(0, lev.residual(y, b))
        y = y + s.prolong(0, s.levels[1].solve_exact_single_slab(rc))
        return first(second(y, b), b)

    S, A = lev.smooth_S, lev.nodal_A
    assert s_sa.levels[1].N == 1
    assert np.array_equal(s_sa.vcycle(0, x, b), two_level(s_sa, A, S))
    assert np.array_equal(s_as.vcycle(0, x, b), two_level(s_as, S, A))


def test_chebyshev_error_is_the_scaled_chebyshev_polynomial():
    """k steps from zero leave the error p(D^{-1} A) e_0 with
    p(lam) = T_k((theta - lam) / delta) / T_k(theta / delta): checked
    eigencomponent by eigencomponent on a random SPD matrix whose spectrum
    lies inside the interval given."""
    from numpy.polynomial import chebyshev as npc
    from oracle.vcycle import chebyshev_solve
    rng = np.random.default_rng(12)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(0.2, 3.0, n)
    Dh = np.diag(rng.uniform(0.5, 2.0, n))            # D^{1/2}
    A = Dh @ Q @ np.diag(lam) @ Q.T @ Dh              # D^{-1/2} A D^{-1/2} = Q lam Q^T
    A = 0.5 * (A + A.T)
    D = np.diag(A)
    # the diagonal of A must be D for the Jacobi preconditioner: rescale
    s = np.sqrt(np.diag(Dh) ** 2 / D)
    A = np.diag(s) @ A @ np.diag(s)
    Dm = np.diag(np.sqrt(np.diag(A)))
    lamD, V = np.linalg.eigh(np.linalg.inv(Dm) @ A @ np.linalg.inv(Dm))
    lmin, lmax = 0.9 * lamD.min(), 1.1 * lamD.max()
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    g = rng.standard_normal(n)
    x = np.linalg.solve(A, g)
    import scipy.sparse as sps
    for k in (1, 2, 5, 9):
        y = chebyshev_solve(sps.csr_matrix(A), g, k, (lmin, lmax))
        c = np.zeros(k + 1)
        c[-1] = 1.0
        p = npc.chebval((theta - lamD) / delta, c) / npc.chebval(theta / delta, c)
        e0 = V.T @ (Dm @ x)                  # error components in the D^{1/2} eigenbasis
        ek = V.T @ (Dm @ (x - y))
        assert np.allclose(ek, p * e0, atol=1e-12 * np.abs(e0).max()), k


def test_chebyshev_bounds_contain_the_spectrum_and_converge():
    from oracle.vcycle import chebyshev_bounds, chebyshev_solve
    s = _solver(4, 2, 1)
    Kn = s.fine.Kn
    lmin, lmax = chebyshev_bounds(Kn)
    Dm = np.diag(1.0 / np.sqrt(Kn.diagonal()))
    ev = np.linalg.eigvalsh(Dm @ Kn.toarray() @ Dm)
    assert ev.max() <= lmax * (1 + 1e-12) and abs(lmin - lmax / 30) <= 1e-15 * lmax
    g = np.random.default_rng(3).standard_normal((Kn.shape[0], 3))
    y = chebyshev_solve(Kn, g, 400, (0.99 * ev.min(), lmax))
    assert np.linalg.norm(y - np.linalg.solve(Kn.toarray(), g)) <= 1e-10 * np.linalg.norm(y)


@pytest.mark.parametrize("pt", [0, 1])
def test_inexact_nodal_vcycle_converges_to_direct_solution(pt):
    s = _solver(4, 8, pt, nodal_cheb=3)
    b = np.random.default_rng(5).standard_normal((8, pt + 1, s.fine.n_e))
    x, hist = s.solve(b, rtol=1e-12, max_cycles=80)
    xd = direct_solve(s, b)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def _twogrid(pt, k=3, box=False):
    from oracle.vcycle import SlabSolverTwoGrid
    prob = (inputs.config_core_box(n=8, Nt=2, pt=pt, seed=3, jitter=0.2) if box else
            inputs.config_block_random(n=8, Nt=2, pt=pt, seed=11, block_hexes=4))
    s = SpaceTimeMultigrid(prob)
    return s, SlabSolverTwoGrid(s.space[0], s.space[1], pt, s.levels[0].tau, k)


@pytest.mark.parametrize("pt", [0, 1])
def test_twogrid_slab_solve_converges_to_the_slab_solve(pt):
    """Preconditioned Richardson with the two-grid cycle converges to the
    exact spatial solve (SuperLU of mu M + tau K); 3 steps reduce the error
    below 0.2, also on the high-contrast jittered case."""
    import scipy.sparse.linalg as spla
    for box in (False, True):
        s, tg = _twogrid(pt, box=box)
        rng = np.random.default_rng(7)
        n = s.fine.n_e
        w = rng.standard_normal((n, 3)) + (1j * rng.standard_normal((n, 3)) if pt else 0)
        exact = spla.splu(tg.A.tocsc()).solve(w)
        tg.k = 150
        assert np.linalg.norm(tg.solve_spatial(w) - exact) <= 1e-10 * np.linalg.norm(exact)
        tg.k = 3
        assert np.linalg.norm(tg.solve_spatial(w) - exact) <= 0.2 * np.linalg.norm(exact)


@pytest.mark.parametrize("pt", [0, 1])
def test_twogrid_cycle_is_symmetric(pt):
    """The two-grid cycle B (smoother, coarse correction, smoother in reversed
    order) is symmetric in the bilinear form u^T B v, as A = mu M + tau K is:
    a step out of order or a transposed transfer breaks it."""
    s, tg = _twogrid(pt)
    rng = np.random.default_rng(8)
    n = s.fine.n_e
    u = rng.standard_normal((n, 1)) + (1j * rng.standard_normal((n, 1)) if pt else 0)
    v = rng.standard_normal((n, 1)) + (1j * rng.standard_normal((n, 1)) if pt else 0)
    a, b = (u.T @ tg.precondition(v)).item(), (v.T @ tg.precondition(u)).item()
    assert abs(a - b) <= 1e-12 * max(abs(a), 1e-300)


@pytest.mark.parametrize("pt", [0, 1])
def test_twogrid_vcycle_converges_to_direct_solution(pt):
    prob = inputs.config_block_random(n=4, Nt=8, pt=pt, seed=11, block_hexes=2)
    s = SpaceTimeMultigrid(prob, slab_solver="twogrid:3")
    assert any(type(lev.slab).__name__ == "SlabSolverTwoGrid" for lev in s.levels)
    b = np.random.default_rng(9).standard_normal((8, pt + 1, s.fine.n_e))
    x, hist = s.solve(b, rtol=1e-12, max_cycles=200)
    assert hist[-1] <= 1e-12
    xd = direct_solve(s, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
