"""Pins of the oracle under the Neumann boundary condition (section 3:
mu^{-1} curl u x n = 0 on the boundary; the condition of the section 5
experiments).

The condition is natural, so every edge stays a degree of freedom. The nodal
space would contain the constants, which the gradient maps to zero; the
oracle leaves the lowest-numbered vertex out of it (a gauge). Each check ties
that reading to something other than the oracle itself:

* G 1 = 0 in exact integers, and the gauge column of G is minus the sum of
  the others, so the remaining columns span the same range (eq. (8)'s
  correction space is unchanged);
* the gauged K_n = G^T M G is SPD (dense Cholesky) and equals the directly
  assembled P1 stiffness of div sigma grad without the gauge row and column;
* with all edges free, the sigma-mass and nu-curl energies of the fields
  c (constant) and b x x (linear), which the lowest-order Nedelec space
  reproduces exactly, equal sigma |c|^2 vol and 4 nu |b|^2 vol;
* P_e G_c = G_f P_n on the gauged spaces, exactly (dyadic rationals);
* the V-cycle's fixed point is the direct sparse LU solution of the whole
  space-time system, and A solves gradient errors exactly, the gauge
  vertex's potential included;
* with exact solves, pure time coarsening contracts by < 0.5 (section 3.1).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1911_09548_amd import inputs
from oracle.fem import assemble_p1_stiffness
from oracle.hierarchy import build_space_levels
from oracle.mesh import NEUMANN, Topology
from oracle.vcycle import SpaceTimeMultigrid, direct_solve


def _problem(n=4, Nt=8, pt=1, seed=11):
    prob = inputs.config_block_random(n=n, Nt=Nt, pt=pt, seed=seed, block_hexes=max(1, n // 2))
    prob.bc = "neumann"
    return prob


@pytest.mark.parametrize("n", [2, 3])
def test_all_edges_free_and_gauge_vertex(n):
    topo = Topology(inputs.kuhn_coords(n), inputs.kuhn_tets(n), NEUMANN)
    assert np.array_equal(topo.interior_edges, np.arange(topo.n_edges))
    assert np.array_equal(topo.interior_vertices, np.arange(1, topo.n_vertices))
    G = topo.gradient().astype(np.int64)
    assert not np.any(G @ np.ones(topo.n_vertices, dtype=np.int64))
    Gd = G.toarray()
    assert np.array_equal(Gd[:, 0], -Gd[:, 1:].sum(axis=1))
    Gi = Gd[:, topo.interior_vertices].astype(np.float64)
    assert np.linalg.matrix_rank(Gi) == topo.n_vertices - 1


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_gauged_nodal_matrix_is_spd_p1_stiffness(jitter):
    prob = inputs.config_block_random(n=4, Nt=2, pt=1, seed=3, block_hexes=2)
    prob.bc = "neumann"
    if jitter:
        prob.levels[0].coords = inputs.jitter_coords(prob.levels[0].coords, 4, jitter,
                                                     np.random.default_rng(5))
    S = build_space_levels(prob)[0]
    Kn = S.Kn.toarray()
    np.linalg.cholesky(Kn)   # raises unless SPD
    Kd = assemble_p1_stiffness(S.topo, prob.sigma).toarray()[1:, 1:]
    assert np.abs(Kn - Kd).max() <= 1e-13 * np.abs(Kd).max()
    # the full (ungauged) matrix has the constants as its null space
    Kfull = assemble_p1_stiffness(S.topo, prob.sigma)
    assert np.abs(Kfull @ np.ones(S.topo.n_vertices)).max() <= 1e-13 * np.abs(Kd).max()
    np.linalg.cholesky(S.M.toarray())


def test_energies_of_reproduced_fields_over_all_edges():
    n = 3
    prob = inputs.config_block_random(n=n, Nt=2, pt=1, seed=3, block_hexes=n)
    prob.bc = "neumann"
    sig, nu = 2.5, 0.75
    prob.sigma[:] = sig
    prob.nu[:] = nu
    prob.levels[0].coords = inputs.jitter_coords(prob.levels[0].coords, n, 0.2,
                                                 np.random.default_rng(9))
    S = build_space_levels(prob)[0]
    X = S.topo.coords
    tail, head = S.topo.edges[:, 0], S.topo.edges[:, 1]
    c = np.array([0.3, -1.2, 0.7])
    uc = (X[head] - X[tail]) @ c                       # line integrals of the constant field
    assert abs(uc @ (S.M @ uc) - sig * (c @ c)) <= 1e-13 * sig * (c @ c)
    assert abs(uc @ (S.K @ uc)) <= 1e-13 * (c @ c)
    b = np.array([0.4, 0.9, -0.5])
    # b x x is linear: its line integral over an edge is (b x midpoint) . (head - tail)
    mid = 0.5 * (X[head] + X[tail])
    ub = np.einsum("ij,ij->i", np.cross(b, mid), X[head] - X[tail])
    assert abs(ub @ (S.K @ ub) - 4.0 * nu * (b @ b)) <= 1e-12 * nu * (b @ b)


def test_edge_and_vertex_prolongations_commute_with_gradient():
    prob = _problem(n=4)
    lv = build_space_levels(prob)
    fine, coarse = lv[0], lv[1]
    lhs = (coarse.Pe @ coarse.G).toarray()
    rhs = (fine.G @ coarse.Pn).toarray()
    assert np.array_equal(lhs, rhs)
    # the coarse edge operators are the Galerkin products over all edges
    assert coarse.n_e == coarse.topo.n_edges


@pytest.mark.parametrize("pt", [0, 1])
@pytest.mark.parametrize("n,Nt", [(2, 4), (4, 8), (4, 16)])
def test_vcycle_converges_to_direct_solution(n, Nt, pt):
    s = SpaceTimeMultigrid(_problem(n, Nt, pt))
    assert s.fine.n_e == s.fine.topo.n_edges
    b = np.random.default_rng(3).standard_normal((Nt, pt + 1, s.fine.n_e))
    x, hist = s.solve(b, rtol=1e-12, max_cycles=60)
    xd = direct_solve(s, b)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("pt", [0, 1])
def test_nodal_correction_solves_gradient_errors(pt):
    s = SpaceTimeMultigrid(_problem(4, 8, pt))
    lev = s.levels[0]
    rng = np.random.default_rng(2)
    Gall = s.fine.topo.gradient()
    # potentials on every vertex, the gauge vertex included
    phi = rng.standard_normal((lev.N, pt + 1, s.fine.topo.n_vertices))
    u = np.stack([(Gall @ phi[:, k].T).T for k in range(pt + 1)], axis=1)
    b = lev.apply_L(u)
    x = lev.nodal_A(np.zeros_like(b), b)
    assert np.linalg.norm(x - u) <= 1e-11 * np.linalg.norm(u)
    r = lev.residual(lev.nodal_A(rng.standard_normal(b.shape), b), b)
    gr = np.stack([(Gall.T @ r[:, k].T).T for k in range(pt + 1)], axis=1)
    assert np.linalg.norm(gr) <= 1e-11 * np.linalg.norm(b)


def test_semi_time_rate_below_one_half():
    s = SpaceTimeMultigrid(_problem(4, 16, 1), allow_space=False)
    rate, _ = s.power_rate(seed=1, max_cycles=20)
    assert rate < 0.5
