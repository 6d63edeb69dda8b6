"""Pins of the oracle's spatial part: topology, Whitney assembly, transfers.

Each check ties the oracle to something other than itself: integer identities
of the de Rham sequence, closed-form counts, exact energies of fields the
lowest-order Nedelec space reproduces, and rediscretisation on nested meshes.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1911_09548_amd import inputs
from oracle.mesh import Topology
from oracle.fem import assemble_edge_matrices, assemble_p1_stiffness, barycentric_gradients
from oracle.hierarchy import edge_prolongation, vertex_prolongation, build_space_levels
from oracle.manufactured import interpolate_edges


def kuhn_edge_count(n):
    # 7 edge directions d in {0,1}^3 \ 0; count of grid positions per direction
    return 3 * n * (n + 1) ** 2 + 3 * n ** 2 * (n + 1) + n ** 3


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_counts_and_euler(n):
    topo = Topology(inputs.kuhn_coords(n), inputs.kuhn_tets(n))
    V, E, F, T = topo.n_vertices, topo.n_edges, topo.faces.shape[0], topo.tets.shape[0]
    assert V == (n + 1) ** 3 and T == 6 * n ** 3
    assert E == kuhn_edge_count(n)
    assert V - E + F - T == 1                         # Euler characteristic of a ball
    assert topo.interior_vertices.size == (n - 1) ** 3
    # boundary edges: 6 triangulated n x n faces (2n(n+1) grid edges + n^2
    # diagonals each), the 12 cube edges of n segments counted twice
    n_bnd = 6 * (2 * n * (n + 1) + n * n) - 12 * n
    assert topo.interior_edges.size == E - n_bnd
    table = {2: (98, 26), 4: (604, 316)}
    if n in table:
        assert (E, topo.interior_edges.size) == table[n]


@pytest.mark.parametrize("n", [2, 3])
def test_curl_grad_is_zero_exactly(n):
    topo = Topology(inputs.kuhn_coords(n), inputs.kuhn_tets(n))
    C = topo.curl().astype(np.int64)
    G = topo.gradient().astype(np.int64)
    CG = (C @ G).toarray()
    assert np.array_equal(CG, np.zeros_like(CG))
    # every row of G has one +1 (head) and one -1 (tail)
    Gd = G.toarray()
    assert np.all(Gd.sum(axis=1) == 0) and np.all(np.abs(Gd).sum(axis=1) == 2)


def _mesh(n, jitter, seed=0):
    rng = np.random.default_rng(seed)
    c = inputs.kuhn_coords(n)
    if jitter:
        c = inputs.jitter_coords(c, n, jitter, rng)
    return Topology(c, inputs.kuhn_tets(n))


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_K_annihilates_gradients(jitter):
    topo = _mesh(3, jitter)
    rng = np.random.default_rng(1)
    sigma = 10 ** rng.uniform(-1, 2, topo.tets.shape[0])
    nu = 10 ** rng.uniform(-1, 2, topo.tets.shape[0])
    M, K = assemble_edge_matrices(topo, sigma, nu)
    G = topo.gradient()
    KG = K @ G
    scale = sp.linalg.norm(K) * sp.linalg.norm(G)
    assert sp.linalg.norm(KG) <= 1e-13 * scale
    # K_n = G^T M G equals the directly assembled P1 stiffness of div sigma grad
    Kn = G.T @ M @ G
    Kd = assemble_p1_stiffness(topo, sigma)
    assert sp.linalg.norm(Kn - Kd) <= 1e-13 * sp.linalg.norm(Kd)


def _tet_quadrature_deg2():
    a, b = 0.5854101966249685, 0.1381966011250105
    pts = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
    return pts, np.full(4, 0.25)


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_exact_energies_of_linear_fields(jitter):
    """u = a + b x x lies in the lowest-order Nedelec space, so its interpolant
    reproduces int sigma |u|^2 and int nu |curl u|^2 = int nu |2b|^2 exactly."""
    topo = _mesh(3, jitter, seed=2)
    rng = np.random.default_rng(3)
    sigma = 10 ** rng.uniform(-1, 1, topo.tets.shape[0])
    nu = 10 ** rng.uniform(-1, 1, topo.tets.shape[0])
    M, K = assemble_edge_matrices(topo, sigma, nu)
    a = np.array([0.3, -1.2, 0.7])
    bv = np.array([0.5, 0.25, -2.0])

    def field(x):
        return a[None, :] + np.cross(bv[None, :], x)

    u = interpolate_edges(topo.coords, topo.edges, field)
    # reference integrals by an exact degree-2 rule per tet
    _, vol = barycentric_gradients(topo.coords, topo.tets)
    pts, w = _tet_quadrature_deg2()
    X = topo.coords[topo.tets]                            # [nt,4,3]
    mass = 0.0
    for p, wi in zip(pts, w):
        xq = np.einsum("v,tvd->td", p, X)
        mass += wi * np.sum(sigma * vol * np.sum(field(xq) ** 2, axis=1))
    curl_energy = np.sum(nu * vol) * np.dot(2 * bv, 2 * bv)
    assert abs(u @ M @ u - mass) <= 1e-12 * mass
    assert abs(u @ K @ u - curl_energy) <= 1e-12 * curl_energy


def test_constant_field_mass():
    topo = _mesh(4, 0.2, seed=4)
    sigma = np.full(topo.tets.shape[0], 2.5)
    M, _ = assemble_edge_matrices(topo, sigma, np.ones_like(sigma))
    c = np.array([1.0, -2.0, 0.5])
    u = (topo.coords[topo.edges[:, 1]] - topo.coords[topo.edges[:, 0]]) @ c
    assert abs(u @ M @ u - 2.5 * 1.0 * c @ c) <= 1e-12 * (2.5 * c @ c)


def test_spd_after_dirichlet_elimination():
    topo = _mesh(3, 0.2, seed=5)
    sig = np.ones(topo.tets.shape[0])
    M, K = assemble_edge_matrices(topo, sig, sig)
    ie = topo.interior_edges
    Mi = M[ie][:, ie].toarray()
    Ki = K[ie][:, ie].toarray()
    assert np.allclose(Mi, Mi.T, atol=1e-15) and np.allclose(Ki, Ki.T, atol=1e-14)
    assert np.linalg.eigvalsh(Mi).min() > 0
    ev = np.linalg.eigvalsh(Ki)
    assert ev.min() > -1e-12 * ev.max()                  # PSD (gradient kernel)


def test_boundary_detection_on_cube():
    n = 3
    topo = _mesh(n, 0.0)
    c = topo.coords
    on_bnd = np.any((c < 1e-12) | (c > 1 - 1e-12), axis=1)
    assert np.array_equal(on_bnd, topo.boundary_vertex)
    # an edge is on the boundary iff both ends lie on one common face plane
    e = topo.edges
    p, q = c[e[:, 0]], c[e[:, 1]]
    same_plane = np.zeros(len(e), dtype=bool)
    for d in range(3):
        for v in (0.0, 1.0):
            same_plane |= (np.abs(p[:, d] - v) < 1e-12) & (np.abs(q[:, d] - v) < 1e-12)
    assert np.array_equal(same_plane, topo.boundary_edge)


def test_prolongations_commute_with_gradient():
    """P_e G_c = G_f P_n exactly (dyadic rationals), on all DOFs."""
    levs = inputs.kuhn_hierarchy(4)
    f = Topology(levs[0].coords, levs[0].tets)
    c = Topology(levs[1].coords, levs[1].tets)
    Pe = edge_prolongation(f, c, levs[1].vertex_parent)
    Pn = vertex_prolongation(f, c, levs[1].vertex_parent)
    lhs = (Pe @ c.gradient()).toarray()
    rhs = (f.gradient() @ Pn).toarray()
    assert np.array_equal(lhs, rhs)
    assert set(np.unique(Pe.data)) <= {-0.5, -0.25, 0.25, 0.5, 1.0, -1.0}


def test_galerkin_equals_rediscretisation_on_nested_meshes():
    prob = inputs.config_block_random(n=4, Nt=2, pt=1, seed=7, block_hexes=2)
    sl = build_space_levels(prob)
    # rediscretise the coarse mesh with the coarse-tet materials (blocks are
    # aligned with coarse hexes, so every coarse tet has one material)
    lev1 = prob.levels[1]
    tp = lev1.tet_parent
    sig_c = np.zeros(lev1.tets.shape[0])
    nu_c = np.zeros(lev1.tets.shape[0])
    sig_c[tp] = prob.sigma
    nu_c[tp] = prob.nu
    topo = Topology(lev1.coords, lev1.tets)
    M, K = assemble_edge_matrices(topo, sig_c, nu_c)
    ie = topo.interior_edges
    for Ag, Ad in ((sl[1].M, M[ie][:, ie]), (sl[1].K, K[ie][:, ie])):
        assert sp.linalg.norm(Ag - Ad) <= 1e-13 * sp.linalg.norm(Ad)


def test_tet_parent_contains_child():
    levs = inputs.kuhn_hierarchy(4)
    f, c = levs[0], levs[1]
    cent = f.coords[f.tets].mean(axis=1)
    Xc = c.coords[c.tets[c.tet_parent]]
    # barycentric coordinates of the fine centroid in the parent: all positive
    B = np.stack([Xc[:, 1] - Xc[:, 0], Xc[:, 2] - Xc[:, 0], Xc[:, 3] - Xc[:, 0]], axis=2)
    lam = np.linalg.solve(B, (cent - Xc[:, 0])[..., None])[..., 0]
    lam0 = 1 - lam.sum(axis=1)
    assert np.all(lam > 0) and np.all(lam0 > 0)
