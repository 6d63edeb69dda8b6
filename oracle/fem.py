"""Lowest-order Nedelec (Whitney) and P1 assembly in FP64 (oracle, test infrastructure).

Section 3 defines (M_h)_ij = int sigma phi_i . phi_j and
(K_h)_ij = int mu^{-1} curl phi_i . curl phi_j on the Nedelec basis; the nodal
correction (eq. (8)) uses K_n, the stiffness of div sigma grad on the nodal
(P1) space. With barycentric coordinates lambda_a and g_a = grad lambda_a on a
tetrahedron T, the Whitney function of the edge i->j is
phi_ij = lambda_i g_j - lambda_j g_i, its curl is 2 g_i x g_j, and
int_T lambda_a lambda_b = vol(T) (1 + delta_ab) / 20.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

LOCAL_EDGES = list(itertools.combinations(range(4), 2))  # (01,02,03,12,13,23)


def barycentric_gradients(coords: np.ndarray, tets: np.ndarray):
    """Return (g [nt,4,3], vol [nt]) for tets given with sorted vertex ids."""
    x = coords[tets]                        # [nt, 4, 3]
    B = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)  # columns
    det = np.linalg.det(B)
    Binv = np.linalg.inv(B)                 # rows are grad lambda_1..3
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:] = Binv
    g[:, 0] = -Binv.sum(axis=1)
    return g, np.abs(det) / 6.0


def whitney_element_matrices(coords, tets, sigma, nu):
    """Element mass and curl-curl matrices [nt, 6, 6] in local edge order."""
    g, vol = barycentric_gradients(coords, tets)
    nt = tets.shape[0]
    gg = np.einsum("tad,tbd->tab", g, g)    # g_a . g_b
    Me = np.zeros((nt, 6, 6))
    Ke = np.zeros((nt, 6, 6))
    curl = np.stack([2.0 * np.cross(g[:, i], g[:, j]) for i, j in LOCAL_EDGES], axis=1)  # [nt,6,3]

    def ll(a, b):  # int lambda_a lambda_b / vol
        return (2.0 if a == b else 1.0) / 20.0

    for p, (i, j) in enumerate(LOCAL_EDGES):
        for q, (k, l) in enumerate(LOCAL_EDGES):
            Me[:, p, q] = (ll(i, k) * gg[:, j, l] - ll(i, l) * gg[:, j, k]
                           - ll(j, k) * gg[:, i, l] + ll(j, l) * gg[:, i, k]) * vol
    Ke = np.einsum("tpd,tqd->tpq", curl, curl) * vol[:, None, None]
    return Me * sigma[:, None, None], Ke * nu[:, None, None], vol


def assemble_edge_matrices(topo, sigma, nu):
    """Global M, K over all edges (before Dirichlet elimination)."""
    Me, Ke, _ = whitney_element_matrices(topo.coords, topo.tets, sigma, nu)
    te = topo.tet_edges                      # [nt, 6] in LOCAL_EDGES order
    rows = np.repeat(te, 6, axis=1).ravel()
    cols = np.tile(te, (1, 6)).ravel()
    E = topo.n_edges
    M = sp.csr_matrix((Me.ravel(), (rows, cols)), shape=(E, E))
    K = sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(E, E))
    M.sum_duplicates()
    K.sum_duplicates()
    return M, K


def assemble_p1_stiffness(topo, sigma):
    """Directly assembled P1 stiffness of div sigma grad over all vertices."""
    g, vol = barycentric_gradients(topo.coords, topo.tets)
    Ae = np.einsum("tad,tbd->tab", g, g) * (sigma * vol)[:, None, None]
    t = topo.tets
    rows = np.repeat(t, 4, axis=1).ravel()
    cols = np.tile(t, (1, 4)).ravel()
    nv = topo.n_vertices
    A = sp.csr_matrix((Ae.ravel(), (rows, cols)), shape=(nv, nv))
    A.sum_duplicates()
    return A
