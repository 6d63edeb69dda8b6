"""Upwind DG-in-time matrices (oracle, test infrastructure).

The paper states its method for implicit Euler with uniform step tau (eq. (1));
the slab block there is A = M + tau K and the coupling to the previous step is
-M. Degree p_t = 1 is the upwind discontinuous Galerkin generalisation: on each
slab I_n = (t_{n-1}, t_n) with reference coordinate s in [0, 1], the local basis
is Legendre psi_0 = 1, psi_1 = 2 s - 1, and testing the semi-discrete system
M u' + K u = f with psi_l on I_n, plus the upwind jump M (u(t_{n-1}^+) -
u(t_{n-1}^-)) psi_l(0), gives

    K_t[l, k] = int_0^1 psi_k'(s) psi_l(s) ds + psi_k(0) psi_l(0)
    M_t[l, k] = tau int_0^1 psi_k psi_l ds
    N_t[l, k] = psi_l(0) psi_k(1)        (data carried in from slab n-1)

so that slab block = K_t (x) M + M_t (x) K and coupling = -N_t (x) M. At
p_t = 0 these are 1, tau, 1: exactly eq. (1). The entries below are those
integrals evaluated by Gauss-Legendre quadrature, which is exact for these
polynomial degrees.
"""
from __future__ import annotations

import numpy as np


def _basis(pt: int, s: np.ndarray):
    """(psi [q, len(s)], dpsi/ds [q, len(s)]) of the Legendre basis on [0,1]."""
    s = np.asarray(s, dtype=np.float64)
    if pt == 0:
        return np.ones((1, s.size)), np.zeros((1, s.size))
    if pt == 1:
        return np.stack([np.ones_like(s), 2 * s - 1]), np.stack([np.zeros_like(s), 2 * np.ones_like(s)])
    raise ValueError("pt must be 0 or 1")


def time_matrices(pt: int, tau: float):
    """Return (K_t, M_t, N_t), each (pt+1) x (pt+1) float64."""
    xg, wg = np.polynomial.legendre.leggauss(4)
    s = 0.5 * (xg + 1.0)
    w = 0.5 * wg
    psi, dpsi = _basis(pt, s)
    psi0, _ = _basis(pt, np.array([0.0]))
    psi1, _ = _basis(pt, np.array([1.0]))
    Kt = (psi * w) @ dpsi.T + psi0 @ psi0.T          # [l, k]
    Mt = tau * (psi * w) @ psi.T
    Nt = psi0 @ psi1.T                                # [l, k] = psi_l(0) psi_k(1)
    return Kt, Mt, Nt


def psi_at(pt: int, s: float) -> np.ndarray:
    """Values psi_k(s) of the slab basis (used for initial data and end values)."""
    return _basis(pt, np.array([s]))[0][:, 0]


def time_prolongation(pt: int) -> np.ndarray:
    """P_t for one coarse slab -> its two fine halves, shape [2q, q].

    A coarse-slab polynomial c(sigma), sigma in [0,1], restricted to the fine
    halves sigma = s/2 and sigma = (1+s)/2 and re-expanded in the fine basis;
    computed here by L2 projection with exact quadrature.
    """
    q = pt + 1
    xg, wg = np.polynomial.legendre.leggauss(4)
    s = 0.5 * (xg + 1.0)
    w = 0.5 * wg
    psi_f, _ = _basis(pt, s)
    gram = (psi_f * w) @ psi_f.T
    P = np.zeros((2 * q, q))
    for half in range(2):
        sig = 0.5 * (s + half)
        psi_c, _ = _basis(pt, sig)
        P[half * q:(half + 1) * q] = np.linalg.solve(gram, (psi_f * w) @ psi_c.T)
    return P
