"""Manufactured eddy-current problem on the unit cube (oracle, test infrastructure).

u(x, t) = u_s(x) e^{-t}, u_s = (sin pi y sin pi z, sin pi x sin pi z, sin pi x sin pi y).
u_s is divergence free, curl curl u_s = 2 pi^2 u_s and u_s x n = 0 on the
boundary of (0,1)^3, so with sigma = nu = 1 the eddy-current equation (4) holds
with f = (2 pi^2 - 1) u_s e^{-t}.

Discrete data:
* Pi_h u_s: Nedelec interpolant, i.e. the line integral of u_s along each edge
  tail -> head (5-point Gauss-Legendre);
* load b_{n,k} = int_{I_n} psi_k(t) e^{-t} dt * (2 pi^2 - 1) M Pi_h u_s (the load
  of the interpolated source; the time integral is exact);
* initial value u0 = Pi_h u_s (t = 0).
"""
from __future__ import annotations

import numpy as np


def field_us(x):
    s = np.sin(np.pi * x)
    return np.stack([s[:, 1] * s[:, 2], s[:, 0] * s[:, 2], s[:, 0] * s[:, 1]], axis=1)


def interpolate_edges(coords, edges, field=field_us, npts=5):
    """Line integrals of `field` along every edge tail -> head."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    s = 0.5 * (xg + 1.0)
    w = 0.5 * wg
    p = coords[edges[:, 0]]
    d = coords[edges[:, 1]] - p
    out = np.zeros(edges.shape[0])
    for si, wi in zip(s, w):
        out += wi * np.einsum("ed,ed->e", field(p + si * d), d)
    return out


def time_weights(pt: int, T: float, Nt: int) -> np.ndarray:
    """c[n, k] = int_{I_n} psi_k(t) e^{-t} dt, exact."""
    tau = T / Nt
    t0 = tau * np.arange(Nt)
    c = np.zeros((Nt, pt + 1))
    em = np.exp(-tau)
    c[:, 0] = np.exp(-t0) * (1.0 - em)
    if pt == 1:
        c[:, 1] = np.exp(-t0) * (2.0 * (1.0 - em * (1.0 + tau)) / tau - (1.0 - em))
    return c


def manufactured_problem(solver):
    """Return (b_all [Nt,q,E], u0_all [E], uT_interp_all [E]) over all edges.

    b is the load functional the library receives (boundary entries zero);
    u0 is the interpolated initial field; uT is Pi_h u(T) for error checks.
    """
    prob = solver.problem
    topo = solver.fine.topo
    us = interpolate_edges(topo.coords, topo.edges)
    ie = solver.fine.ie
    Mus = solver.fine.M @ us[ie]
    c = time_weights(prob.pt, prob.T, prob.Nt)
    b_int = (2.0 * np.pi ** 2 - 1.0) * c[:, :, None] * Mus[None, None, :]
    b = np.zeros((prob.Nt, prob.pt + 1, topo.n_edges))
    b[..., ie] = b_int
    u0 = us.copy()
    u0[topo.boundary_edge] = 0.0
    uT = np.exp(-prob.T) * u0
    return b, u0, uT


def end_value(x, pt: int):
    """u_h(T^-) from the last slab's coefficients (psi_k(1) = 1 for all k)."""
    return x[-1].sum(axis=0) if pt == 1 else x[-1, 0]
