"""Pins of the oracle's DG-in-time part and time transfers.

* Degree 0 is implicit Euler (eq. (1)): slab block 1*M + tau*K, coupling -M.
* Degree 1 upwind DG is the two-stage Radau IIA method, whose stability
  function is the (1,2) Pade approximant (1 - z/3) / (1 + 2z/3 + z^2/6) of
  e^{-z} for u' + lambda u = 0 (the paper's test equation (5)), z = lambda tau.
* DG of degree p reproduces solutions that are polynomials of degree <= p.
* Time coarsening: P_t^T L_fine P_t equals the operator rediscretised with 2 tau.
"""
import numpy as np
import pytest

from oracle.dgtime import time_matrices, time_prolongation, psi_at


def test_degree0_is_implicit_euler():
    Kt, Mt, Nt = time_matrices(0, 0.37)
    assert np.allclose(Kt, [[1.0]], atol=0) and np.allclose(Mt, [[0.37]], atol=1e-16)
    assert np.allclose(Nt, [[1.0]], atol=0)


@pytest.mark.parametrize("z", [0.01, 0.3, 1.0, 7.0, 50.0])
def test_degree1_stability_is_pade_12(z):
    tau = 0.25
    lam = z / tau
    Kt, Mt, Nt = time_matrices(1, tau)
    # one slab of u' + lam u = 0 from u(0^-) = 1: (K_t + lam M_t) x = N_t [u_prev coefficients]
    prev = np.array([1.0, 0.0])           # constant 1 carried in (end value 1)
    x = np.linalg.solve(Kt + lam * Mt, Nt @ prev)
    end = psi_at(1, 1.0) @ x
    pade = (1 - z / 3) / (1 + 2 * z / 3 + z * z / 6)
    assert abs(end - pade) <= 2e-16 * max(1.0, abs(pade)) + 1e-16


@pytest.mark.parametrize("pt", [0, 1])
def test_dg_reproduces_polynomials(pt):
    """u(t) = a + c t (degree <= pt) solves u' + lam u = f exactly in DG(pt)."""
    tau, lam, N = 0.2, 3.0, 5
    a, c = 1.3, (-0.7 if pt == 1 else 0.0)
    Kt, Mt, Nt = time_matrices(pt, tau)
    xg, wg = np.polynomial.legendre.leggauss(6)
    s, w = 0.5 * (xg + 1), 0.5 * wg
    q = pt + 1
    prev = np.zeros(q)
    prev_end_coeffs = None
    for n in range(N):
        t = tau * (n + s)
        f = c + lam * (a + c * t)
        psi = np.stack([np.ones_like(s), 2 * s - 1])[:q]
        b = tau * (psi * w) @ f
        if n == 0:
            b = b + psi_at(pt, 0.0) * a       # initial value u(0) = a
            rhs = b
        else:
            rhs = b + Nt @ prev
        x = np.linalg.solve(Kt + lam * Mt, rhs)
        # exact coefficients of a + c t on this slab in the Legendre basis
        mid = a + c * tau * (n + 0.5)
        exact = np.array([mid, c * tau / 2])[:q]
        assert np.allclose(x, exact, atol=1e-13, rtol=0)
        prev = x


def test_eigenvalues_of_time_block():
    tau = 0.125
    Kt, Mt, _ = time_matrices(1, tau)
    ev = np.sort_complex(np.linalg.eigvals(np.linalg.solve(Mt, Kt)) * tau)
    assert np.allclose(ev, [2 - 1j * np.sqrt(2), 2 + 1j * np.sqrt(2)], atol=1e-14)


@pytest.mark.parametrize("pt", [0, 1])
@pytest.mark.parametrize("lam", [0.0, 2.0, 40.0])
def test_time_galerkin_equals_rediscretisation(pt, lam):
    tau = 0.1
    Ktf, Mtf, Ntf = time_matrices(pt, tau)
    Ktc, Mtc, Ntc = time_matrices(pt, 2 * tau)
    q = pt + 1
    P = time_prolongation(pt)
    # two coarse slabs <-> four fine slabs, scalar operator u' + lam u
    Af = Ktf + lam * Mtf
    Lf = np.zeros((4 * q, 4 * q))
    for n in range(4):
        Lf[n * q:(n + 1) * q, n * q:(n + 1) * q] = Af
        if n:
            Lf[n * q:(n + 1) * q, (n - 1) * q:n * q] = -Ntf
    Lc = np.zeros((2 * q, 2 * q))
    for n in range(2):
        Lc[n * q:(n + 1) * q, n * q:(n + 1) * q] = Ktc + lam * Mtc
        if n:
            Lc[n * q:(n + 1) * q, (n - 1) * q:n * q] = -Ntc
    Pfull = np.zeros((4 * q, 2 * q))
    Pfull[:2 * q, :q] = P
    Pfull[2 * q:, q:] = P
    assert np.allclose(Pfull.T @ Lf @ Pfull, Lc, atol=1e-14, rtol=0)


def test_time_prolongation_is_exact_embedding():
    """A coarse polynomial evaluated through P_t equals its values on the halves."""
    P = time_prolongation(1)
    c = np.array([0.8, -1.7])
    for half in range(2):
        for s in (0.0, 0.3, 1.0):
            sig = 0.5 * (s + half)
            coarse_val = c[0] + c[1] * (2 * sig - 1)
            fine = P[2 * half:2 * half + 2] @ c
            assert abs(fine[0] + fine[1] * (2 * s - 1) - coarse_val) < 1e-15
