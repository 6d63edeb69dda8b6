"""GPU numeric factorisation against the host factorisation and the oracle.

The device setup assembles every front on the GPU, factors it (diagonal
blocks in LDS, panel triangular solves and rank-64 symmetric updates) and
forms the selective-inversion panels P_s = [inv(L11); -L21 inv(L11)]. Its
FP64 panels are copied back and
* compared with the host factorisation of the same matrix: the same
  symbolic structure, and solves with either set of panels both have a
  normwise backward error <= 1e-14 (the panel difference and the forward
  difference of the two solves, which grows with the conditioning, are
  printed);
* applied to solve the oracle's slab block (mu M + tau K, mu = 2 + i sqrt2,
  or M + tau K) and nodal matrix K_n: normwise backward error <= 1e-14
  (infinity norms, per right-hand side), a bound that does not depend on
  the conditioning.
"""
import numpy as np
import pytest
from paper_1911_09548_amd import inputs
from _parity import BWD64, backward_error, fwd

pytestmark = pytest.mark.gpu

CASES = {
    "unit_n4_N16_p1": lambda: inputs.config_unit_manufactured(4, 16, 1),
    "block_n8_N16_p1": lambda: inputs.config_block_random(n=8, Nt=16, pt=1, seed=3, block_hexes=4),
    "block_n8_N8_p0": lambda: inputs.config_block_random(n=8, Nt=8, pt=0, seed=4, block_hexes=4),
    "jitter_n6_N16_p1": lambda: inputs.config_core_box(n=6, Nt=16, pt=1, seed=1, jitter=0.2),
    "request_n12_N32_p1": lambda: inputs.config_request(12, 32, 1, 9),
}


def _apply_factor(F, b):
    """x = A^{-1} b from exported panels (forward then backward sweep)."""
    n = F["perm"].size
    X = np.zeros((n,) + b.shape[1:], dtype=np.result_type(F["panel"].dtype, b.dtype))
    X[:] = b[F["perm"]]
    blocks = []
    for s in range(F["col0"].size - 1):
        c0, c1 = F["col0"][s], F["col0"][s + 1]
        w = c1 - c0
        R = F["rows"][F["rptr"][s]:F["rptr"][s + 1]]
        P = F["panel"][F["panel_off"][s]:F["panel_off"][s + 1]].reshape(w, w + R.size).T
        blocks.append((c0, c1, R, P[:w], P[w:]))
    for c0, c1, R, Li, W in blocks:
        top = X[c0:c1].copy()
        X[R] += W @ top
        X[c0:c1] = Li @ top
    for c0, c1, R, Li, W in reversed(blocks):
        X[c0:c1] = Li.T @ X[c0:c1] + W.T @ X[R]
    out = np.empty_like(X)
    out[F["perm"]] = X
    return out


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    from paper_1911_09548_amd import stmg
    from oracle.vcycle import SpaceTimeMultigrid
    prob = CASES[request.param]()
    print(f"\n[case] device factorisation {request.param}", flush=True)
    dev = stmg.Solver(prob, device_factor=1)
    host = stmg.Solver(prob, host_only=1)
    ora = SpaceTimeMultigrid(prob)
    yield request.param, prob, dev, host, ora
    dev.close()
    host.close()


def _matrices(prob, lev):
    sd = lev.space
    slab = ((2 + 1j * np.sqrt(2)) * sd.M + lev.tau * sd.K) if prob.pt == 1 else (sd.M + lev.tau * sd.K)
    return slab.tocsr(), sd.Kn.tocsr()


def test_device_panels_match_host(pair):
    name, prob, dev, host, ora = pair
    rng = np.random.default_rng(12)
    for l, lev in enumerate(ora.levels):
        sd = lev.space
        for which, A in enumerate(_matrices(prob, lev)):
            if which == 1 and sd.n_v == 0:
                continue
            Fd, Fh = dev.export_factor(l, which), host.export_factor(l, which)
            for key in ("perm", "col0", "rptr", "rows", "panel_off"):
                assert np.array_equal(Fd[key], Fh[key]), (name, l, which, key)
            rel = np.linalg.norm(Fd["panel"] - Fh["panel"]) / np.linalg.norm(Fh["panel"])
            b = rng.standard_normal((A.shape[0], 3))
            if np.iscomplexobj(Fd["panel"]):
                b = b + 1j * rng.standard_normal(b.shape)
            xd, xh = _apply_factor(Fd, b), _apply_factor(Fh, b)
            ed, eh = backward_error(A, xd, b), backward_error(A, xh, b)
            print(f"[factor] {name} level {l} {'slab' if which == 0 else 'nodal'}: "
                  f"|P_dev - P_host| / |P_host| = {rel:.2e}, backward error dev {ed:.1e} host {eh:.1e}, "
                  f"solves differ {fwd(xd, xh):.1e}")
            assert ed <= BWD64 and eh <= BWD64, (name, l, which, ed, eh)


def test_device_panels_solve_oracle_systems(pair):
    name, prob, dev, host, ora = pair
    rng = np.random.default_rng(11)
    for l, lev in enumerate(ora.levels):
        sd = lev.space
        A, Kn = _matrices(prob, lev)
        F = dev.export_factor(l, 0)
        b = rng.standard_normal((sd.n_e, 3))
        if prob.pt == 1:
            b = b + 1j * rng.standard_normal((sd.n_e, 3))
        x = _apply_factor(F, b)
        assert backward_error(A, x, b) <= BWD64, (name, l, backward_error(A, x, b))
        if sd.n_v > 0:
            Fn = dev.export_factor(l, 1)
            bn = rng.standard_normal((sd.n_v, 2))
            xn = _apply_factor(Fn, bn)
            assert backward_error(Kn, xn, bn) <= BWD64, (name, l, backward_error(Kn, xn, bn))
