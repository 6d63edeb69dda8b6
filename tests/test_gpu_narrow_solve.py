"""GPU parity of the supernode solves with narrow right-hand sides.

Levels with at most 16 slabs solve with 64 x 16 GEMM tiles, whose columns
beyond the level's width are padding. On 8^3 meshes with N_t = 16 (widths
16, 8, 4, 2, 1 over the levels) the slab solve of every level is checked
by its normwise backward error against the oracle's slab block (<= 1e-14),
its forward difference from the oracle's sparse direct solve (<= 1e-10),
and against the same solve whose backward sweep reads P_s instead of the
stored transpose (<= 1e-12), with automatic and forced K splits and the GPU
factorisation. The nodal correction is checked by the gradient component of
the new residual and its forward difference (tests/_parity.py).
"""
import numpy as np
import pytest

from paper_1911_09548_amd import inputs
from _parity import BWD64, FWD64, fwd, gradient_orthogonality, slab_backward_error

pytestmark = pytest.mark.gpu

CASES = {  # name: (Nt, pt, options)
    "N16_p1": (16, 1, {}),
    "N16_p0": (16, 0, {}),
    "N16_p1_split5": (16, 1, {"gemm_splitk": 5}),
    "N8_p1_split2_devfactor": (8, 1, {"gemm_splitk": 2, "device_factor": 1}),
}


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module", params=list(CASES))
def trio(request):
    from paper_1911_09548_amd import stmg
    from oracle.vcycle import SpaceTimeMultigrid
    Nt, pt, opts = CASES[request.param]
    prob = inputs.config_block_random(n=8, Nt=Nt, pt=pt, seed=41, block_hexes=4)
    print(f"\n[case] narrow solve {request.param}", flush=True)
    gpu = stmg.Solver(prob, **opts)
    alt = stmg.Solver(prob, factor_transpose=0)
    ora = SpaceTimeMultigrid(prob)
    yield request.param, prob, gpu, alt, ora
    gpu.close()
    alt.close()


def test_slab_solve_every_width(trio):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, alt, ora = trio
    for l in range(gpu.n_levels):
        lev = ora.levels[l]
        r = np.random.default_rng(100 + l).standard_normal((lev.N, ora.q, lev.space.n_e))
        ref = lev.slab.solve(r)
        got = _host(gpu.level_apply(l, stmg.OP_SLAB_SOLVE, _dev(r)))
        other = _host(alt.level_apply(l, stmg.OP_SLAB_SOLVE, _dev(r)))
        eta = slab_backward_error(lev, got, r)
        print(f"[narrow] {name} level {l} (N={lev.N}): backward error {eta:.1e}, oracle {fwd(got, ref):.2e}, "
              f"backward sweep from P {fwd(got, other):.2e}")
        assert eta <= BWD64 and fwd(got, ref) <= FWD64, (name, l, eta)
        assert fwd(got, other) <= 1e-12, (name, l)


def test_nodal_correction(trio):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, alt, ora = trio
    for l in range(gpu.n_levels):
        lev = ora.levels[l]
        if lev.space.n_v <= 1:
            continue
        rng = np.random.default_rng(200 + l)
        x = rng.standard_normal((lev.N, ora.q, lev.space.n_e))
        b = rng.standard_normal((lev.N, ora.q, lev.space.n_e))
        got = _host(gpu.level_apply(l, stmg.OP_NODAL_A, _dev(x), _dev(b)))
        assert gradient_orthogonality(lev, got, b) <= 1e-13, (name, l)
        assert fwd(got, lev.nodal_A(x, b)) <= FWD64, (name, l)


def test_solve_meets_tolerance(trio):
    name, prob, gpu, alt, ora = trio
    b_all = np.random.default_rng(7).standard_normal((prob.Nt, prob.pt + 1, gpu.n_edges))
    b = ora.to_interior(b_all)
    x, rep = gpu.solve(_dev(b_all))
    rr = np.linalg.norm(ora.levels[0].residual(ora.to_interior(_host(x)), b)) / np.linalg.norm(b)
    print(f"[narrow] {name}: cycles {rep['cycles']}, oracle residual {rr:.2e}")
    assert rep["rel_res"] <= 1e-8 and rr <= 1e-8 * (1 + 1e-6)
