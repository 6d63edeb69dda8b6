"""GPU parity for long time horizons: rows of 256 to 8192 values per spatial DOF.

The residual reads a row of N q values as interleaved 2-value packets (one
wave per row, or per group of 4 rows of the Hilbert order, from N q = 64 q
on) and splits rows longer than 64 C values (C the values per lane: the
stream_chunk option, at most 8 for grouped rows) into segments run as
consecutive launches, each handing the end value of its last slab to the next
for the DG coupling; the nodal time scan carries its running sum across
packets and segments.
These cases put every lane-chunk width (1, 2, 4, 8, 16 values per lane), 1 to
32 segments, the grouped and the per-row kernel and all visiting orders
through the residual, the nodal correction and a whole V-cycle, on a 4^3 mesh
so the oracle stays fast. Bounds as in the main parity suite (none depends
on a condition number): 1e-13 for sparse-only steps; for the nodal
correction the gradient component of the new residual (<= 1e-13 of its
rounding scale) and the forward difference (<= 1e-10); SAS forward <= 1e-10.
"""
import numpy as np
import pytest

from paper_1911_09548_amd import inputs
from _parity import FWD64, SPARSE64, fwd, gradient_orthogonality

pytestmark = pytest.mark.gpu

CASES = {  # name: (Nt, pt, stream_chunk, row_schedule); chunk 0 = the default
    # grouped rows (row_schedule 0): at most 8 values per lane
    "N128_p1": (128, 1, 0, 0),         # 256 values per row: 4 per lane, one segment
    "N256_p1_c4": (256, 1, 4, 0),      # 512: 2 segments of 256
    "N256_p1_c8": (256, 1, 8, 0),      # 512: one segment, 8 per lane
    "N512_p1_c16": (512, 1, 16, 0),    # 1024: 2 segments of 512
    "N1024_p1": (1024, 1, 0, 0),       # 2048: 4 segments of 512
    "N2048_p0": (2048, 0, 0, 0),       # 2048 with one value per slab: 4 segments
    "N2048_p0_c1": (2048, 0, 1, 0),    # one value per lane: 32 segments of 64
    "N4096_p1_c8": (4096, 1, 8, 0),    # 8192: 16 segments of 512
    # one row per wave, Hilbert order (row_schedule 2) or storage order (1); Morton groups (3)
    "N512_p1_c16_rows": (512, 1, 16, 2),    # 1024: one segment, 16 per lane
    "N1024_p1_c16_rows": (1024, 1, 16, 2),  # 2048: 2 segments of 1024
    "N1024_p0_rows": (1024, 0, 0, 2),       # 1024 one value per slab: one segment of 16 per lane
    "N2048_p0_c1_rows": (2048, 0, 1, 2),    # 32 segments of 64
    "N256_p1_storage": (256, 1, 0, 1),      # 512: one segment, storage order
    "N256_p1_morton": (256, 1, 0, 3),       # 512: grouped rows in Morton order
    "N512_p1_tiles": (512, 1, 32, 0),  # LDS-tiled residual: 64 segments of 16 values per tile
    "N1024_p0_tiles": (1024, 0, 32, 0),
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
def pair(request):
    from paper_1911_09548_amd import stmg
    from oracle.vcycle import SpaceTimeMultigrid
    Nt, pt, chunk, sched = CASES[request.param]
    prob = inputs.config_block_random(n=4, Nt=Nt, pt=pt, seed=21, block_hexes=2)
    print(f"\n[case] long horizon {request.param}", flush=True)
    gpu = stmg.Solver(prob, stream_chunk=chunk, row_schedule=sched)
    ora = SpaceTimeMultigrid(prob)
    yield request.param, prob, gpu, ora
    gpu.close()


def _vec(ora, l, seed):
    lev = ora.levels[l]
    return np.random.default_rng(seed).standard_normal((lev.N, ora.q, lev.space.n_e))


def test_residual_every_level(pair):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora = pair
    for l in range(gpu.n_levels):
        x, b = _vec(ora, l, 1), _vec(ora, l, 2)
        got = _host(gpu.level_apply(l, stmg.OP_RESIDUAL, _dev(x), _dev(b)))
        assert fwd(got, ora.levels[l].residual(x, b)) <= SPARSE64, (name, l)


def test_nodal_correction_and_sas(pair):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora = pair
    for l in (0, 1):
        lev = ora.levels[l]
        x, b = _vec(ora, l, 3), _vec(ora, l, 4)
        got = _host(gpu.level_apply(l, stmg.OP_NODAL_A, _dev(x), _dev(b)))
        assert gradient_orthogonality(lev, got, b) <= 1e-13, (name, l)
        assert fwd(got, lev.nodal_A(x, b)) <= FWD64, (name, l)
        got = _host(gpu.level_apply(l, stmg.OP_SAS, _dev(x), _dev(b)))
        assert fwd(got, lev.smooth_SAS(x, b, 0.5, True)) <= FWD64, (name, l)


def test_solve_meets_tolerance(pair):
    name, prob, gpu, ora = pair
    rng = np.random.default_rng(5)
    b_all = rng.standard_normal((prob.Nt, prob.pt + 1, gpu.n_edges))
    b = ora.to_interior(b_all)
    x, rep = gpu.solve(_dev(b_all))
    rr = np.linalg.norm(ora.levels[0].residual(ora.to_interior(_host(x)), b)) / np.linalg.norm(b)
    print(f"[long horizon] {name}: {gpu.n_levels} levels, cycles {rep['cycles']}, oracle residual {rr:.2e}")
    assert rep["rel_res"] <= 1e-8 and rr <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("name", ["N1024_p1", "N2048_p0", "N1024_p1_c16_rows"])
def test_precision_form_long_rows(name):
    from paper_1911_09548_amd import stmg
    from oracle.vcycle import SpaceTimeMultigrid
    Nt, pt, chunk, sched = CASES[name]
    prob = inputs.config_block_random(n=4, Nt=Nt, pt=pt, seed=22, block_hexes=2)
    gpu = stmg.Solver(prob, precision=stmg.FP32_REFINED, stream_chunk=chunk, row_schedule=sched)
    ora = SpaceTimeMultigrid(prob)
    b_all = np.random.default_rng(6).standard_normal((Nt, pt + 1, gpu.n_edges))
    b = ora.to_interior(b_all)
    x, rep = gpu.solve(_dev(b_all))
    rr = np.linalg.norm(ora.levels[0].residual(ora.to_interior(_host(x)), b)) / np.linalg.norm(b)
    print(f"[long horizon fp32-refined] {name}: cycles {rep['cycles']}, oracle residual {rr:.2e}")
    gpu.close()
    assert rr <= 1e-8 * (1 + 1e-6)
