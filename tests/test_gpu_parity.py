"""GPU parity: every step of the HIP V-cycle against the CPU oracle.

Each level operation (residual, smoother S, nodal correction A, SAS, slab
solve, restriction, prolongation, V-cycle) is called through the C ABI on
seeded inputs and compared element by element with the oracle's result for
the same inputs. Sizes are chosen so the solves span several supernode
heights, diagonal blocks of more than 64 columns, several right-hand-side
column tiles and ragged tails, with both DG degrees.

Tolerances (FP64, relative to the output norm): a step that applies sparse
operators only is compared at 1e-13; a step that goes through a triangular
solve at 50 * kappa * u (u = 2^-53, kappa the 2-norm condition number of the
SPD matrix it factors: M + tau K for the slab block, K_n for the nodal
correction), never tighter than 1e-12. Backward-stable solves in either
implementation differ by at most a small multiple of kappa * u.
"""
import functools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_1911_09548_amd import inputs

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


U = 2.0 ** -53


def _cond_spd(A):
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    return float(lmax / lmin)


@functools.lru_cache(maxsize=None)
def _tols(name, l):
    ora = _ORACLES[name]
    lev = ora.levels[l]
    ks = _cond_spd((lev.space.M + lev.tau * lev.space.K).tocsc())
    kn = _cond_spd(lev.space.Kn.tocsc()) if lev.space.n_v > 1 else 1.0
    return max(1e-12, 50 * ks * U), max(1e-12, 50 * kn * U)


_ORACLES = {}


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


CASES = {
    # name: (problem factory, description)
    "unit_n4_N16_p1": lambda: inputs.config_unit_manufactured(4, 16, 1),
    "block_n8_N32_p1": lambda: inputs.config_block_random(n=8, Nt=32, pt=1, seed=5, block_hexes=4),
    "block_n8_N8_p0": lambda: inputs.config_block_random(n=8, Nt=8, pt=0, seed=6, block_hexes=4),
    "jitter_n6_N16_p1": lambda: inputs.config_core_box(n=6, Nt=16, pt=1, seed=2, jitter=0.2),
    # forced 64-row GEMM tiles (the per-launch choice picks 32 rows on small meshes)
    "block_n8_N64_p1_rows64": lambda: inputs.config_block_random(n=8, Nt=64, pt=1, seed=8, block_hexes=4),
    "block_n8_N16_p0_rows64": lambda: inputs.config_block_random(n=8, Nt=16, pt=0, seed=9, block_hexes=4),
    # backward read from P (no stored transpose) and forced split-K backward
    "block_n8_N32_p1_noT_split3": lambda: inputs.config_block_random(n=8, Nt=32, pt=1, seed=12, block_hexes=4),
    "unit_n4_N16_p0_split2": lambda: inputs.config_unit_manufactured(4, 16, 0),
    # numeric factorisation on the GPU (automatic only for large factors)
    "block_n8_N32_p1_devfactor": lambda: inputs.config_block_random(n=8, Nt=32, pt=1, seed=14, block_hexes=4),
    "jitter_n6_N16_p0_devfactor": lambda: inputs.config_core_box(n=6, Nt=16, pt=0, seed=3, jitter=0.2),
}
OPTS = {"block_n8_N64_p1_rows64": dict(gemm_rows=64), "block_n8_N16_p0_rows64": dict(gemm_rows=64),
        "block_n8_N32_p1": dict(gemm_rows=32),
        "block_n8_N32_p1_noT_split3": dict(factor_transpose=0, gemm_splitk=3),
        "unit_n4_N16_p0_split2": dict(gemm_splitk=2),
        "block_n8_N32_p1_devfactor": dict(device_factor=1),
        "jitter_n6_N16_p0_devfactor": dict(device_factor=1)}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    from paper_1911_09548_amd import stmg
    from oracle.vcycle import SpaceTimeMultigrid
    prob = CASES[request.param]()
    print(f"\n[case] {request.param}", flush=True)
    gpu = stmg.Solver(prob, **OPTS.get(request.param, {}))
    ora = SpaceTimeMultigrid(prob)
    _ORACLES[request.param] = ora
    yield request.param, prob, gpu, ora
    gpu.close()


def test_hierarchy_matches(pair):
    name, prob, gpu, ora = pair
    assert gpu.n_levels == len(ora.specs)
    for l, spec in enumerate(ora.specs):
        li = gpu.level_info(l)
        assert (li.mesh, li.N) == (spec.space, spec.N)
        assert abs(li.tau - spec.tau) <= 1e-15 * spec.tau


def _vec(ora, l, seed):
    lev = ora.levels[l]
    rng = np.random.default_rng(seed)
    return rng.standard_normal((lev.N, ora.q, lev.space.n_e))


def test_residual(pair):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora = pair
    for l in range(gpu.n_levels):
        x, b = _vec(ora, l, 1), _vec(ora, l, 2)
        ref = ora.levels[l].residual(x, b)
        got = _host(gpu.level_apply(l, stmg.OP_RESIDUAL, _dev(x), _dev(b)))
        assert _rel(got, ref) <= 1e-13, (name, l)


def test_slab_solve(pair):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora = pair
    for l in range(gpu.n_levels):
        r = _vec(ora, l, 3)
        ref = ora.levels[l].slab.solve(r)
        got = _host(gpu.level_apply(l, stmg.OP_SLAB_SOLVE, _dev(r)))
        tol = _tols(name, l)[0]
        print(f"[slab] {name} level {l}: rel {_rel(got, ref):.2e} tol {tol:.1e}")
        assert _rel(got, ref) <= tol, (name, l, _rel(got, ref))


@pytest.mark.parametrize("op", ["S", "A", "SAS"])
def test_smoothers(pair, op):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora = pair
    code = {"S": stmg.OP_SMOOTH_S, "A": stmg.OP_NODAL_A, "SAS": stmg.OP_SAS}[op]
    for l in range(gpu.n_levels):
        lev = ora.levels[l]
        x, b = _vec(ora, l, 4), _vec(ora, l, 5)
        if op == "S":
            ref = lev.smooth_S(x, b, 0.5)
        elif op == "A":
            ref = lev.nodal_A(x, b)
        else:
            ref = lev.smooth_SAS(x, b, 0.5, True)
        got = _host(gpu.level_apply(l, code, _dev(x), _dev(b)))
        ts, tn = _tols(name, l)
        tol = {"S": ts, "A": tn, "SAS": max(ts, tn)}[op]
        print(f"[{op}] {name} level {l}: rel {_rel(got, ref):.2e} tol {tol:.1e}")
        assert _rel(got, ref) <= tol, (name, op, l, _rel(got, ref))


def test_transfers(pair):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora = pair
    for l in range(gpu.n_levels - 1):
        r = _vec(ora, l, 6)
        ref = ora.restrict(l, r)
        got = _host(gpu.level_apply(l, stmg.OP_RESTRICT, _dev(r)))
        assert _rel(got, ref) <= 1e-13, (name, "restrict", l)
        e = _vec(ora, l + 1, 7)
        ref = ora.prolong(l, e)
        got = _host(gpu.level_apply(l + 1, stmg.OP_PROLONG, _dev(e)))
        assert _rel(got, ref) <= 1e-13, (name, "prolong", l)


def test_vcycle(pair):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora = pair
    x, b = _vec(ora, 0, 8), _vec(ora, 0, 9)
    ref = ora.vcycle(0, x, b)
    got = _host(gpu.level_apply(0, stmg.OP_VCYCLE, _dev(x), _dev(b)))
    tol = max(max(_tols(name, l)) for l in range(gpu.n_levels))
    print(f"[vcycle] {name}: rel {_rel(got, ref):.2e} tol {tol:.1e}")
    assert _rel(got, ref) <= tol, (name, _rel(got, ref))


def test_full_solve_history_and_solution(pair):
    name, prob, gpu, ora = pair
    rng = np.random.default_rng(10)
    E = gpu.n_edges
    b_all = rng.standard_normal((prob.Nt, prob.pt + 1, E))
    u0 = rng.standard_normal(E)
    b = ora.fold_initial(ora.to_interior(b_all), u0)
    x_ref, hist_ref = ora.solve(b, rtol=1e-11, max_cycles=60)
    # split API: the same number of cycles as the oracle needed for 1e-11
    gpu.load(_dev(b_all), _dev(u0))
    hist = gpu.cycles(len(hist_ref))
    x = _host(gpu.store())
    # per-cycle relative residuals agree to 1e-8 relative, down to a floor of
    # 1e-15 (roundoff of ||b - Lx|| / ||b|| itself)
    for k, (h, hr) in enumerate(zip(hist, hist_ref)):
        assert abs(h - hr) <= 1e-8 * hr + 1e-15, (name, k, h, hr)
    assert hist[-1] <= 1e-10
    # the oracle's residual of the GPU solution
    x_int = ora.to_interior(x)
    rr = np.linalg.norm(ora.levels[0].residual(x_int, b)) / np.linalg.norm(b)
    assert rr <= 1e-10, (name, rr)
    tol = max(1e-9, max(max(_tols(name, l)) for l in range(gpu.n_levels)))
    print(f"[solve] {name}: cycles {len(hist)} oracle-residual {rr:.2e} "
          f"|x - x_oracle|/|x_oracle| {_rel(x_int, x_ref):.2e} tol {tol:.1e}")
    assert _rel(x_int, x_ref) <= tol
    bnd = np.ones(E, dtype=bool)
    bnd[ora.fine.ie] = False
    assert np.all(x[..., bnd] == 0.0)


def test_full_layout_residual(pair):
    name, prob, gpu, ora = pair
    rng = np.random.default_rng(11)
    E = gpu.n_edges
    b_all = rng.standard_normal((prob.Nt, prob.pt + 1, E))
    x_all = rng.standard_normal((prob.Nt, prob.pt + 1, E))
    u0 = rng.standard_normal(E)
    r = _host(gpu.residual(_dev(x_all), _dev(b_all), _dev(u0)))
    b = ora.fold_initial(ora.to_interior(b_all), u0)
    ref = ora.levels[0].residual(ora.to_interior(x_all), b)
    assert _rel(ora.to_interior(r), ref) <= 1e-13
    bnd = np.ones(E, dtype=bool)
    bnd[ora.fine.ie] = False
    assert np.all(r[..., bnd] == 0.0)


def test_edge_numbering_matches_definition(pair):
    name, prob, gpu, ora = pair
    assert np.array_equal(gpu.edges(), ora.fine.topo.edges)
