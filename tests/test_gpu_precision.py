"""GPU parity of the precision form: FP32 smoother, SpMV, slab and nodal
solves inside an FP64 refinement loop (FP64 outer residual, FP64 factors
rounded to FP32, FP64 coarsest solve).

* Each FP32 level operation is compared with the FP64 oracle on the same
  inputs at 50 * kappa * u32 (u32 = 2^-24, kappa the 2-norm condition number
  of the SPD matrix the step factors), never tighter than 1e-5; sparse-only
  steps at 1e-5.
* A refined solve to 1e-8 must have an oracle-computed relative residual
  <= 1e-8; its distance to the oracle's FP64 solution is reported per case.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_1911_09548_amd import inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24

CASES = {
    "unit_n4_N16_p1": lambda: inputs.config_unit_manufactured(4, 16, 1),
    "block_n8_N32_p1": lambda: inputs.config_block_random(n=8, Nt=32, pt=1, seed=5, block_hexes=4),
    "block_n8_N8_p0": lambda: inputs.config_block_random(n=8, Nt=8, pt=0, seed=6, block_hexes=4),
    "block_n8_N16_p1_devfactor": lambda: inputs.config_block_random(n=8, Nt=16, pt=1, seed=7, block_hexes=4),
}
OPTS = {"block_n8_N16_p1_devfactor": dict(device_factor=1)}


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _cond_spd(A):
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    return float(lmax / lmin)


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    from paper_1911_09548_amd import stmg
    from oracle.vcycle import SpaceTimeMultigrid
    prob = CASES[request.param]()
    print(f"\n[case] {request.param} (precision form)", flush=True)
    gpu = stmg.Solver(prob, precision=stmg.FP32_REFINED, rtol=1e-8, **OPTS.get(request.param, {}))
    ora = SpaceTimeMultigrid(prob)
    tols = []
    for lev in ora.levels:
        ks = _cond_spd((lev.space.M + lev.tau * lev.space.K).tocsc())
        kn = _cond_spd(lev.space.Kn.tocsc()) if lev.space.n_v > 1 else 1.0
        tols.append((max(1e-5, 50 * ks * U32), max(1e-5, 50 * kn * U32)))
    yield request.param, prob, gpu, ora, tols
    gpu.close()


def _vec(ora, l, seed):
    lev = ora.levels[l]
    return np.random.default_rng(seed).standard_normal((lev.N, ora.q, lev.space.n_e))


def test_fp32_steps(pair):
    from paper_1911_09548_amd import stmg
    name, prob, gpu, ora, tols = pair
    last = len(ora.levels) - 1
    for l, lev in enumerate(ora.levels):
        x, b = _vec(ora, l, 1), _vec(ora, l, 2)
        got = _host(gpu.level_apply(l, stmg.OP_RESIDUAL, _dev(x), _dev(b)))
        assert _rel(got, lev.residual(x, b)) <= 1e-5, (name, "residual", l)
        got = _host(gpu.level_apply(l, stmg.OP_SLAB_SOLVE, _dev(x)))
        tol = tols[l][0] if l < last else 1e-11 * max(1.0, tols[l][0] / 1e-5)  # coarsest: FP64
        assert _rel(got, lev.slab.solve(x)) <= tol, (name, "slab", l, _rel(got, lev.slab.solve(x)))
        if l == last:
            continue
        ts, tn = tols[l]
        for code, ref, tol in ((stmg.OP_SMOOTH_S, lev.smooth_S(x, b, 0.5), ts),
                               (stmg.OP_NODAL_A, lev.nodal_A(x, b), tn),
                               (stmg.OP_SAS, lev.smooth_SAS(x, b, 0.5, True), max(ts, tn))):
            got = _host(gpu.level_apply(l, code, _dev(x), _dev(b)))
            print(f"[fp32 op {code}] {name} level {l}: rel {_rel(got, ref):.2e} tol {tol:.1e}")
            assert _rel(got, ref) <= tol, (name, code, l, _rel(got, ref))


def test_refined_solve(pair):
    name, prob, gpu, ora, tols = pair
    rng = np.random.default_rng(13)
    E = gpu.n_edges
    b_all = rng.standard_normal((prob.Nt, prob.pt + 1, E))
    u0 = rng.standard_normal(E)
    b = ora.fold_initial(ora.to_interior(b_all), u0)
    x_ref, hist_ref = ora.solve(b, rtol=1e-12, max_cycles=60)
    x, rep = gpu.solve(_dev(b_all), _dev(u0))
    xi = ora.to_interior(_host(x))
    rr = np.linalg.norm(ora.levels[0].residual(xi, b)) / np.linalg.norm(b)
    err = _rel(xi, x_ref)
    print(f"[fp32-refined] {name}: cycles {rep['cycles']} (FP64 oracle needs "
          f"{next(k + 1 for k, h in enumerate(hist_ref) if h <= 1e-8)} for 1e-8), "
          f"oracle residual {rr:.2e}, |x - x_fp64| / |x_fp64| = {err:.2e}")
    assert rep["rel_res"] <= 1e-8
    assert rr <= 1e-8
    assert err <= 1e-6
    fp64_cycles = next(k + 1 for k, h in enumerate(hist_ref) if h <= 1e-8)
    assert rep["cycles"] <= fp64_cycles + 3
