"""GPU parity of the precision form: FP32 smoother, SpMV, slab and nodal
solves inside an FP64 refinement loop (FP64 outer residual, FP64 factors
rounded to FP32, FP64 coarsest solve).

Each FP32 level operation is checked with bounds that do not depend on a
condition number (tests/_parity.py):
* residual: 1e-5 relative, norm-wise and entry-wise (FP32 sparse sums);
* slab solve: normwise backward error against the oracle's FP64 slab block
  <= 1e-6 (the coarsest level solves in FP64: <= 1e-14 and forward <= 1e-10);
* S as a solve A (x' - x) = omega (b - L x): backward error <= 1e-6;
* A: the new residual's gradient component <= 1e-6 of its rounding scale
  (exact nodal solves; with k Chebyshev steps the refined solve below is
  the check);
* SAS: bitwise equal to the GPU's S, A, S applied by three separate calls.
* inexact slab solves (k two-grid Richardson steps in FP32, section 5): the
  slab solve and S against the oracle's FP64 iteration of the same k steps,
  forward <= 1e-3. The difference is FP32 rounding carried through the FP32
  coarse solves and grows with the level's tau (measured 2.5e-6 on the top
  level to 1.1e-4 on the coarsest two-grid level); the bound catches a wrong
  step (an O(1) difference), and the refined solve's oracle residual below
  is the accuracy check. The backward errors above belong to exact solves.
A refined solve to 1e-8 must have an oracle-computed relative residual
<= 1e-8; its distance to the oracle's FP64 solution is reported per case.
One-slab problems (the coarsest level is the finest) are solved in both
forms and compared with the oracle's direct slab solve.
"""
import numpy as np
import pytest

from paper_1911_09548_amd import inputs
from _parity import BWD32, BWD64, FWD64, fwd, gradient_orthogonality, slab_backward_error, smoother_backward_error

pytestmark = pytest.mark.gpu

CASES = {
    "unit_n4_N16_p1": lambda: inputs.config_unit_manufactured(4, 16, 1),
    "block_n8_N32_p1": lambda: inputs.config_block_random(n=8, Nt=32, pt=1, seed=5, block_hexes=4),
    "block_n8_N8_p0": lambda: inputs.config_block_random(n=8, Nt=8, pt=0, seed=6, block_hexes=4),
    "block_n8_N16_p1_devfactor": lambda: inputs.config_block_random(n=8, Nt=16, pt=1, seed=7, block_hexes=4),
    "tg2_block_n8_N64_p1": lambda: inputs.config_block_random(n=8, Nt=64, pt=1, seed=21, block_hexes=4),
    "tg1_block_n8_N16_p0_devfactor": lambda: inputs.config_block_random(n=8, Nt=16, pt=0, seed=20, block_hexes=4),
    "neumann_block_n8_N16_p1": lambda: _neumann(inputs.config_block_random(n=8, Nt=16, pt=1, seed=26, block_hexes=4)),
    "cheb3_block_n8_N32_p1": lambda: inputs.config_block_random(n=8, Nt=32, pt=1, seed=27, block_hexes=4),
}
OPTS = {"block_n8_N16_p1_devfactor": dict(device_factor=1), "tg2_block_n8_N64_p1": dict(slab=2),
        "tg1_block_n8_N16_p0_devfactor": dict(slab=1, device_factor=1), "cheb3_block_n8_N32_p1": dict(nodal=3)}
ORACLE_OPTS = {"tg2_block_n8_N64_p1": dict(slab_solver="twogrid:2"),
               "tg1_block_n8_N16_p0_devfactor": dict(slab_solver="twogrid:1"),
               "cheb3_block_n8_N32_p1": dict(nodal_cheb=3)}
FWD32_INEXACT = 1e-3


def _neumann(prob):
    prob.bc = "neumann"
    return prob


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
    prob = CASES[request.param]()
    print(f"\n[case] {request.param} (precision form)", flush=True)
    gpu = stmg.Solver(prob, precision=stmg.FP32_REFINED, rtol=1e-8, **OPTS.get(request.param, {}))
    ora = SpaceTimeMultigrid(prob, **ORACLE_OPTS.get(request.param, {}))
    tols = None
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
        assert fwd(got, lev.residual(x, b)) <= 1e-5, (name, "residual", l)
        got = _host(gpu.level_apply(l, stmg.OP_SLAB_SOLVE, _dev(x)))
        inexact = type(lev.slab).__name__ == "SlabSolverTwoGrid"
        eta, d = (0.0 if inexact else slab_backward_error(lev, got, x)), fwd(got, lev.slab.solve(x))
        print(f"[fp32 slab] {name} level {l}: backward error {eta:.1e}, forward {d:.1e}")
        if l == last:
            assert eta <= BWD64 and d <= FWD64, (name, "slab", l, eta, d)
            continue
        assert eta <= BWD32 and (not inexact or d <= FWD32_INEXACT), (name, "slab", l, eta, d)
        got = _host(gpu.level_apply(l, stmg.OP_SMOOTH_S, _dev(x), _dev(b)))
        e = 0.0 if inexact else smoother_backward_error(lev, x, b, got)
        dS = fwd(got, lev.smooth_S(x, b))
        print(f"[fp32 S] {name} level {l}: backward error {e:.1e}, forward {dS:.1e}")
        assert e <= BWD32 and (not inexact or dS <= FWD32_INEXACT), (name, "S", l, e, dS)
        got = _host(gpu.level_apply(l, stmg.OP_NODAL_A, _dev(x), _dev(b)))
        if lev.space.n_v > 0 and lev.nodal_cheb == 0:  # only an exact nodal solve removes the gradient part
            e = gradient_orthogonality(lev, got, b)
            print(f"[fp32 A] {name} level {l}: gradient residual {e:.1e}, forward {fwd(got, lev.nodal_A(x, b)):.1e}")
            assert e <= 1e-6, (name, "A", l, e)
        got = _host(gpu.level_apply(l, stmg.OP_SAS, _dev(x), _dev(b)))
        s1 = gpu.level_apply(l, stmg.OP_SMOOTH_S, _dev(x), _dev(b))
        a1 = gpu.level_apply(l, stmg.OP_NODAL_A, s1, _dev(b))
        s2 = _host(gpu.level_apply(l, stmg.OP_SMOOTH_S, a1, _dev(b)))
        assert np.array_equal(got, s2), (name, "SAS", l)


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


@pytest.mark.parametrize("pt", [0, 1])
@pytest.mark.parametrize("form", ["fp64", "fp32_refined"])
def test_one_slab(pt, form):
    """N_t = 1: the only level is the coarsest, solved exactly with the FP64
    factor; in the precision form each refinement iteration solves the FP32
    residual in FP64. The result is the oracle's direct slab solve."""
    from paper_1911_09548_amd import stmg
    from oracle.vcycle import SpaceTimeMultigrid
    prob = inputs.config_block_random(n=8, Nt=1, pt=pt, seed=31, block_hexes=4)
    print(f"\n[case] one slab pt={pt} {form}", flush=True)
    prec = stmg.FP64 if form == "fp64" else stmg.FP32_REFINED
    gpu = stmg.Solver(prob, precision=prec, rtol=1e-10, max_cycles=20)
    ora = SpaceTimeMultigrid(prob)
    assert gpu.n_levels == 1 and len(ora.levels) == 1
    b_all = np.random.default_rng(32).standard_normal((1, pt + 1, gpu.n_edges))
    b = ora.to_interior(b_all)
    x_ref = ora.levels[0].solve_exact_single_slab(b)
    for rep_i in range(2):  # a second solve on the same handle starts clean
        x, rep = gpu.solve(_dev(b_all))
        xi = ora.to_interior(_host(x))
        rr = np.linalg.norm(ora.levels[0].residual(xi, b)) / np.linalg.norm(b)
        print(f"[one slab] pt={pt} {form}: cycles {rep['cycles']}, oracle residual {rr:.2e}, "
              f"forward {fwd(xi, x_ref):.2e}")
        assert rep["rel_res"] <= 1e-10 and rr <= 1e-10
        assert fwd(xi, x_ref) <= FWD64
        assert rep["cycles"] <= (1 if form == "fp64" else 10)
    gpu.close()
