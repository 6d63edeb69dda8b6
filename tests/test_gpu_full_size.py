"""GPU parity at the benchmark's full size: 32^3 x 6 Kuhn tets (220,256
interior edges), N_t = 256, p_t = 1, block-random sigma and nu, seed 1, in
the launch configuration bench.py times (default options, GPU
factorisation).

The oracle's full V-cycle needs exact slab and nodal factors at this size
(minutes of setup, tens of GB), so these checks use what the oracle computes
here in seconds: its space-time operator L of eq. (1) and the slab block of
eq. (2) (assembly of M and K, the row formulas in the DG(1) time basis):
* the GPU residual b - L x against the oracle's, every entry (relative
  1e-13, as in the small parity suites);
* the level-0 slab solve, the path of the dominant kernels: its normwise
  backward error against the oracle's slab block is <= 1e-14 (a bound that
  does not depend on the conditioning);
* the FP64 solve to 1e-10: the oracle's relative residual of the GPU's final
  iterate is <= 1e-10 (the FP64 parity target); the precision form's solve
  to 1e-8 likewise <= 1e-8, with its distance to the FP64 solution printed.
"""
import os

import numpy as np
import pytest

from paper_1911_09548_amd import inputs
from _parity import BWD64, SPARSE64, fwd, slab_backward_error

pytestmark = pytest.mark.gpu

N, PT = 256, 1


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def full():
    from paper_1911_09548_amd import stmg
    from oracle.hierarchy import finest_space
    from oracle.vcycle import Level
    prob = inputs.config_block_random(n=32, Nt=N, pt=PT, seed=1, block_hexes=8)
    print("\n[case] full size 32^3 x 256, p_t = 1", flush=True)
    space = finest_space(prob)
    lev = Level.operator_only(space, PT, N, prob.T / N)
    gpu = stmg.Solver(prob, rtol=1e-10, max_cycles=100)
    assert gpu.level_info(0).n_e == space.n_e and gpu.level_info(0).N == N
    yield prob, space, lev, gpu
    gpu.close()


def test_residual_full_size(full):
    prob, space, lev, gpu = full
    rng = np.random.default_rng(21)
    x_all = rng.standard_normal((N, PT + 1, gpu.n_edges))
    b_all = rng.standard_normal((N, PT + 1, gpu.n_edges))
    got = _host(gpu.residual(_dev(x_all), _dev(b_all)))[..., space.ie]
    ref = lev.residual(x_all[..., space.ie], b_all[..., space.ie])
    print(f"[full] residual: rel {fwd(got, ref):.2e}")
    assert fwd(got, ref) <= SPARSE64


def test_slab_solve_full_size(full):
    from paper_1911_09548_amd import stmg
    prob, space, lev, gpu = full
    r = np.random.default_rng(22).standard_normal((N, PT + 1, space.n_e))
    z = _host(gpu.level_apply(0, stmg.OP_SLAB_SOLVE, _dev(r)))
    eta = slab_backward_error(lev, z, r)
    print(f"[full] slab solve: backward error {eta:.2e}, relative residual {_rel(lev.apply_slab(z), r):.2e}")
    assert eta <= BWD64


_X64 = {}


@pytest.mark.parametrize("form", ["fp64", "fp32_refined"])
def test_solve_full_size(full, form):
    from paper_1911_09548_amd import stmg
    prob, space, lev, gpu = full
    b_all = inputs.gaussian_rhs(gpu.n_edges, N, PT, seed=2)
    solver = gpu if form == "fp64" else stmg.Solver(prob, rtol=1e-8, max_cycles=100,
                                                    precision=stmg.FP32_REFINED)
    x, rep = solver.solve(_dev(b_all))
    if solver is not gpu:
        solver.close()
    b = b_all[..., space.ie]
    xi = _host(x)[..., space.ie]
    rr = np.linalg.norm(lev.residual(xi, b)) / np.linalg.norm(b)
    target = 1e-10 if form == "fp64" else 1e-8
    extra = ""
    if form == "fp64":
        _X64["x"] = xi
    elif "x" in _X64:
        extra = f", |x - x_fp64| / |x_fp64| = {_rel(xi, _X64['x']):.2e}"
    print(f"[full] solve {form}: {rep['cycles']} cycles, library {rep['rel_res']:.2e}, "
          f"oracle residual {rr:.2e}{extra}")
    assert rep["rel_res"] <= target and rr <= target * (1 + 1e-6)


@pytest.mark.parametrize("form", ["fp64", "fp32_refined"])
def test_core_box_solve(form):
    """The jittered high-contrast core box (sigma 1e4 / 1e-2, nu 1e-3 / 1) at
    24^3 x 128 slabs, larger than the parity suites' 6^3: the oracle's
    relative residual of the GPU's final iterate is <= 1e-10 in the FP64
    form and <= 1e-8 in the precision form."""
    from paper_1911_09548_amd import stmg
    from oracle.hierarchy import finest_space
    from oracle.vcycle import Level
    prob = inputs.config_core_box(n=24, Nt=128, pt=1, seed=3, jitter=0.2)
    print(f"\n[case] core box 24^3 x 128 {form}", flush=True)
    space = finest_space(prob)
    lev = Level.operator_only(space, 1, 128, prob.T / 128)
    prec = stmg.FP64 if form == "fp64" else stmg.FP32_REFINED
    target = 1e-10 if form == "fp64" else 1e-8
    gpu = stmg.Solver(prob, rtol=target, max_cycles=100, precision=prec)
    b_all = inputs.gaussian_rhs(gpu.n_edges, 128, 1, seed=2)
    x, rep = gpu.solve(_dev(b_all))
    levels = [(gpu.level_info(l).mesh, gpu.level_info(l).N) for l in range(gpu.n_levels)]
    gpu.close()
    b = b_all[..., space.ie]
    rr = np.linalg.norm(lev.residual(_host(x)[..., space.ie], b)) / np.linalg.norm(b)
    print(f"[core box] {form}: levels {levels}, {rep['cycles']} cycles, library {rep['rel_res']:.2e}, "
          f"oracle residual {rr:.2e}")
    assert rep["rel_res"] <= target and rr <= target * (1 + 1e-6)


@pytest.mark.skipif(os.environ.get("STMG_CORE_BOX_64") != "1",
                    reason="the 64^3 x 128 core box takes a minute of setup, up to two of solve and about "
                           "200 GB; run with STMG_CORE_BOX_64=1 (and a test timeout of 600 s)")
@pytest.mark.parametrize("form", ["fp32_refined", "fp64", "fp64_twogrid3", "fp32_refined_twogrid3"])
def test_core_box_64_full_size(form):
    """The high-contrast case at its stated size: 64^3 jittered Kuhn mesh
    (1,798,336 interior edges), N_t = 128, p_t = 1, without stored factor
    transposes. Either the setup refuses by its device-memory estimate
    (STMG_ENOMEM, before allocating: the exact slab factors of all eight
    levels on the 64^3 mesh), or the solve reaches the oracle's relative
    residual target (1e-8 precision form, 1e-10 FP64). With 3 two-grid
    Richardson steps per slab solve (section 5's inexact spatial solves) the
    levels above the coarsest keep only 32^3 slab factors and the case fits
    one GPU."""
    from paper_1911_09548_amd import stmg
    from oracle.hierarchy import finest_space
    from oracle.vcycle import Level
    prob = inputs.config_core_box(n=64, Nt=128, pt=1, seed=3, jitter=0.2)
    print(f"\n[case] core box 64^3 x 128 {form}", flush=True)
    prec = stmg.FP32_REFINED if form.startswith("fp32_refined") else stmg.FP64
    target = 1e-8 if form.startswith("fp32_refined") else 1e-10
    slab = 3 if form.endswith("twogrid3") else 0
    try:
        gpu = stmg.Solver(prob, rtol=target, max_cycles=100, precision=prec, factor_transpose=0, slab=slab)
    except stmg.StmgError as e:
        print(f"[core box 64] {form}: setup refused: {e}", flush=True)
        assert e.code == stmg.STMG_ENOMEM and "GB" in str(e) and slab == 0
        return
    b_all = inputs.gaussian_rhs(gpu.n_edges, 128, 1, seed=2)
    x, rep = gpu.solve(_dev(b_all))
    xh = _host(x)
    gpu.close()
    del x
    print(f"[core box 64] {form}: {rep['cycles']} cycles, {rep['solve_s']:.2f}s, setup {rep['setup_s']:.1f}s, "
          f"library {rep['rel_res']:.2e}", flush=True)
    space = finest_space(prob)
    lev = Level.operator_only(space, 1, 128, prob.T / 128)
    b = b_all[..., space.ie]
    rr = np.linalg.norm(lev.residual(xh[..., space.ie], b)) / np.linalg.norm(b)
    print(f"[core box 64] {form}: oracle residual {rr:.2e}", flush=True)
    assert rep["rel_res"] <= target and rr <= target * (1 + 1e-6)
