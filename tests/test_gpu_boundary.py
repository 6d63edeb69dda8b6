"""GPU checks of entry points around the solver (no oracle needed):

* stmg_vcycle (one cycle on caller data) gives bitwise the iterate of one
  cycle of the split form (stmg_load / stmg_cycles / stmg_store) from the
  same start, in both forms, and k calls give k cycles;
* allocation failures injected at device allocations of a setup return
  STMG_ENOMEM and release every device buffer the setup had made: free
  device memory returns to its level before the call, and a following setup
  on the same process solves normally;
* the setup's parallel slab factorisations give bitwise the factors and
  solves of a setup on one stream.
"""
import numpy as np
import pytest

from paper_1911_09548_amd import inputs

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("precision", [0, 1])
def test_vcycle_equals_split_cycles(precision):
    import torch
    from paper_1911_09548_amd import stmg
    prob = inputs.config_block_random(n=8, Nt=16, pt=1, seed=21, block_hexes=4)
    print(f"\n[case] stmg_vcycle, 8^3 x 16, precision {precision}", flush=True)
    gpu = stmg.Solver(prob, precision=precision)
    try:
        rng = np.random.default_rng(4)
        E = gpu.n_edges
        b = _dev(rng.standard_normal((prob.Nt, 2, E)))
        x0 = _dev(rng.standard_normal((prob.Nt, 2, E)))
        for k in (1, 3):
            x = x0.clone()
            for _ in range(k):
                gpu.vcycle(b, x)
            gpu.load(b, None, x0)
            gpu.cycles(k, want_residuals=False)
            ref = gpu.store()
            torch.cuda.synchronize()
            assert torch.equal(x, ref), (precision, k)
    finally:
        gpu.close()


def test_injected_device_allocation_failures_release_memory():
    import torch
    from paper_1911_09548_amd import stmg
    prob = inputs.config_block_random(n=8, Nt=16, pt=1, seed=22, block_hexes=4)
    print("\n[case] allocation failures, 8^3 x 16", flush=True)
    torch.cuda.synchronize()
    stmg.debug_fail_alloc(0)
    ok = stmg.Solver(prob, device_factor=1)
    n = stmg.debug_fail_alloc(0)
    ok.close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    # every device-phase point sits after the host phase's points; sample
    # the whole range including the last point
    ks = sorted(set(list(range(1, n + 1, max(1, n // 12))) + [n]))
    for k in ks:
        stmg.debug_fail_alloc(k)
        with pytest.raises(stmg.StmgError) as e:
            stmg.Solver(prob, device_factor=1)
        assert e.value.code == stmg.STMG_ENOMEM, (k, e.value)
        torch.cuda.synchronize()
        free = torch.cuda.mem_get_info()[0]
        assert free0 - free < (64 << 20), (k, free0 - free)
    stmg.debug_fail_alloc(0)
    gpu = stmg.Solver(prob, device_factor=1, rtol=1e-8)
    try:
        rng = np.random.default_rng(5)
        b = _dev(rng.standard_normal((prob.Nt, 2, gpu.n_edges)))
        _, rep = gpu.solve(b)
        assert rep["rel_res"] <= 1e-8
    finally:
        gpu.close()


def test_setup_refuses_before_allocating_beyond_free_memory():
    """A handle whose estimated device bytes exceed the free device memory
    (12^3 mesh, 2^19 slabs: hundreds of GB of vectors) is refused with
    STMG_ENOMEM by the estimate, before any device allocation."""
    import torch
    from paper_1911_09548_amd import stmg
    prob = inputs.config_block_random(n=12, Nt=2 ** 19, pt=1, seed=23, block_hexes=4)
    print("\n[case] 12^3 x 2^19 slabs: refused by the estimate", flush=True)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    stmg.debug_fail_alloc(0)
    with pytest.raises(stmg.StmgError) as e:
        stmg.Solver(prob, device_factor=0)
    n_alloc = stmg.debug_fail_alloc(0)
    assert e.value.code == stmg.STMG_ENOMEM and "free" in str(e.value), e.value
    torch.cuda.synchronize()
    assert abs(torch.cuda.mem_get_info()[0] - free0) < (64 << 20)
    print(f"[enomem] {e.value}; host-phase allocation points {n_alloc}")


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_equals_eager_launches(precision):
    """Iterations replayed from the captured HIP graph give bitwise the
    iterates and residual norms of eager launches, over several replays with
    eager work (a residual, a layout conversion) and synchronisations between
    them, and in stmg_solve."""
    import torch
    from paper_1911_09548_amd import stmg
    prob = inputs.config_block_random(n=8, Nt=32, pt=1, seed=24, block_hexes=4)
    print(f"\n[case] graph replay, 8^3 x 32, precision {precision}", flush=True)
    rng = np.random.default_rng(6)
    solvers = {g: stmg.Solver(prob, precision=precision, graph=g) for g in (1, 0)}
    try:
        b = _dev(rng.standard_normal((prob.Nt, 2, solvers[0].n_edges)))
        got = {}
        for g, s in solvers.items():
            s.load(b)
            seq = []
            for k in (1, 3, 2):
                h = s.cycles(k)
                x = s.store().clone()
                r = s.residual(x, b)          # eager work between replays
                torch.cuda.synchronize()
                seq.append((h, x, r))
            x_solve, rep = s.solve(b)
            torch.cuda.synchronize()
            got[g] = (seq, x_solve.clone(), rep["history"])
        for (hg, xg, rg), (he, xe, re_) in zip(got[1][0], got[0][0]):
            assert np.array_equal(hg, he)
            assert torch.equal(xg, xe) and torch.equal(rg, re_)
        assert torch.equal(got[1][1], got[0][1]) and got[1][2] == got[0][2]
        print(f"[graph] {len(got[1][2])} solve cycles, replays bitwise equal to eager launches")
    finally:
        for s in solvers.values():
            s.close()


def test_parallel_setup_equals_one_stream(monkeypatch):
    """The slab factorisations on worker threads (the default) give bitwise
    the factors, iterates and residual history of a setup on one stream
    (STMG_SETUP_THREADS=1), in both forms."""
    import torch
    from paper_1911_09548_amd import stmg
    prob = inputs.config_block_random(n=8, Nt=64, pt=1, seed=25, block_hexes=4)
    print("\n[case] parallel setup against one stream, 8^3 x 64", flush=True)
    for precision in (0, 1):
        out = {}
        for threads in ("1", "8"):
            monkeypatch.setenv("STMG_SETUP_THREADS", threads)
            s = stmg.Solver(prob, precision=precision, device_factor=1, rtol=1e-9)
            try:
                b = _dev(np.random.default_rng(8).standard_normal((prob.Nt, 2, s.n_edges)))
                x, rep = s.solve(b)
                torch.cuda.synchronize()
                out[threads] = (x.clone(), rep["history"], [s.export_factor(l, 0)["panel"]
                                                           for l in range(s.n_levels) if precision == 0])
            finally:
                s.close()
        (x1, h1, f1), (x8, h8, f8) = out["1"], out["8"]
        assert torch.equal(x1, x8) and h1 == h8, precision
        assert all(np.array_equal(a, c) for a, c in zip(f1, f8)), precision
    monkeypatch.delenv("STMG_SETUP_THREADS")
