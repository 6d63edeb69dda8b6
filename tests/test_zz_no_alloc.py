"""The no-allocation residual entry point against the allocating one.

stmg_residual_noalloc computes r = b - L x (eq. (1)) with its temporaries in
the library's fixed device array; stmg_residual allocates them on its first
call. Both run the same kernels in the same order, so their results agree
bitwise. Checked on two calls in a row, the second on a smaller problem (the
array keeps the first call's contents), that the no-allocation call leaves
the handle's device memory unchanged, and that a problem beyond the array's
size is refused with STMG_EINVAL.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1911_09548_amd import inputs

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case(n, Nt, pt, seed):
    from paper_1911_09548_amd import stmg
    prob = inputs.config_block_random(n=n, Nt=Nt, pt=pt, seed=seed, block_hexes=max(1, n // 2))
    gpu = stmg.Solver(prob)
    rng = np.random.default_rng(seed)
    E = gpu.n_edges
    x = rng.standard_normal((Nt, pt + 1, E))
    b = rng.standard_normal((Nt, pt + 1, E))
    u0 = rng.standard_normal(E)
    return gpu, _dev(x), _dev(b), _dev(u0)


def _device_bytes(gpu):
    from paper_1911_09548_amd import stmg
    info = stmg.Info()
    assert stmg.lib().stmg_info(gpu._h, C.byref(info)) == 0
    return info.device_bytes


@pytest.mark.parametrize("with_u0", [False, True])
def test_noalloc_residual_equals_residual(with_u0):
    import torch
    big = _case(6, 64, 1, 31)
    small = _case(4, 8, 0, 32)
    try:
        for name, (gpu, x, b, u0) in (("6^3 x 64, p_t 1", big), ("4^3 x 8, p_t 0", small)):
            print(f"\n[case] {name}, u0={with_u0}", flush=True)
            u = u0 if with_u0 else None
            before = _device_bytes(gpu)
            r_na = torch.full_like(b, np.nan)
            gpu.residual_noalloc(x, b, r_na, u0=u)
            torch.cuda.synchronize()
            assert _device_bytes(gpu) == before, "the no-allocation call allocated device memory"
            r = gpu.residual(x, b, u0=u)
            torch.cuda.synchronize()
            assert torch.equal(r_na, r)
            assert torch.isfinite(r).all()
    finally:
        big[0].close()
        small[0].close()


def test_noalloc_refuses_problems_beyond_the_array():
    from paper_1911_09548_amd import stmg
    import torch
    print("\n[case] 12^3 x 256, p_t 1 (over the array size)", flush=True)
    gpu, x, b, _ = _case(12, 256, 1, 33)
    try:
        r = torch.zeros_like(b)
        with pytest.raises(stmg.StmgError) as e:
            gpu.residual_noalloc(x, b, r)
        assert e.value.code == stmg.STMG_EINVAL
        assert "too large" in str(e.value)
    finally:
        gpu.close()
