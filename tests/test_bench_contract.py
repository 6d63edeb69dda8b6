"""CPU checks of bench.py's contract that need no GPU.

* More than one GPU is refused with exit code 2 and a message.
* The committed HBM-traffic summary was taken with the current kernel source
  (its hash matches), so the benchmark line reports `roofline.traffic` for the
  dominant solve kernel and the level-0 residual instead of null.
* The counter-summary parser maps rocprofv3 kernel names onto the library
  profiler's instantiation names.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_recorded_traffic_matches_current_kernels():
    import bench
    for kernel in ("k_sn_gemm<cd,32,32,bwdT>", "k_sn_gemm<cd,32,32,fwd>", "k_residual_grp<double,8,2>"):
        t = bench.recorded_traffic(kernel)
        assert t is not None and t > 0, (kernel, bench._source_sha())


def test_rocprof_names_map_to_profiler_names():
    import bench
    assert bench._kernel_key("void stmg::k_sn_gemm<stmg::cd, 32, 32, 2>(stmg::FactorDev, int)") == \
        "k_sn_gemm<cd,32,32,bwdT>"
    assert bench._kernel_key("void stmg::k_residual<double, 2, 2, false>(stmg::ResidualArgsT<double>, int, int)") == \
        "k_residual<double,2,2>"
    assert bench._kernel_key("void stmg::k_residual_grp<double, 8, 2>(stmg::ResidualArgsT<double>, int, int)") == \
        "k_residual_grp<double,8,2>"
