"""Benchmark: space-time DOF-updates/s per V-cycle on one MI355X.

Workload (default): unit cube, 32^3 hexes x 6 Kuhn tetrahedra, N_t = 256
slabs, DG degree 1 in time, sigma in [1, 1e3] and nu in [1, 100] log-uniform
on 8^3-hex blocks (seed 1), Gaussian right-hand side (seed 2), T = 1; FP64.
A step is one solver iteration: a full V-cycle over all levels (SAS
smoothing, nodal auxiliary correction, coarse-grid correction) followed by
the fine-level residual norm. Inputs are resident in HBM when timing starts.
The value comes from K timed steps without per-launch events; K more steps
with per-launch events give the kernel table and the rooflines.

Besides the FP64 line the run reports the precision form (FP32 V-cycle inside
FP64 refinement) on the same workload, the serving form (a seeded Poisson
stream of requests through the continuous-batching server: p50/p99 latency
and throughput), the roofline of the dominant kernel and of the residual, and
the CPU oracle on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--n 32 --Nt 256 --pt 1]
    python bench.py --pmc-summary FETCH.csv WRITE.csv   # counter summary, no GPU
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
KERNEL_SOURCE = os.path.join(ROOT, "paper_1911_09548_amd", "csrc", "kernels.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_32cube_Nt256_pt1_fp64.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(args):
    """Time the oracle on a bounded sample (runs in a child process, 1 thread)."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-sample",
           "--sample-n", str(args.sample_n), "--sample-Nt", str(args.sample_Nt), "--pt", str(args.pt),
           "--n", str(args.n), "--Nt", str(args.Nt)]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        log(r.stderr[-2000:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def _host_description():
    """CPU model, core count and the thread settings the oracle ran with."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    try:
        from threadpoolctl import threadpool_info
        threads["blas_pools"] = [{"api": d.get("internal_api"), "num_threads": d.get("num_threads")}
                                 for d in threadpool_info()]
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "threads": threads}


def oracle_sample(args):
    """Child: oracle V-cycles on the same material recipe at a smaller mesh,
    then the oracle's residual (eq. (1)) on the benchmark's own inputs."""
    import numpy as np
    from paper_1911_09548_amd import inputs
    from oracle.vcycle import SpaceTimeMultigrid, Level
    from oracle.hierarchy import finest_space
    prob = inputs.config_block_random(n=args.sample_n, Nt=args.sample_Nt, pt=args.pt, seed=1,
                                      block_hexes=max(1, args.sample_n // 4))
    t0 = time.perf_counter()
    ora = SpaceTimeMultigrid(prob, slab_solver="complex" if args.pt == 1 else "real")
    setup = time.perf_counter() - t0
    rng = np.random.default_rng(2)
    b = rng.standard_normal((prob.Nt, prob.pt + 1, ora.fine.n_e))
    x = np.zeros_like(b)
    times = []
    t_start = time.perf_counter()
    while len(times) < 2 or (time.perf_counter() - t_start < 10.0 and len(times) < 5):
        t = time.perf_counter()
        x = ora.vcycle(0, x, b)
        np.linalg.norm(ora.levels[0].residual(x, b))
        times.append(time.perf_counter() - t)
    t_cycle = float(np.median(times))
    dofs = ora.fine.n_e * prob.Nt * (prob.pt + 1)
    out = {"value": dofs / t_cycle, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
           "sample": (f"oracle V-cycle + residual norm, median of {len(times)} cycles, "
                      f"{args.sample_n}^3 Kuhn mesh ({ora.fine.n_e} interior edges), "
                      f"N_t={prob.Nt}, p_t={prob.pt}, same block-random material recipe; "
                      f"setup {setup:.1f}s excluded; 1 thread (SuperLU, scipy)"),
           "s_per_cycle": t_cycle, "host": _host_description()}
    if args.n > 0:
        # the residual of the benchmark's workload itself (the full oracle
        # V-cycle there needs the complex slab factors of every level: far
        # beyond a bounded sample)
        big = inputs.config_block_random(n=args.n, Nt=args.Nt, pt=args.pt, seed=1, block_hexes=8)
        sp = finest_space(big)
        t = time.perf_counter()
        lev = Level.operator_only(sp, big.pt, big.Nt, big.T / big.Nt, nodal=True)
        t_kn = time.perf_counter() - t
        xb = np.random.default_rng(3).standard_normal((big.Nt, big.pt + 1, sp.n_e))
        bb = np.random.default_rng(2).standard_normal(xb.shape)
        t = time.perf_counter()
        lev.residual(xb, bb)
        t_res = time.perf_counter() - t
        t = time.perf_counter()
        lev.nodal_A(xb, bb)
        t_nod = time.perf_counter() - t
        dofs_big = sp.n_e * big.Nt * (big.pt + 1)
        out["same_inputs"] = {"workload": f"{args.n}^3 x 6 Kuhn tets, N_t={big.Nt}, p_t={big.pt} (the GPU line's)",
                              "residual_s": t_res, "residual_dof_per_s": dofs_big / t_res,
                              "nodal_correction_s": t_nod, "nodal_factor_s": t_kn,
                              "note": ("one space-time residual b - L x (eq. (1)) and one nodal correction A "
                                       "(eq. (8): its residual, G^T, the K_n solve of all N_t (p_t+1) columns "
                                       "with the SuperLU factor, the time scan, G), 1 thread; the slab factors "
                                       "of this size do not fit a bounded sample")}
    print(json.dumps(out))


def serving_bench(args):
    """Serving form: a seeded Poisson stream of solve requests through the
    continuous-batching server (FP32 smoother, FP64 refinement to 1e-8).
    Arrivals run at 0.8x the single-stream capacity measured on the first
    requests of the same stream; latency is submission to result."""
    import numpy as np
    from paper_1911_09548_amd import inputs, stmg
    sizes = tuple(int(v) for v in args.serve_sizes.split(","))
    horizons = tuple(int(v) for v in args.serve_horizons.split(","))
    stream = inputs.request_stream(n_requests=args.serve_requests, rate=1.0, seed=5, sizes=sizes,
                                   horizons=horizons, degrees=(0, 1))
    problems = []
    log(f"[bench] serving: building {len(stream)} requests")
    for r in stream:
        prob = inputs.config_request(r["n"], r["Nt"], r["pt"], r["seed"])
        E = inputs.count_edges(prob.levels[0].tets, prob.levels[0].coords.shape[0])
        rhs = np.random.default_rng(r["seed"]).standard_normal((r["Nt"], r["pt"] + 1, E))
        problems.append((prob, rhs))
        if len(problems) % 8 == 0:
            log(f"[bench] serving: {len(problems)} requests built")
    opts32 = dict(precision=stmg.FP32_REFINED, rtol=1e-8, max_cycles=60)
    opts64 = dict(precision=stmg.FP64, rtol=1e-8, max_cycles=60)

    def one_at_a_time(opts, k):
        srv = stmg.Server(max_active=1, setup_threads=1)
        t = time.perf_counter()
        for prob, rhs in problems[:k]:
            tk = srv.submit(prob, rhs, **opts)
            assert srv.wait(tk, 600)
            rc, _, _ = srv.poll(tk, rhs.shape)
            assert rc == stmg.STMG_OK, rc
        dt = (time.perf_counter() - t) / k
        srv.close()
        return dt

    k = min(args.serve_probe, len(problems))
    single32 = one_at_a_time(opts32, k)
    single64 = one_at_a_time(opts64, k)
    log(f"[bench] serving: single-stream {single32:.3f} s/request (FP32 refined), {single64:.3f} (FP64), "
        f"first {k} requests one at a time")

    def closed_loop(batch):
        # saturated: every request submitted at once
        srv = stmg.Server(max_active=args.serve_active, setup_threads=args.serve_threads, batch=batch)
        tks = [srv.submit(prob, rhs, **opts32) for prob, rhs in problems]
        good = True
        for i, ((prob, rhs), tk) in enumerate(zip(problems, tks)):
            assert srv.wait(tk, 900)
            rc, _, _ = srv.poll(tk, rhs.shape)
            good &= rc == stmg.STMG_OK
            if (i + 1) % 8 == 0:
                log(f"[bench] serving (closed loop, batch={batch}): {i + 1} of {len(problems)} requests done")
        cst = srv.stats()
        srv.close()
        return {"throughput_req_s": cst["throughput_req_s"], "throughput_dof_updates_s": cst["throughput_dofs"],
                "p50_s": cst["p50_s"], "p99_s": cst["p99_s"], "batched_iterations": cst["batched_iterations"],
                "batched_request_iterations": cst["batched_members"], "all_converged": bool(good)}

    # the server's capacity on this mix: all requests submitted at once
    closed = {"batched": closed_loop(True)}
    if args.serve_closed:
        closed["unbatched"] = closed_loop(False)
    capacity = closed["batched"]["throughput_req_s"]
    log(f"[bench] serving, all submitted at once: {capacity:.2f} requests/s batched" +
        (f", {closed['unbatched']['throughput_req_s']:.2f} unbatched" if "unbatched" in closed else "") +
        f"; {1.0 / single32:.2f} requests/s single-stream (first {k} requests)")
    # Poisson arrivals at 0.8x that capacity: latency under load
    rate = 0.8 * capacity
    srv = stmg.Server(max_active=args.serve_active, setup_threads=args.serve_threads)
    t0 = time.perf_counter()
    tickets = []
    for (prob, rhs), r in zip(problems, stream):
        delay = r["arrival"] / rate - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(prob, rhs, **opts32))
    worst, ok = 0.0, True
    for i, ((prob, rhs), tk) in enumerate(zip(problems, tickets)):
        assert srv.wait(tk, 900)
        rc, _, rep = srv.poll(tk, rhs.shape)
        ok &= rc == stmg.STMG_OK
        worst = max(worst, rep["rel_res"])
        if (i + 1) % 8 == 0:
            log(f"[bench] serving: {i + 1} of {len(problems)} requests done")
    st = srv.stats()
    srv.close()
    log(f"[bench] serving: p50 {st['p50_s']:.3f} s, p99 {st['p99_s']:.3f} s, "
        f"{st['throughput_req_s']:.2f} requests/s, {st['throughput_dofs']:.3e} DOF-updates/s, "
        f"{st['batched_iterations']} batched iterations ({st['batched_members']} request iterations)")
    return {"form": "continuous batching, fp32 smoother + fp64 refinement to 1e-8",
            "requests": len(problems),
            "mix": (f"n in {sizes} (x6 Kuhn tets), N_t in {horizons}, p_t in (0, 1), "
                    "block-random sigma in [1e-2,1e4], nu in [1e-3,100], Gaussian rhs (seeded)"),
            "arrivals": f"Poisson, {rate:.3f} requests/s = 0.8x the saturated throughput of the same mix",
            "p50_s": st["p50_s"], "p99_s": st["p99_s"], "mean_s": st["mean_s"],
            "throughput_req_s": st["throughput_req_s"], "throughput_dof_updates_s": st["throughput_dofs"],
            "single_stream_s_per_request": {"fp32_refined": single32, "fp64": single64, "requests": k},
            "max_active": args.serve_active, "hbm_peak_bytes": st["hbm_peak"],
            "batched_iterations": st["batched_iterations"], "batched_request_iterations": st["batched_members"],
            "all_converged": bool(ok), "max_final_rel_res": worst, "closed_loop": closed}


def _source_sha():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _kernel_key(name):
    """rocprofv3 kernel name -> the profiler's instantiation name."""
    import re
    n = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("stmg::", "")
    n = n.replace(" ", "")
    m = re.match(r"k_sn_gemm<(\w+),(\d+),(\d+),(\d)>", n)
    if m:
        return f"k_sn_gemm<{m.group(1)},{m.group(2)},{m.group(3)},{['fwd', 'bwd', 'bwdT'][int(m.group(4))]}>"
    m = re.match(r"k_residual<(\w+),(\d+),(\d+),(true|false)>", n)
    if m:
        return f"k_residual<{m.group(1)},{m.group(2)},{m.group(3)}>"
    return n


def pmc_summary(fetch_csv, write_csv):
    """Per-kernel HBM bytes per dispatch from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by what the same
    counter reads for the plain copy kernel of known size in the same run
    (--hbm-calibrate). Prints a markdown table and one machine-readable line
    per kernel: `traffic <kernel> <fetch B> <write B> <kernels.hip sha>`."""
    import collections
    import csv

    def load(path, counter):
        agg = collections.defaultdict(lambda: [0, 0.0])
        calib = None
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if "neg_kernel" in r["Kernel_Name"]:
                calib = v
                continue
            a = agg[_kernel_key(r["Kernel_Name"])]
            a[0] += 1
            a[1] += v
        return agg, calib

    f, cf = load(fetch_csv, "FETCH_SIZE")
    w, cw = load(write_csv, "WRITE_SIZE")
    copy_kib = 1024.0 * 1024.0  # the calibration copy of the counter runs: --hbm-calibrate 1024
    sf, sw = copy_kib / cf, copy_kib / cw
    sha = _source_sha()
    print(f"Calibration: the 1 GiB copy reads FETCH_SIZE {cf:.0f} KiB (scale {sf:.3f}) and WRITE_SIZE "
          f"{cw:.0f} KiB (scale {sw:.3f}).\n")
    print("| kernel | dispatches | fetch MB / dispatch | write MB / dispatch |")
    print("|---|---|---|---|")
    rows = sorted(f.items(), key=lambda kv: -kv[1][1])
    for k, (n, tot) in rows[:20]:
        wn, wt = w.get(k, [1, 0.0])
        print(f"| `{k}` | {n} | {tot / n * sf / 1024:.1f} | {wt / max(wn, 1) * sw / 1024:.1f} |")
    print()
    for k, (n, tot) in rows[:20]:
        wn, wt = w.get(k, [1, 0.0])
        print(f"traffic {k} {tot / n * sf * 1024:.0f} {wt / max(wn, 1) * sw * 1024:.0f} {sha}")


def stats_summary(stats_csv, top=24):
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv):
    calls, total and average duration per kernel, with the library
    profiler's names beside rocprofv3's."""
    import csv
    rows = []
    for r in csv.DictReader(open(stats_csv)):
        rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
                     float(r.get("Percentage", 0.0))))
    rows.sort(key=lambda t: -t[2])
    cycle = ("k_sn_gemm", "k_sn_reduce", "k_residual", "k_fwd_asm", "k_slab_", "k_grad", "k_time_scan",
             "k_restrict", "k_prolong", "k_sum", "k_to_", "k_add_float", "k_fill", "k_cheb", "k_tg_",
             "k_csr_slabs", "k_scale_slabs", "k_axpy")
    for title, sel in (("Kernels of the V-cycle", lambda k: k.startswith(cycle)),
                       ("Other kernels (setup: numeric factorisation, uploads, layout changes)",
                        lambda k: not k.startswith(cycle))):
        print(f"### {title}\n")
        print("| kernel (rocprofv3) | profiler name | calls | total ms | avg us | % of GPU time |")
        print("|---|---|---|---|---|---|")
        for name, calls, tot, avg, pct in [r for r in rows if sel(_kernel_key(r[0]))][:top]:
            short = name if len(name) < 70 else name[:67] + "..."
            key = _kernel_key(name)
            key = key if len(key) < 48 else key[:45] + "..."
            print(f"| `{short}` | `{key}` | {calls} | {tot:.2f} | {avg:.2f} | {pct:.2f} |")
        print()


def sq_summary(sq_csv, cache_csv, top=14):
    """Shader and cache counters per kernel from two rocprofv3 --pmc runs:
    MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs x 1024
    SIMDs); waves per SIMD = 4 SQ_WAVE_CYCLES / (GRBM_GUI_ACTIVE / 8 x 1024);
    issue wait = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; L2 hit = TCC_HIT /
    (TCC_HIT + TCC_MISS). Sums over each kernel's dispatches."""
    import collections
    import csv

    def load(path):
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(set)
        for r in csv.DictReader(open(path)):
            k = _kernel_key(r["Kernel_Name"])
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k].add(r.get("Dispatch_Id", r.get("Correlation_Id", "")))
        return agg, disp

    sq, disp = load(sq_csv)
    cache, _ = load(cache_csv)
    rows = sorted(sq.items(), key=lambda kv: -kv[1].get("GRBM_GUI_ACTIVE", 0.0))
    print("| kernel | dispatches | MFMA busy % | waves per SIMD | issue wait % | L2 hit % | LDS bank conflicts |")
    print("|---|---|---|---|---|---|---|")
    for k, c in rows[:top]:
        active = c.get("GRBM_GUI_ACTIVE", 0.0) / 8.0 * 1024.0
        if active <= 0:
            continue
        mfma = 100.0 * c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / active
        waves = 4.0 * c.get("SQ_WAVE_CYCLES", 0.0) / active
        wait = 100.0 * c.get("SQ_WAIT_INST_ANY", 0.0) / max(c.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        h = cache.get(k, {})
        hit = 100.0 * h.get("TCC_HIT_sum", 0.0) / max(h.get("TCC_HIT_sum", 0.0) + h.get("TCC_MISS_sum", 0.0), 1.0)
        print(f"| `{k}` | {len(disp[k])} | {mfma:.1f} | {waves:.1f} | {wait:.1f} | {hit:.1f} | "
              f"{c.get('SQ_LDS_BANK_CONFLICT', 0.0):.0f} |")


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when it is absent or the kernel source changed since."""
    try:
        lines = open(TRAFFIC_SUMMARY).read().splitlines()
    except OSError:
        return None
    sha = _source_sha()
    for ln in lines:
        p = ln.split()
        if len(p) == 5 and p[0] == "traffic" and p[1] == kernel and p[4] == sha:
            return float(p[2]) + float(p[3])
    return None


def rate_sweep(args):
    """Convergence rates against the anisotropy (section 5.1): the power
    iteration of the SAS V-cycle on a two-mesh Kuhn hierarchy with sigma =
    nu = 1, coarsened in space on its top level ("Full": lambda_crit = 0)
    or in time only ("Semi-time"), for tau / h^2 from 2^-7 to 2^5 and both
    DG degrees; then the smoother orders of section 4 at three values of
    lambda. lambda is the library's eq. (3) value of the top level. Prints
    one JSON line."""
    import numpy as np
    import torch
    from paper_1911_09548_amd import inputs, stmg

    n, Nt, cycles = args.sweep_n, args.sweep_Nt, args.sweep_cycles
    meshes = inputs.kuhn_hierarchy(n)[:2]
    nt = meshes[0].tets.shape[0]
    rows = []
    for pt in (0, 1):
        for e in range(-7, 6):
            T = 2.0 ** e * Nt / n ** 2  # tau n^2 = 2^e
            prob = inputs.Problem(meshes, np.ones(nt), np.ones(nt), T, Nt, pt,
                                  meta={"name": f"rate sweep n={n} Nt={Nt} pt={pt} T={T}"})
            row = {"pt": pt, "T": T}
            for name, opts in (("full", dict(lambda_crit=0.0)), ("semi_time", dict(allow_space_coarsening=0))):
                s = stmg.Solver(prob, **opts)
                row["lambda"] = s.level_info(0).lambda_
                x0 = torch.from_numpy(np.random.default_rng(7).uniform(0.0, 1.0, (Nt, pt + 1, s.n_edges))).cuda()
                t0 = time.perf_counter()
                rate, rates = s.power_rate(x0, max_cycles=cycles)
                dt = time.perf_counter() - t0
                row[name] = rate
                row[name + "_ms_per_cycle"] = 1e3 * dt / max(1, len(rates))
                s.close()
            rows.append(row)
            log(f"[sweep] pt={pt} lambda={row['lambda']:.4g}: full {row['full']:.4f}, "
                f"semi-time {row['semi_time']:.4f}")
    # smoother orders (section 4), p_t = 1, hierarchy by the default rule
    # (lambda_crit = 0.1): rate, time per cycle and the cycles' cost of one
    # decade of error reduction
    orders = []
    for e in (-7, 0, 5):
        T = 2.0 ** e * Nt / n ** 2
        prob = inputs.Problem(meshes, np.ones(nt), np.ones(nt), T, Nt, 1,
                              meta={"name": f"smoother orders n={n} Nt={Nt} T={T}"})
        for seq, code in stmg.SMOOTHERS.items():
            s = stmg.Solver(prob, smoother=code)
            x0 = torch.from_numpy(np.random.default_rng(7).uniform(0.0, 1.0, (Nt, 2, s.n_edges))).cuda()
            t0 = time.perf_counter()
            rate, rates = s.power_rate(x0, max_cycles=cycles)
            ms = 1e3 * (time.perf_counter() - t0) / max(1, len(rates))
            row = {"lambda": s.level_info(0).lambda_, "smoother": seq, "rate": rate, "ms_per_cycle": ms,
                   "ms_per_decade": ms * np.log(10.0) / -np.log(rate) if 0.0 < rate < 1.0 else None}
            s.close()
            orders.append(row)
            log(f"[sweep] lambda={row['lambda']:.4g} {seq}: rate {rate:.4f}, {ms:.1f} ms per cycle")
    print(json.dumps({"rate_sweep": {"mesh": f"{n}^3 x 6 Kuhn tets, two meshes, sigma = nu = 1",
                                     "Nt": Nt, "cycles": cycles, "start": "uniform [0, 1], seed 7",
                                     "rows": rows, "smoother_orders": orders}}), flush=True)


TWO_LAMBDA_LAMBDAS = (1.0, 0.5, 0.25, 0.125, 0.0625, 0.03125, 0.015625, 0.01)
TWO_LAMBDA_NU2 = (1.0, 1e1, 1e2, 1e3, 1e4, 1e5, 1e6)


def two_lambda(args, lambdas=TWO_LAMBDA_LAMBDAS, nu2s=TWO_LAMBDA_NU2):
    """The "Two lambda" experiment (section 5.2, Table 2) on Kuhn meshes: the
    cube's halves carry nu = 1 and nu = nu2 (sigma = 1, Neumann boundary), so
    the smaller anisotropy lambda = tau / h_T^2 is set by tau alone while nu2
    raises the other half's. "Full" method: two meshes, coarsened in space
    and time on the top level (lambda_crit = 0). The rate is the largest
    per-cycle reduction factor of the power iteration over at most
    args.two_lambda_cycles cycles from a start uniform in [0, 1] (seed 7).
    Returns the table as a dict."""
    import numpy as np
    import torch
    from paper_1911_09548_amd import inputs, stmg

    n, Nt, cycles = args.sweep_n, args.sweep_Nt, args.two_lambda_cycles
    h_T = np.sqrt(3.0) / n   # longest edge of a Kuhn tetrahedron
    rows = []
    for nu2 in nu2s:
        row = {"nu2": nu2, "rates": {}, "ms_per_cycle": {}}
        for lam in lambdas:
            T = Nt * lam * h_T ** 2
            prob = inputs.config_two_lambda(n, Nt, 1, T, nu2)
            s = stmg.Solver(prob, lambda_crit=0.0)
            got = s.level_info(0).lambda_
            assert abs(got - lam) <= 1e-9 * lam, (got, lam)
            x0 = torch.from_numpy(np.random.default_rng(7).uniform(0.0, 1.0, (Nt, 2, s.n_edges))).cuda()
            t0 = time.perf_counter()
            rate, rates = s.power_rate(x0, max_cycles=cycles)
            row["rates"][f"{lam:g}"] = rate
            row["ms_per_cycle"][f"{lam:g}"] = 1e3 * (time.perf_counter() - t0) / max(1, len(rates))
            s.close()
        rows.append(row)
        log(f"[two-lambda] nu2={nu2:g}: " + ", ".join(f"{k}: {v:.3f}" for k, v in row["rates"].items()))
    return {"mesh": f"{n}^3 x 6 Kuhn tets (two meshes), halves x < 1/2 (nu = 1) and x > 1/2 (nu = nu2), "
                    "sigma = 1, Neumann boundary", "Nt": Nt, "pt": 1, "method": "Full (lambda_crit = 0)",
            "cycles": cycles, "start": "uniform [0, 1], seed 7", "rows": rows}


def core_box(args):
    """The unstructured high-contrast case (jittered Kuhn mesh, conducting
    core box [0.3, 0.7]^3 with sigma = 1e4 and nu = 1e-3 inside, sigma = 1e-2
    outside): setup, then the solve to 1e-8 in the FP64 and in the precision
    form with exact slab solves, or (--core-box-slab k) with k two-grid
    Richardson steps per slab solve, which keeps only the coarser mesh's slab
    factors on the levels above the coarsest (the size that the exact factors
    do not fit on one GPU). Cycles run one at a time with a
    progress line every 10 s; the time to 1e-8 covers the cycles up to the
    first residual at or below 1e-8. Prints one JSON line."""
    import numpy as np
    import torch
    from paper_1911_09548_amd import inputs, stmg

    n, Nt, pt = args.core_box, args.core_box_Nt, 1
    prob = inputs.config_core_box(n=n, Nt=Nt, pt=pt, seed=3, jitter=0.2)
    rhs = None
    k = args.core_box_slab
    out = {"workload": f"jittered core box, {n}^3 x 6 Kuhn tets (vertices moved by up to 20% of h), "
                       f"N_t={Nt}, p_t={pt}, Gaussian rhs", "factor_transpose": args.core_box_transpose,
           "slab_steps": k, "forms": {}}
    sfx = f"_twogrid{k}" if k > 0 else ""
    forms = (("fp64" + sfx, stmg.FP64), ("fp32_refined" + sfx, stmg.FP32_REFINED))
    max_cycles = args.core_box_cycles
    for form, prec in forms:
        log(f"[core box] setup {form} n={n} Nt={Nt}")
        t0 = time.perf_counter()
        try:
            s = stmg.Solver(prob, rtol=1e-8, max_cycles=max_cycles, precision=prec,
                            factor_transpose=args.core_box_transpose, slab=k,
                            device_factor={"auto": -1, "gpu": 1, "host": 0}[args.factor])
        except stmg.StmgError as e:
            # refused by the device-memory estimate (or out of memory)
            out["forms"][form] = {"refused": str(e), "code": e.code, "after_s": time.perf_counter() - t0}
            log(f"[core box] {form}: {e}")
            continue
        setup_s = time.perf_counter() - t0
        if "levels" not in out:
            out["levels"] = [{"mesh": li.mesh, "N": li.N, "lambda": li.lambda_, "n_e": li.n_e,
                              "slab_factor_mesh": li.slab_factor_mesh, "slab_steps": li.slab_steps,
                              "slab_factor_entries": li.factor_nnz_slab}
                             for li in (s.level_info(l) for l in range(s.n_levels))]
            rhs = torch.from_numpy(inputs.gaussian_rhs(s.n_edges, Nt, pt, seed=2)).cuda()
        info = stmg.Info()
        stmg.lib().stmg_info(s._h, stmg.C.byref(info))
        out["forms"].setdefault(form, {})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.load(rhs)
        hist, t_log = [], t0
        while len(hist) < max_cycles and (not hist or (hist[-1] > 1e-8 and np.isfinite(hist[-1]))):
            hist.append(float(s.cycles(1)[0]))
            if time.perf_counter() - t_log > 10.0:
                t_log = time.perf_counter()
                log(f"[core box] {form}: cycle {len(hist)}, rel res {hist[-1]:.2e}, {t_log - t0:.1f}s")
        solve_s = time.perf_counter() - t0
        out["forms"][form] = {"setup_s": setup_s, "device_bytes": info.device_bytes,
                              "factor_bytes": info.factor_bytes, "cycles": len(hist), "time_to_1e-8_s": solve_s,
                              "ms_per_cycle": 1e3 * solve_s / max(1, len(hist)),
                              "final_rel_res": hist[-1], "converged": hist[-1] <= 1e-8, "history": hist}
        log(f"[core box] {form}: setup {setup_s:.1f}s, {len(hist)} cycles, {solve_s:.2f}s, "
            f"rel res {hist[-1]:.2e}")
        s.close()
        torch.cuda.empty_cache()
    print(json.dumps({"core_box": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--Nt", type=int, default=256)
    ap.add_argument("--pt", type=int, default=1)
    ap.add_argument("--sample-n", type=int, default=8)
    ap.add_argument("--sample-Nt", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-8 solve")
    ap.add_argument("--no-fp32", action="store_true", help="skip the precision-form measurement")
    ap.add_argument("--factor", choices=("auto", "gpu", "host"), default="auto",
                    help="where the numeric factorisation of the setup runs")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-form measurement")
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-sizes", default="8,12,16")
    ap.add_argument("--serve-horizons", default="16,64,128")
    ap.add_argument("--serve-probe", type=int, default=4, help="requests timed one at a time")
    ap.add_argument("--serve-active", type=int, default=8)
    ap.add_argument("--serve-threads", type=int, default=4)
    ap.add_argument("--serve-only", action="store_true", help="only the serving-form measurement")
    ap.add_argument("--serve-closed", type=int, default=1,
                    help="also measure the saturated (closed-loop) throughput, batched and unbatched")
    ap.add_argument("--hbm-calibrate", type=int, default=0, metavar="MiB",
                    help="first run one plain device copy of this many MiB (read + write), so that "
                         "hardware byte counters can be scaled by a kernel of known traffic")
    ap.add_argument("--sq-summary", nargs=2, metavar=("SQ_CSV", "CACHE_CSV"),
                    help="summarise the shader and cache counter runs (no GPU work)")
    ap.add_argument("--stats-summary", metavar="KERNEL_STATS_CSV",
                    help="summarise a rocprofv3 --stats kernel table (no GPU work)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 counter runs (no GPU work)")
    ap.add_argument("--rate-sweep", action="store_true",
                    help="only the convergence-rate sweep against lambda (power iteration)")
    ap.add_argument("--sweep-n", type=int, default=16)
    ap.add_argument("--sweep-Nt", type=int, default=64)
    ap.add_argument("--sweep-cycles", type=int, default=60)
    ap.add_argument("--two-lambda", action="store_true",
                    help="only the full Two-lambda table (section 5.2): 7 values of nu2 x 8 of lambda")
    ap.add_argument("--two-lambda-cycles", type=int, default=100)
    ap.add_argument("--nodal-steps", type=int, default=3,
                    help="also measure the form with inexact nodal solves (k Chebyshev steps; 0 skips)")
    ap.add_argument("--slab-steps", type=int, default=2,
                    help="also measure the form with inexact slab solves (k two-grid Richardson steps; 0 skips)")
    ap.add_argument("--no-two-lambda", action="store_true",
                    help="skip the Two-lambda subset of the default run")
    ap.add_argument("--core-box", type=int, default=0, metavar="N",
                    help="only the jittered high-contrast core-box case on an N^3 mesh")
    ap.add_argument("--core-box-Nt", type=int, default=128)
    ap.add_argument("--core-box-slab", type=int, default=0, metavar="K",
                    help="inexact slab solves: K two-grid Richardson steps")
    ap.add_argument("--core-box-cycles", type=int, default=100, help="cycle cap of the core-box solves")
    ap.add_argument("--core-box-transpose", type=int, default=-1, choices=(-1, 0, 1),
                    help="keep P^T for the backward solves: -1 auto, 0 never (half the factor memory)")
    ap.add_argument("--oracle-sample", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_sample:
        oracle_sample(args)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.stats_summary:
        stats_summary(args.stats_summary)
        return
    if args.sq_summary:
        sq_summary(*args.sq_summary)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU only (the multi-GPU time sharding is a design "
              "note, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.rate_sweep:
        rate_sweep(args)
        return
    if args.serve_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"serving_form": serving_bench(args)}), flush=True)
        return
    if args.two_lambda:
        print(json.dumps({"two_lambda": two_lambda(args)}), flush=True)
        return
    import numpy as np
    import torch
    from paper_1911_09548_amd import inputs, stmg

    torch.cuda.set_device(0)
    if args.hbm_calibrate > 0:
        n = args.hbm_calibrate << 17  # doubles
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # reads and writes n * 8 bytes
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {n * 8} bytes read, {n * 8} bytes written")
        del src, dst
    if args.core_box > 0:
        core_box(args)
        return
    prob = inputs.config_block_random(n=args.n, Nt=args.Nt, pt=args.pt, seed=1, block_hexes=8)
    log(f"[bench] setup n={args.n} Nt={args.Nt} pt={args.pt}")
    t0 = time.perf_counter()
    dev_factor = {"auto": -1, "gpu": 1, "host": 0}[args.factor]
    solver = stmg.Solver(prob, rtol=1e-8, max_cycles=100, device_factor=dev_factor)
    setup_s = time.perf_counter() - t0
    levels = [solver.level_info(l) for l in range(solver.n_levels)]
    log(f"[bench] setup {setup_s:.1f}s, levels " +
        ", ".join(f"(mesh {li.mesh}, N {li.N})" for li in levels))
    q = args.pt + 1
    rng = np.random.default_rng(2)
    rhs = torch.from_numpy(rng.standard_normal((args.Nt, q, solver.n_edges))).cuda()
    n_e = levels[0].n_e
    dofs = n_e * args.Nt * q

    solver.load(rhs)
    solver.cycles(args.warmup)
    torch.cuda.synchronize()
    # the library runs on torch's current stream: events on it bracket the
    # timed region (no per-launch events inside: value and ms_per_step)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    res = solver.cycles(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log(f"[bench] {ms:.2f} ms per V-cycle, residuals {res[-1]:.2e}")
    # a second timed region of the same length with per-launch events on the
    # same stream: each kernel's duration and algorithmic work (rooflines)
    solver.profile(True)
    e0.record(stream)
    solver.cycles(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_prof = e0.elapsed_time(e1) / args.steps
    kernels = solver.profile_report()
    solver.profile(False)
    log(f"[bench] {ms_prof:.2f} ms per V-cycle with per-launch events")
    for k in kernels:
        log(f"[bench]   {k['kernel']:28s} {k['ms'] / args.steps:8.2f} ms/step {k['launches'] // args.steps:5d} launches/step "
            f"{k['flops'] / (k['ms'] * 1e-3) / 1e12:7.2f} TFLOP/s {k['bytes'] / (k['ms'] * 1e-3) / 1e9:8.1f} GB/s")
    # a supernode GEMM is timed together with its split-K reduce (named
    # after the GEMM's shape); the dominant kernel has the largest such total
    by_name = {k["kernel"]: k for k in kernels}

    def combined_ms(k):
        if k["kernel"].startswith("k_sn_gemm"):
            red = by_name.get(k["kernel"].replace("k_sn_gemm", "k_sn_reduce"))
            return k["ms"] + (red["ms"] if red else 0.0)
        return k["ms"]

    top = max((k for k in kernels if not k["kernel"].startswith("k_sn_reduce")), key=combined_ms)
    avg_s = combined_ms(top) * 1e-3 / top["launches"]
    if top["kernel"].startswith("k_sn_gemm"):
        achieved = top["flops"] / top["launches"] / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None}
    else:
        achieved = top["bytes"] / top["launches"] / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    roof["traffic"] = recorded_traffic(top["kernel"])
    red = by_name.get(top["kernel"].replace("k_sn_gemm", "k_sn_reduce"))
    roof.update({"kernel": top["kernel"], "avg_launch_us": avg_s * 1e6, "launches": top["launches"],
                 "gemm_avg_launch_us": top["ms"] * 1e3 / top["launches"],
                 "reduce_us_per_launch": (red["ms"] * 1e3 / top["launches"]) if red else 0.0,
                 "flops_per_launch": top["flops"] / top["launches"],
                 "work_count": "8 flops per structural nonzero of L and complex right-hand side",
                 "nnz_L_struct_level0": levels[0].factor_nnz_slab_struct,
                 "nnz_L_stored_level0": levels[0].factor_nnz_slab,
                 "profiled_ms_per_step": ms_prof})
    # the HBM-bound residual (largest total time among its shapes), against HBM peak
    res = max((k for k in kernels if k["kernel"].startswith("k_residual")), key=lambda k: k["ms"], default=None)
    roof_res = None
    if res:
        r_avg = res["ms"] * 1e-3 / res["launches"]
        r_ach = res["bytes"] / res["launches"] / r_avg / 1e9
        roof_res = {"bound": "hbm", "achieved": r_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": r_ach / HBM_PEAK_GBS, "traffic": recorded_traffic(res["kernel"]),
                    "kernel": res["kernel"], "avg_launch_us": r_avg * 1e6, "launches": res["launches"]}
    breakdown = [{"kernel": k["kernel"], "ms_per_step": k["ms"] / args.steps,
                  "launches_per_step": k["launches"] // args.steps,
                  "tflops": k["flops"] / (k["ms"] * 1e-3) / 1e12,
                  "gbs": k["bytes"] / (k["ms"] * 1e-3) / 1e9} for k in kernels[:24]]

    extra = {}
    x64 = None
    if not args.no_solve:
        t = time.perf_counter()
        x64, rep = solver.solve(rhs)
        torch.cuda.synchronize()
        extra = {"time_to_1e-8_s": time.perf_counter() - t, "cycles_to_1e-8": rep["cycles"],
                 "final_rel_res": rep["rel_res"]}
        log(f"[bench] solve to 1e-8: {extra['time_to_1e-8_s']:.2f}s in {rep['cycles']} cycles")

    prec = None
    if not args.no_fp32:
        # precision form on the same workload: FP32 V-cycle inside FP64
        # refinement; same metric (one refinement iteration = one V-cycle)
        solver.close()
        del solver
        torch.cuda.empty_cache()
        log("[bench] setup of the precision form (FP32 smoother, FP64 refinement)")
        t0 = time.perf_counter()
        s32 = stmg.Solver(prob, rtol=1e-8, max_cycles=100, precision=stmg.FP32_REFINED, device_factor=dev_factor)
        setup32 = time.perf_counter() - t0
        s32.load(rhs)
        s32.cycles(args.warmup)
        torch.cuda.synchronize()
        e0.record(stream)
        s32.cycles(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms32 = e0.elapsed_time(e1) / args.steps
        # the FP32 iteration's kernels with per-launch events (same stream);
        # the dominant FP32 supernode GEMM with its split-K reduce against the
        # FP32 matrix-core peak
        s32.profile(True)
        s32.cycles(args.steps)
        torch.cuda.synchronize()
        k32 = s32.profile_report()
        s32.profile(False)
        by32 = {k["kernel"]: k for k in k32}

        def comb32(k):
            red = by32.get(k["kernel"].replace("k_sn_gemm", "k_sn_reduce"))
            return k["ms"] + (red["ms"] if red and k["kernel"].startswith("k_sn_gemm") else 0.0)

        top32 = max((k for k in k32 if k["kernel"].startswith("k_sn_gemm<c")), key=comb32, default=None)
        roof32 = None
        if top32:
            avg32 = comb32(top32) * 1e-3 / top32["launches"]
            ach32 = top32["flops"] / top32["launches"] / avg32 / 1e12
            roof32 = {"bound": "mfma", "achieved": ach32, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": ach32 / FP32_PEAK_TFLOPS, "kernel": top32["kernel"], "avg_launch_us": avg32 * 1e6,
                      "launches": top32["launches"]}
        t = time.perf_counter()
        x32, rep32 = s32.solve(rhs)
        torch.cuda.synchronize()
        tts32 = time.perf_counter() - t
        prec = {"form": "fp32 smoother + fp64 refinement", "value": dofs / (ms32 * 1e-3),
                "ms_per_step": ms32, "time_to_1e-8_s": tts32, "cycles_to_1e-8": rep32["cycles"],
                "final_rel_res": rep32["rel_res"], "setup_s": setup32, "roofline_fp32_solve": roof32,
                "kernels": [{"kernel": k["kernel"], "ms_per_step": k["ms"] / args.steps,
                             "launches_per_step": k["launches"] // args.steps,
                             "tflops": k["flops"] / (k["ms"] * 1e-3) / 1e12,
                             "gbs": k["bytes"] / (k["ms"] * 1e-3) / 1e9} for k in k32[:12]]}
        if x64 is not None:
            # distance to the FP64 form's solution of the same system (both
            # solved to 1e-8; final_rel_res is already the FP64 residual)
            prec["rel_diff_vs_fp64_solution"] = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        log(f"[bench] precision form: {ms32:.2f} ms per iteration, 1e-8 in {rep32['cycles']} cycles "
            f"({tts32:.2f}s)" + (f"; {roof32['kernel']} {roof32['achieved']:.1f} TFLOP/s = "
                                 f"{roof32['frac']:.2f} of the FP32 peak" if roof32 else ""))
        s32.close()

    def inexact_form(label, key, what, **opts):
        # the same workload and FP64 form with inexact spatial solves (section 5)
        torch.cuda.empty_cache()
        log(f"[bench] setup with inexact {label} solves ({what})")
        t0 = time.perf_counter()
        sc = stmg.Solver(prob, rtol=1e-8, max_cycles=100, device_factor=dev_factor, **opts)
        setup_c = time.perf_counter() - t0
        sc.load(rhs)
        sc.cycles(args.warmup)
        torch.cuda.synchronize()
        e0.record(stream)
        sc.cycles(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_c = e0.elapsed_time(e1) / args.steps
        t = time.perf_counter()
        _, rep_c = sc.solve(rhs)
        torch.cuda.synchronize()
        tts_c = time.perf_counter() - t
        info = stmg.Info()
        stmg.lib().stmg_info(sc._h, stmg.C.byref(info))
        res = {key: what, "value": dofs / (ms_c * 1e-3), "ms_per_step": ms_c, "time_to_1e-8_s": tts_c,
               "cycles_to_1e-8": rep_c["cycles"], "final_rel_res": rep_c["rel_res"], "setup_s": setup_c,
               "device_bytes": info.device_bytes, "factor_bytes": info.factor_bytes}
        log(f"[bench] inexact {label}: {ms_c:.2f} ms per V-cycle, 1e-8 in {rep_c['cycles']} cycles ({tts_c:.2f}s), "
            f"setup {setup_c:.1f}s, factors {info.factor_bytes / 1e9:.2f} GB")
        sc.close()
        return res

    inexact = inexact_slab = None
    if args.nodal_steps > 0:
        # k Chebyshev steps instead of the exact K_n solve; no nodal factor
        inexact = inexact_form("nodal", "nodal", f"{args.nodal_steps} Jacobi-preconditioned Chebyshev steps",
                               nodal=args.nodal_steps)
    if args.slab_steps > 0:
        # k two-grid Richardson steps instead of the exact slab solves on the
        # levels whose mesh has a coarser one; those keep the coarser slab factor
        inexact_slab = inexact_form("slab", "slab", f"{args.slab_steps} Richardson steps with a two-grid cycle",
                                    slab=args.slab_steps)

    out = {
        "metric": "space-time DOF-updates/s per V-cycle",
        "value": dofs / (ms * 1e-3),
        "unit": "DOF-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"eddy-current space-time V-cycle, {args.n}^3x6 Kuhn tets, N_t={args.Nt}, "
                                f"p_t={args.pt}, block-random sigma in [1,1e3], nu in [1,100], Gaussian rhs"),
                   "n_interior_edges": n_e, "space_time_dofs": dofs, "levels": len(levels),
                   "setup_s": setup_s, **extra},
        "roofline": roof,
        "roofline_residual": roof_res,
        "kernels": breakdown,
    }
    if prec:
        out["precision_form"] = prec
    if inexact:
        out["inexact_nodal_form"] = inexact
    if inexact_slab:
        out["inexact_slab_form"] = inexact_slab
    if not args.no_serving:
        torch.cuda.empty_cache()
        out["serving_form"] = serving_bench(args)
    if not args.no_two_lambda:
        torch.cuda.empty_cache()
        out["two_lambda"] = two_lambda(args, lambdas=(1.0, 0.125, 0.015625), nu2s=(1.0, 1e3, 1e6))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        cb = cpu_baseline(args)
        if cb:
            cb.pop("s_per_cycle", None)
            out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
