"""Benchmark of the CSR SpMV / Jacobi-PCG hot path on one MI355X.

Default line (no flags): one step is
  - C2, 3D 7-point Laplacian 128^3 (n = 2,097,152, nnz = 14,581,760): one FP64
    and one mixed-precision Jacobi-PCG solve to rtol 1e-8 and 100 standalone
    FP64 SpMVs;
  - C3, 3D 27-point lognormal diffusion 160^3 (n = 4,096,000,
    nnz = 109,215,352): one FP64 and one mixed solve to rtol 1e-8, and a
    100-iteration FP64 PCG run whose SpMV products are each timed with a HIP
    event pair on the solve stream (the roofline of the PCG product).
All inputs are resident in HBM before the clock starts; every call goes
through the C ABI of libspk.so on the current torch stream.  `value` is the
step's algorithmic HBM traffic (SpMV 12 nnz + 4(n+1) + 16n bytes, PCG
iteration 12 nnz + 4(n+1) + 88n, FP32 inner iteration 8 nnz + 4(n+1) + 44n,
refinement steps and setup/true-residual products) divided by its wall time.
After the timed steps, outside the clock: the C2 SpMV after evicting the
Infinity Cache, the served stream (C5: Poisson arrivals, p50/p99 latency, a
closed loop for solves/s against one-at-a-time solves), the single-reduction,
Chebyshev, multi-right-hand-side and multigrid legs, and the CPU oracle
(serial and all host cores).

Other workloads (one JSON line each): --workload c2 (the C2 part alone),
c3, c4 (power-law n = 4M SpMV by kernel family), serve, spectrum, mg.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# rocprofv3 names of the standalone FP64 SpMV kernel of each family
SPMV_KERNELS = {
    "stream": "k_spmv_stream<double>",
    "sell": "k_spmv_sell<double, CI>",
    "vector": "k_spmv_vector<double, L>",
    "merge": "k_spmv_merge<double> + k_merge_fixup<double>",
}


def sell_ci(info):
    """Offset type in the SELL kernels' names: int16 per lane ("short"), or
    int32 (per lane, or shared per slice: info.lanes 0)."""
    return "short" if info.lanes == 16 else "int"


def spmv_kernel_name(spk, info):
    return SPMV_KERNELS[spk.KERNEL_NAMES[info.kernel]].replace("CI", sell_ci(info))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="all", choices=["all", "c2", "c3", "c4", "serve", "spectrum", "mg"])
    p.add_argument("--spmvs", type=int, default=100)
    p.add_argument("--cold-spmvs", type=int, default=20,
                   help="SpMVs timed after evicting the Infinity Cache (after the timed steps)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-iters", type=int, default=200)
    p.add_argument("--graph-k", type=int, default=8)
    p.add_argument("--serve-seconds", type=float, default=60.0)
    p.add_argument("--serve-rate", type=float, default=200.0)
    p.add_argument("--serve-closed", type=int, default=0,
                   help="closed-loop saturation run with this many requests queued at t=0")
    p.add_argument("--c5-seconds", type=float, default=20.0,
                   help="default line: seconds of the open-loop served stream")
    p.add_argument("--c5-closed", type=int, default=500,
                   help="default line: requests of the closed-loop run (0: none)")
    p.add_argument("--c3-probe-iters", type=int, default=100,
                   help="default line: FP64 PCG iterations whose products are event-timed on C3")
    p.add_argument("--no-extras", action="store_true",
                   help="default line: skip the single-reduction, Chebyshev, multi-RHS and multigrid legs")
    p.add_argument("--c4-band", type=int, default=0,
                   help="c4 workload: columns within +-band of the row (the banded diagnostic variant)")
    p.add_argument("--cpu-c5-seconds", type=float, default=15.0,
                   help="CPU oracle floor of the served stream: seconds of sequential solves")
    return p.parse_args()


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def pct(a, q):
    import numpy as np

    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def source_hash(files=("spmv.hpp", "common.hpp")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2011_00715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key, bytes_per_launch):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, or None if
    absent or taken on a different kernel source (the entry lists the source
    files its kernel is built from)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel_key)
    if not e or e.get("source_hash") != source_hash(tuple(e.get("sources", ("spmv.hpp", "common.hpp")))):
        return None
    return e.get("hbm_bytes_per_launch")


def dev(a):
    import numpy as np
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mixed_outer_bytes(n, spmv64):
    # per refinement step: x += s d (read d 4n, x 8n, write x 8n), r = b - A x
    # (SpMV + read b + write r), r32/z32/p32/d32 setup (read r 8n, dinv32 4n,
    # write 16n)
    return spmv64 + 16 * n + 20 * n + 28 * n


def solve_bytes(info, res):
    n = info.n
    if res.inner_iterations or res.outer_steps:
        b = res.inner_iterations * info.bytes_pcg_iter_f32
        b += (res.outer_steps + 1) * mixed_outer_bytes(n, info.bytes_spmv_f64)
        b += res.iterations * info.bytes_pcg_iter_f64
        return b + info.bytes_spmv_f64  # final true residual
    # setup residual + iterations + true residual
    return res.iterations * info.bytes_pcg_iter_f64 + 2 * info.bytes_spmv_f64


def cpu_info():
    import os

    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "model": model}


def cpu_baseline(A, b, info, iters):
    """The serial oracle on a bounded sample: `iters` FP64 PCG iterations of
    the C2 system (plus its setup and final residual products)."""
    import oracle

    t = time.perf_counter()
    _, r, _ = oracle.pcg(A, b, rtol=0.0, maxit=iters)
    dt = time.perf_counter() - t
    bytes_ = r["iterations"] * info.bytes_pcg_iter_f64 + 2 * info.bytes_spmv_f64
    return {
        "value": bytes_ / dt / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{r['iterations']} FP64 Jacobi-PCG iterations of the same 128^3 7-point system "
                  f"(plus its setup and final residual products), serial C oracle, {dt:.2f} s; "
                  f"{dt / max(r['iterations'], 1) * 1e3:.1f} ms per iteration",
        "seconds": dt,
    }


def cpu_baselines(A1, A2, b2, info2, serve_reqs, args):
    """The oracle timed on the host: the OpenMP build on every core it is
    given (full C2 and C1 solves, and a sequential floor of the served
    stream), and the serial build on a bounded C2 sample."""
    import numpy as np

    import oracle
    import spkgen

    lo = oracle.load_omp()
    threads = oracle.threads(lo)
    t = time.perf_counter()
    _, r2, _ = oracle.pcg(A2, b2, lib=lo)
    dt2 = time.perf_counter() - t
    bytes2 = r2["iterations"] * info2.bytes_pcg_iter_f64 + 2 * info2.bytes_spmv_f64
    c1 = []
    for seed in range(5):
        b1 = spkgen.rhs_uniform(A1.n, seed)
        t = time.perf_counter()
        _, r1, _ = oracle.pcg(A1, b1, lib=lo)
        c1.append((time.perf_counter() - t, r1["iterations"]))
    serial = cpu_baseline(A2, b2, info2, args.cpu_iters)
    # served stream, one request after the other (FP64 oracle solve of each),
    # for at most cpu_c5_seconds
    lat, t_all = [], time.perf_counter()
    for r in serve_reqs:
        if time.perf_counter() - t_all > args.cpu_c5_seconds:
            break
        A = spkgen.serve_matrix(r)
        bq = spkgen.rhs_uniform(A.n, r.rhs_seed % (2**31))
        t = time.perf_counter()
        _, rq, _ = oracle.pcg(A, bq, lib=lo)
        lat.append(time.perf_counter() - t)
        assert rq["reason"] > 0
    span = time.perf_counter() - t_all
    return {
        "value": bytes2 / dt2 / 1e9,
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"one full FP64 Jacobi-PCG solve of the 128^3 7-point system to rtol 1e-8 "
                   f"({r2['iterations']} iterations, {dt2:.2f} s, {1 / dt2:.2f} solves/s), OpenMP build of "
                   f"the oracle on {threads} threads"),
        "host": cpu_info(),
        "c2_solve": {"seconds": dt2, "solves_per_s": 1 / dt2, "iterations": r2["iterations"],
                     "ms_per_iter": dt2 * 1e3 / max(r2["iterations"], 1)},
        "c1_solves": {"ms_p50": float(np.median([c[0] for c in c1])) * 1e3,
                      "solves_per_s": 1 / float(np.median([c[0] for c in c1])),
                      "iterations": [c[1] for c in c1]},
        "c5_sequential": {"requests": len(lat), "seconds": span,
                          "solves_per_s": len(lat) / span if span > 0 else None,
                          "solve_ms_p50": pct(lat, 50) * 1e3 if lat else None,
                          "solve_ms_p99": pct(lat, 99) * 1e3 if lat else None,
                          "note": "the first requests of the closed-loop set, solved one after the other "
                                  "(FP64 oracle PCG to rtol 1e-8)"},
        "serial_1_core": serial,
    }


def c2_extra_legs(spk, M, A, b, bd, xs, info, args, jacobi_s):
    """The C2 legs of the other hot-path rows, outside the timed steps:
    Chebyshev-Jacobi smoother, single-reduction CG, multiple right-hand
    sides, multigrid-preconditioned CG."""
    import numpy as np
    import torch

    import spkgen

    # Chebyshev-Jacobi smoother (multigrid smoothing of Sec. 5.3), default
    # interval [g/10, g] from the Gershgorin bound; outside the timed steps
    cheb = {}
    xc = torch.zeros_like(xs)
    mat_bytes = 12 * info.nnz + 4 * (info.n + 1)
    for steps in (2, 8):
        us = []
        for _ in range(20):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            spk.pc_chebyshev(M, bd, xc, steps)
            e1.record()
            torch.cuda.synchronize()
            us.append(e0.elapsed_time(e1) * 1e3)
        nb = 40 * info.n + (steps - 1) * (mat_bytes + 56 * info.n) + 24 * info.n
        t = float(np.median(us))
        cheb[f"steps_{steps}"] = {"us_p50": t, "bytes": nb, "gbps": nb / (t * 1e-6) / 1e9}
    cheb["note"] = ("x0 = 0, no residual output: 40n (init) + (steps-1) x (12 nnz + 4(n+1) + 56n) "
                    "fused SpMV+update passes + 24n (last x += d)")

    # single-reduction (Chronopoulos-Gear) FP64 solve of the same system
    osr = spk.ksp_opts(graph_k=args.graph_k, single_reduction=1)
    xsr = torch.zeros_like(xs)
    rsr = spk.ksp_solve(M, bd, xsr, osr)
    tsr = []
    for _ in range(3):
        rsr = spk.ksp_solve(M, bd, xsr, osr)
        tsr.append(rsr.seconds)
    sr = {"solves_per_s": 1.0 / float(np.median(tsr)), "ms_p50": float(np.median(tsr)) * 1e3,
          "iterations": rsr.iterations, "us_per_iter": float(np.median(tsr)) * 1e6 / max(rsr.iterations, 1),
          "true_rel_residual": rsr.true_rel_residual, "reason": spk.reason_str(rsr.reason)}

    # multiple right-hand sides (k = 8): SpMM, and 8 solves sharing each SpMM
    kk = 8
    Xm = torch.stack([xs] * kk, dim=1).contiguous()
    Ym = torch.empty_like(Xm)
    for _ in range(5):  # warm-up
        spk.mat_mult_multi(M, Xm, Ym)
    groups = []
    for _ in range(5):  # five groups of 20 back-to-back launches; the median group
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            spk.mat_mult_multi(M, Xm, Ym)
        e1.record()
        torch.cuda.synchronize()
        groups.append(e0.elapsed_time(e1) * 1e3 / 20)
    spmm_us = float(np.median(groups))
    Bm = torch.stack([dev(spkgen.rhs_uniform(A.n, sd)) for sd in range(kk)], dim=1).contiguous()
    Xs = torch.zeros_like(Bm)
    spk.ksp_solve_multi(M, Bm, Xs, spk.ksp_opts(graph_k=args.graph_k))
    ts = []
    for _ in range(3):
        Xs.zero_()
        rs = spk.ksp_solve_multi(M, Bm, Xs, spk.ksp_opts(graph_k=args.graph_k))
        ts.append(rs[0].seconds)
    tm = float(np.median(ts))
    spmm_bytes = 12 * info.nnz + 4 * (info.n + 1) + 16 * kk * info.n
    multi = {"k": kk, "spmm_us": spmm_us, "spmm_us_groups": groups, "spmm_bytes": spmm_bytes,
             "spmm_gbps": spmm_bytes / (spmm_us * 1e-6) / 1e9,
             "spmm_us_per_rhs": spmm_us / kk,
             "solve_ms": tm * 1e3, "rhs_solved_per_s": kk / tm,
             "iterations": [r.iterations for r in rs],
             "worst_true_rel_residual": max(r.true_rel_residual for r in rs),
             "note": "SpMM: 5 warm-up launches, then the median of 5 groups of 20 back-to-back launches "
                     "(each group's mean in spmm_us_groups); bytes: CSR matrix once + k x (8n gather + 8n "
                     "write); solves: k FP64 Jacobi-PCG columns sharing each SpMM, per-column scalars and "
                     "stopping"}

    mg = mg_legs(spk, M, A, b, bd, 128, jacobi_s)
    return cheb, sr, multi, mg


def bench_c2(args):
    import numpy as np
    import torch

    import spkgen
    from paper_2011_00715_amd import spk

    N = 128
    log("generating 7-point 128^3")
    A = spkgen.laplace3d7(N)
    b = spkgen.rhs_uniform(A.n, 0)
    M = spk.mat_create_csr(dev(A.rowptr), dev(A.col), dev(A.val), flags=spk.MAT_MIXED)
    info = M.info
    bd = dev(b)
    xs = dev(b)  # SpMV input: rhs of seed 0
    ys = torch.empty_like(xs)
    x64 = torch.zeros_like(xs)
    xmx = torch.zeros_like(xs)
    o64 = spk.ksp_opts(graph_k=args.graph_k)
    omx = spk.ksp_opts(graph_k=args.graph_k, precision=spk.PREC_MIXED)
    S = args.spmvs
    # one event pair on the launch stream around the S back-to-back SpMVs:
    # the average launch duration without per-launch event overhead
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def step(record):
        r64 = spk.ksp_solve(M, bd, x64, o64)
        rmx = spk.ksp_solve(M, bd, xmx, omx)
        if record:
            ev[0].record()
        for i in range(S):
            spk.mat_mult(M, xs, ys)
        if record:
            ev[1].record()
        return r64, rmx

    log("warmup")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("timed steps")
    step_ms, t64, tmx, spmv_us = [], [], [], []
    bytes_total = 0
    r64 = rmx = None
    t_all = time.perf_counter()
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r64, rmx = step(True)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        t64.append(r64.seconds * 1e3)
        tmx.append(rmx.seconds * 1e3)
        spmv_us.append(ev[0].elapsed_time(ev[1]) * 1e3 / S)
        bytes_total += solve_bytes(info, r64) + solve_bytes(info, rmx) + S * info.bytes_spmv_f64
    elapsed = time.perf_counter() - t_all
    ms_per_step = float(np.mean(step_ms))

    # parity of the last results against the FP64 definition (oracle)
    import oracle

    xg = x64.cpu().numpy()
    xm = xmx.cpu().numpy()
    bn = oracle.nrm2(b)
    rel64 = oracle.nrm2(b - oracle.spmv(A, xg)) / bn
    relmx = oracle.nrm2(b - oracle.spmv(A, xm)) / bn
    spmv_avg_us = float(np.mean(spmv_us))
    achieved = info.bytes_spmv_f64 / (spmv_avg_us * 1e-6) / 1e9
    kname = spk.KERNEL_NAMES[info.kernel]
    spmv_kernel = spmv_kernel_name(spk, info)
    traffic = traffic_from_profiles(spmv_kernel + "@c2", info.bytes_spmv_f64)

    # cold Infinity Cache: each SpMV after reading 1 GiB of scratch (outside
    # the timed steps; events bracket the SpMV only)
    scratch = torch.zeros((1 << 30) // 8, dtype=torch.float64, device="cuda")
    cold_us = []
    for _ in range(args.cold_spmvs):
        spk.cache_flush(scratch)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        spk.mat_mult(M, xs, ys)
        e1.record()
        torch.cuda.synchronize()
        cold_us.append(e0.elapsed_time(e1) * 1e3)
    del scratch
    cold_avg = float(np.mean(cold_us)) if cold_us else float("nan")

    cheb, sr, multi, mg = c2_extra_legs(spk, M, A, b, bd, xs, info, args, float(np.median(t64)) * 1e-3)

    out = {
        "metric": "CSR SpMV HBM GB/s; PCG solves/s to rtol 1e-8, FP64 vs mixed; p50/p99 lat",
        "value": bytes_total / elapsed / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (mixed solve: f32 inner / f64 outer)",
        "data": "synthetic",
        "config": {
            "workload": "3D 7-point Laplacian 128^3 (n=2097152, nnz=14581760), FP64 CSR int32, "
                        "rhs uniform[-1,1) seed 0; step = FP64 Jacobi-PCG + mixed Jacobi-PCG to "
                        f"rtol 1e-8 + {S} standalone SpMVs",
            "n": info.n, "nnz": info.nnz, "spmv_kernel": kname,
            "kernel_param": info.lanes, "cached_loads": info.cached_loads, "graph_k": args.graph_k,
        },
        "spmv": {
            "us_avg": spmv_avg_us, "us_step_min": min(spmv_us), "us_step_max": max(spmv_us),
            "gbps": achieved, "bytes": info.bytes_spmv_f64,
            "format_bytes": info.format_bytes_spmv_f64,
            "format_gbps": info.format_bytes_spmv_f64 / (spmv_avg_us * 1e-6) / 1e9,
            "stored_nnz": info.stored_nnz,
            "cold_us_avg": cold_avg,
            "cold_gbps": info.bytes_spmv_f64 / (cold_avg * 1e-6) / 1e9,
            "cold_format_gbps": info.format_bytes_spmv_f64 / (cold_avg * 1e-6) / 1e9,
        },
        "pcg_fp64": {
            "solves_per_s": 1e3 / float(np.median(t64)), "ms_p50": pct(t64, 50), "ms_p99": pct(t64, 99),
            "iterations": r64.iterations, "us_per_iter": float(np.median(t64)) * 1e3 / max(r64.iterations, 1),
            "gbps": solve_bytes(info, r64) / (float(np.median(t64)) * 1e-3) / 1e9,
            "true_rel_residual_oracle": rel64, "reason": spk.reason_str(r64.reason),
        },
        "pcg_fp64_single_reduction": sr,
        "chebyshev": cheb,
        "multi_rhs": multi,
        "multigrid_pcg": mg,
        "pcg_mixed": {
            "solves_per_s": 1e3 / float(np.median(tmx)), "ms_p50": pct(tmx, 50), "ms_p99": pct(tmx, 99),
            "inner_iterations": rmx.inner_iterations, "outer_steps": rmx.outer_steps,
            "fallback_fp64": rmx.fallback_fp64,
            "true_rel_residual_oracle": relmx, "reason": spk.reason_str(rmx.reason),
            "error_vs_fp64": float(np.linalg.norm(xm - xg) / np.linalg.norm(xg)),
            "speedup_vs_fp64": float(np.median(t64)) / float(np.median(tmx)),
        },
        "roofline": {
            "kernel": spmv_kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": info.bytes_spmv_f64,
            "format_bytes_per_launch": info.format_bytes_spmv_f64,
            "achieved_cold": info.bytes_spmv_f64 / (cold_avg * 1e-6) / 1e9,
            "frac_cold": info.bytes_spmv_f64 / (cold_avg * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "note": "achieved = 12 nnz + 4 (n+1) + 16 n algorithmic (CSR, FP64) bytes per launch / "
                    "average launch duration (one event pair around the back-to-back launches of "
                    "each timed step, on the launch stream); the "
                    "kernel reads format_bytes_per_launch from its own storage, and its working "
                    "set can be partly served by the 256 MB Infinity Cache (spmv.cold_* gives "
                    "the same launch after evicting it)",
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(A, b, info, args.cpu_iters)
    M.close()
    return out


def wide_product(info):
    """Whether the PCG runs the one-wavefront-per-slice SELL product (the
    library's rule: more than 96 stored entries per lane of a grid of
    min(1024, ceil(n / 256)) blocks, rounded down to a multiple of 8)."""
    tiles = (info.n + 255) // 256
    nblk = tiles if tiles < 8 else min(tiles, 1024) - min(tiles, 1024) % 8
    return info.kernel == 4 and info.stored_nnz > 96 * 256 * nblk  # 4 = SPK_KERNEL_SELL


def bench_all(args):
    """The default line (see the module docstring)."""
    import numpy as np
    import torch

    import oracle
    import spkgen
    from paper_2011_00715_amd import spk

    log("generating C2 (7-point 128^3) and C3 (27-point lognormal 160^3)")
    A2 = spkgen.laplace3d7(128)
    b2 = spkgen.rhs_uniform(A2.n, 0)
    A3 = spkgen.diffusion3d27_lognormal(160, seed=0)
    b3 = spkgen.rhs_uniform(A3.n, 0)
    M2 = spk.mat_create_csr(dev(A2.rowptr), dev(A2.col), dev(A2.val), flags=spk.MAT_MIXED)
    M3 = spk.mat_create_csr(dev(A3.rowptr), dev(A3.col), dev(A3.val), flags=spk.MAT_MIXED)
    i2, i3 = M2.info, M3.info
    assert spk.KERNEL_NAMES[i3.kernel] == "sell" and i3.lanes in (0, 16) and wide_product(i3)
    bd2, bd3 = dev(b2), dev(b3)
    xs2 = dev(b2)
    ys2 = torch.empty_like(xs2)
    x64_2, xmx_2 = torch.zeros_like(xs2), torch.zeros_like(xs2)
    x64_3, xmx_3, xpr_3 = torch.zeros_like(bd3), torch.zeros_like(bd3), torch.zeros_like(bd3)
    o64 = spk.ksp_opts(graph_k=args.graph_k)
    omx = spk.ksp_opts(graph_k=args.graph_k, precision=spk.PREC_MIXED)
    P = args.c3_probe_iters
    oprobe = spk.ksp_opts(rtol=0.0, atol=0.0, maxit=P, profile=1)
    S = args.spmvs
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def step(record):
        r = {"c2_64": spk.ksp_solve(M2, bd2, x64_2, o64), "c2_mx": spk.ksp_solve(M2, bd2, xmx_2, omx)}
        if record:
            ev[0].record()
        for _ in range(S):
            spk.mat_mult(M2, xs2, ys2)
        if record:
            ev[1].record()
        r["c3_64"] = spk.ksp_solve(M3, bd3, x64_3, o64)
        r["c3_mx"] = spk.ksp_solve(M3, bd3, xmx_3, omx)
        r["c3_probe"] = spk.ksp_solve(M3, bd3, xpr_3, oprobe)
        return r

    def step_bytes(r):
        return (solve_bytes(i2, r["c2_64"]) + solve_bytes(i2, r["c2_mx"]) + S * i2.bytes_spmv_f64
                + solve_bytes(i3, r["c3_64"]) + solve_bytes(i3, r["c3_mx"]) + solve_bytes(i3, r["c3_probe"]))

    log("warmup")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("timed steps")
    step_ms, spmv_us, bytes_total = [], [], 0
    rec = {k: [] for k in ("c2_64", "c2_mx", "c3_64", "c3_mx", "c3_probe")}
    t_all = time.perf_counter()
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = step(True)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        spmv_us.append(ev[0].elapsed_time(ev[1]) * 1e3 / S)
        bytes_total += step_bytes(r)
        for k in rec:
            rec[k].append(r[k])
    elapsed = time.perf_counter() - t_all
    last = {k: v[-1] for k, v in rec.items()}

    # the products of the C3 probe: an event pair around each launch
    prod_ms = sum(x.product_ms for x in rec["c3_probe"])
    prod_n = sum(x.product_launches for x in rec["c3_probe"])
    prod_us = prod_ms * 1e3 / max(prod_n, 1)
    achieved = i3.bytes_spmv_f64 / (prod_us * 1e-6) / 1e9

    log("oracle checks of the last solutions")
    res = {}
    for cfg, A, b, M_info, xk in (("c2", A2, b2, i2, (x64_2, xmx_2)), ("c3", A3, b3, i3, (x64_3, xmx_3))):
        bn = oracle.nrm2(b)
        xg, xm = xk[0].cpu().numpy(), xk[1].cpu().numpy()
        res[cfg] = (oracle.nrm2(b - oracle.spmv(A, xg)) / bn, oracle.nrm2(b - oracle.spmv(A, xm)) / bn,
                    float(np.linalg.norm(xm - xg) / np.linalg.norm(xg)))

    def solve_entry(cfg, info, lst64, lstmx):
        t64 = [x.seconds for x in lst64]
        tmx = [x.seconds for x in lstmx]
        r64, rmx = lst64[-1], lstmx[-1]
        m64, mmx = float(np.median(t64)), float(np.median(tmx))
        return {
            "fp64": {"solves_per_s": 1 / m64, "ms_p50": m64 * 1e3, "ms_p99": pct(t64, 99) * 1e3,
                     "iterations": r64.iterations, "us_per_iter": m64 * 1e6 / max(r64.iterations, 1),
                     "iter_gbps": info.bytes_pcg_iter_f64 * r64.iterations / m64 / 1e9,
                     "solve_gbps": solve_bytes(info, r64) / m64 / 1e9,
                     "true_rel_residual_oracle": res[cfg][0], "reason": spk.reason_str(r64.reason)},
            "mixed": {"solves_per_s": 1 / mmx, "ms_p50": mmx * 1e3, "ms_p99": pct(tmx, 99) * 1e3,
                      "inner_iterations": rmx.inner_iterations, "outer_steps": rmx.outer_steps,
                      "fallback_fp64": rmx.fallback_fp64,
                      "us_per_inner_iter": mmx * 1e6 / max(rmx.inner_iterations, 1),
                      "solve_gbps": solve_bytes(info, rmx) / mmx / 1e9,
                      "true_rel_residual_oracle": res[cfg][1], "error_vs_fp64": res[cfg][2],
                      "reason": spk.reason_str(rmx.reason)},
            "speedup_mixed_vs_fp64": m64 / mmx,
        }

    c2 = solve_entry("c2", i2, rec["c2_64"], rec["c2_mx"])
    c3 = solve_entry("c3", i3, rec["c3_64"], rec["c3_mx"])

    # C2 SpMV with a cold Infinity Cache: each launch after reading 1 GiB
    log("cold SpMVs")
    scratch = torch.zeros((1 << 30) // 8, dtype=torch.float64, device="cuda")
    cold_us = []
    for _ in range(args.cold_spmvs):
        spk.cache_flush(scratch)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        spk.mat_mult(M2, xs2, ys2)
        e1.record()
        torch.cuda.synchronize()
        cold_us.append(e0.elapsed_time(e1) * 1e3)
    del scratch
    log("streaming bandwidth (copy, read)")
    stream_bw = measured_stream_gbps()
    warm = float(np.mean(spmv_us))
    cold = float(np.mean(cold_us)) if cold_us else float("nan")
    c2["spmv"] = {
        "kernel": spmv_kernel_name(spk, i2), "bytes": i2.bytes_spmv_f64,
        "format_bytes": i2.format_bytes_spmv_f64,
        "cold_us_avg": cold, "cold_gbps": i2.bytes_spmv_f64 / cold / 1e3,
        "cold_frac": i2.bytes_spmv_f64 / cold / 1e3 / HBM_PEAK_GBS,
        "warm_us_avg": warm, "warm_gbps": i2.bytes_spmv_f64 / warm / 1e3,
        "warm_frac": i2.bytes_spmv_f64 / warm / 1e3 / HBM_PEAK_GBS,
        "traffic_warm": traffic_from_profiles(spmv_kernel_name(spk, i2) + "@c2", i2.bytes_spmv_f64),
        "note": "cold: an event pair around each launch after 1 GiB of scratch was read (the SELL layout, "
                "%.0f MB, no longer in the 256 MB Infinity Cache; includes one launch's dispatch); warm: one "
                "event pair around the step's 100 back-to-back launches" % (i2.format_bytes_spmv_f64 / 1e6),
    }

    extras = None
    if not args.no_extras:
        log("extra legs (single reduction, Chebyshev, multi-RHS, multigrid)")
        cheb, sr, multi, mg = c2_extra_legs(spk, M2, A2, b2, bd2, xs2, i2, args, c2["fp64"]["ms_p50"] * 1e-3)
        extras = {"c2_single_reduction": sr, "c2_chebyshev": cheb, "c2_multi_rhs": multi, "c2_multigrid_pcg": mg}
    M3.close()

    serve = None
    reqs_closed = []
    if args.c5_seconds > 0 or args.c5_closed > 0:
        serve = {}
        if args.c5_seconds > 0:
            reqs = spkgen.serve_stream(seed=0, rate=args.serve_rate, duration=args.c5_seconds)
            log(f"served stream, open loop: {len(reqs)} requests over {args.c5_seconds:g} s")
            serve["open_loop"] = serve_run(spk, reqs, False, args.graph_k)
            serve["open_loop"]["workload"] = f"Poisson {args.serve_rate:g} req/s for {args.c5_seconds:g} s, seed 0"
        if args.c5_closed > 0:
            reqs_closed = spkgen.serve_stream(seed=0, rate=args.serve_rate, duration=60.0, count=args.c5_closed)
            log(f"served stream, closed loop: {len(reqs_closed)} requests")
            serve["closed_loop"] = serve_run(spk, reqs_closed, True, args.graph_k)
            for name, prec, flags in (("mixed", spk.PREC_MIXED, spk.MAT_MIXED), ("fp64", spk.PREC_FP64, 0)):
                log(f"one request at a time ({name})")
                seq = sequential_run(spk, reqs_closed, prec, flags, args.graph_k)
                seq["batching_gain"] = serve["closed_loop"]["solves_per_s"] / seq["solves_per_s"]
                serve["closed_loop"]["sequential_" + name] = seq
        serve["mix"] = SERVE_MIX

    out = {
        "metric": "CSR SpMV HBM GB/s; PCG solves/s to rtol 1e-8, FP64 vs mixed; p50/p99 lat",
        "value": bytes_total / elapsed / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (mixed solves: f32 inner / f64 outer)",
        "data": "synthetic",
        "config": {
            "workload": ("step = C2 3D 7-point Laplacian 128^3 (n=2097152, nnz=14581760): FP64 and mixed "
                         f"Jacobi-PCG to rtol 1e-8 + {S} FP64 SpMVs; C3 3D 27-point lognormal diffusion 160^3 "
                         "(n=4096000, nnz=109215352): FP64 and mixed Jacobi-PCG to rtol 1e-8 + a "
                         f"{P}-iteration FP64 PCG run with event-timed products; FP64 CSR int32, rhs "
                         "uniform[-1,1) seed 0"),
            "value": ("algorithmic HBM GB/s of the timed steps: SpMV 12nnz+4(n+1)+16n, PCG iteration "
                      "12nnz+4(n+1)+88n, FP32 inner iteration 8nnz+4(n+1)+44n, refinement steps and "
                      "setup/true-residual products, summed over the steps / their wall time"),
            "c2_kernel": spk.KERNEL_NAMES[i2.kernel], "c3_kernel": spk.KERNEL_NAMES[i3.kernel],
            "c3_kernel_param": i3.lanes, "graph_k": args.graph_k,
        },
        "c2": c2,
        "c3": c3,
        "c5_served": serve,
        "roofline": {
            "kernel": "k_pcg_spmv_sell_wide<double, %s> (C3 FP64 PCG product q = A p with p.q partials%s)"
                      % (sell_ci(i3), ", column offsets shared per slice" if i3.lanes == 0 else ""),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_from_profiles("k_pcg_spmv_sell_wide<double, %s>@c3" % sell_ci(i3),
                                             i3.bytes_spmv_f64),
            "bytes_per_launch": i3.bytes_spmv_f64, "format_bytes_per_launch": i3.format_bytes_spmv_f64,
            "us_avg": prod_us, "launches_timed": prod_n,
            "measured_gbps": stream_bw, "frac_of_copy": achieved / stream_bw["copy"],
            "frac_of_axpy": achieved / stream_bw["axpy"],
            "note": "achieved = 12 nnz + 4(n+1) + 16n algorithmic bytes of one C3 FP64 product (q = A p with "
                    "the per-block p.q partials) / its average duration: an event pair on the solve stream "
                    "around each of the probe's product kernels in the timed steps (the one-block fold of the "
                    "partials, about 4.6 us, runs after the pair); the SELL layout (format_bytes_per_launch "
                    "with p and q) is several times the 256 MB Infinity Cache, so the bytes come from HBM; "
                    "format bytes below the algorithmic ones are the layout's index compression",
        },
        "extras": extras,
    }
    if not args.no_cpu_baseline:
        log("cpu baselines (oracle)")
        A1 = spkgen.laplace2d5(64)
        out["cpu_baseline"] = cpu_baselines(A1, A2, b2, i2, reqs_closed, args)
    M2.close()
    return out


def mg_legs(spk, M, A, b, bd, N, jacobi_s):
    """Geometric multigrid as the CG preconditioner (the V- and W-cycles of
    Sec. 5.3 with Chebyshev-Jacobi smoothing), FP64 and FP32 cycles, on the
    N^3 Laplacian handle M; jacobi_s = the FP64 Jacobi-PCG solve time."""
    import numpy as np
    import torch

    import oracle

    bn = oracle.nrm2(b)
    xs = bd
    mg = {}
    for name, cyc, prec in (("v_cycle", 1, spk.PREC_FP64), ("w_cycle", 2, spk.PREC_FP64),
                            ("v_cycle_fp32", 1, spk.PREC_MIXED), ("w_cycle_fp32", 2, spk.PREC_MIXED)):
        t0 = time.perf_counter()
        G = spk.mg_create(M, (N, N, N), spk.mg_opts(cycle=cyc, precision=prec))
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        xg_ = torch.zeros_like(xs)
        og = spk.ksp_opts(graph_k=1)
        spk.ksp_solve_mg(G, bd, xg_, og)
        tg = []
        for _ in range(5):
            rg = spk.ksp_solve_mg(G, bd, xg_, og)
            tg.append(rg.seconds)
        xz = torch.zeros_like(xs)
        spk.mg_apply(G, bd, xz)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            spk.mg_apply(G, bd, xz)
        e1.record()
        torch.cuda.synchronize()
        level_ms = spk.mg_profile(G, bd, xz, reps=20)
        tmed = float(np.median(tg))
        mg[name] = {
            "levels": [G.info.n[l] for l in range(G.levels)],
            "setup_ms": setup_ms, "iterations": rg.iterations, "reason": spk.reason_str(rg.reason),
            "solves_per_s": 1.0 / tmed, "ms_p50": tmed * 1e3, "us_per_iter": tmed * 1e6 / max(rg.iterations, 1),
            "cycle_us": e0.elapsed_time(e1) * 1e3 / 20,
            "level_us": [v * 1e3 for v in level_ms],
            "true_rel_residual": rg.true_rel_residual,
            "speedup_vs_jacobi_pcg": jacobi_s / tmed,
        }
        if cyc == 1:
            xv = xg_.cpu().numpy()
            mg[name]["true_rel_residual_oracle"] = oracle.nrm2(b - oracle.spmv(A, xv)) / bn
        if prec == spk.PREC_MIXED:
            ref = mg[name.replace("_fp32", "")]
            mg[name]["speedup_vs_fp64_cycle"] = ref["ms_p50"] / mg[name]["ms_p50"]
        G.close()
    mg["note"] = ("CG preconditioned by one cycle per iteration: aggregation (2x2x2) transfers, "
                  "Galerkin coarse operators, 2+2 Chebyshev-Jacobi steps on [g/10, g], omega 2, "
                  "dense inverse on the coarsest level (<= 1000 rows); level_us = each level's own "
                  "kernels per cycle (the per-level breakdown of Sec. 5.3); *_fp32: the cycle in "
                  "FP32 (values, vectors, arithmetic) inside the FP64 CG")

    return mg


def bench_mg(args):
    """Multigrid-preconditioned CG on the 128^3 Laplacian (the C2 system)."""
    import numpy as np
    import torch

    import spkgen
    from paper_2011_00715_amd import spk

    N = 128
    A = spkgen.laplace3d7(N)
    b = spkgen.rhs_uniform(A.n, 0)
    M = spk.mat_create_csr(dev(A.rowptr), dev(A.col), dev(A.val))
    bd = dev(b)
    x = torch.zeros_like(bd)
    o = spk.ksp_opts(graph_k=args.graph_k)
    spk.ksp_solve(M, bd, x, o)
    tj = float(np.median([spk.ksp_solve(M, bd, x, o).seconds for _ in range(3)]))
    mg = mg_legs(spk, M, A, b, bd, N, tj)
    v = mg["v_cycle"]
    out = {
        "metric": "multigrid-preconditioned CG solves/s to rtol 1e-8",
        "value": v["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 5, "warmup": 1,
        "ms_per_step": v["ms_p50"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (the *_fp32 legs: f32 cycle inside f64 CG)", "data": "synthetic",
        "config": {"workload": "3D 7-point Laplacian 128^3, rhs uniform seed 0; CG preconditioned by one "
                               "multigrid cycle per iteration, graph_k 1", "jacobi_pcg_ms": tj * 1e3},
        "multigrid_pcg": mg,
    }
    M.close()
    return out


def measured_stream_gbps(reps=10):
    """Bandwidth plain streaming kernels reach on this GPU, for the roofline
    beside the 8 TB/s spec peak: the library's copy (1 GiB into 1 GiB, 2 GiB
    moved) and its AXPY y = a x + y (two 1 GiB inputs, 3 GiB moved, the
    paper's VecAXPY), 4-12x the Infinity Cache; GB/s of the median of `reps`
    event-timed launches."""
    import statistics

    import torch

    from paper_2011_00715_amd import spk

    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.zeros_like(a)

    def timed(fn):
        for _ in range(2):
            fn()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return statistics.median(ts)

    t_copy = timed(lambda: spk.bw_copy(a, c))
    t_axpy = timed(lambda: spk.vec_axpy(0.5, a, c))
    out = {"copy": 2 * n * 8 / t_copy / 1e9, "axpy": 3 * n * 8 / t_axpy / 1e9,
           "note": "copy 1 GiB -> 1 GiB (read + written bytes) and AXPY over 1 GiB vectors (2 reads + "
                   "1 write), median of %d launches; the product's bytes are almost all reads, which "
                   "HBM serves faster than a read/write mix" % reps}
    del a, c
    return out


def calibration_copy():
    """One plain copy of 256 MiB (known traffic: 256 MiB read + 256 MiB
    written), so PMC byte counters can be scaled against it: the smallest
    k_copy dispatch of a run (the streaming-bandwidth figure of the roofline
    copies 1 GiB)."""
    import torch

    from paper_2011_00715_amd import spk

    n = (256 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    spk.bw_copy(a, c)
    torch.cuda.synchronize()
    del a, c


def solve_pair(spk, M, bd, graph_k):
    import torch

    x64 = torch.zeros_like(bd)
    xmx = torch.zeros_like(bd)
    r64 = spk.ksp_solve(M, bd, x64, spk.ksp_opts(graph_k=graph_k))
    rmx = spk.ksp_solve(M, bd, xmx, spk.ksp_opts(graph_k=graph_k, precision=spk.PREC_MIXED))
    return x64, r64, xmx, rmx


def bench_c3(args):
    """27-point lognormal diffusion 160^3: FP64 vs mixed-precision solves."""
    import numpy as np
    import torch

    import oracle
    import spkgen
    from paper_2011_00715_amd import spk

    log("generating 27-point lognormal 160^3")
    A = spkgen.diffusion3d27_lognormal(160, seed=0)
    b = spkgen.rhs_uniform(A.n, 0)
    log("solving")
    M = spk.mat_create_csr(dev(A.rowptr), dev(A.col), dev(A.val), flags=spk.MAT_MIXED)
    info = M.info
    bd = dev(b)
    for _ in range(args.warmup):
        solve_pair(spk, M, bd, args.graph_k)
    t64, tmx = [], []
    for _ in range(args.steps):
        x64, r64, xmx, rmx = solve_pair(spk, M, bd, args.graph_k)
        t64.append(r64.seconds)
        tmx.append(rmx.seconds)
    xg, xm = x64.cpu().numpy(), xmx.cpu().numpy()
    bn = oracle.nrm2(b)
    rel64 = oracle.nrm2(b - oracle.spmv(A, xg)) / bn
    relmx = oracle.nrm2(b - oracle.spmv(A, xm)) / bn
    m64, mmx = float(np.median(t64)), float(np.median(tmx))
    out = {
        "metric": "PCG solves/s to rtol 1e-8, FP64 vs mixed",
        "value": 1.0 / mmx, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": (m64 + mmx) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 inner / f64 outer", "data": "synthetic",
        "config": {"workload": "3D 27-point lognormal diffusion 160^3 (n=4096000, nnz=109215352), "
                               "rhs uniform seed 0; mixed CG (FP32 values/accumulate inside, FP64 "
                               "residual/update/test) vs FP64", "kernel": spk.KERNEL_NAMES[info.kernel],
                   "kernel_param": info.lanes, "cached_loads": info.cached_loads},
        "fp64": {"solves_per_s": 1 / m64, "ms": m64 * 1e3, "iterations": r64.iterations,
                 "us_per_iter": m64 * 1e6 / max(r64.iterations, 1),
                 "gbps": solve_bytes(info, r64) / m64 / 1e9, "true_rel_residual_oracle": rel64},
        "mixed": {"solves_per_s": 1 / mmx, "ms": mmx * 1e3, "inner_iterations": rmx.inner_iterations,
                  "outer_steps": rmx.outer_steps, "fallback_fp64": rmx.fallback_fp64,
                  "us_per_inner_iter": mmx * 1e6 / max(rmx.inner_iterations, 1),
                  "gbps": solve_bytes(info, rmx) / mmx / 1e9, "true_rel_residual_oracle": relmx,
                  "error_vs_fp64": float(np.linalg.norm(xm - xg) / np.linalg.norm(xg))},
        "speedup_mixed_vs_fp64": m64 / mmx,
    }
    log("multigrid")
    out["multigrid_pcg"] = mg_legs(spk, M, A, b, bd, 160, m64)
    M.close()
    return out


def bench_c4(args):
    """Power-law SPD n = 4M: FP64 and FP32-value SpMV per kernel family."""
    import numpy as np
    import torch

    import oracle
    import spkgen
    from paper_2011_00715_amd import spk

    log("generating power-law n=4M" + (f", columns within +-{args.c4_band}" if args.c4_band else ""))
    A = spkgen.powerlaw_spd(4_000_000, seed=0, band=args.c4_band or None)
    log(f"nnz {A.nnz}; timing kernels")
    M = spk.mat_create_csr(dev(A.rowptr), dev(A.col), dev(A.val), flags=spk.MAT_MIXED)
    info = M.info
    auto = spk.KERNEL_NAMES[info.kernel]
    xh = spkgen.rhs_uniform(A.n, 0)
    x = dev(xh)
    y = torch.empty_like(x)
    x32 = x.float()
    y32 = torch.empty_like(x32)
    rows = np.random.default_rng(0).integers(0, A.n, 2000)
    yo, ya = oracle.spmv_rows(A, xh, rows)
    res = {}
    for name, k, p in [("auto", spk.KERNEL_AUTO, 0),
                       ("sliced", spk.KERNEL_SLICED, 2048), ("sliced_lanes4", spk.KERNEL_SLICED, 4),
                       ("merge", spk.KERNEL_MERGE, 0),
                       ("vector32", spk.KERNEL_VECTOR, 32), ("vector8", spk.KERNEL_VECTOR, 8),
                       ("stream", spk.KERNEL_STREAM, 0), ("sell", spk.KERNEL_SELL, 0),
                       ("sell_sigma_4096", spk.KERNEL_SELL_SIGMA, 4096),
                       ("sell_sigma_65536", spk.KERNEL_SELL_SIGMA, 65536),
                       ("sell_sigma_all", spk.KERNEL_SELL_SIGMA, (A.n + 63) // 64 * 64)]:
        try:
            spk.mat_set_kernel(M, k, p)
        except spk.SpkError as e:
            res[name] = {"refused": str(e)}
            continue
        for _ in range(args.warmup + 1):
            spk.mat_mult(M, x, y)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for e0, e1 in ev:
            e0.record()
            spk.mat_mult(M, x, y)
            e1.record()
        torch.cuda.synchronize()
        us = float(np.median([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev]))
        err = float(np.max(np.abs(y.cpu().numpy()[rows] - yo) / ya))
        for _ in range(args.warmup + 1):
            spk.mat_mult_f32(M, x32, y32)
        for e0, e1 in ev:
            e0.record()
            spk.mat_mult_f32(M, x32, y32)
            e1.record()
        torch.cuda.synchronize()
        us32 = float(np.median([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev]))
        mi = M.info
        res[name] = {"us": us, "gbps": info.bytes_spmv_f64 / us / 1e3, "max_err_rel_abs_sum": err,
                     "f32_us": us32, "f32_gbps": info.bytes_spmv_f32 / us32 / 1e3,
                     "kernel": spk.KERNEL_NAMES[mi.kernel], "param": mi.lanes,
                     "stored_nnz": mi.stored_nnz, "format_bytes_f64": mi.format_bytes_spmv_f64,
                     "format_gbps": mi.format_bytes_spmv_f64 / us / 1e3}
    out = {
        "metric": "CSR SpMV HBM GB/s (algorithmic), power-law rows",
        "value": res["auto"]["gbps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["auto"]["us"] / 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"random SPD, n=4000000, nnz={info.nnz}, Zipf(1.8) row picks clipped "
                               "to [3,4000], symmetric pattern"
                               + (f", columns within +-{args.c4_band} of the row" if args.c4_band else
                                  ", uniform columns"), "auto_kernel": auto,
                   "row_mean": info.row_mean, "row_max": info.row_max, "row_cv": info.row_cv},
        "kernels": res,
        "bytes_f64": info.bytes_spmv_f64, "bytes_f32": info.bytes_spmv_f32,
        "note": "gbps = algorithmic CSR bytes (12 nnz + 4(n+1) + 16n; FP32 8 nnz + 4(n+1) + 8n) per "
                "median launch time; the sliced family also moves 4(8n+1) row pointers and writes and "
                "reads 8n partial products (format_bytes_f64)",
    }
    M.close()
    return out


SERVE_CLIENTS = 8  # client threads submitting to the server


def serve_run(spk, reqs, closed, graph_k, pinned_bytes=None):
    """Serve `reqs` through one spk_server: open loop (each request submitted
    at its arrival time) or closed (all queued at t = 0).  Latency = finish
    - scheduled arrival (host clock).  The client forms each request before
    it arrives (producer thread); patterns are built before the clock.
    SERVE_CLIENTS client threads submit, the main thread drives the server."""
    import queue
    import threading

    import numpy as np

    import spkgen

    for r in reqs:
        spkgen.serve_matrix(r)
    opts = spk.server_opts_default()
    opts.hbm_budget_bytes = 32 << 30
    opts.max_slots = 64
    # pinned pool: room for the requests queued ahead of admission (a closed
    # loop queues them all at once: its host arrays, capped at 48 GiB)
    need = sum(12 * spkgen.serve_matrix(r).nnz + 20 * spkgen.serve_matrix(r).n for r in reqs) if closed else 0
    opts.pinned_bytes = pinned_bytes or max(8 << 30, min(int(need * 1.05), 48 << 30))
    opts.graph_k = graph_k
    S = spk.server_create(opts)
    o = spk.ksp_opts(precision=spk.PREC_MIXED)
    prepared = queue.Queue(maxsize=512)

    def producer():
        for r in reqs:
            A = spkgen.serve_matrix(r)
            prepared.put((r, A, spkgen.rhs_uniform(A.n, r.rhs_seed % (2**31))))

    threading.Thread(target=producer, daemon=True).start()
    if closed:  # queue everything at t = 0
        while prepared.qsize() < min(len(reqs), 512) and prepared.qsize() < len(reqs):
            time.sleep(0.01)
    # client threads submit the requests at their arrival times (the copy of
    # a large system runs there, outside the server's lock, and a small
    # request is not held behind a large one's copy) while this thread keeps
    # the GPU fed: progress, the completion queue, collection
    lock, take = threading.Lock(), threading.Lock()
    pending, early, err = {}, [], []
    lat, iters = [], []
    worst_rel = 0.0
    old_si = sys.getswitchinterval()
    sys.setswitchinterval(0.0005)
    t0 = spk.now()

    def submitter():
        try:
            while True:
                with take:  # the next arrival, in order
                    if not left_to_take[0]:
                        return
                    left_to_take[0] -= 1
                    r, A, b = prepared.get()
                if not closed:
                    delay = r.t_arrival - (spk.now() - t0)
                    if delay > 0:
                        time.sleep(delay)
                t_arr = t0 + (0.0 if closed else r.t_arrival)
                t = spk.server_submit(S, A.rowptr, A.col, A.val, b, o)
                with lock:
                    pending[t] = (t_arr, A.n)
        except BaseException as e:  # noqa: BLE001 - re-raised on the main thread
            err.append(e)

    left_to_take = [len(reqs)]
    ths = [threading.Thread(target=submitter, daemon=True) for _ in range(SERVE_CLIENTS)]
    for th in ths:
        th.start()
    try:
        while len(lat) < len(reqs):
            if err:
                raise err[0]
            left = spk.server_progress(S, 1)
            done = spk.server_completed(S)
            if early:  # finished before the client thread recorded the ticket
                done, early = early + done, []
            for t in done:
                with lock:
                    ent = pending.pop(t, None)
                if ent is None:
                    early.append(t)
                    continue
                t_arr, n = ent
                res, tdone = spk.server_poll(S, t, np.empty(n))
                lat.append(tdone - t_arr)
                iters.append(res.inner_iterations + res.iterations)
                worst_rel = max(worst_rel, res.true_rel_residual)
                assert res.reason > 0, spk.reason_str(res.reason)
            if left == 0 and not done:
                time.sleep(5e-5)
    finally:
        sys.setswitchinterval(old_si)
    for th in ths:
        th.join()
    elapsed = spk.now() - t0
    S.close()
    return {"requests": len(lat), "seconds": elapsed, "solves_per_s": len(lat) / elapsed,
            "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3, "max": max(lat) * 1e3},
            "iterations_mean": float(np.mean(iters)), "worst_true_rel_residual": worst_rel}


def sequential_run(spk, reqs, prec, flags, graph_k):
    """The same requests one at a time through spk_ksp_solve (matrix upload,
    solve, x back to the host); input formation is not timed."""
    import torch

    import spkgen

    os_ = spk.ksp_opts(graph_k=graph_k, precision=prec)
    tseq = 0.0
    for r in reqs:
        A = spkgen.serve_matrix(r)
        b = spkgen.rhs_uniform(A.n, r.rhs_seed % (2**31))
        ts = spk.now()
        M = spk.mat_create_csr(A.rowptr, A.col, A.val, flags=flags)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = spk.ksp_solve(M, dev(b), x, os_)
        x.cpu()
        M.close()
        tseq += spk.now() - ts
        assert res.reason > 0
    return {"solves_per_s": len(reqs) / tseq, "seconds": tseq}


SERVE_MIX = "2D 5-point side 32-256 / 3D 7-point side 16-96, diagonal shift U[0,1), rhs U[-1,1)"


def bench_serve(args):
    """Served solve stream: Poisson arrivals of shifted 2D/3D Laplacians."""
    import spkgen
    from paper_2011_00715_amd import spk

    reqs = spkgen.serve_stream(seed=0, rate=args.serve_rate, duration=args.serve_seconds,
                               count=args.serve_closed or None)
    log(f"{len(reqs)} requests; serving")
    closed = bool(args.serve_closed)
    run = serve_run(spk, reqs, closed, args.graph_k)
    seq = None
    if closed:
        # mixed precision as served, and plain FP64, for the batching gain
        seq = {}
        for name, prec, flags in (("mixed", spk.PREC_MIXED, spk.MAT_MIXED), ("fp64", spk.PREC_FP64, 0)):
            log(f"sequential baseline ({name})")
            seq[name] = sequential_run(spk, reqs, prec, flags, args.graph_k)
            seq[name]["batching_gain"] = run["solves_per_s"] / seq[name]["solves_per_s"]
    return {
        "metric": "served PCG solves/s to rtol 1e-8; p50/p99 latency",
        "value": run["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": run["requests"],
        "warmup": 0, "ms_per_step": run["seconds"] * 1e3 / max(run["requests"], 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 inner / f64 outer", "data": "synthetic",
        "config": {"workload": ("closed loop: %d requests queued at t=0" % len(reqs)) if closed else
                   f"open loop: Poisson {args.serve_rate:g} req/s for {args.serve_seconds:g} s",
                   "requests": len(reqs), "mix": SERVE_MIX, "graph_k": args.graph_k},
        "latency_ms": run["latency_ms"], "iterations_mean": run["iterations_mean"],
        "worst_true_rel_residual": run["worst_true_rel_residual"],
        "sequential": seq,
    }


def bench_spectrum(args):
    """Work-time spectrum (Sec. 5.1): time per operation against the work it
    moves, from latency-bound to bandwidth-bound sizes, for VecAXPY
    (3 accesses per entry), a streaming copy (2), the FP64 SpMV and a
    Jacobi-PCG iteration on 3D 7-point Laplacians."""
    import numpy as np
    import torch

    import spkgen
    from paper_2011_00715_amd import spk

    def timed(fn, reps=20):
        us = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            us.append(e0.elapsed_time(e1) * 1e3)
        return float(np.median(us))

    vec = []
    for e in range(6, 17):  # n = 10^3 ... 10^8 in half decades
        n = 2 * int(round(10 ** (e / 2) / 2))  # the copy kernel moves pairs
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.ones(n, dtype=torch.float64, device="cuda")
        fn_axpy = lambda: spk.vec_axpy(0.5, x, y)  # noqa: E731
        fn_copy = lambda: spk.bw_copy(x, y)  # noqa: E731
        fn_axpy(), fn_copy()
        ta, tc = timed(fn_axpy), timed(fn_copy)
        vec.append({"n": n, "axpy_us": ta, "axpy_gbps": 24 * n / ta / 1e3,
                    "copy_us": tc, "copy_gbps": 16 * n / tc / 1e3})
        log(f"vec n={n}: axpy {ta:.2f} us, copy {tc:.2f} us")
        del x, y
    mat = []
    for N in (10, 16, 25, 40, 64, 100, 128, 160, 200):
        A = spkgen.laplace3d7(N)
        M = spk.mat_create_csr(dev(A.rowptr), dev(A.col), dev(A.val))
        info = M.info
        xs = dev(spkgen.rhs_uniform(A.n, 0))
        ys = torch.empty_like(xs)
        spk.mat_mult(M, xs, ys)
        t_spmv = timed(lambda: spk.mat_mult(M, xs, ys))
        b = xs
        xx = torch.zeros_like(xs)
        def iter_us(single_reduction):
            secs = {}
            for its in (20, 60):
                o = spk.ksp_opts(rtol=0.0, atol=0.0, maxit=its, graph_k=args.graph_k,
                                 single_reduction=single_reduction)
                spk.ksp_solve(M, b, xx, o)
                secs[its] = float(np.median([spk.ksp_solve(M, b, xx, o).seconds for _ in range(5)]))
            return (secs[60] - secs[20]) / 40 * 1e6

        t_it = iter_us(0)
        t_sr = iter_us(1)
        mat.append({"N": N, "n": info.n, "nnz": info.nnz, "kernel": spk.KERNEL_NAMES[info.kernel],
                    "spmv_us": t_spmv, "spmv_gbps": info.bytes_spmv_f64 / t_spmv / 1e3,
                    "pcg_iter_us": t_it, "pcg_iter_gbps": info.bytes_pcg_iter_f64 / t_it / 1e3,
                    "pcg_sr_iter_us": t_sr})
        log(f"3D {N}^3: spmv {t_spmv:.2f} us, pcg iteration {t_it:.2f} us, single-reduction {t_sr:.2f} us")
        M.close()
    big = mat[-1]
    return {
        "metric": "work-time spectrum: time per operation vs bytes moved (latency and asymptotic bandwidth)",
        "value": big["spmv_gbps"], "unit": "GB/s", "n_gpus": 1, "steps": len(vec) + len(mat),
        "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "VecAXPY / copy n = 10^3..10^8; 3D 7-point Laplacian N^3, N = 10..200 "
                               "(SpMV, and Jacobi-PCG iterations from (t(60 its) - t(20 its)) / 40)"},
        "vectors": vec, "laplace3d": mat,
        "latency_us": {"axpy": vec[0]["axpy_us"], "copy": vec[0]["copy_us"], "spmv": mat[0]["spmv_us"],
                       "pcg_iter": mat[0]["pcg_iter_us"], "pcg_sr_iter": mat[0]["pcg_sr_iter_us"]},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (sharding the path across "
                          "GPUs is not built)"}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    calibration_copy()
    fn = {"all": bench_all, "c2": bench_c2, "c3": bench_c3, "c4": bench_c4, "serve": bench_serve,
          "spectrum": bench_spectrum, "mg": bench_mg}[args.workload]
    out = fn(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
