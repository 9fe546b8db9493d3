"""Benchmark of the CSR SpMV / Jacobi-PCG hot path on one MI355X.

Default workload: 3D 7-point Laplacian on a 128^3 grid (n = 2,097,152,
nnz = 14,581,760), FP64 CSR with int32 indices, rhs uniform[-1, 1) from seed 0.
One step = one FP64 Jacobi-PCG solve to rtol 1e-8 + one mixed-precision solve
(FP32 inner CG, FP64 refinement) to rtol 1e-8 + 100 standalone FP64 SpMVs,
all through the C ABI of libspk.so on the current torch stream.

Prints one JSON line.  `value` is the whole step's algorithmic HBM traffic
divided by its wall time (GB/s); solves/s, solve latency percentiles and the
SpMV rate are reported beside it.  `roofline` covers the SpMV kernel, timed
with HIP events around each launch on the stream it runs on.

Other workloads (one JSON line each): --workload c3 (27-point lognormal
160^3, FP64 vs mixed), c4 (power-law n = 4M SpMV by kernel family), serve
(served solve stream).
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
SPMV_KERNEL = "k_spmv_stream<double>"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "serve"])
    p.add_argument("--spmvs", type=int, default=100)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-iters", type=int, default=200)
    p.add_argument("--graph-k", type=int, default=8)
    p.add_argument("--serve-seconds", type=float, default=60.0)
    p.add_argument("--serve-rate", type=float, default=200.0)
    p.add_argument("--serve-closed", type=int, default=0,
                   help="closed-loop saturation run with this many requests queued at t=0")
    return p.parse_args()


def pct(a, q):
    import numpy as np

    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def source_hash():
    h = hashlib.sha256()
    for f in ("spmv.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2011_00715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key, bytes_per_launch):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, or None if
    absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel_key)
    if not e or e.get("source_hash") != source_hash():
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


def cpu_baseline(A, b, info, iters):
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


def bench_c2(args):
    import numpy as np
    import torch

    import spkgen
    from paper_2011_00715_amd import spk

    N = 128
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
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(S)]

    def step(record):
        r64 = spk.ksp_solve(M, bd, x64, o64)
        rmx = spk.ksp_solve(M, bd, xmx, omx)
        for i in range(S):
            if record:
                ev[i][0].record()
            spk.mat_mult(M, xs, ys)
            if record:
                ev[i][1].record()
        return r64, rmx

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
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
        spmv_us.extend(e0.elapsed_time(e1) * 1e3 for e0, e1 in ev)
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
    traffic = traffic_from_profiles(SPMV_KERNEL + "@c2", info.bytes_spmv_f64)

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
            "n": info.n, "nnz": info.nnz, "spmv_kernel": spk.KERNEL_NAMES[info.kernel],
            "rows_per_tile": info.lanes, "graph_k": args.graph_k,
        },
        "spmv": {
            "us_avg": spmv_avg_us, "us_p50": pct(spmv_us, 50), "us_p99": pct(spmv_us, 99),
            "gbps": achieved, "bytes": info.bytes_spmv_f64,
        },
        "pcg_fp64": {
            "solves_per_s": 1e3 / float(np.median(t64)), "ms_p50": pct(t64, 50), "ms_p99": pct(t64, 99),
            "iterations": r64.iterations, "us_per_iter": float(np.median(t64)) * 1e3 / max(r64.iterations, 1),
            "gbps": solve_bytes(info, r64) / (float(np.median(t64)) * 1e-3) / 1e9,
            "true_rel_residual_oracle": rel64, "reason": spk.reason_str(r64.reason),
        },
        "pcg_mixed": {
            "solves_per_s": 1e3 / float(np.median(tmx)), "ms_p50": pct(tmx, 50), "ms_p99": pct(tmx, 99),
            "inner_iterations": rmx.inner_iterations, "outer_steps": rmx.outer_steps,
            "fallback_fp64": rmx.fallback_fp64,
            "true_rel_residual_oracle": relmx, "reason": spk.reason_str(rmx.reason),
            "error_vs_fp64": float(np.linalg.norm(xm - xg) / np.linalg.norm(xg)),
            "speedup_vs_fp64": float(np.median(t64)) / float(np.median(tmx)),
        },
        "roofline": {
            "kernel": SPMV_KERNEL, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": info.bytes_spmv_f64,
            "note": "12 nnz + 4 (n+1) + 16 n algorithmic bytes per launch; back-to-back launches, "
                    "so the 217 MB working set can be partly served by the 256 MB Infinity Cache",
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, b, info, args.cpu_iters)
    M.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(the multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "c2":
        out = bench_c2(args)
    else:
        out = {"error": f"workload {args.workload} not available"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
