#!/usr/bin/env python3
"""Benchmark of the tiled GEMM C = alpha*A*B + beta*C on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--no-cpu]

One step is one full GEMM on device-resident inputs (square FP64, N = 8192,
entries uniform[-1,1], alpha = beta = 1).  The K timed steps are bracketed by a
device synchronisation on both sides and timed with HIP events on the stream the
kernels run on; TFLOP/s = 2N^3 / time (the paper's Eq. 4, in TFLOP/s).  Prints
one JSON line.  The CPU baseline is the oracle (plain FP64 triple loop, all host
cores) on a bounded sample of rows of the same product.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GEMM TFLOP/s (% peak): FP64 vs split-precision at equal error; tuner regret"
PEAK_F64_TFLOPS = 78.6       # MI355X FP64 matrix peak (published)
PEAK_F32_TFLOPS = 157.3
HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(n, A, B, C, budget_s):
    """Times the oracle on a row sample of the same product; scales to TFLOP/s."""
    import oracle
    cores = oracle.num_procs()
    # calibrate with 4 rows, then size the sample to the time budget
    t = time.perf_counter()
    oracle.gemm_f64(1.0, A[:4], B, 1.0, C[:4], nthreads=cores)
    dt = max(time.perf_counter() - t, 1e-6)
    rows = int(max(cores, min(n, 4 * budget_s / dt)))
    rows = max(cores, (rows // cores) * cores)
    t = time.perf_counter()
    oracle.gemm_f64(1.0, A[:rows], B, 1.0, C[:rows], nthreads=cores)
    dt = time.perf_counter() - t
    flops = 2.0 * rows * n * n
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"first {rows} of {n} rows of the N={n} FP64 product "
                      f"({flops / 1e9:.1f} GFLOP in {dt:.1f} s, OpenMP over rows)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (the library is single-GPU)")
        return 2
    import torch
    import synth
    import paper_1706_10086_amd as mg

    if not torch.cuda.is_available():
        log("bench.py: no GPU visible")
        return 3
    mg.lib()
    dev = torch.device("cuda:0")
    n = args.n
    log(f"bench: generating N={n} inputs")
    sa, sb, sc = synth.seeds_for(1, int(np.log2(n)))
    A = synth.uniform_pm1((n, n), sa)
    B = synth.uniform_pm1((n, n), sb)
    C0 = synth.uniform_pm1((n, n), sc)
    tA = torch.from_numpy(A).to(dev)
    tB = torch.from_numpy(B).to(dev)
    tC = torch.from_numpy(C0).to(dev)
    stream = torch.cuda.current_stream()

    def step():
        mg.gemm(tA, tB, tC, 1.0, 1.0, stream=stream)

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    total_ms = ev[0].elapsed_time(ev[-1])
    ms = total_ms / args.steps
    flops = 2.0 * n ** 3
    tflops = flops / (ms * 1e-3) / 1e12
    kern_ms = float(np.mean(per))
    best_ms = float(np.min(per))

    # accuracy of this exact run against the oracle on sampled rows
    rows = np.arange(0, n, max(1, n // 16))
    steps_done = args.warmup + args.steps
    log("bench: accuracy check on sampled rows")
    import oracle
    # C was updated steps_done times: C_s = A B + C_{s-1}; recompute on the rows
    ref = C0[rows].copy()
    AB = oracle.gemm_f64(1.0, A[rows], B, 0.0, None, nthreads=oracle.num_procs())
    for _ in range(steps_done):
        ref = AB + ref
    got = tC[torch.from_numpy(rows).to(dev)].cpu().numpy()
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    cpu = None
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline(n, A, B, C0, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"square DGEMM N={n}, FP64 row-major, A,B,C uniform[-1,1], "
                               f"alpha=1, beta=1, default tile configuration",
                   "n": n, "alpha": 1.0, "beta": 1.0, "parallelism": "single GPU"},
        "pct_peak": round(100.0 * tflops / PEAK_F64_TFLOPS, 2),
        "best_step_tflops": round(flops / (best_ms * 1e-3) / 1e12, 3),
        "wall_s": round(wall, 3),
        "sampled_rel_err_vs_oracle": err,
        "roofline": {"bound": "mfma", "achieved": round(flops / (kern_ms * 1e-3) / 1e12, 3),
                     "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(flops / (kern_ms * 1e-3) / 1e12 / PEAK_F64_TFLOPS, 4),
                     "traffic": None,
                     "kernel": "gemm_tiled_kernel<double,...> (one launch per step)",
                     "kernel_avg_ms": round(kern_ms, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
