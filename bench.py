#!/usr/bin/env python3
"""Benchmark of the tiled GEMM C = alpha*A*B + beta*C on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--no-cpu] [--no-extras]

One step is one full FP64 GEMM on device-resident inputs (square N = 8192, entries
uniform[-1,1], alpha = beta = 1): the paper's benchmark computation (Sec. 2, Eq. 1) at
the headline size.  The K timed steps are bracketed by a device synchronisation on both
sides and timed with HIP events on the stream the kernels run on; TFLOP/s = 2N^3 / time
(Eq. 4).  ``value`` is that throughput.

The same JSON line also carries (unless --no-extras):
  split    the split-precision emulated FP64 GEMM (bf16 and int8 slices) and plain FP64
           on the wide-range stress inputs at N = 8192: FP64-equivalent TFLOP/s and
           normwise error against the double-double oracle on sampled rows;
  batched  2048 uneven FP64 problems (m, n, k log-uniform in [16, 1024]): one captured
           persistent launch against one launch per problem;
  tuner    the learned configuration predictor (trained here by the library's MLP
           kernels on the tuner database in paper_1706_10086_amd/data) on the held-out
           shapes: achieved fraction of the exhaustive best, against the single tuned
           configuration per dtype.
The CPU baseline is the oracle (plain FP64 triple loop, all host cores) on a bounded
sample of rows of the same product.
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

from paper_1706_10086_amd import perfmodel as pm  # noqa: E402  (closed forms, Eq. 2-8)

METRIC = "GEMM TFLOP/s (% peak): FP64 vs split-precision at equal error; tuner regret"
# MI355X dense matrix peaks (published; Eq. 8 with 256 CUs at 2.4 GHz gives the same
# to 0.1 %, perfmodel.mi355x_peak)
PEAK_F64_TFLOPS = 78.6
PEAK_F32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2516.6
PEAK_FP8_TFLOPS = 5033.2
PEAK_INT8_TOPS = 5033.2
# Measured HBM traffic of the N = 8192 FP64 launch (FETCH_SIZE x 2.0 + WRITE_SIZE x
# 1.0, the factors a plain copy of known size gives); valid for the kernel as
# profiled -- to be re-measured whenever the FP64 tile kernel changes.
TRAFFIC_F64_N8192 = 22.05e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="only the FP64 headline leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--leg", choices=["parity", "sweep", "split", "batched", "batched_plan", "tuner",
                                       "memory", "copy"],
                    default=None,
                    help="run only this extra leg and print its JSON (for profiling runs; "
                         "'copy' is the calibration workload of the traffic counters)")
    ap.add_argument("--cfg", default=None,
                    help="bm,bn,bk,waves,ept,dbuf,occ: time this registered configuration "
                         "instead of the library's choice (profiling runs)")
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy leg: MiB per copy")
    ap.add_argument("--copy-reps", type=int, default=3, help="copy leg: number of copies")
    return ap.parse_args()


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or 'unknown'."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def leg_copy(torch, dev, mib=1024, reps=3):
    """Calibration workload for the HBM traffic counters: a device-to-device copy
    of a known number of bytes (torch's copy kernel), ``reps`` times.  Run under
    rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE), the reading per copied byte
    scales the same counters of the GEMM kernels to bytes."""
    n = mib * 1024 * 1024 // 8
    src = torch.rand(n, device=dev, dtype=torch.float64)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"bytes_per_copy": 8 * n, "copies": reps}


def kernel_name(c: dict) -> str:
    """The FP64 kernel a registered configuration runs on aligned rows (as the
    profiler names it)."""
    wgm = 4 if c["waves"] == 8 and c["bm"] >= c["bn"] else 2
    wgn = c["waves"] // wgm
    if c["double_buffer"] == 2:
        return f"gemm_pipe_kernel<double,{c['bm']},{c['bn']},{c['bk']},{wgm},{wgn}>"
    return (f"gemm_tiled_kernel<double,{c['bm']},{c['bn']},{c['bk']},...> "
            f"({c['waves']} waves, {c['elems_per_thread']} per thread, "
            f"{c['double_buffer'] + 1} stage(s), occupancy {c['occupancy']})")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(fn, stream, reps, warmup=1):
    """Per-call device times (ms) of fn() with HIP events on ``stream``."""
    import torch
    for _ in range(warmup):
        fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(reps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]


def timed_batches(fn, stream, batches=5, warm_s=0.1, batch_s=0.05):
    """Per-call device time (ms) of back-to-back calls of fn(): one event pair
    around each batch of calls (events between every call add a few microseconds
    each, which small products would count); warmed up for warm_s seconds first
    (clocks ramp up) and each batch sized to about batch_s seconds."""
    import torch
    est = timed(fn, stream, 3, warmup=2)
    per = max(min(est), 1e-3) / 1e3
    for _ in range(max(3, int(warm_s / per))):
        fn()
    reps = max(3, int(batch_s / per))
    out = []
    for _ in range(batches):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / reps)
    return out


def cpu_baseline(n, A, B, C, budget_s):
    """Times the oracle on a row sample of the same product; scales to TFLOP/s."""
    import oracle
    cores = oracle.num_procs()
    rows = max(cores, 16)
    t = time.perf_counter()
    oracle.gemm_f64(1.0, A[:rows], B, 1.0, C[:rows], nthreads=cores)
    dt = max(time.perf_counter() - t, 1e-6)
    rows = int(min(n, rows * budget_s / dt))
    rows = max(cores, (rows // cores) * cores)
    t = time.perf_counter()
    oracle.gemm_f64(1.0, A[:rows], B, 1.0, C[:rows], nthreads=cores)
    dt = time.perf_counter() - t
    flops = 2.0 * rows * n * n
    # one thread on the whole N = 1024 product, extrapolated by N^3 to this N
    import synth
    a1 = synth.uniform_pm1((1024, 1024), 9001)
    b1 = synth.uniform_pm1((1024, 1024), 9002)
    t1 = time.perf_counter()
    oracle.gemm_f64(1.0, a1, b1, 0.0, None, nthreads=1)
    t1 = time.perf_counter() - t1
    return {"value": round(flops / dt / 1e12, 5), "unit": "TFLOP/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {rows} of {n} rows of the N={n} FP64 product "
                      f"({flops / 1e9:.1f} GFLOP in {dt:.1f} s, OpenMP over rows)",
            "single_thread_n1024_s": round(t1, 3),
            "single_thread_extrapolated_s": round(t1 * (n / 1024) ** 3, 1)}


def leg_split(mg, torch, dev, n=8192, with_small=True):
    """The emulated FP64 dtypes and plain FP64 on the wide-range stress inputs at
    N = 8192 (256 rows spread evenly over the matrix checked) and N / 2 (every
    element checked): time, FP64-equivalent TFLOP/s, and the normwise error
    against the double-double (Dot2) oracle and against the plain FP64 oracle."""
    import oracle
    import synth
    out = {"inputs": "u*2^e, u uniform[-1,1], e uniform integer in [-20,20]; alpha 1, beta 0",
           "error": "normwise, against the double-double (Dot2) oracle (rel_err) and the plain "
                    "FP64 oracle (rel_err_vs_f64_oracle)"}
    sizes = [(n, 256)] + ([(n // 2, None)] if with_small else [])
    for size, count in sizes:
        log(f"bench: split leg, N={size} wide-range inputs")
        sa, sb, _ = synth.seeds_for(2, int(np.log2(size)))
        A = synth.wide_range((size, size), sa)
        B = synth.wide_range((size, size), sb)
        rows = np.arange(size) if count is None else np.linspace(0, size - 1, count).astype(np.int64)
        log(f"bench: split leg, Dot2 and FP64 oracles on {len(rows)} rows")
        ref = oracle.gemm_dot2(1.0, A[rows], B, nthreads=oracle.num_procs())
        ref64 = oracle.gemm_f64(1.0, A[rows], B, nthreads=oracle.num_procs())
        tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        del A, B
        tC = torch.zeros((size, size), device=dev, dtype=torch.float64)
        trows = torch.from_numpy(rows).to(dev)
        stream = torch.cuda.current_stream()
        res = {"n": size, "rows_checked": len(rows),
               "f64_oracle_vs_dot2": float(np.linalg.norm(ref64 - ref) / np.linalg.norm(ref))}
        for name, dt in (("f64", mg.F64), ("bf16", mg.SPLIT_BF16), ("fp8", mg.SPLIT_FP8),
                         ("int8", mg.SPLIT_INT8), ("crt_int8", mg.CRT_INT8)):
            ts = timed(lambda: mg.gemm(tA, tB, tC, 1.0, 0.0, dtype=dt, stream=stream), stream, 5)
            got = tC[trows].cpu().numpy()
            ms = float(np.mean(ts))
            res[name] = {"ms": round(ms, 4), "tflops_fp64_equiv": round(2.0 * size ** 3 / ms / 1e9, 3),
                         "pct_fp64_peak": round(100 * 2.0 * size ** 3 / ms / 1e9 / PEAK_F64_TFLOPS, 2),
                         "rel_err": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                         "rel_err_vs_f64_oracle": float(np.linalg.norm(got - ref64) / np.linalg.norm(ref64))}
            log(f"  n={size} {name}: {ms:.3f} ms, err {res[name]['rel_err']:.2e} (Dot2), "
                f"{res[name]['rel_err_vs_f64_oracle']:.2e} (FP64 oracle)")
        res["bf16"]["mfma_util"] = round(21 * 2.0 * size ** 3 / (res["bf16"]["ms"] * 1e9) / PEAK_BF16_TFLOPS, 4)
        res["fp8"]["mfma_util"] = round(66 * 2.0 * size ** 3 / (res["fp8"]["ms"] * 1e9) / PEAK_FP8_TFLOPS, 4)
        res["int8"]["mfma_util"] = round(36 * 2.0 * size ** 3 / (res["int8"]["ms"] * 1e9) / PEAK_INT8_TOPS, 4)
        # 16 int8 GEMMs of the zero-padded operands (one per modulus)
        npad = -(-size // 256) * 256
        kpad = -(-size // 64) * 64
        res["crt_int8"]["mfma_util"] = round(16 * 2.0 * npad * npad * kpad /
                                             (res["crt_int8"]["ms"] * 1e9) / PEAK_INT8_TOPS, 4)
        if size == n:
            out.update(res)
        else:
            out[f"n{size}"] = res
        del tA, tB, tC
        torch.cuda.empty_cache()
    return out


def leg_parity(mg, torch, dev):
    """The parity case: m = n = k = 256, uniform inputs, alpha 1.5, beta 0.5; the
    GPU time (latency-bound), the oracle's single-thread wall time and the
    normwise error against it."""
    import oracle
    import synth
    n = 256
    sa, sb, sc = synth.seeds_for(0, 8)
    A, B, C = synth.uniform_pm1((n, n), sa), synth.uniform_pm1((n, n), sb), synth.uniform_pm1((n, n), sc)
    tA, tB, tC0 = (torch.from_numpy(x).to(dev) for x in (A, B, C))
    tC = tC0.clone()
    stream = torch.cuda.current_stream()
    mg.gemm(tA, tB, tC, 1.5, 0.5, stream=stream)
    got = tC.cpu().numpy()
    t = time.perf_counter()
    want = oracle.gemm_f64(1.5, A, B, 0.5, C, nthreads=1)
    t_orc = time.perf_counter() - t
    ts = timed(lambda: mg.gemm(tA, tB, tC, 1.5, 0.5, stream=stream), stream, 50, warmup=5)
    return {"n": n, "gpu_us": round(1e3 * float(np.mean(ts)), 2),
            "gpu_tflops": round(2.0 * n ** 3 / float(np.mean(ts)) / 1e9, 3),
            "oracle_single_thread_s": round(t_orc, 4),
            "rel_err": float(np.linalg.norm(got - want) / np.linalg.norm(want))}


def leg_sweep(mg, torch, dev, sizes=(1024, 2048, 3072, 4096, 6144, 7680, 8192, 16384)):
    """The square sweep: FP64 and FP32 with the library's default configuration,
    uniform[-1,1) inputs drawn on the device, alpha = beta = 1; each size records
    the plan (tile, k ranges, rows run whole), and where the plan is a split tail
    (N = 3072 FP64, 7680) also the rate of its 128 x 128 tile run whole."""
    log("bench: square sweep, FP64 and FP32")
    stream = torch.cuda.current_stream()
    out = {"inputs": "uniform[-1,1) on the device, alpha = beta = 1",
           "timing": "back-to-back calls after 0.1 s of warm-up, one event pair per batch "
                     "of about 50 ms; ms = mean over the batches",
           "f64": {}, "f32": {}}
    for name, tdt, dt, peak in (("f64", torch.float64, mg.F64, PEAK_F64_TFLOPS),
                                ("f32", torch.float32, mg.F32, PEAK_F32_TFLOPS)):
        for n in sizes:
            g = torch.Generator(device=dev)
            g.manual_seed(7000 + n)
            A = torch.rand((n, n), device=dev, dtype=tdt, generator=g) * 2 - 1
            B = torch.rand((n, n), device=dev, dtype=tdt, generator=g) * 2 - 1
            C = torch.rand((n, n), device=dev, dtype=tdt, generator=g) * 2 - 1
            ts = timed_batches(lambda: mg.gemm(A, B, C, 1.0, 1.0, stream=stream), stream,
                               batches=5 if n <= 8192 else 3)
            ms = float(np.mean(ts))
            tf = 2.0 * n ** 3 / ms / 1e9
            c, splits, whole = mg.choice(n, n, n, dt, rows=True)
            rec = {"ms": round(ms, 4), "tflops": round(tf, 3),
                   "pct_peak": round(100 * tf / peak, 2),
                   "best_tflops": round(2.0 * n ** 3 / min(ts) / 1e9, 3),
                   "plan": {"tile": f"{c.bm}x{c.bn}x{c.bk}", "k_ranges": splits,
                            "whole_rows": whole}}
            if splits > 1 and whole > 0:
                tw = timed_batches(lambda: mg.gemm(A, B, C, 1.0, 1.0, cfg=c, stream=stream),
                                   stream, batches=3)
                rec["tile_whole_tflops"] = round(2.0 * n ** 3 / float(np.mean(tw)) / 1e9, 3)
            out[name][str(n)] = rec
            log(f"  {name} N={n}: {ms:.3f} ms, {tf:.1f} TFLOP/s")
            del A, B, C
        torch.cuda.empty_cache()
    return out


def leg_batched(mg, torch, dev, plan_only=False):
    """The batched workload: FP64 and FP32 plans, each against per-problem launches
    and (FP64) the oracle.  plan_only: the plan executions alone (a profiling run
    with few dispatches)."""
    import synth
    log("bench: batched leg, 2048 uneven FP64 problems")
    cnt = 2048
    ms = synth.log_uniform_int(cnt, 4001, 16, 1024)
    ns = synth.log_uniform_int(cnt, 4002, 16, 1024)
    ks = synth.log_uniform_int(cnt, 4003, 16, 1024)
    # every operand is a view into one buffer (each starting on a 512-byte
    # boundary, as a separate allocation would): one fill instead of thousands;
    # beta = 0, so C's initial values are never read
    sizes = [int(s) for m, n, k in zip(ms, ns, ks) for s in (m * k, k * n, m * n)]
    offs = np.concatenate([[0], np.cumsum([(s + 63) // 64 * 64 for s in sizes])])
    g = torch.Generator(device=dev)
    g.manual_seed(4004)
    buf = torch.rand(int(offs[-1]), device=dev, dtype=torch.float64, generator=g) * 2 - 1
    views = [buf[int(offs[i]):int(offs[i]) + sizes[i]] for i in range(len(sizes))]
    As = [views[3 * i].view(int(m), int(k)) for i, (m, k) in enumerate(zip(ms, ks))]
    Bs = [views[3 * i + 1].view(int(k), int(n)) for i, (k, n) in enumerate(zip(ks, ns))]
    Cs = [views[3 * i + 2].view(int(m), int(n)) for i, (m, n) in enumerate(zip(ms, ns))]
    flops = float(sum(pm.gemm_flops(m, n, k) for m, n, k in zip(ms, ns, ks)))
    stream = torch.cuda.current_stream()
    plan = mg.BatchedPlan(As, Bs, Cs, 1.0, 0.0, stream=stream)
    tp = timed(plan.execute, stream, 10, warmup=2)
    log("bench: FP64 plan timed")
    info = plan.info()
    plan.destroy()
    tuned = None
    if not plan_only:
        tuned = tuned_plan(mg, As, Bs, Cs, mg.F64, stream, flops, PEAK_F64_TFLOPS)
        log(f"bench: FP64 plan tuned ({tuned['rule']})")
    if plan_only:
        tl = [float("nan")]
    else:
        tl = timed(lambda: mg.gemm_batched(As, Bs, Cs, 1.0, 0.0), stream, 3, warmup=1)
        log("bench: FP64 per-problem launches timed")
    nbytes = float(sum(8.0 * (m * k + k * n + m * n) for m, n, k in zip(ms, ns, ks)))
    gms = float(np.mean(tp))
    # the batch's time bound problem by problem: sum over problems of max(F / peak, B / BW)
    bound_s = float(sum(max(pm.gemm_flops(m, n, k) / (PEAK_F64_TFLOPS * 1e12),
                            8.0 * (m * k + k * n + m * n) / 8e12) for m, n, k in zip(ms, ns, ks)))
    out = {"problems": cnt, "flops": flops, "bytes": nbytes, "buckets": info["buckets"],
           "tiles": info["tiles"], "graph_ms": round(gms, 4),
           "graph_tflops": round(flops / gms / 1e9, 3),
           # max(sum F / peak, sum B / bandwidth) / t: the batch's roofline fraction
           "roofline_frac": round(max(flops / (PEAK_F64_TFLOPS * 1e12), nbytes / 8e12) / (gms * 1e-3), 4),
           "roofline_frac_per_problem": round(bound_s / (gms * 1e-3), 4),
           "per_problem_ms": None if plan_only else round(float(np.mean(tl)), 4),
           "per_problem_tflops": None if plan_only else round(flops / float(np.mean(tl)) / 1e9, 3),
           "speedup": None if plan_only else round(float(np.mean(tl)) / gms, 3),
           "tuned": tuned}
    if not plan_only:
        # the oracle on every problem of the batch, all host cores (the first 512
        # problems, scaled by FLOP to the whole batch)
        import oracle
        sub = 512
        t = time.perf_counter()
        for i in range(sub):
            oracle.gemm_f64(1.0, As[i].cpu().numpy(), Bs[i].cpu().numpy(), 0.0, None,
                            nthreads=oracle.num_procs())
        t_sub = time.perf_counter() - t
        f_sub = float(sum(2.0 * m * n * k for m, n, k in zip(ms[:sub], ns[:sub], ks[:sub])))
        out["oracle_batch_s_estimate"] = round(t_sub * flops / f_sub, 2)
    # FP32 variant of the same batch
    buf32 = buf.float()
    del As, Bs, Cs, views, buf
    views = [buf32[int(offs[i]):int(offs[i]) + sizes[i]] for i in range(len(sizes))]
    As32 = [views[3 * i].view(int(m), int(k)) for i, (m, k) in enumerate(zip(ms, ks))]
    Bs32 = [views[3 * i + 1].view(int(k), int(n)) for i, (k, n) in enumerate(zip(ks, ns))]
    Cs32 = [views[3 * i + 2].view(int(m), int(n)) for i, (m, n) in enumerate(zip(ms, ns))]
    plan = mg.BatchedPlan(As32, Bs32, Cs32, 1.0, 0.0, stream=stream)
    tp = timed(plan.execute, stream, 10, warmup=2)
    log("bench: FP32 plan timed")
    plan.destroy()
    tuned32 = None
    if not plan_only:
        tuned32 = tuned_plan(mg, As32, Bs32, Cs32, mg.F32, stream, flops, PEAK_F32_TFLOPS)
        log(f"bench: FP32 plan tuned ({tuned32['rule']})")
    if plan_only:
        tl = [float("nan")]
    else:
        tl = timed(lambda: mg.gemm_batched(As32, Bs32, Cs32, 1.0, 0.0), stream, 3, warmup=1)
        log("bench: FP32 per-problem launches timed")
    g32 = float(np.mean(tp))
    out["f32"] = {"graph_ms": round(g32, 4), "graph_tflops": round(flops / g32 / 1e9, 3),
                  "roofline_frac": round(max(flops / (PEAK_F32_TFLOPS * 1e12), nbytes / 2 / 8e12) /
                                         (g32 * 1e-3), 4),
                  "per_problem_ms": None if plan_only else round(float(np.mean(tl)), 4),
                  "speedup": None if plan_only else round(float(np.mean(tl)) / g32, 3),
                  "tuned": tuned32}
    return out


def tuned_plan(mg, As, Bs, Cs, dtype, stream, flops, peak_tflops):
    """The batch tuner's choice for this batch (every candidate rule's plan timed,
    5 runs each), re-timed on its own over 10 runs."""
    from paper_1706_10086_amd import tune
    cands = tune.tune_batch(As, Bs, Cs, 1.0, 0.0, dtype, reps=5, stream=stream)
    name, _, _, cfgs = cands[0]
    t, nb = tune.time_plan(As, Bs, Cs, 1.0, 0.0, dtype, cfgs, reps=10, stream=stream)
    ms = float(np.mean(t))
    return {"rule": name, "buckets": nb, "graph_ms": round(ms, 4),
            "graph_tflops": round(flops / ms / 1e9, 3),
            "mfma_frac": round(flops / (ms * 1e-3) / (peak_tflops * 1e12), 4),
            "candidates_ms": {c[0]: round(c[1], 4) for c in cands}}


def leg_memory(mg, torch, dev, sizes=(1024, 2048, 4096, 8192)):
    """Operands in device memory against operands in host memory (the paper's
    unified-against-device-memory comparison, Sec. 3): square FP64 GEMM,
    alpha = beta = 1, with (a) A, B, C resident in device memory, (b) A, B, C in
    pinned host memory copied in and C copied back around every call, (c) A, B, C
    in pinned, mapped host memory read and written in place by the kernel
    (coherent: uncached; non-coherent: the GPU may cache it)."""
    log("bench: memory leg, device vs explicit copy vs zero-copy host memory")
    stream = torch.cuda.current_stream()
    out = {"inputs": "uniform[-1,1) on the device, alpha = beta = 1, library's default tile choice"}
    last = {}    # mode -> (n, ms): a host-memory mode is skipped once its time,
    #              scaled by n^3 from the previous size, would pass 3 s per call
    for n in sizes:
        reps = 2 if n >= 8192 else 3
        g = torch.Generator(device=dev)
        g.manual_seed(5000 + n)
        tA, tB, tC = (torch.rand((n, n), device=dev, dtype=torch.float64, generator=g) * 2 - 1
                      for _ in range(3))
        hA, hB, hC = (t.cpu().pin_memory() for t in (tA, tB, tC))
        flops = pm.gemm_flops(n, n, n)
        row = {}
        t = timed(lambda: mg.gemm(tA, tB, tC, 1.0, 1.0, stream=stream), stream, reps)
        row["device_ms"] = round(float(np.mean(t)), 3)

        def explicit():
            tA.copy_(hA, non_blocking=True)
            tB.copy_(hB, non_blocking=True)
            tC.copy_(hC, non_blocking=True)
            mg.gemm(tA, tB, tC, 1.0, 1.0, stream=stream)
            hC.copy_(tC, non_blocking=True)
        t = timed(explicit, stream, reps)
        row["explicit_copy_ms"] = round(float(np.mean(t)), 3)
        t = timed(lambda: tA.copy_(hA, non_blocking=True), stream, reps)
        row["h2d_GBps"] = round(8.0 * n * n / (float(np.mean(t)) * 1e6), 1)
        for name, coh in (("zero_copy_coherent_ms", True), ("zero_copy_noncoherent_ms", False)):
            if name in last and last[name][1] * (n / last[name][0]) ** 3 > 3000.0:
                row[name] = None
                continue
            bufs = [mg.HostBuffer(8 * n * n, coh) for _ in range(3)]
            for b, h in zip(bufs, (hA, hB, hC)):
                b.array((n, n))[...] = h.numpy()
            a, b, c = (x.dev for x in bufs)
            t = timed(lambda: mg._check(mg.gemm_ex_raw(n, n, n, 1.0, a, n, b, n, 1.0, c, n, mg.F64,
                                                       None, stream.cuda_stream)), stream, reps)
            row[name] = round(float(np.mean(t)), 3)
            last[name] = (n, row[name])
            for x in bufs:
                x.free()
        for key in list(row):
            if key.endswith("_ms") and row[key] is not None:
                row[key[:-3] + "_tflops"] = round(flops / (row[key] * 1e9), 3)
        out[str(n)] = row
        log(f"bench: memory leg N={n}: {row}")
        del tA, tB, tC, hA, hB, hC
        torch.cuda.empty_cache()
    return out


def live_recheck(mg, pred, table, count=8):
    """Re-times held-out FP64 shapes now: TFLOP/s of the predicted configuration,
    and of the library's built-in choice (no configuration named), over the best of
    all registered configurations, measured in this run (each configuration once
    after one untimed run, a second time unless more than twice the best so far)."""
    import torch
    from paper_1706_10086_amd import learn, tune
    shapes = [s for s in tune.shape_set("heldout") if 2.0 * s[0] * s[1] * s[2] < 2e11][:count]
    choice = learn.predict(pred, [(mg.F64, *s) for s in shapes])
    fr, fb = [], []
    for (m, n, k), c in zip(shapes, choice):
        ops = tune.Operands(m, n, k, mg.F64)
        tf = {}
        best = None
        for cfg in mg.configs(mg.F64):
            t = tune.time_config(ops, mg.F64, cfg, warmup=1, reps=2,
                                 abandon_ms=None if best is None else 2.0 * best)
            best = min(t) if best is None else min(best, min(t))
            tf[cfg.as_tuple()] = tune.flops(m, n, k) / (min(t) * 1e9)
        t = tune.time_config(ops, mg.F64, None, warmup=1, reps=3)
        fr.append(tf[table[c][1]] / max(tf.values()))
        fb.append(tune.flops(m, n, k) / (min(t) * 1e9) / max(tf.values()))
        del ops
    torch.cuda.empty_cache()
    return learn.summarize(np.array(fr)), learn.summarize(np.array(fb))


def occupancy_gain(db, shapes, dtype):
    """The occupancy axis (waves per SIMD, the paper's hardware threads per core)
    on the held-out shapes of ``dtype``, from the database: per shape, the best
    occupancy-2 configuration over the best occupancy-1 configuration among the
    tiles compiled at both occupancies (geometric mean over shapes, and per tile
    family); and the exhaustive best with against without occupancy-2 points."""
    by = {}
    for r in db.records:
        if r["dtype"] == dtype:
            by.setdefault((r["m"], r["n"], r["k"]), {})[tuple(r["cfg"])] = r["tflops"]
    cfgs = {c for row in by.values() for c in row}
    fam1 = {c[:6] for c in cfgs if c[6] == 1}
    both = {f for f in fam1 if f + (2,) in cfgs}
    best_ratio, with_without, per_tile = [], [], {f: [] for f in both}
    for sh in shapes:
        row = by.get(tuple(sh))
        if not row:
            continue
        o1 = [row[f + (1,)] for f in both if f + (1,) in row]
        o2 = [row[f + (2,)] for f in both if f + (2,) in row]
        if o1 and o2:
            best_ratio.append(max(o2) / max(o1))
        without = [v for c, v in row.items() if c[6] != 2]
        if without:
            with_without.append(max(row.values()) / max(without))
        for f in both:
            if f + (1,) in row and f + (2,) in row:
                per_tile[f].append(row[f + (2,)] / row[f + (1,)])
    gm = lambda x: float(np.exp(np.mean(np.log(x)))) if len(x) else None  # noqa: E731
    tiles = {f: gm(v) for f, v in per_tile.items() if v}
    return {"tile_families_at_both": len(both), "shapes": len(best_ratio),
            "best_occ2_over_best_occ1": gm(best_ratio),
            "share_shapes_occ2_faster": float(np.mean(np.array(best_ratio) > 1.0)) if best_ratio else None,
            "exhaustive_with_over_without_occ2": gm(with_without),
            "per_tile_family_geomean_min": min(tiles.values()) if tiles else None,
            "per_tile_family_geomean_max": max(tiles.values()) if tiles else None,
            "tile_families_occ2_faster": sum(1 for v in tiles.values() if v > 1.0)}


def model_latency(mg, pred, shapes, tmpdir):
    """Inference latency of the learned model through the C ABI: a model file
    written from ``pred``, loaded with mgemm_model_load; mgemm_model_predict per
    shape on first sight (one forward pass on the GPU) and again (cached)."""
    path = os.path.join(tmpdir, "bench_model.txt")
    pred.save(path)
    mg.model_load(path)
    try:
        t = time.perf_counter()
        for (dt, m, n, k) in shapes:
            mg.model_predict(m, n, k, dt)
        first = (time.perf_counter() - t) / len(shapes)
        t = time.perf_counter()
        for (dt, m, n, k) in shapes:
            mg.model_predict(m, n, k, dt)
        cached = (time.perf_counter() - t) / len(shapes)
    finally:
        mg.model_load(None)
    return {"shapes": len(shapes), "first_call_us": round(1e6 * first, 1),
            "cached_call_us": round(1e6 * cached, 2)}


def leg_tuner(mg):
    from paper_1706_10086_amd import learn, tune
    path = os.path.join(ROOT, "paper_1706_10086_amd", "data", "tune_db.json.gz")
    if not os.path.exists(path):
        return {"status": "no tuner database"}
    log("bench: tuner leg, training the MLP on the tuner database")
    db = tune.load_compact(path)
    table = learn.config_table()
    dtr, dho = learn.datasets(db, table)
    if not dtr.shapes or not dho.shapes:
        return {"status": "tuner database does not match the configuration registry"}
    settings = learn.TRAIN_SETTINGS
    steps = settings["steps"] + settings.get("final_steps", 0)
    t0 = time.time()
    pred = learn.train(dtr, table, **settings)
    t_train = time.time() - t0
    t0 = time.time()
    choice = learn.predict(pred, dho.shapes)
    t_pred = time.time() - t0
    base = learn.single_best_baseline(dtr, table)
    mlp = learn.summarize(learn.achieved(dho, choice))
    single = learn.summarize(learn.achieved(dho, [base[s[0]] for s in dho.shapes]))
    top3 = learn.summarize(learn.top_k_fallback(dho, pred, 3))
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        lat = model_latency(mg, pred, dho.shapes[:50], td)
    occ = {name: occupancy_gain(db, tune.shape_set("heldout"), dt)
           for name, dt in (("f64", mg.F64), ("f32", mg.F32))}
    per = {}
    for name, dt in (("f64", mg.F64), ("f32", mg.F32)):
        rows = [i for i, s in enumerate(dho.shapes) if s[0] == dt]
        per[name] = learn.summarize(learn.achieved(dho, choice)[rows]) if rows else None
    log("bench: tuner leg, live re-timing of held-out shapes")
    live, builtin = live_recheck(mg, pred, table)
    return {"database": "paper_1706_10086_amd/data/tune_db.json.gz (MI355X sweep, m,n,k log-uniform "
                        "in [64,16384], FP64 and FP32, every registered configuration)",
            "configurations": {"f64": len(mg.configs(mg.F64)), "f32": len(mg.configs(mg.F32))},
            "train_rows": len(dtr.shapes), "heldout_rows": len(dho.shapes),
            "training": dict(settings, target_power=learn.TARGET_POWER,
                             sets=list(learn.TRAIN_SETS)),
            "train_s": round(t_train, 2), "adam_steps": steps,
            "ms_per_adam_step": round(1e3 * t_train / steps, 4),
            "predict_heldout_ms": round(1e3 * t_pred, 2), "model_predict_c_abi": lat,
            "mlp": mlp, "mlp_per_dtype": per, "single_best_config": single,
            "mlp_top3_measured": top3, "regret_geomean": round(1.0 - mlp["geomean"], 4),
            "gain_over_single": round(mlp["geomean"] / single["geomean"], 4),
            "occupancy_axis": occ,
            "live_recheck_f64": live, "builtin_choice_live_f64": builtin}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
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
    if args.leg:
        # (a profiling run of one leg: the split leg at N only)
        legs = {"split": lambda: leg_split(mg, torch, dev, n, with_small=False),
                "sweep": lambda: leg_sweep(mg, torch, dev),
                "parity": lambda: leg_parity(mg, torch, dev),
                "batched": lambda: leg_batched(mg, torch, dev),
                "batched_plan": lambda: leg_batched(mg, torch, dev, plan_only=True),
                "tuner": lambda: leg_tuner(mg),
                "memory": lambda: leg_memory(mg, torch, dev),
                "copy": lambda: leg_copy(torch, dev, args.copy_mib, args.copy_reps)}
        print(json.dumps({args.leg: legs[args.leg]()}), flush=True)
        return 0
    cfg = None
    if args.cfg:
        want = tuple(int(x) for x in args.cfg.split(","))
        cfg = next((c for c in mg.configs(mg.F64) if c.as_tuple() == want), None)
        if cfg is None:
            log(f"bench.py: {args.cfg} is not a registered FP64 configuration")
            return 2
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
        mg.gemm(tA, tB, tC, 1.0, 1.0, cfg=cfg, stream=stream)

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
    flops = pm.gemm_flops(n, n, n)
    tflops = flops / (ms * 1e-3) / 1e12
    kern_ms = float(np.mean(per))
    best_ms = float(np.min(per))
    median_ms = float(np.median(per))

    # accuracy of this run against the oracle on sampled rows: C_s = A B + C_{s-1}
    import oracle
    log("bench: accuracy check on sampled rows")
    rows = np.arange(0, n, max(1, n // 16))
    steps_done = args.warmup + args.steps
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
    del tA, tB, tC

    if cfg is not None:
        cfg_used, splits, whole_rows = cfg.as_dict(), 1, n
    else:
        c, splits, whole_rows = mg.choice(n, n, n, mg.F64, rows=True)
        cfg_used = c.as_dict()
    if splits == 1:
        launches = kernel_name(cfg_used) + " (one launch per step)"
    elif whole_rows == 0:
        launches = (f"split-k of {kernel_name(cfg_used)}, k in {splits} ranges, and the sum of "
                    "the planes (two launches per step; kernel_avg_ms is their total)")
    else:
        launches = (f"{kernel_name(cfg_used)} on the first {whole_rows} rows, its split-k on "
                    f"the other {n - whole_rows} rows with k in {splits} ranges, and the sum of "
                    "the planes (three launches per step; kernel_avg_ms is their total)")
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
                               f"alpha=1, beta=1 ("
                               f"{'explicit' if cfg is not None else 'library' + chr(39) + 's default'}"
                               f" tile configuration)",
                   "n": n, "alpha": 1.0, "beta": 1.0, "tile_config": cfg_used,
                   "k_ranges": splits, "whole_rows": whole_rows,
                   "parallelism": "single GPU"},
        "pct_peak": round(100.0 * tflops / PEAK_F64_TFLOPS, 2),
        "best_step_tflops": round(flops / (best_ms * 1e-3) / 1e12, 3),
        "median_ms_per_step": round(median_ms, 4),
        "median_step_tflops": round(flops / (median_ms * 1e-3) / 1e12, 3),
        "wall_s": round(wall, 3),
        "sampled_rel_err_vs_oracle": err,
        "roofline": {"bound": "mfma", "achieved": round(flops / (kern_ms * 1e-3) / 1e12, 3),
                     "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(flops / (kern_ms * 1e-3) / 1e12 / PEAK_F64_TFLOPS, 4),
                     # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE runs in
                     # profiles/gemm_pipe_f64_N8192_traffic.md (copy-calibrated)
                     "traffic": TRAFFIC_F64_N8192 if n == 8192 and cfg is None else None,
                     "traffic_unit": "bytes per launch",
                     "kernel": launches,
                     "kernel_avg_ms": round(kern_ms, 4),
                     "work_per_launch": f"2*N^3 = {flops:.4g} FLOP",
                     # Eq. 6 for the kernel's 256 x 128 tiles: the bytes with no cache
                     # reuse, against the algorithmic minimum (A, B, C read, C written)
                     "traffic_model": {"tiles_no_reuse": pm.tile_traffic_bytes(
                                           n, n, n, cfg_used["bm"], cfg_used["bn"], 8),
                                       "algorithmic": 4.0 * 8 * n * n}},
        "cpu_baseline": cpu,
    }
    if not args.no_extras:
        for name, fn in (("parity", lambda: leg_parity(mg, torch, dev)),
                         ("sweep", lambda: leg_sweep(mg, torch, dev)),
                         ("split", lambda: leg_split(mg, torch, dev)),
                         ("batched", lambda: leg_batched(mg, torch, dev)),
                         ("memory", lambda: leg_memory(mg, torch, dev)),
                         ("tuner", lambda: leg_tuner(mg))):
            try:
                out[name] = fn()
            except Exception as e:  # an extra leg must not hide the headline line
                out[name] = {"status": f"failed: {type(e).__name__}: {e}"}
                log(f"bench: {name} leg failed: {e}")
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
