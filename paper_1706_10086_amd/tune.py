"""Autotuner: time every registered tile configuration of a dtype on a set of
shapes, keep the results in an append-only JSONL database, and pick the
exhaustive best.

The procedure follows the paper's parameter tuning (Sec. 2.3 "Multidimensional
parameter tuning" and Sec. 3, Tab. 4): a grid of tile parameters is searched,
each point measured several times and the best kept, at a main size and checked
at a control size.  Here the grid searched is the library's configuration
registry (tile M/N/K, waves per work-group, elements per thread, double
buffering, occupancy), the compiled subset of the valid points of the raw grid
defined below (``raw_grid``, ``grid_violations``); the measurement is the device time of one gemm_ex call from HIP
events (warm-up, then ``reps`` timed runs; median and best kept), and a
configuration whose first timed run is more than ``abandon`` times slower than
the best so far for that shape is not measured further.

Database records (one JSON object per line) are keyed by
(device, build, dtype, m, n, k, cfg); a sweep skips keys already present, so an
interrupted sweep resumes where it stopped.  Lines that do not parse are skipped
and counted.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from dataclasses import dataclass

import numpy as np

from . import F32, F64, SPLIT_BF16, LIB_PATH, Cfg, configs, gemm


def build_id() -> str:
    h = hashlib.sha1()
    with open(LIB_PATH, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:12]


def device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def key_of(rec: dict) -> tuple:
    return (rec["device"], rec["build"], rec["dtype"], rec["m"], rec["n"], rec["k"],
            tuple(rec["cfg"]))


@dataclass
class DB:
    path: str
    records: list
    bad_lines: int = 0

    @classmethod
    def load(cls, path: str) -> "DB":
        recs, bad = [], 0
        if os.path.exists(path):
            with open(path) as f:
                for line in f:
                    line = line.strip()
                    if not line:
                        continue
                    try:
                        r = json.loads(line)
                        key_of(r)
                        recs.append(r)
                    except (ValueError, KeyError, TypeError):
                        bad += 1
        return cls(path, recs, bad)

    def keys(self) -> set:
        return {key_of(r) for r in self.records}

    def append(self, rec: dict) -> None:
        self.records.append(rec)
        with open(self.path, "a") as f:
            f.write(json.dumps(rec) + "\n")
            f.flush()

    def for_shape(self, dtype: int, m: int, n: int, k: int) -> list:
        return [r for r in self.records if r["dtype"] == dtype and (r["m"], r["n"], r["k"]) == (m, n, k)]


def flops(m, n, k) -> float:
    return 2.0 * m * n * k


# The raw tuning grid (the paper's powers-of-two search of Sec. 2.3 and Tab. 4,
# widened to the GPU's tile parameters): tile M/N/K, waves per work-group,
# elements per thread, one or two LDS stages.  Every point is a kernel of its own
# (tile shapes are template parameters), so the library compiles a subset: the
# registry.  ``grid_violations`` is the filter that decides which points can be
# compiled at all; the kernels' static assertions enforce the same rules.
GRID_TILES = (32, 64, 128, 256)
GRID_WAVES = (1, 2, 4, 8)
GRID_EPT = (4, 8, 16)
GRID_DBUF = (0, 1)
# the registry also uses k-steps of 16 and runs of 2 elements (one 16-byte FP64
# load): a 256 x 128 FP64 tile with three stages fits the LDS only at bk = 16
EXT_BK = (16,)
EXT_EPT = (2,)
LDS_BYTES = 160 * 1024          # per compute unit
ACC_VGPRS = 256                 # accumulator registers one lane may hold
MFMA_TILE = 16                  # 16 x 16 output block of the FP64 and FP32 instructions


def raw_grid():
    """All 4^3 * 4 * 3 * 2 = 1536 points (bm, bn, bk, waves, ept, dbuf)."""
    return [(bm, bn, bk, w, e, d) for bm in GRID_TILES for bn in GRID_TILES for bk in GRID_TILES
            for w in GRID_WAVES for e in GRID_EPT for d in GRID_DBUF]


def grid_violations(dtype: int, bm: int, bn: int, bk: int, waves: int, ept: int,
                    dbuf: int) -> list:
    """Names of the rules a configuration breaks (empty: it can be compiled).

    * ``lds``:   the A and B stages, (bm bk + bk bn) S bytes each, fit in the LDS
                 (``dbuf`` 0, 1, 2: one, two, three stages);
    * ``acc``:   each lane's share of the bm x bn accumulators fits in 256 VGPRs;
    * ``mfma``:  the waves split the tile into a WGM x WGN grid of wave tiles that
                 are whole 16 x 16 instruction blocks;
    * ``loads``: both slabs split into runs of ``ept`` consecutive elements, at
                 least one per thread, each within one row of the slab.
    """
    S = 4 if dtype == F32 else 8
    out = []
    if (bm * bk + bk * bn) * S * (1 + dbuf) > LDS_BYTES:
        out.append("lds")
    if bm * bn * (S // 4) > ACC_VGPRS * 64 * waves:
        out.append("acc")
    if not any(waves % wgm == 0 and bm % (wgm * MFMA_TILE) == 0
               and bn % ((waves // wgm) * MFMA_TILE) == 0 for wgm in GRID_WAVES if wgm <= waves):
        out.append("mfma")
    per_pass = 64 * waves * ept
    if (bm * bk) % per_pass or (bk * bn) % per_pass or bm * bk < per_pass \
            or bk * bn < per_pass or ept > bk or ept > bn or ept % 2:
        out.append("loads")
    return out


def extended_grid():
    """``raw_grid`` with k-steps of 16 and runs of 2 elements added (2560 points)."""
    return [(bm, bn, bk, w, e, d) for bm in GRID_TILES for bn in GRID_TILES
            for bk in EXT_BK + GRID_TILES for w in GRID_WAVES for e in EXT_EPT + GRID_EPT
            for d in GRID_DBUF]


def valid_grid(dtype: int, extended: bool = False):
    """The points of ``raw_grid`` (or ``extended_grid``) that break no rule."""
    return [p for p in (extended_grid() if extended else raw_grid())
            if not grid_violations(dtype, *p)]


class Operands:
    """Device buffers for one shape; values are uniform[-1,1) drawn on the device
    (timing of the FP64/FP32 kernels does not depend on the values)."""

    def __init__(self, m, n, k, dtype):
        import torch
        tdt = torch.float32 if dtype == F32 else torch.float64
        g = torch.Generator(device="cuda")
        g.manual_seed(m * 1_000_003 + n * 1009 + k)
        self.A = torch.rand((m, k), device="cuda", dtype=tdt, generator=g) * 2 - 1
        self.B = torch.rand((k, n), device="cuda", dtype=tdt, generator=g) * 2 - 1
        self.C = torch.zeros((m, n), device="cuda", dtype=tdt)


def time_config(ops: Operands, dtype: int, cfg, warmup: int = 1, reps: int = 3,
                abandon_ms: float | None = None) -> list[float]:
    """Device times (ms) of ``reps`` gemm calls after ``warmup`` untimed ones.
    Stops after the first timed run if it exceeds ``abandon_ms``."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        gemm(ops.A, ops.B, ops.C, 1.0, 0.0, dtype=dtype, cfg=cfg, stream=stream)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        gemm(ops.A, ops.B, ops.C, 1.0, 0.0, dtype=dtype, cfg=cfg, stream=stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
        if abandon_ms is not None and times[-1] > abandon_ms:
            break
    return times


def sweep(shapes, dtype: int, db: DB, cfgs=None, reps: int = 3, abandon: float = 2.0,
          log=None) -> int:
    """Times every configuration on every shape not yet in ``db``; returns the
    number of new records."""
    dev, bid = device_name(), build_id()
    cfgs = list(cfgs if cfgs is not None else configs(dtype))
    done = db.keys()
    new = 0
    for (m, n, k) in shapes:
        todo = [c for c in cfgs if (dev, bid, dtype, m, n, k, c.as_tuple()) not in done]
        if not todo:
            continue
        ops = Operands(m, n, k, dtype)
        best = min((r["best_ms"] for r in db.for_shape(dtype, m, n, k)
                    if r["device"] == dev and r["build"] == bid), default=None)
        for c in todo:
            t = time_config(ops, dtype, c, reps=reps,
                            abandon_ms=None if best is None else abandon * best)
            rec = {"device": dev, "build": bid, "dtype": dtype, "m": m, "n": n, "k": k,
                   "cfg": list(c.as_tuple()), "times_ms": [round(x, 5) for x in t],
                   "best_ms": min(t), "median_ms": float(np.median(t)),
                   "tflops": flops(m, n, k) / (float(np.median(t)) * 1e-3) / 1e12,
                   "abandoned": len(t) < reps, "ts": time.time()}
            db.append(rec)
            new += 1
            best = rec["best_ms"] if best is None else min(best, rec["best_ms"])
            if log:
                log(f"  {dtype} {m}x{n}x{k} {c} median {rec['median_ms']:.4f} ms "
                    f"{rec['tflops']:.2f} TF")
        del ops
    return new


def exhaustive_best(db: DB, dtype: int, m: int, n: int, k: int):
    """(cfg tuple, TFLOP/s) of the configuration with the highest median
    TFLOP/s among the measured ones (abandoned runs included: their one time is
    an upper bound of their speed)."""
    rs = db.for_shape(dtype, m, n, k)
    if not rs:
        return None, 0.0
    r = max(rs, key=lambda r: r["tflops"])
    return tuple(r["cfg"]), r["tflops"]


def regret(db: DB, dtype: int, m: int, n: int, k: int, cfg) -> float:
    """1 - TFLOP/s(cfg) / TFLOP/s(exhaustive best) on one shape."""
    rs = db.for_shape(dtype, m, n, k)
    best = max(r["tflops"] for r in rs)
    mine = [r["tflops"] for r in rs if tuple(r["cfg"]) == tuple(cfg)]
    if not mine:
        raise KeyError("configuration not measured on this shape")
    return 1.0 - max(mine) / best


# ---------------------------------------------------------------------------
# Shape sets of the learned-tuner workload and the sweep driver.
# ---------------------------------------------------------------------------
TRAIN_SEEDS = (5001, 5002, 5003)
HELDOUT_SEEDS = (5011, 5012, 5013)
ALIGNED_SEEDS = (5021, 5022, 5023)


def shape_set(which: str, count: int | None = None, lo: int = 64, hi: int = 16384):
    """'train' (3000 shapes), 'heldout' (500 shapes, none also in 'train') or
    'aligned' (800 shapes rounded up to multiples of 4, so every row is a whole
    16-byte load in FP64 and FP32; none in the other two sets): m, n, k each
    log-uniform in [lo, hi] from their own seeded streams."""
    import synth
    if which == "train":
        seeds, cnt = TRAIN_SEEDS, 3000 if count is None else count
    elif which == "heldout":
        seeds, cnt = HELDOUT_SEEDS, 500 if count is None else count
    elif which == "aligned":
        seeds, cnt = ALIGNED_SEEDS, 800 if count is None else count
    else:
        raise ValueError(which)
    ms, ns, ks = (synth.log_uniform_int(cnt + 64, s, lo, hi) for s in seeds)
    shapes = [(int(a), int(b), int(c)) for a, b, c in zip(ms, ns, ks)]
    if which == "aligned":
        shapes = [tuple(-(-x // 4) * 4 for x in sh) for sh in shapes]
    if which in ("heldout", "aligned"):
        tr = set(shape_set("train", lo=lo, hi=hi))
        if which == "aligned":
            tr |= set(shape_set("heldout", lo=lo, hi=hi))
        shapes = [s for s in shapes if s not in tr]
    out, seen = [], set()
    for s in shapes:
        if s not in seen:
            seen.add(s)
            out.append(s)
    return out[:cnt]


class Arena:
    """One device allocation per operand, sized for the largest shape of a sweep
    and filled once with uniform[-1,1) values; shapes take contiguous views."""

    def __init__(self, shapes, dtype):
        import torch
        tdt = torch.float32 if dtype == F32 else torch.float64
        ma = max(m * k for m, n, k in shapes)
        mb = max(k * n for m, n, k in shapes)
        mc = max(m * n for m, n, k in shapes)
        g = torch.Generator(device="cuda")
        g.manual_seed(12345)
        self.a = torch.rand(ma, device="cuda", dtype=tdt, generator=g) * 2 - 1
        self.b = torch.rand(mb, device="cuda", dtype=tdt, generator=g) * 2 - 1
        self.c = torch.zeros(mc, device="cuda", dtype=tdt)

    def operands(self, m, n, k):
        o = Operands.__new__(Operands)
        o.A = self.a[:m * k].view(m, k)
        o.B = self.b[:k * n].view(k, n)
        o.C = self.c[:m * n].view(m, n)
        return o


def sweep_set(shapes, dtype, db: DB, reps=2, abandon=2.0, log=print, every=25):
    """Resumable sweep of every registered configuration over ``shapes``."""
    dev, bid = device_name(), build_id()
    cfgs = list(configs(dtype))
    done = db.keys()
    todo = [s for s in shapes
            if any((dev, bid, dtype, s[0], s[1], s[2], c.as_tuple()) not in done for c in cfgs)]
    if not todo:
        log(f"sweep dtype={dtype}: nothing to do ({len(shapes)} shapes already measured)")
        return 0
    arena = Arena(todo, dtype)
    t0 = time.time()
    new = 0
    for i, (m, n, k) in enumerate(todo):
        ops = arena.operands(m, n, k)
        best = None
        for c in cfgs:
            key = (dev, bid, dtype, m, n, k, c.as_tuple())
            if key in done:
                continue
            t = time_config(ops, dtype, c, reps=reps,
                            abandon_ms=None if best is None else abandon * best)
            rec = {"device": dev, "build": bid, "dtype": dtype, "m": m, "n": n, "k": k,
                   "cfg": list(c.as_tuple()), "times_ms": [round(x, 5) for x in t],
                   "best_ms": min(t), "median_ms": float(np.median(t)),
                   "tflops": flops(m, n, k) / (float(np.median(t)) * 1e-3) / 1e12,
                   "abandoned": len(t) < reps, "ts": time.time()}
            db.append(rec)
            new += 1
            best = rec["best_ms"] if best is None else min(best, rec["best_ms"])
        if (i + 1) % every == 0 or i + 1 == len(todo):
            log(f"sweep dtype={dtype}: {i + 1}/{len(todo)} shapes, {new} records, "
                f"{time.time() - t0:.0f} s")
    return new


# ---------------------------------------------------------------------------
# Batched plans: which tile configuration each problem of a batch runs with.
# The problems of a plan share the GPU, so a choice is scored by timing the
# whole captured plan, not problem by problem.
# ---------------------------------------------------------------------------
def batch_rules(dtype: int) -> dict:
    """Candidate rules, each mapping a problem (m, n, k) to a configuration tuple:
    one registered configuration for every problem (three-stage entries are left
    out: in a plan they run their two-stage fallback, registered on its own), and
    mixtures of the 64 x 64 four-wave tile with the smallest tile for thin
    problems (min(m, n) <= T) or a 128 x 128 tile for large ones (min(m, n) >= T)."""
    cs = [c.as_tuple() for c in configs(dtype) if c.double_buffer < 2]
    rules = {f"all {c}": (lambda m, n, k, c=c: c) for c in cs}
    mid = next((c for c in cs if c[:4] == (64, 64, 16, 4)), None)
    small = min(cs, key=lambda c: (c[0] * c[1], c[2]))
    big = next((c for c in cs if c[:4] == (128, 128, 16, 4) and c[6] == 0), None)
    if mid is not None:
        for T in (32, 48, 64):
            rules[f"min(m,n) <= {T}: {small}, else {mid}"] = \
                (lambda m, n, k, T=T: small if min(m, n) <= T else mid)
        if big is not None:
            for T in (256, 512):
                rules[f"min(m,n) >= {T}: {big}, else {mid}"] = \
                    (lambda m, n, k, T=T: big if min(m, n) >= T else mid)
    return rules


def time_plan(As, Bs, Cs, alphas, betas, dtype, cfgs, reps=5, warmup=2, stream=None):
    """Device times (ms) of ``reps`` executions of one captured plan, and its
    bucket count."""
    import torch
    from . import BatchedPlan
    stream = stream or torch.cuda.current_stream()
    plan = BatchedPlan(As, Bs, Cs, alphas, betas, dtype=dtype, cfgs=cfgs, stream=stream)
    try:
        for _ in range(warmup):
            plan.execute()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for i in range(reps):
            plan.execute()
            ev[i + 1].record(stream)
        ev[-1].synchronize()
        return [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)], plan.info()["buckets"]
    finally:
        plan.destroy()


def tune_batch(As, Bs, Cs, alphas=1.0, betas=0.0, dtype=F64, rules=None, reps=5, stream=None):
    """Times the plan of every candidate rule (``batch_rules``) on this batch;
    returns [(name, median ms, buckets, per-problem configurations)], fastest first."""
    rules = rules or batch_rules(dtype)
    shapes = [(A.shape[0], B.shape[1], A.shape[1]) for A, B in zip(As, Bs)]
    out = []
    for name, rule in rules.items():
        cfgs = [rule(m, n, k) for m, n, k in shapes]
        t, nb = time_plan(As, Bs, Cs, alphas, betas, dtype, cfgs, reps=reps, stream=stream)
        out.append((name, float(np.median(t)), nb, cfgs))
    out.sort(key=lambda r: r[1])
    return out


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="autotuner sweep (resumable JSONL database)")
    ap.add_argument("--set", choices=["train", "heldout", "aligned"], required=True)
    ap.add_argument("--dtype", choices=["f64", "f32"], required=True)
    ap.add_argument("--db", required=True)
    ap.add_argument("--count", type=int, default=None)
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args(argv)
    dt = F64 if a.dtype == "f64" else F32
    db = DB.load(a.db)
    if db.bad_lines:
        print(f"tune: skipped {db.bad_lines} unreadable database lines", flush=True)
    shapes = shape_set(a.set, a.count)
    n = sweep_set(shapes, dt, db, reps=a.reps, log=lambda s: print(s, flush=True))
    print(f"tune: {n} new records in {a.db}", flush=True)


if __name__ == "__main__":
    main()


# ---------------------------------------------------------------------------
# Compact, read-only form of a database (shipped with the package).
# ---------------------------------------------------------------------------
def save_compact(db: DB, path: str) -> None:
    """gzip'd JSON: one row per (dtype, m, n, k) with the TFLOP/s of every
    measured configuration (the best of duplicate measurements)."""
    import gzip
    cfgs, rows = {}, {}
    for r in db.records:
        dt = r["dtype"]
        c = tuple(r["cfg"])
        lst = cfgs.setdefault(dt, [])
        if c not in lst:
            lst.append(c)
        key = (dt, r["m"], r["n"], r["k"])
        row = rows.setdefault(key, {})
        row[c] = max(row.get(c, 0.0), r["tflops"])
    devices = sorted({r["device"] for r in db.records})
    out = {"devices": devices, "configs": {str(dt): [list(c) for c in cs] for dt, cs in cfgs.items()},
           "rows": [[dt, m, n, k, [round(row.get(c, -1.0), 4) for c in cfgs[dt]]]
                    for (dt, m, n, k), row in sorted(rows.items())]}
    with gzip.open(path, "wt") as f:
        json.dump(out, f, separators=(",", ":"))


def load_compact(path: str) -> DB:
    """A DB (records without timings) from save_compact's file."""
    import gzip
    with gzip.open(path, "rt") as f:
        d = json.load(f)
    dev = d["devices"][0] if d["devices"] else "unknown"
    recs = []
    for dt, m, n, k, tf in d["rows"]:
        for c, v in zip(d["configs"][str(dt)], tf):
            if v < 0:
                continue
            recs.append({"device": dev, "build": "compact", "dtype": dt, "m": m, "n": n, "k": k,
                         "cfg": list(c), "tflops": v, "best_ms": flops(m, n, k) / (v * 1e9),
                         "median_ms": flops(m, n, k) / (v * 1e9)})
    return DB(path, recs, 0)
