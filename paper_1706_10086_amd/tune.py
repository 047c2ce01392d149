"""Autotuner: time every registered tile configuration of a dtype on a set of
shapes, keep the results in an append-only JSONL database, and pick the
exhaustive best.

The procedure follows the paper's parameter tuning (Sec. 2.3 "Multidimensional
parameter tuning" and Sec. 3, Tab. 4): a grid of tile parameters is searched and
each point measured, the best kept.  Here the grid searched is the library's
configuration registry (tile M/N/K, waves per work-group, elements per thread,
LDS stages, occupancy): the hand-registered kernels and the compiled subset of
the valid points of the raw grid defined below (``raw_grid``,
``grid_violations``).  The measurement is the device time of one gemm_ex call
from HIP events on the stream it runs on: one timed run, ``reps`` in all unless
the first is more than ``abandon`` times slower than the shape's best so far
(then its one time stands, an upper bound of its speed).  Every kernel is run
once before the sweep, so no timed run loads code.

Database lines are JSON objects of two kinds: a shape record (one line per
device, dtype and shape: every configuration measured, with its times) written
by ``sweep``, and the older per-configuration record; ``DB.load`` reads both as
per-configuration records.  A sweep skips the (device, dtype, shape) triples
already present, so an interrupted sweep resumes at the shape it stopped in.
Lines that do not parse are skipped and counted.
"""
from __future__ import annotations

import hashlib
import json
import math
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


def flops(m, n, k) -> float:
    return 2.0 * m * n * k


def expand_shape_record(r: dict) -> list:
    """The per-configuration records of one shape record."""
    out = []
    for c, t in zip(r["cfgs"], r["ms"]):
        med = float(np.median(t))
        out.append({"device": r["device"], "build": r["build"], "dtype": r["dtype"],
                    "m": r["m"], "n": r["n"], "k": r["k"], "cfg": list(c), "times_ms": t,
                    "best_ms": min(t), "median_ms": med,
                    "tflops": flops(r["m"], r["n"], r["k"]) / (med * 1e-3) / 1e12,
                    "abandoned": len(t) < r.get("reps", len(t)),
                    "refined": bool(r.get("refine", False))})
    return out


def prefer_refined(records: list) -> list:
    """Drops the sweep's measurement of a (device, dtype, shape, configuration)
    that a refinement pass measured again (``refine``): the refined median of
    more runs replaces it."""
    ref = {(r["device"], r["dtype"], r["m"], r["n"], r["k"], tuple(r["cfg"]))
           for r in records if r.get("refined")}
    if not ref:
        return records
    return [r for r in records if r.get("refined") or
            (r["device"], r["dtype"], r["m"], r["n"], r["k"], tuple(r["cfg"])) not in ref]


@dataclass
class DB:
    path: str
    records: list
    bad_lines: int = 0

    @classmethod
    def load(cls, path: str, raw: bool = False) -> "DB":
        """The database at ``path`` (empty if absent); unreadable lines are
        counted, not fatal.  Refined measurements replace the sweep's unless
        ``raw`` (every record as written)."""
        recs, bad = [], 0
        if os.path.exists(path):
            with open(path) as f:
                for line in f:
                    line = line.strip()
                    if not line:
                        continue
                    try:
                        r = json.loads(line)
                        if "cfgs" in r:
                            if len(r["cfgs"]) != len(r["ms"]) or not all(r["ms"]):
                                raise ValueError("shape record")
                            rs = expand_shape_record(r)
                        else:
                            rs = [r]
                        for x in rs:
                            key_of(x)
                        recs.extend(rs)
                    except (ValueError, KeyError, TypeError):
                        bad += 1
        return cls(path, recs if raw else prefer_refined(recs), bad)

    def keys(self) -> set:
        return {key_of(r) for r in self.records}

    def shapes_done(self, device: str) -> set:
        """(dtype, m, n, k) measured on ``device`` by a sweep."""
        return {(r["dtype"], r["m"], r["n"], r["k"]) for r in self.records
                if r["device"] == device and not r.get("refined")}

    def shapes_refined(self, device: str) -> set:
        """(dtype, m, n, k) measured on ``device`` by a refinement pass."""
        return {(r["dtype"], r["m"], r["n"], r["k"]) for r in self.records
                if r["device"] == device and r.get("refined")}

    def append(self, rec: dict) -> None:
        """Appends one record (a shape record is kept expanded in memory)."""
        self.records.extend(expand_shape_record(rec) if "cfgs" in rec else [rec])
        if rec.get("refine"):
            self.records = prefer_refined(self.records)
        self.write_line(rec)

    def write_line(self, rec: dict) -> None:
        """Appends one record to the file only (``load`` reads it back)."""
        with open(self.path, "a") as f:
            f.write(json.dumps(rec, separators=(",", ":")) + "\n")
            f.flush()

    def for_shape(self, dtype: int, m: int, n: int, k: int) -> list:
        return [r for r in self.records if r["dtype"] == dtype and (r["m"], r["n"], r["k"]) == (m, n, k)]


# The raw tuning grid (the paper's powers-of-two search of Sec. 2.3 and Tab. 4,
# widened to the GPU's tile parameters): tile M/N/K, waves per work-group,
# elements per thread, one or two LDS stages, and occupancy -- waves per SIMD,
# the GPU counterpart of the paper's hardware threads per core (Sec. 3, Tab. 4,
# Fig. 4).  Every point is a kernel of its own (tile shapes are template
# parameters), so the library compiles a subset: the registry.
# ``grid_violations`` decides which points can run as specified; it models the
# kernels' real LDS layout and register use.
GRID_TILES = (32, 64, 128, 256)
GRID_WAVES = (1, 2, 4, 8)
GRID_EPT = (4, 8, 16)
GRID_DBUF = (0, 1)
GRID_OCC = (1, 2)
# the hand-registered kernels also use k-steps of 16 and runs of 2 elements (one
# 16-byte FP64 load): a 256 x 128 FP64 tile with three stages fits the LDS only
# at bk = 16
EXT_BK = (16,)
EXT_EPT = (2,)
LDS_BYTES = 160 * 1024          # per compute unit
SIMDS = 4                       # per compute unit
LANE_REGS = 512                 # 32-bit registers per lane of one SIMD
ACC_VGPRS = 256                 # accumulator registers one lane may hold
MFMA_TILE = 16                  # 16 x 16 output block of the FP64 and FP32 instructions
BASE_REGS = 24                  # addresses, loop counters and the like
# Headroom the compiler needs (hipcc for gfx950, checked against its register and
# scratch report for every grid kernel): tiles whose accumulators fill all 256
# accumulator registers, or whose estimate at two waves per SIMD passes 240, spill.
ACC_HEADROOM = 8
OCC2_HEADROOM = 16
HOIST_GROUPS = 2                # 8-deep k groups whose fragments are live at once


def wave_layout(bm: int, bn: int, waves: int):
    """(WGM, WGN): the waves' grid over the tile -- whole 16 x 16 instruction
    blocks per wave, the wave tile closest to square (fewer rows of waves on a
    tie) -- or None if there is none."""
    best = None
    for wgm in GRID_WAVES:
        if wgm > waves or waves % wgm:
            continue
        wgn = waves // wgm
        if bm % (wgm * MFMA_TILE) or bn % (wgn * MFMA_TILE):
            continue
        key = (abs(math.log2((bm // wgm) / (bn // wgn))), wgm)
        if best is None or key < best[0]:
            best = (key, (wgm, wgn))
    return None if best is None else best[1]


def lds_bytes(dtype: int, bm: int, bn: int, bk: int, dbuf: int) -> int:
    """LDS one work-group needs: the two-stage kernel's padded A and B tiles (A
    rows bk + 2, B rows bn + 8 FP64 / + 16 FP32 elements) per stage (dbuf 0, 1:
    one, two stages); the three-stage kernel's 16-byte units (A rows one unit
    longer, B rows 4 FP64 / 2 FP32 units longer) times three (dbuf 2)."""
    S = 4 if dtype == F32 else 8
    if dbuf == 2:
        au = bk * S // 16 + 1
        bu = bn * S // 16 + (4 if S == 8 else 2)
        return 3 * 16 * (bm * au + bk * bu)
    return (bm * (bk + 2) + bk * (bn + (8 if S == 8 else 16))) * S * (1 + dbuf)


def reg_estimate(dtype: int, bm: int, bn: int, bk: int, waves: int, ept: int, dbuf: int):
    """(accumulator registers, other registers) per lane: the C fragments; the
    staged loads (two-stage kernels: the next k-step's tile in registers), the
    operand fragments of HOIST_GROUPS k groups (the compiler reads the next group
    from LDS during the current one), run coordinates and BASE_REGS.  None
    without a wave layout."""
    lay = wave_layout(bm, bn, waves)
    if lay is None:
        return None
    s4 = (4 if dtype == F32 else 8) // 4
    nt = 64 * waves
    fm, fn = bm // lay[0] // MFMA_TILE, bn // lay[1] // MFMA_TILE
    acc = bm * bn // nt * s4
    if dbuf == 2:      # all fragments of a k-step held, one load offset per instruction
        loads = -(-lds_bytes(dtype, bm, bn, bk, 2) // (3 * 16 * nt))
        return acc, (bk // 8) * (2 * fm + 2 * fn) * s4 + loads + BASE_REGS
    stage = (bm * bk + bk * bn) // nt * s4
    runs = 2 * ((bm * bk) // (ept * nt) + (bk * bn) // (ept * nt))
    frag = (2 * fm + 2 * fn) * s4 * min(bk // 8, HOIST_GROUPS)
    return acc, stage + frag + runs + BASE_REGS


def grid_violations(dtype: int, bm: int, bn: int, bk: int, waves: int, ept: int,
                    dbuf: int, occ: int = 0) -> list:
    """Names of the rules a configuration breaks (empty: it runs as specified).

    * ``mfma``:  the waves split the tile into whole 16 x 16 instruction blocks
                 (``wave_layout``);
    * ``loads``: both slabs split into runs of ``ept`` consecutive elements, at
                 least one per thread, each within one row of the slab;
    * ``occ``:   ``occ`` waves per SIMD leave room for at least one work-group
                 (waves <= 4 occ);
    * ``lds``:   the LDS of the g work-groups that run ``occ`` waves per SIMD
                 (g = max(1, 4 occ / waves); one for occ 0) fits in 160 KiB;
    * ``acc``:   the accumulators fit the 256 accumulator registers of a lane
                 (with ACC_HEADROOM to spare);
    * ``regs``:  the registers fit 512 / occ per lane (occ 0 or 1: 256 besides
                 the accumulators; occ 2: 256 in all, OCC2_HEADROOM to spare).
    """
    out = []
    lay = wave_layout(bm, bn, waves)
    if lay is None:
        out.append("mfma")
    per_pass = 64 * waves * ept
    if (bm * bk) % per_pass or (bk * bn) % per_pass or bm * bk < per_pass \
            or bk * bn < per_pass or ept > bk or ept > bn or ept % 2:
        out.append("loads")
    groups = 1
    if occ > 0:
        groups = SIMDS * occ // waves
        if groups < 1:
            out.append("occ")
            groups = 1
    if lds_bytes(dtype, bm, bn, bk, dbuf) * groups > LDS_BYTES:
        out.append("lds")
    if lay is not None:
        acc, other = reg_estimate(dtype, bm, bn, bk, waves, ept, dbuf)
        if acc > ACC_VGPRS - ACC_HEADROOM:
            out.append("acc")
        elif (occ <= 1 and other > LANE_REGS - ACC_VGPRS) or \
                (occ >= 2 and acc + other > LANE_REGS // occ - OCC2_HEADROOM):
            out.append("regs")
    return out


def raw_grid():
    """All 4^3 * 4 * 3 * 2 * 2 = 3072 points (bm, bn, bk, waves, ept, dbuf, occ)."""
    return [(bm, bn, bk, w, e, d, o) for bm in GRID_TILES for bn in GRID_TILES
            for bk in GRID_TILES for w in GRID_WAVES for e in GRID_EPT for d in GRID_DBUF
            for o in GRID_OCC]


def extended_grid():
    """``raw_grid`` with k-steps of 16, runs of 2 elements and occupancy 0 (the
    compiler's choice) added: 4*4*5*4*4*2*3 = 7680 points."""
    return [(bm, bn, bk, w, e, d, o) for bm in GRID_TILES for bn in GRID_TILES
            for bk in EXT_BK + GRID_TILES for w in GRID_WAVES for e in EXT_EPT + GRID_EPT
            for d in GRID_DBUF for o in (0,) + GRID_OCC]


def valid_grid(dtype: int, extended: bool = False):
    """The points of ``raw_grid`` (or ``extended_grid``) that break no rule."""
    return [p for p in (extended_grid() if extended else raw_grid())
            if not grid_violations(dtype, *p)]


def both_occupancy_tiles(dtype: int):
    """Tiles (bm, bn, bk, waves, ept, dbuf) of the raw grid valid at occupancy 1
    and at occupancy 2 (the pairs whose comparison measures the occupancy axis)."""
    v = set(valid_grid(dtype))
    return sorted({p[:6] for p in v if p[6] == 1} & {p[:6] for p in v if p[6] == 2})


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
                abandon_ms: float | None = None, stream=None) -> list[float]:
    """Device times (ms) of ``reps`` gemm calls after ``warmup`` untimed ones, from
    HIP events on the stream the calls run on.  Stops after the first timed run if
    it exceeds ``abandon_ms``."""
    import torch
    stream = stream or torch.cuda.current_stream()
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
TRAIN2_SEEDS = (5031, 5032, 5033)


def shape_set(which: str, count: int | None = None, lo: int = 64, hi: int = 16384):
    """'train' (3000 shapes), 'heldout' (500 shapes, none also in 'train'),
    'aligned' (800 shapes rounded up to multiples of 4, so every row is a whole
    16-byte load in FP64 and FP32; none in the other two sets) or 'train2' (3000
    more training shapes, none in the other three sets): m, n, k each log-uniform
    in [lo, hi] from their own seeded streams."""
    import synth
    if which == "train":
        seeds, cnt = TRAIN_SEEDS, 3000 if count is None else count
    elif which == "heldout":
        seeds, cnt = HELDOUT_SEEDS, 500 if count is None else count
    elif which == "aligned":
        seeds, cnt = ALIGNED_SEEDS, 800 if count is None else count
    elif which == "train2":
        seeds, cnt = TRAIN2_SEEDS, 3000 if count is None else count
    else:
        raise ValueError(which)
    ms, ns, ks = (synth.log_uniform_int(cnt + 64, s, lo, hi) for s in seeds)
    shapes = [(int(a), int(b), int(c)) for a, b, c in zip(ms, ns, ks)]
    if which == "aligned":
        shapes = [tuple(-(-x // 4) * 4 for x in sh) for sh in shapes]
    if which != "train":
        taken = set(shape_set("train", lo=lo, hi=hi))
        if which in ("aligned", "train2"):
            taken |= set(shape_set("heldout", lo=lo, hi=hi))
        if which == "train2":
            taken |= set(shape_set("aligned", lo=lo, hi=hi))
        shapes = [s for s in shapes if s not in taken]
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


def sweep(shapes, dtype: int, db: DB, cfgs=None, reps: int = 2, abandon: float = 2.0,
          log=None, every: int = 25, seconds: float | None = None) -> int:
    """Times every configuration (default: all registered ones of dtype) on every
    shape not yet in ``db`` for this device, appending one shape record per shape;
    returns the number of new records.  Configurations are tried in the order of
    their mean log relative speed over the shapes swept so far (the likely fastest
    first, so that slow ones are abandoned after one run).  With ``seconds``, no
    new shape is started after that many seconds."""
    import torch
    log = log or (lambda s: None)
    dev, bid = device_name(), build_id()
    cfgs = list(cfgs if cfgs is not None else configs(dtype))
    done = db.shapes_done(dev)
    todo = [tuple(s) for s in shapes if (dtype, *s) not in done]
    if not todo:
        log(f"sweep dtype={dtype}: nothing to do ({len(shapes)} shapes already measured)")
        return 0
    arena = Arena(todo + [(64, 64, 64)], dtype)
    stream = torch.cuda.current_stream()
    # load every kernel's code before anything is timed
    warm = arena.operands(64, 64, 64)
    for c in cfgs:
        gemm(warm.A, warm.B, warm.C, 1.0, 0.0, dtype=dtype, cfg=c, stream=stream)
    torch.cuda.synchronize()
    score = np.zeros(len(cfgs))
    t0 = time.time()
    new = 0
    for i, (m, n, k) in enumerate(todo):
        if seconds is not None and time.time() - t0 > seconds:
            log(f"sweep dtype={dtype}: time budget reached after {i} shapes")
            break
        ops = arena.operands(m, n, k)
        best = None
        times = [None] * len(cfgs)
        for j in np.argsort(-score, kind="stable"):
            t = time_config(ops, dtype, cfgs[j], warmup=0, reps=reps,
                            abandon_ms=None if best is None else abandon * best, stream=stream)
            times[j] = [round(x, 5) for x in t]
            best = min(t) if best is None else min(best, min(t))
        db.append({"device": dev, "build": bid, "dtype": dtype, "m": m, "n": n, "k": k,
                   "reps": reps, "cfgs": [list(c.as_tuple()) for c in cfgs], "ms": times,
                   "ts": round(time.time(), 1)})
        new += 1
        med = np.array([float(np.median(t)) for t in times])
        score += np.log(med.min() / med)
        if (i + 1) % every == 0 or i + 1 == len(todo):
            log(f"sweep dtype={dtype}: {i + 1}/{len(todo)} shapes, {time.time() - t0:.0f} s")
    return new


def refine(shapes, dtype: int, db: DB, top: int = 8, min_ms: float = 2.0, max_reps: int = 40,
           log=None, every: int = 100, seconds: float | None = None) -> int:
    """Measures again, with more runs, the ``top`` configurations the sweep found
    fastest on each shape of ``shapes`` in ``db`` (this device): each is run once
    untimed, then timed ``reps`` times, ``reps`` = enough runs for ``min_ms`` of
    kernel time (at least 5, at most ``max_reps``), and its median kept.  Near-ties
    between configurations (about half the shapes have a runner-up within 2 % of
    the best, and one run of a short kernel varies by several per cent) are thus
    decided on a median of many runs; the refined measurements replace the sweep's
    for those configurations (``prefer_refined``) when the database is loaded
    again.  Appends one record per shape to the database's file; returns the
    number of new records.  Shapes already refined are skipped."""
    import torch
    log = log or (lambda s: None)
    dev, bid = device_name(), build_id()
    valid = {c.as_tuple(): c for c in configs(dtype)}
    done = db.shapes_refined(dev)
    todo = [tuple(s) for s in shapes if (dtype, *s) not in done]
    if not todo:
        return 0
    arena = Arena(todo + [(64, 64, 64)], dtype)
    stream = torch.cuda.current_stream()
    warm = arena.operands(64, 64, 64)
    for c in valid.values():
        gemm(warm.A, warm.B, warm.C, 1.0, 0.0, dtype=dtype, cfg=c, stream=stream)
    torch.cuda.synchronize()
    want = set(todo)
    by_shape = {}
    for r in db.records:
        if r["dtype"] == dtype and r["device"] == dev and (r["m"], r["n"], r["k"]) in want \
                and tuple(r["cfg"]) in valid:
            by_shape.setdefault((r["m"], r["n"], r["k"]), []).append(r)
    t0 = time.time()
    new = 0
    for i, (m, n, k) in enumerate(todo):
        if seconds is not None and time.time() - t0 > seconds:
            log(f"refine dtype={dtype}: time budget reached after {i} shapes")
            break
        rs = by_shape.get((m, n, k), [])
        if not rs:
            continue
        rs.sort(key=lambda r: r["median_ms"])
        pick = [tuple(r["cfg"]) for r in rs[:top]]
        ops = arena.operands(m, n, k)
        reps = int(min(max_reps, max(5, math.ceil(min_ms / max(rs[0]["median_ms"], 1e-3)))))
        times = []
        for c in pick:
            t = time_config(ops, dtype, valid[c], warmup=1, reps=reps, stream=stream)
            times.append([round(x, 5) for x in t])
        # written to the file only: the refined medians take effect when the
        # database is loaded again
        db.write_line({"device": dev, "build": bid, "dtype": dtype, "m": m, "n": n, "k": k,
                       "reps": reps, "refine": True, "cfgs": [list(c) for c in pick], "ms": times,
                       "ts": round(time.time(), 1)})
        new += 1
        if (i + 1) % every == 0 or i + 1 == len(todo):
            log(f"refine dtype={dtype}: {i + 1}/{len(todo)} shapes, {time.time() - t0:.0f} s")
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
    from . import CFG_BATCHED
    cs = [c.as_tuple() for c in configs(dtype, CFG_BATCHED) if c.double_buffer < 2]
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


def _parse_cfg(text: str) -> tuple:
    v = tuple(int(x) for x in text.split(","))
    if len(v) != 7:
        raise ValueError(f"a configuration is 7 integers (bm,bn,bk,waves,ept,dbuf,occ): {text}")
    return v


def shapes_with_top(db: DB, dtype: int, shapes, cfgs, top: int) -> list:
    """The shapes of ``shapes`` on which one of ``cfgs`` is among the ``top``
    fastest configurations measured in ``db``."""
    by = {}
    for r in db.records:
        if r["dtype"] == dtype:
            by.setdefault((r["m"], r["n"], r["k"]), {})[tuple(r["cfg"])] = r["median_ms"]
    out = []
    for s in shapes:
        d = by.get(tuple(s), {})
        best = sorted(d, key=lambda c: d[c])[:top]
        if any(c in best for c in cfgs):
            out.append(tuple(s))
    return out


def merge_databases(base_paths, update_paths, out: str) -> DB:
    """One compact database from sweep and refinement databases (JSONL or compact):
    the ``update_paths`` hold later measurements (configurations registered since,
    and refinements of the shapes where one of them ranks among the fastest); their
    refinement records replace the earlier ones of the same shapes (the later pass
    re-timed that shape's current fastest configurations together)."""
    def load(p):
        d = load_compact(p) if p.endswith(".gz") else DB.load(p, raw=True)
        if d.bad_lines:
            raise ValueError(f"{p}: {d.bad_lines} unreadable lines")
        return d.records
    base = [r for p in base_paths for r in load(p)]
    upd = [r for p in update_paths for r in load(p)]
    again = {(r["device"], r["dtype"], r["m"], r["n"], r["k"]) for r in upd if r.get("refined")}
    kept = [r for r in base if not (r.get("refined") and
                                    (r["device"], r["dtype"], r["m"], r["n"], r["k"]) in again)]
    db = DB(out, prefer_refined(kept + upd), 0)
    save_compact(db, out)
    return db


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="autotuner sweep (resumable JSONL database)")
    ap.add_argument("--set", choices=["train", "heldout", "aligned", "train2"])
    ap.add_argument("--dtype", choices=["f64", "f32"])
    ap.add_argument("--db")
    ap.add_argument("--count", type=int, default=None)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--seconds", type=float, default=None,
                    help="start no new shape after this many seconds")
    ap.add_argument("--refine", type=int, default=0,
                    help="instead of sweeping: re-time the N fastest configurations of every "
                         "shape of the set already in --db (and --from databases)")
    ap.add_argument("--from", dest="sources", action="append", default=[],
                    help="(with --refine) further databases holding the sweep's records "
                         "(JSONL, or the compact .json.gz form); (with --merge) the earlier "
                         "databases")
    ap.add_argument("--only", action="append", default=[],
                    help="bm,bn,bk,waves,ept,dbuf,occ: sweep only these registered "
                         "configurations (into a database of their own); with --refine, "
                         "refine only the shapes where one of them is among the N fastest")
    ap.add_argument("--skip", default=None,
                    help="text file of 'dtype m n k' lines: shapes measured elsewhere (for "
                         "sweeps split over several databases)")
    ap.add_argument("--merge", default=None,
                    help="write this compact database from the --from databases and the "
                         "--update ones (whose refinements replace earlier ones of a shape)")
    ap.add_argument("--update", action="append", default=[])
    a = ap.parse_args(argv)
    if a.merge:
        db = merge_databases(a.sources, a.update, a.merge)
        print(f"tune: {len(db.records)} records -> {a.merge}", flush=True)
        return
    if not (a.set and a.dtype and a.db):
        ap.error("--set, --dtype and --db are required unless --merge is given")
    dt = F64 if a.dtype == "f64" else F32
    only = [_parse_cfg(t) for t in a.only]
    db = DB.load(a.db)
    if db.bad_lines:
        print(f"tune: skipped {db.bad_lines} unreadable database lines", flush=True)
    shapes = shape_set(a.set, a.count)
    if a.refine:
        for src in a.sources:
            extra = load_compact(src) if src.endswith(".gz") else DB.load(src)
            db.records = prefer_refined(db.records + extra.records)
        if only:
            shapes = shapes_with_top(db, dt, shapes, only, a.refine)
        n = refine(shapes, dt, db, top=a.refine, log=lambda s: print(s, flush=True),
                   seconds=a.seconds)
        print(f"tune: {n} new refinement records in {a.db}", flush=True)
        return
    if a.skip:
        with open(a.skip) as f:
            done = {tuple(int(x) for x in line.split()) for line in f if line.strip()}
        shapes = [s for s in shapes if (dt, *s) not in done]
    cfgs = None
    if only:
        cfgs = [c for c in configs(dt) if c.as_tuple() in only]
        if len(cfgs) != len(set(only)):
            ap.error("--only names a configuration this library does not register")
    n = sweep(shapes, dt, db, cfgs=cfgs, reps=a.reps, log=lambda s: print(s, flush=True),
              seconds=a.seconds)
    print(f"tune: {n} new shape records in {a.db}", flush=True)


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


if __name__ == "__main__":
    main()
