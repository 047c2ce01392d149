"""Autotuner: time every registered tile configuration of a dtype on a set of
shapes, keep the results in an append-only JSONL database, and pick the
exhaustive best.

The procedure follows the paper's parameter tuning (Sec. 2.3 "Multidimensional
parameter tuning" and Sec. 3, Tab. 4): a grid of tile parameters is searched,
each point measured several times and the best kept, at a main size and checked
at a control size.  Here the grid is the library's configuration registry
(tile M/N/K, waves per work-group, elements per thread, double buffering,
occupancy), the measurement is the device time of one gemm_ex call from HIP
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
