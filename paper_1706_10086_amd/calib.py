"""Calibration workload for hardware traffic counters: a plain device-to-device
copy of a known number of bytes, run under a profiler so that the counter
reading per copied byte can scale the counters of the GEMM kernels.

    python -m paper_1706_10086_amd.calib [--mib 1024] [--reps 3]

Each repetition reads and writes ``mib`` MiB once (torch's copy kernel).
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    import torch
    n = a.mib * 1024 * 1024 // 8
    src = torch.rand(n, device="cuda", dtype=torch.float64)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"calib: copied {a.mib} MiB x {a.reps}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
