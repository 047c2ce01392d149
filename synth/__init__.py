"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module holds no GEMM arithmetic.  It only turns a seed into numbers:

* ``splitmix64(seed, count)`` is the SplitMix64 sequence (Steele, Lea and Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014) started from
  state ``seed``: output ``i`` mixes ``seed + (i + 1) * 0x9E3779B97F4A7C15``.
  Every output is a pure function of ``(seed, i)``, so any slice of a stream can be
  regenerated without the rest.
* ``unit(seed, count)``: ``(x >> 11) * 2**-53`` in [0, 1).
* ``uniform_pm1``: ``2u - 1`` in [-1, 1) -- the dense workloads of the square and
  batched benchmarks.
* ``wide_range``: ``u * 2**e`` with ``u`` in [-1, 1) and ``e`` a uniform integer in
  [-20, 20] -- the stress input of the split-precision path.
* ``log_uniform_int``: integers log-uniform in [a, b] -- the uneven batched shapes
  and the tuner's shapes.
* ``integer_valued``: uniform integers in [-r, r] -- inputs whose products and
  partial sums are exact in floating point.

Large matrices are generated in row blocks so that a 16384 x 16384 operand never
needs more than a few hundred MB of temporaries.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream of ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
        return _mix(state)


def unit(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1) with 53 random bits each."""
    x = splitmix64(seed, count, start)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _fill(shape, seed, per_elem, fn) -> np.ndarray:
    """Fills a C-contiguous float64 array chunk by chunk; ``fn(seed, n, start)``
    returns ``n`` values for elements starting at flat index ``start // per_elem``."""
    total = int(np.prod(shape)) if len(shape) else 1
    out = np.empty(total, dtype=np.float64)
    for s in range(0, total, _CHUNK):
        n = min(_CHUNK, total - s)
        out[s:s + n] = fn(seed, n, s * per_elem)
    return out.reshape(shape)


def uniform_pm1(shape, seed: int) -> np.ndarray:
    """i.i.d. uniform[-1, 1) doubles, element ``i`` from stream output ``i``."""
    return _fill(shape, seed, 1, lambda sd, n, st: 2.0 * unit(sd, n, st) - 1.0)


def wide_range(shape, seed: int, emin: int = -20, emax: int = 20) -> np.ndarray:
    """``u * 2**e``: element ``i`` takes ``u`` from output ``2i`` (uniform[-1,1)) and
    ``e`` from output ``2i+1`` (uniform integer in [emin, emax])."""
    span = emax - emin + 1

    def gen(sd, n, st):
        r = unit(sd, 2 * n, st)
        u = 2.0 * r[0::2] - 1.0
        e = emin + np.floor(r[1::2] * span).astype(np.int64)
        return np.ldexp(u, e)

    return _fill(shape, seed, 2, gen)


def integer_valued(shape, seed: int, r: int) -> np.ndarray:
    """Uniform integers in [-r, r] stored as doubles."""
    span = 2 * r + 1
    return _fill(shape, seed, 1,
                 lambda sd, n, st: np.floor(unit(sd, n, st) * span) - r)


def log_uniform_int(count: int, seed: int, lo: int, hi: int) -> np.ndarray:
    """``count`` integers log-uniform in [lo, hi]:
    ``floor(2**(log2 lo + u*(log2(hi+1) - log2 lo)))`` clamped to ``hi``."""
    u = unit(seed, count)
    a = np.log2(lo)
    b = np.log2(hi + 1)
    v = np.floor(np.exp2(a + u * (b - a))).astype(np.int64)
    return np.clip(v, lo, hi)


def seeds_for(config: int, tag: int) -> tuple[int, int, int]:
    """Seeds of (A, B, C) for a workload: ``s = 1000*config + tag``."""
    s = 1000 * config + tag
    return s, s + 1, s + 2
