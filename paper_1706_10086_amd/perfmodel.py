"""The paper's performance model (Sec. 2, Eq. 2-7; Sec. 3, Eq. 8) and its
generalisation to rectangular tiles, as used for the measurements' roofline and
traffic figures.

Square N x N matrices, tile size T, S bytes per element:

* ``ops(N)``          operations of one GEMM, Eq. 2 (3N^2 for the alpha/beta
                      update plus 2N^3 for the product; the 2N^3 term is what
                      Eq. 4 and every TFLOP/s figure here count).
* ``blocks(N, e, t)`` blocks per grid dimension for e elements per thread and t
                      threads per block, Eq. 3.
* ``perf_gflops``     GFLOP/s from a time in seconds, Eq. 4.
* ``cache_bytes``     bytes of one A tile and one B tile, Eq. 5.
* ``mem_ops``         element loads of the tiled algorithm: every C tile reads
                      N/T tiles of A and of B and its own C tile once, Eq. 6.
* ``intensity``       operations per element loaded, Eq. 7 (tends to T).
* ``peak``            clock x operations per cycle and core x cores, Eq. 8.

Generalisations for BM x BN tiles of C and k-steps of BK: ``gemm_flops`` (2mnk),
``tile_traffic_bytes`` (Eq. 6 per tile: the A panel BM x k and B panel k x BN,
plus C read and written once) and ``lds_stage_bytes`` (Eq. 5 for one k-step).
"""
from __future__ import annotations

# MI355X: 256 compute units at 2.4 GHz; operations per clock and compute unit of
# the dense matrix cores for each type (the published peaks divided by 256 x 2.4e9)
MI355X_CUS = 256
MI355X_CLOCK_HZ = 2.4e9
MI355X_OPS_PER_CLK_CU = {"f64": 128, "f32": 256, "bf16": 4096, "int8": 8192}


def ops(N: float) -> float:
    """Eq. 2: 3 N^2 + 2 N^3."""
    return 3.0 * N * N + 2.0 * N ** 3


def gemm_flops(m: float, n: float, k: float) -> float:
    """The counted work of one m x n x k GEMM (the 2 N^3 term of Eq. 2 and 4)."""
    return 2.0 * m * n * k


def blocks(N: float, e: float, t: float) -> float:
    """Eq. 3: blocks per grid dimension, N / (t e)."""
    return N / (t * e)


def perf_gflops(N: float, seconds: float) -> float:
    """Eq. 4: 2 N^3 / t * 1e-9."""
    return 2.0 * N ** 3 / seconds * 1e-9


def cache_bytes(S: float, T: float) -> float:
    """Eq. 5: one T x T tile of A and one of B, S bytes per element."""
    return 2.0 * T * T * S


def mem_ops(N: float, T: float) -> float:
    """Eq. 6: N^2 (2 N / T + 1) element loads."""
    return N * N * (2.0 * N / T + 1.0)


def intensity(N: float, T: float) -> float:
    """Eq. 7: 2 N T / (2 N + T) operations per element loaded."""
    return 2.0 * N * T / (2.0 * N + T)


def peak(f: float, o: float, n: float) -> float:
    """Eq. 8: clock f times operations per cycle and core o times cores n."""
    return f * o * n


def mi355x_peak(kind: str) -> float:
    """Eq. 8 for the MI355X matrix cores (operations per second)."""
    return peak(MI355X_CLOCK_HZ, MI355X_OPS_PER_CLK_CU[kind], MI355X_CUS)


def tile_traffic_bytes(m: int, n: int, k: int, bm: int, bn: int, S: int,
                       read_c: bool = True) -> float:
    """Eq. 6 for BM x BN tiles without any cache reuse: each of the
    ceil(m/BM) ceil(n/BN) tiles reads its A panel (BM x k) and B panel (k x BN);
    C is read (if beta != 0) and written once."""
    tiles = -(-m // bm) * -(-n // bn)
    return float(tiles * (bm * k + k * bn) * S + (2 if read_c else 1) * m * n * S)


def lds_stage_bytes(bm: int, bn: int, bk: int, S: int) -> int:
    """Eq. 5 for one k-step of a BM x BN tile: the BM x BK slab of A and the
    BK x BN slab of B (before padding)."""
    return (bm * bk + bk * bn) * S
