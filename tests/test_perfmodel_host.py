"""Pins of the performance model (Sec. 2, Eq. 2-7; Sec. 3, Eq. 8): each closed form
against the paper's other form of the same quantity or against a count done
another way (exact rational arithmetic, explicit tile enumeration)."""
from fractions import Fraction

import pytest

from paper_1706_10086_amd import perfmodel as pm


def test_eq6_closed_form_equals_tile_count():
    # N/T tiles per dimension; every C tile loads N/T tiles of A and of B (T^2
    # elements each) and itself once
    for N, T in [(64, 8), (1024, 16), (8192, 128), (8192, 256), (300, 30)]:
        nb = Fraction(N, T)
        counted = nb * nb * (2 * T * T * nb + T * T)
        assert Fraction(pm.mem_ops(N, T)) == counted
    assert pm.mem_ops(8192, 128) == 129 * 8192 ** 2


def test_eq7_is_ops_over_memory_and_tends_to_T():
    for N, T in [(1024, 16), (8192, 256), (100, 7)]:
        exact = Fraction(2 * N ** 3) / Fraction(N * N * (2 * N + T), T)
        assert abs(Fraction(pm.intensity(N, T)) - exact) <= exact * Fraction(1, 10 ** 12)
    assert round(pm.intensity(8192, 256), 1) == 252.1
    assert abs(pm.intensity(1e15, 64) - 64) < 1e-9


def test_eq2_eq4_eq3_eq5():
    assert pm.ops(10) == 3 * 100 + 2 * 1000
    assert pm.gemm_flops(8192, 8192, 8192) == 2 * 8192 ** 3
    assert pm.ops(8192) - pm.gemm_flops(8192, 8192, 8192) == 3 * 8192 ** 2
    assert pm.perf_gflops(1000, 2.0) == 1.0          # 2e9 operations in 2 s
    assert pm.blocks(1024, 4, 16) == 16
    assert pm.cache_bytes(8, 16) == 4096             # two 16 x 16 FP64 tiles
    assert pm.lds_stage_bytes(16, 16, 16, 8) == pm.cache_bytes(8, 16)


def test_eq8_mi355x_peaks_match_published():
    published = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2516.6e12, "int8": 5033.2e12}
    for kind, value in published.items():
        assert abs(pm.mi355x_peak(kind) / value - 1) < 1e-3, kind
    assert pm.peak(2.0, 3.0, 5.0) == 30.0


@pytest.mark.parametrize("m,n,k,bm,bn", [(8192, 8192, 8192, 256, 128), (1000, 300, 77, 64, 64),
                                         (33, 65, 5, 32, 32)])
def test_tile_traffic_by_enumeration(m, n, k, bm, bn):
    total = 0
    for i0 in range(0, m, bm):
        for j0 in range(0, n, bn):
            total += (bm * k + k * bn) * 8
    total += 2 * m * n * 8
    assert pm.tile_traffic_bytes(m, n, k, bm, bn, 8) == total
    assert pm.tile_traffic_bytes(m, n, k, bm, bn, 8, read_c=False) == total - m * n * 8


def test_square_tiles_reduce_to_eq6():
    # with BM = BN = T and S = 1 the generalisation is Eq. 6 plus the C write
    for N, T in [(1024, 64), (8192, 256)]:
        assert pm.tile_traffic_bytes(N, N, N, T, T, 1, read_c=True) == pm.mem_ops(N, T) + N * N
    # the A and B panel reads of the 2048 tiles of the N = 8192 FP64 kernel: 51.5e9 B
    panels = pm.tile_traffic_bytes(8192, 8192, 8192, 256, 128, 8, read_c=False) - 8192 ** 2 * 8
    assert abs(panels - 51.5e9) < 0.1e9
