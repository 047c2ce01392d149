"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every
symbol include/mgemm.h declares, and rejects invalid arguments with the -i code of
the first bad argument (BLAS convention) before touching the device."""
import ctypes
import os
import re

import pytest

import paper_1706_10086_amd as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "mgemm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:MGEMM_API\s+)?(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M))


@pytest.fixture(scope="module")
def L():
    try:
        return mg.lib()
    except mg.MgemmNotBuilt:
        pytest.skip("libmgemm.so not built")


def test_every_declared_symbol_is_exported(L):
    syms = header_symbols()
    assert {"gemm", "gemm_ex", "mgemm_last_error"} <= syms
    for s in syms:
        assert hasattr(L, s), s
    assert set(mg.EXPORTED) == syms


P = 1 << 20   # a fake, never dereferenced device address


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 1.0, P, 4, P, 4, 0.0, P * 2, 4, 0), -1),
    ((4, -1, 4, 1.0, P, 4, P, 4, 0.0, P * 2, 4, 0), -2),
    ((4, 4, -1, 1.0, P, 4, P, 4, 0.0, P * 2, 4, 0), -3),
    ((4, 4, 4, 1.0, 0, 4, P, 4, 0.0, P * 2, 4, 0), -5),
    ((4, 4, 8, 1.0, P, 7, P, 4, 0.0, P * 2, 4, 0), -6),
    ((4, 4, 4, 1.0, P, 4, 0, 4, 0.0, P * 2, 4, 0), -7),
    ((4, 5, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 5, 0), -8),
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, 0, 4, 0), -10),
    ((4, 5, 4, 1.0, P, 4, P * 4, 5, 0.0, P * 2, 4, 0), -11),
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 4, 7), -12),
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 4, 6), -12),
    # every emulated dtype is accepted: the bad leading dimension is reported
    ((4, 4, 8, 1.0, P, 7, P, 4, 0.0, P * 2, 4, 2), -6),
    ((4, 4, 8, 1.0, P, 7, P, 4, 0.0, P * 2, 4, 3), -6),
    ((4, 4, 8, 1.0, P, 7, P, 4, 0.0, P * 2, 4, 4), -6),
    ((4, 4, 8, 1.0, P, 7, P, 4, 0.0, P * 2, 4, 5), -6),
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 4, -1), -12),
    # C overlapping A
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P + 64, 4, 0), -10),
    # the first bad argument wins
    ((-1, -1, 4, 1.0, 0, 0, 0, 0, 0.0, 0, 0, 9), -1),
    ((4, 4, 4, 1.0, 0, 1, 0, 1, 0.0, 0, 1, 9), -5),
])
def test_invalid_arguments(L, args, code):
    assert mg.gemm_raw(*args) == code
    assert mg.last_error() != ""


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 1.0, P, 4, P, 4, 0.0, P * 2, 4, 0), -1),
    ((4, 4, 8, 1.0, P, 7, P, 4, 0.0, P * 2, 4, 1), -6),
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P + 64, 4, 0), -10),
    # the emulated dtypes need the library workspace
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 4, 2), -12),
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 4, 5), -12),
    ((4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 4, 9), -12),
])
def test_noalloc_invalid_arguments(L, args, code):
    assert mg.gemm_ex_noalloc_raw(*args) == code
    assert mg.last_error() != ""
    # empty problems return before any device work
    assert mg.gemm_ex_noalloc_raw(0, 4, 4, 1.0, 0, 4, 0, 4, 0.0, 0, 4, 0) == 0


def test_empty_problems_return_without_device_work(L):
    # m == 0 or n == 0: nothing to do, NULL pointers allowed
    assert mg.gemm_raw(0, 4, 4, 1.0, 0, 4, 0, 4, 0.0, 0, 4, 0) == 0
    assert mg.gemm_raw(4, 0, 4, 1.0, 0, 4, 0, 1, 0.0, 0, 1, 1) == 0
    # lda >= max(1, k) also when k == 0
    assert mg.gemm_raw(0, 0, 0, 1.0, 0, 1, 0, 1, 0.0, 0, 1, 0) == 0
    assert mg.gemm_raw(0, 0, 0, 1.0, 0, 0, 0, 1, 0.0, 0, 1, 0) == -6


def test_unregistered_config_rejected(L):
    bad = mg.Cfg(48, 48, 16, 4, 2, 1, 0)
    assert mg.gemm_ex_raw(4, 4, 4, 1.0, P, 4, P * 4, 4, 0.0, P * 2, 4, 0, bad, None) == -13


@pytest.mark.parametrize("dtype", [mg.SPLIT_BF16, mg.SPLIT_FP8, mg.SPLIT_INT8, mg.CRT_INT8])
@pytest.mark.parametrize("alpha,k", [(1.0, 4), (0.0, 4), (1.0, 0)])
def test_split_dtype_with_config_rejected_whatever_alpha(L, dtype, alpha, k):
    # the check comes before the alpha == 0 / k == 0 quick return, so the verdict on
    # a call does not depend on the value of alpha
    cfg = mg.Cfg(64, 64, 16, 4, 2, 1, 0)
    assert mg.gemm_ex_raw(4, 4, k, alpha, P, 4, P * 4, 4, 0.0, P * 2, 4, dtype, cfg, None) == -13
    assert "split dtypes" in mg.last_error()


def test_config_registry(L):
    for dt in (mg.F64, mg.F32):
        cs = mg.configs(dt)
        assert len(cs) >= 1
        for c in cs:
            assert c.bm % 16 == 0 and c.bn % 16 == 0 and c.bk % 8 == 0
            assert c.waves in (1, 2, 4, 8) and c.double_buffer in (0, 1, 2) and c.occupancy in (0, 1, 2)
        assert len({c.as_tuple() for c in cs}) == len(cs)
    assert L.mgemm_config_count(9) < 0
    c = mg.Cfg()
    assert L.mgemm_config_get(mg.F64, 10 ** 6, ctypes.byref(c)) == -2


def test_choice_argument_errors(L):
    """mgemm_choice checks its arguments before asking the device anything."""
    c, s = mg.Cfg(), ctypes.c_int32()
    cases = [((0, 4, 4, 4, 4, mg.F64), -1), ((4, 0, 4, 4, 4, mg.F64), -2),
             ((4, 4, 0, 4, 4, mg.F64), -3), ((4, 4, 8, 7, 4, mg.F64), -4),
             ((4, 8, 4, 4, 7, mg.F64), -5), ((4, 4, 4, 4, 4, mg.SPLIT_BF16), -6)]
    for args, code in cases:
        assert L.mgemm_choice(*args, ctypes.byref(c), ctypes.byref(s), None) == code, args
    assert L.mgemm_choice(4, 4, 4, 4, 4, mg.F64, None, ctypes.byref(s), None) == -7
    assert L.mgemm_choice(4, 4, 4, 4, 4, mg.F64, ctypes.byref(c), None, None) == -8


def test_host_alloc_argument_errors(L):
    # both are rejected before any HIP call
    h, d = ctypes.c_void_p(), ctypes.c_void_p()
    assert L.mgemm_host_alloc(0, 1, ctypes.byref(h), ctypes.byref(d)) == -1
    assert L.mgemm_host_alloc(-5, 0, ctypes.byref(h), ctypes.byref(d)) == -1
    assert h.value is None and d.value is None
    assert L.mgemm_host_alloc(64, 1, None, ctypes.byref(d)) == -2
    assert L.mgemm_host_alloc(64, 1, ctypes.byref(h), None) == -2
    assert L.mgemm_host_free(None) == 0
