"""Oracle of the tiled GEMM -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It wraps ``oracle.c`` (plain C, built with gcc, no FMA contraction) through
ctypes and shares nothing with the GPU library.

Functions take numpy float64 matrices that are row-major with unit column stride
(views with a larger row stride are passed with that stride as the leading
dimension) and return new arrays; the caller's inputs are never modified.

* ``gemm_f64``   -- C = alpha*A*B + beta*C (paper, Sec. 2, Eq. 1), each element summed
                    over increasing k.
* ``gemm_dot2``  -- the same result with double-double accumulation (Ogita, Rump,
                    Oishi 2005, Dot2), the high-accuracy reference.
* ``split_*``    -- the split-precision (Ozaki) emulation: exponents, slices, exact
                    slice-pair products and the full recombined product.
* ``crt_gemm``   -- the modular-integer emulation (Ozaki scheme II): the exact product
                    of the operands truncated to ``bits`` bits per row / column, rounded
                    once; ``crt_bits`` is the operand width the scheme uses for a given k.
* ``mlp_*``      -- the FP64 MLP cost model (see ``oracle/mlp.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared", "-std=c11"]

FMT_BF16 = 0
FMT_E4M3 = 1
FMT_INT8 = 2
DEFAULT_SLICES = {FMT_BF16: 6, FMT_E4M3: 11, FMT_INT8: 8}
ERR_NONFINITE = 3


def build() -> str:
    """Compiles ``liboracle.so`` with gcc (always; a few seconds)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        i64, d, p, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        for name in ("orc_gemm_f64", "orc_gemm_dot2"):
            fn = getattr(L, name)
            fn.argtypes = [i64, i64, i64, d, p, i64, p, i64, d, p, i64, i32]
            fn.restype = None
        L.orc_split_gemm.argtypes = [i64, i64, i64, d, p, i64, p, i64, d, p, i64, i32, i32, i32]
        L.orc_split_gemm.restype = i32
        L.orc_split_row_exponents.argtypes = [i64, i64, p, i64, p]
        L.orc_split_col_exponents.argtypes = [i64, i64, p, i64, p]
        L.orc_split_slices_rows.argtypes = [i64, i64, p, i64, p, i32, i32, p, p]
        L.orc_split_slices_cols.argtypes = [i64, i64, p, i64, p, i32, i32, p, p]
        L.orc_split_pair_product.argtypes = [i64, i64, i64, p, p, p]
        L.orc_split_bits.argtypes = [i32, p, p]
        L.orc_split_bits.restype = i32
        L.orc_crt_gemm.argtypes = [i64, i64, i64, d, p, i64, p, i64, d, p, i64, i32, i32]
        L.orc_crt_gemm.restype = i32
        L.orc_num_procs.restype = i32
        _lib = L
    return _lib


def _mat(X: np.ndarray) -> tuple[np.ndarray, int]:
    """Returns (array, leading dimension) for a row-major float64 matrix view."""
    X = np.asarray(X)
    if X.dtype != np.float64:
        X = X.astype(np.float64)
    if X.ndim != 2:
        raise ValueError("matrix expected")
    if ((X.shape[1] > 1 and X.strides[1] != 8) or X.strides[0] % 8
            or (X.shape[0] > 1 and X.strides[0] < 8 * X.shape[1])):
        X = np.ascontiguousarray(X)
    ld = X.strides[0] // 8 if X.shape[0] > 1 else max(1, X.shape[1])
    return X, max(ld, 1)


def _ptr(X: np.ndarray) -> int:
    return X.ctypes.data


def num_procs() -> int:
    return int(lib().orc_num_procs())


def _gemm(fn, alpha, A, B, beta, C, nthreads):
    A, lda = _mat(A)
    B, ldb = _mat(B)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = np.zeros((m, n))
    C = np.array(C, dtype=np.float64, order="C", copy=True)
    if C.shape != (m, n):
        raise ValueError("C shape")
    fn(m, n, k, float(alpha), _ptr(A), lda, _ptr(B), ldb, float(beta), _ptr(C),
       max(1, n), int(nthreads))
    return C


def gemm_f64(alpha, A, B, beta=0.0, C=None, nthreads: int = 1) -> np.ndarray:
    """alpha*A@B + beta*C in plain FP64, k summed in increasing order."""
    return _gemm(lib().orc_gemm_f64, alpha, A, B, beta, C, nthreads)


def gemm_dot2(alpha, A, B, beta=0.0, C=None, nthreads: int = 1) -> np.ndarray:
    """alpha*A@B + beta*C with double-double accumulation (about u^2 error)."""
    return _gemm(lib().orc_gemm_dot2, alpha, A, B, beta, C, nthreads)


def split_bits(fmt: int) -> tuple[int, int]:
    b1 = ctypes.c_int()
    b = ctypes.c_int()
    if lib().orc_split_bits(fmt, ctypes.byref(b1), ctypes.byref(b)) != 0:
        raise ValueError("unknown slice format")
    return b1.value, b.value


def split_gemm(alpha, A, B, beta=0.0, C=None, fmt: int = FMT_BF16, S: int | None = None,
               nthreads: int = 1) -> np.ndarray:
    """Split-precision emulated FP64 GEMM.  Raises FloatingPointError on
    non-finite input (the C code's status 3)."""
    A, lda = _mat(A)
    B, ldb = _mat(B)
    m, k = A.shape
    _, n = B.shape
    S = DEFAULT_SLICES[fmt] if S is None else S
    C = np.zeros((m, n)) if C is None else np.array(C, dtype=np.float64, order="C", copy=True)
    rc = lib().orc_split_gemm(m, n, k, float(alpha), _ptr(A), lda, _ptr(B), ldb,
                              float(beta), _ptr(C), max(1, n), fmt, S, int(nthreads))
    if rc == ERR_NONFINITE:
        raise FloatingPointError("non-finite input")
    if rc == -14:
        raise OverflowError("k too large for the exact level sum")
    if rc != 0:
        raise ValueError(f"split_gemm status {rc}")
    return C


def split_row_exponents(A) -> np.ndarray:
    A, lda = _mat(A)
    e = np.zeros(A.shape[0], dtype=np.int32)
    lib().orc_split_row_exponents(A.shape[0], A.shape[1], _ptr(A), lda, _ptr(e))
    return e


def split_col_exponents(B) -> np.ndarray:
    B, ldb = _mat(B)
    f = np.zeros(B.shape[1], dtype=np.int32)
    lib().orc_split_col_exponents(B.shape[0], B.shape[1], _ptr(B), ldb, _ptr(f))
    return f


def split_slices_rows(A, e, fmt: int, S: int):
    """(Q, rem): Q[s] is the integer slice s+1 of A (m x k, int16); rem the last
    remainder in units of the last slice."""
    A, lda = _mat(A)
    e = np.ascontiguousarray(e, dtype=np.int32)
    m, k = A.shape
    Q = np.zeros((S, m, k), dtype=np.int16)
    rem = np.zeros((m, k))
    lib().orc_split_slices_rows(m, k, _ptr(A), lda, _ptr(e), fmt, S, _ptr(Q), _ptr(rem))
    return Q, rem


def split_slices_cols(B, f, fmt: int, S: int):
    """(Q, rem) for B sliced per column: Q[t] is k x n."""
    B, ldb = _mat(B)
    f = np.ascontiguousarray(f, dtype=np.int32)
    k, n = B.shape
    Q = np.zeros((S, k, n), dtype=np.int16)
    rem = np.zeros((k, n))
    lib().orc_split_slices_cols(k, n, _ptr(B), ldb, _ptr(f), fmt, S, _ptr(Q), _ptr(rem))
    return Q, rem


def split_pair_product(QA: np.ndarray, QB: np.ndarray) -> np.ndarray:
    """Exact int64 product of an m x k and a k x n int16 slice."""
    QA = np.ascontiguousarray(QA, dtype=np.int16)
    QB = np.ascontiguousarray(QB, dtype=np.int16)
    m, k = QA.shape
    _, n = QB.shape
    G = np.zeros((m, n), dtype=np.int64)
    lib().orc_split_pair_product(m, n, k, _ptr(QA), _ptr(QB), _ptr(G))
    return G


# The modular emulation carries the exact product of the truncated operands in
# residues modulo 16 pairwise coprime moduli whose product exceeds 2^125; the
# reconstruction is unambiguous while |sum| <= 2^123 (a quarter of that product).
# Operands of b bits give |sum| < k 2^(2b), hence the widest safe b for a given k:
CRT_SUM_BITS = 123


def crt_bits(k: int) -> int:
    """Largest b with k * 2^(2b) <= 2^123 (b <= 62)."""
    if k < 1:
        raise ValueError("k >= 1")
    b = 62
    while k * (1 << (2 * b)) > (1 << CRT_SUM_BITS):
        b -= 1
    return b


def crt_gemm(alpha, A, B, beta=0.0, C=None, bits: int | None = None,
             nthreads: int = 1) -> np.ndarray:
    """Modular-integer emulated FP64 GEMM: exact product of the operands truncated
    to ``bits`` bits (default ``crt_bits(k)``), rounded once.  Raises
    FloatingPointError on non-finite input."""
    A, lda = _mat(A)
    B, ldb = _mat(B)
    m, k = A.shape
    _, n = B.shape
    if bits is None:
        bits = crt_bits(max(k, 1))
    C = np.zeros((m, n)) if C is None else np.array(C, dtype=np.float64, order="C", copy=True)
    rc = lib().orc_crt_gemm(m, n, k, float(alpha), _ptr(A), lda, _ptr(B), ldb,
                            float(beta), _ptr(C), max(1, n), int(bits), int(nthreads))
    if rc == ERR_NONFINITE:
        raise FloatingPointError("non-finite input")
    if rc == -14:
        raise OverflowError("k * 2^(2 bits) too large for the exact sum")
    if rc != 0:
        raise ValueError(f"crt_gemm status {rc}")
    return C
