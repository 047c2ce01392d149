"""mgemm: tiled GEMM C = alpha*A*B + beta*C on AMD MI355X (gfx950).

A thin ctypes binding of ``libmgemm.so`` (built in-tree by ``build.py``).  Every
step of the computation runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch is used for device memory and streams.  If the
library has not been built, importing works but every call raises
``MgemmNotBuilt`` -- there is no fallback.

Entry points mirror ``include/mgemm.h``:

* ``gemm_raw`` / ``gemm_ex_raw``: the C functions with integer pointers.
* ``gemm(A, B, C, alpha, beta, dtype, cfg, stream)``: the same on torch tensors.
* ``configs(dtype)``: the registered tile configurations.
"""
from __future__ import annotations

import ctypes
import os
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgemm.so")

F64, F32, SPLIT_BF16, SPLIT_FP8, SPLIT_INT8, CRT_INT8 = 0, 1, 2, 3, 4, 5
DTYPE_NAMES = {F64: "f64", F32: "f32", SPLIT_BF16: "split_bf16", SPLIT_FP8: "split_fp8",
               SPLIT_INT8: "split_int8", CRT_INT8: "crt_int8"}
SPLIT_SLICES = {SPLIT_BF16: 6, SPLIT_FP8: 11, SPLIT_INT8: 8}
ERR_HIP, ERR_NOMEM, ERR_NONFINITE, ERR_NOCONFIG, ERR_PLAN = 1, 2, 3, 4, 5

# Every symbol include/mgemm.h declares.
EXPORTED = [
    "gemm", "gemm_ex", "mgemm_set_stream", "mgemm_last_error", "mgemm_config_count",
    "mgemm_config_get", "mgemm_release_workspace", "mgemm_probe_mfma", "mgemm_probe_mfma_raw",
    "gemm_batched", "gemm_batched_plan_create", "gemm_batched_plan_execute",
    "gemm_batched_plan_destroy", "gemm_batched_plan_info", "mgemm_host_alloc", "mgemm_host_free",
    "mgemm_config_flags", "gemm_ex_noalloc", "mgemm_choice",
]
CFG_GEMM, CFG_BATCHED, CFG_SPLITK = 1, 2, 4


class MgemmNotBuilt(RuntimeError):
    pass


class MgemmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mgemm error {code}: {msg}")
        self.code = code


class Cfg(ctypes.Structure):
    _fields_ = [("bm", ctypes.c_int32), ("bn", ctypes.c_int32), ("bk", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("elems_per_thread", ctypes.c_int32),
                ("double_buffer", ctypes.c_int32), ("occupancy", ctypes.c_int32)]

    def as_tuple(self):
        return (self.bm, self.bn, self.bk, self.waves, self.elems_per_thread, self.double_buffer,
                self.occupancy)

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return "Cfg(%d,%d,%d,w%d,e%d,d%d,o%d)" % self.as_tuple()


_lib = None


def lib():
    """Loads libmgemm.so (once) and declares its prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MgemmNotBuilt(f"{LIB_PATH} is missing: run `python -m paper_1706_10086_amd.build`")
    # torch (device memory and streams for the binding) is loaded first: with the
    # library's HIP runtime loaded before torch's, torch finds no GPU
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, d, p = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    L.gemm.argtypes = [i64, i64, i64, d, p, i64, p, i64, d, p, i64, i32]
    L.gemm.restype = i32
    L.gemm_ex.argtypes = [i64, i64, i64, d, p, i64, p, i64, d, p, i64, i32,
                          ctypes.POINTER(Cfg), p]
    L.gemm_ex.restype = i32
    L.gemm_ex_noalloc.argtypes = L.gemm_ex.argtypes
    L.gemm_ex_noalloc.restype = i32
    L.mgemm_set_stream.argtypes = [p]
    L.mgemm_set_stream.restype = i32
    L.mgemm_last_error.argtypes = []
    L.mgemm_last_error.restype = ctypes.c_char_p
    L.mgemm_config_count.argtypes = [i32]
    L.mgemm_config_count.restype = i32
    L.mgemm_config_get.argtypes = [i32, i32, ctypes.POINTER(Cfg)]
    L.mgemm_config_get.restype = i32
    L.mgemm_config_flags.argtypes = [i32, i32]
    L.mgemm_config_flags.restype = i32
    L.mgemm_choice.argtypes = [i64, i64, i64, i64, i64, i32, ctypes.POINTER(Cfg),
                               ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.mgemm_choice.restype = i32
    L.mgemm_release_workspace.argtypes = []
    L.mgemm_release_workspace.restype = i32
    L.mgemm_probe_mfma.argtypes = [i32, p, p, p, p]
    L.mgemm_probe_mfma.restype = i32
    L.mgemm_probe_mfma_raw.argtypes = [i32, p, p, p, p]
    L.mgemm_probe_mfma_raw.restype = i32
    arr = [i64, p, p, p, p, p, p, p, p, p, p, p, i32]
    L.gemm_batched.argtypes = arr
    L.gemm_batched.restype = i32
    L.gemm_batched_plan_create.argtypes = arr + [p, p, ctypes.POINTER(p)]
    L.gemm_batched_plan_create.restype = i32
    L.gemm_batched_plan_execute.argtypes = [p]
    L.gemm_batched_plan_execute.restype = i32
    L.gemm_batched_plan_destroy.argtypes = [p]
    L.gemm_batched_plan_destroy.restype = i32
    L.gemm_batched_plan_info.argtypes = [p, p, p, p]
    L.gemm_batched_plan_info.restype = i32
    L.mgemm_host_alloc.argtypes = [i64, i32, ctypes.POINTER(p), ctypes.POINTER(p)]
    L.mgemm_host_alloc.restype = i32
    L.mgemm_host_free.argtypes = [p]
    L.mgemm_host_free.restype = i32
    _lib = L
    return L


def last_error() -> str:
    return lib().mgemm_last_error().decode()


def _check(code: int) -> int:
    if code != 0:
        raise MgemmError(code, last_error())
    return code


def _cfg_ptr(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, Cfg):
        return ctypes.pointer(cfg)
    return ctypes.pointer(Cfg(*cfg))


def gemm_raw(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype) -> int:
    """The C ``gemm``; pointers are integers (device addresses).  Returns the code."""
    return lib().gemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype)


def gemm_ex_raw(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, cfg=None, stream=None) -> int:
    return lib().gemm_ex(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, _cfg_ptr(cfg),
                         stream)


def gemm_ex_noalloc_raw(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, cfg=None,
                        stream=None) -> int:
    """The C ``gemm_ex_noalloc`` (no device allocation); returns the code."""
    return lib().gemm_ex_noalloc(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype,
                                 _cfg_ptr(cfg), stream)


class HostBuffer:
    """Pinned host memory mapped for the GPU (mgemm_host_alloc): ``dev`` is the
    address kernels use, ``array`` a numpy view of the host side."""

    def __init__(self, nbytes: int, coherent: bool = True):
        h, d = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().mgemm_host_alloc(int(nbytes), 1 if coherent else 0, ctypes.byref(h),
                                      ctypes.byref(d)))
        self.host, self.dev, self.nbytes = h.value, d.value, int(nbytes)

    def array(self, shape, dtype=np.float64, offset: int = 0) -> np.ndarray:
        """numpy view of ``shape`` elements starting ``offset`` bytes in."""
        dt = np.dtype(dtype)
        count = int(np.prod(shape))
        if offset < 0 or offset + count * dt.itemsize > self.nbytes:
            raise ValueError("view beyond the buffer")
        raw = (ctypes.c_char * (count * dt.itemsize)).from_address(self.host + offset)
        return np.frombuffer(raw, dtype=dt).reshape(shape)

    def free(self) -> None:
        if self.host:
            _check(lib().mgemm_host_free(self.host))
            self.host = self.dev = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def choice(m: int, n: int, k: int, dtype: int = F64, lda: int | None = None,
           ldb: int | None = None, rows: bool = False):
    """(configuration, k ranges) that gemm with no configuration runs for an
    m x n x k product with aligned operands (mgemm_choice); with rows, also the
    rows that run whole (m, 0, or the rows before a split tail)."""
    c = Cfg()
    s = ctypes.c_int32()
    r = ctypes.c_int64()
    _check(lib().mgemm_choice(m, n, k, k if lda is None else lda, n if ldb is None else ldb,
                              dtype, ctypes.byref(c), ctypes.byref(s), ctypes.byref(r)))
    return (c, int(s.value), int(r.value)) if rows else (c, int(s.value))


def configs(dtype: int, need: int = 0) -> list[Cfg]:
    """The registered configurations of dtype, in registry order; with ``need``
    (CFG_BATCHED, CFG_SPLITK bits) only those that take part in all of it."""
    L = lib()
    n = L.mgemm_config_count(dtype)
    if n < 0:
        raise MgemmError(n, "bad dtype")
    out = []
    for i in range(n):
        if need and (L.mgemm_config_flags(dtype, i) & need) != need:
            continue
        c = Cfg()
        _check(L.mgemm_config_get(dtype, i, ctypes.byref(c)))
        out.append(c)
    return out


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ld(t) -> int:
    if t.dim() != 2:
        raise ValueError("2-D tensor expected")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("unit column stride required")
    return max(t.stride(0), 1) if t.shape[0] > 1 else max(t.shape[1], 1)


def dtype_of(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise ValueError(f"unsupported tensor dtype {t.dtype}")


def _check_operands(dtype: int, *ts) -> None:
    """The C ABI takes bare device pointers, so the element type and the device
    are checked here: FP32 needs float32 tensors, every other dtype float64, all
    on the current GPU."""
    import torch
    want = torch.float32 if dtype == F32 else torch.float64
    dev = torch.cuda.current_device() if torch.cuda.is_available() else None
    for t in ts:
        if not isinstance(t, torch.Tensor):
            raise TypeError("torch tensors expected")
        if t.dtype != want:
            raise ValueError(f"{DTYPE_NAMES.get(dtype, dtype)} takes {want} tensors, got {t.dtype}")
    for t in ts:
        if not t.is_cuda or t.device.index != dev:
            raise ValueError("tensors must live on the current GPU")


def gemm(A, B, C, alpha: float = 1.0, beta: float = 0.0, dtype: int | None = None,
         cfg=None, stream=None):
    """C <- alpha*A@B + beta*C on the GPU, in place; returns C.

    A (m x k), B (k x n), C (m x n) are torch tensors on the current device with
    unit column stride (row stride = leading dimension).  ``dtype`` defaults to
    the tensors' type; the emulated dtypes (SPLIT_*, CRT_INT8) take float64 tensors."""
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    if dtype is None:
        dtype = dtype_of(A)
    _check_operands(dtype, A, B, C)
    s = _stream_handle(stream)
    _check(gemm_ex_raw(m, n, k, float(alpha), A.data_ptr(), _ld(A), B.data_ptr(), _ld(B),
                       float(beta), C.data_ptr(), _ld(C), dtype, cfg, s))
    return C


def set_stream(stream) -> None:
    _check(lib().mgemm_set_stream(_stream_handle(stream)))


def release_workspace() -> None:
    _check(lib().mgemm_release_workspace())


def probe_mfma(dtype: int, A, B, D, stream=None) -> None:
    """One matrix-core step (16x4 times 4x16) with the fragment layout the tiled
    kernels assume; D receives the 16x16 product."""
    _check(lib().mgemm_probe_mfma(dtype, A.data_ptr(), B.data_ptr(), D.data_ptr(),
                                  _stream_handle(stream)))


def probe_mfma_raw(kind: int, a, b, d, stream=None) -> None:
    """Raw-register matrix-core step (see mgemm.h): a, b are 64x16-byte device
    tensors, d a 64x16 32-bit device tensor."""
    _check(lib().mgemm_probe_mfma_raw(kind, a.data_ptr(), b.data_ptr(), d.data_ptr(),
                                      _stream_handle(stream)))


class _BatchArrays:
    """Host arrays (kept alive) describing a list of problems."""

    def __init__(self, As, Bs, Cs, alphas, betas):
        import numpy as np
        cnt = len(As)
        self.count = cnt
        self.m = np.array([a.shape[0] for a in As], dtype=np.int64)
        self.k = np.array([a.shape[1] for a in As], dtype=np.int64)
        self.n = np.array([b.shape[1] for b in Bs], dtype=np.int64)
        self.lda = np.array([_ld(a) for a in As], dtype=np.int64)
        self.ldb = np.array([_ld(b) for b in Bs], dtype=np.int64)
        self.ldc = np.array([_ld(c) for c in Cs], dtype=np.int64)
        self.alpha = np.ascontiguousarray(np.broadcast_to(np.asarray(alphas, dtype=np.float64), (cnt,)))
        self.beta = np.ascontiguousarray(np.broadcast_to(np.asarray(betas, dtype=np.float64), (cnt,)))
        self.A = (ctypes.c_void_p * cnt)(*[a.data_ptr() for a in As])
        self.B = (ctypes.c_void_p * cnt)(*[b.data_ptr() for b in Bs])
        self.C = (ctypes.c_void_p * cnt)(*[c.data_ptr() for c in Cs])
        for a, b, c in zip(As, Bs, Cs):
            if a.shape[1] != b.shape[0] or tuple(c.shape) != (a.shape[0], b.shape[1]):
                raise ValueError("shape mismatch in batch")

    def args(self):
        P = lambda x: x.ctypes.data if hasattr(x, "ctypes") else ctypes.cast(x, ctypes.c_void_p).value
        return (self.count, P(self.m), P(self.n), P(self.k), P(self.alpha), P(self.A), P(self.lda),
                P(self.B), P(self.ldb), P(self.beta), P(self.C), P(self.ldc))


def gemm_batched(As, Bs, Cs, alphas=1.0, betas=0.0, dtype=None) -> None:
    """C_i <- alpha_i A_i B_i + beta_i C_i, one library launch per problem."""
    if not As:
        return
    dtype = dtype_of(As[0]) if dtype is None else dtype
    _check_operands(dtype, *As, *Bs, *Cs)
    arrs = _BatchArrays(As, Bs, Cs, alphas, betas)
    _check(lib().gemm_batched(*arrs.args(), dtype))


class BatchedPlan:
    """A captured batched launch (see gemm_batched_plan_create in mgemm.h).
    ``cfgs``: None (library choice) or one Cfg / tuple per problem."""

    def __init__(self, As, Bs, Cs, alphas=1.0, betas=0.0, dtype=None, cfgs=None, stream=None):
        self.handle = ctypes.c_void_p()
        self.dtype = dtype_of(As[0]) if dtype is None and As else (dtype or F64)
        if self.dtype in (F64, F32):
            _check_operands(self.dtype, *As, *Bs, *Cs)
        # the plan reads A, B and writes C at every execution through the raw
        # addresses it keeps, so the tensors themselves are held until destroy():
        # memory the caching allocator reused would otherwise be written
        self._tensors = (list(As), list(Bs), list(Cs))
        self._arrs = _BatchArrays(As, Bs, Cs, alphas, betas)
        cfg_arr = None
        if cfgs is not None:
            cfg_arr = (Cfg * len(cfgs))(*[c if isinstance(c, Cfg) else Cfg(*c) for c in cfgs])
        self._cfgs = cfg_arr
        _check(lib().gemm_batched_plan_create(
            *self._arrs.args(), self.dtype,
            ctypes.cast(cfg_arr, ctypes.c_void_p).value if cfg_arr is not None else None,
            _stream_handle(stream), ctypes.byref(self.handle)))

    def execute(self) -> None:
        _check(lib().gemm_batched_plan_execute(self.handle))

    def info(self):
        b = ctypes.c_int32()
        t = ctypes.c_int64()
        f = ctypes.c_double()
        _check(lib().gemm_batched_plan_info(self.handle, ctypes.byref(b), ctypes.byref(t),
                                            ctypes.byref(f)))
        return {"buckets": b.value, "tiles": t.value, "flops": f.value}

    def destroy(self) -> None:
        if self.handle:
            lib().gemm_batched_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()
        self._tensors = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


MLP_SYMBOLS = ["mlp_create", "mlp_param_count", "mlp_set_params", "mlp_get_params",
               "mlp_set_data", "mlp_loss_grad", "mlp_train", "mlp_forward", "mlp_predict",
               "mlp_destroy", "mlp_save", "mgemm_model_load", "mgemm_model_predict"]
ERR_MODEL = 6
EXPORTED += MLP_SYMBOLS


def _mlp_lib():
    L = lib()
    if getattr(L, "_mlp_ready", False):
        return L
    i64, i32, p, f = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_float
    L.mlp_create.argtypes = [i32, i32, i32, p, ctypes.POINTER(p)]
    L.mlp_param_count.argtypes = [p]
    L.mlp_param_count.restype = i64
    L.mlp_set_params.argtypes = [p, p]
    L.mlp_get_params.argtypes = [p, p]
    L.mlp_set_data.argtypes = [p, i64, p, p, p]
    L.mlp_loss_grad.argtypes = [p, p, p]
    L.mlp_train.argtypes = [p, i32, f, f, f, f, p]
    L.mlp_forward.argtypes = [p, i64, p, p]
    L.mlp_predict.argtypes = [p, i64, p, p, p]
    L.mlp_destroy.argtypes = [p]
    L.mlp_save.argtypes = [p, ctypes.c_char_p, p, p, p, p]
    L.mgemm_model_load.argtypes = [ctypes.c_char_p]
    L.mgemm_model_predict.argtypes = [i64, i64, i64, i32, ctypes.POINTER(Cfg)]
    for n in ("mlp_create", "mlp_set_params", "mlp_get_params", "mlp_set_data", "mlp_loss_grad",
              "mlp_train", "mlp_forward", "mlp_predict", "mlp_destroy", "mlp_save",
              "mgemm_model_load", "mgemm_model_predict"):
        getattr(L, n).restype = i32
    L._mlp_ready = True
    return L


def model_load(path) -> None:
    """Loads a tile-configuration model file (mgemm_model_load); None unloads."""
    _check(_mlp_lib().mgemm_model_load(None if path is None else os.fsencode(path)))


def model_predict(m: int, n: int, k: int, dtype: int = F64) -> Cfg:
    """The loaded model's configuration for an m x n x k product (mgemm_model_predict)."""
    c = Cfg()
    _check(_mlp_lib().mgemm_model_predict(int(m), int(n), int(k), int(dtype), ctypes.byref(c)))
    return c


def mlp_rows_check(name: str, shape: tuple, cols: int, rows: int | None = None) -> None:
    """Raises ValueError unless ``shape`` is (rows, cols) (any rows when None)."""
    if len(shape) != 2 or shape[1] != cols or (rows is not None and shape[0] != rows):
        want = f"({'rows' if rows is None else rows}, {cols})"
        raise ValueError(f"{name} has shape {shape}, expected {want}")


class MLP:
    """The library's FP32 MLP cost model (see mlp_* in mgemm.h).  Parameters are
    exchanged as flat float32 numpy arrays; data as float32 torch tensors."""

    def __init__(self, in_dim: int, hidden: int, out_dim: int, init_params):
        import numpy as np
        L = _mlp_lib()
        self.dims = (in_dim, hidden, out_dim)
        init = np.ascontiguousarray(init_params, dtype=np.float32)
        self.handle = ctypes.c_void_p()
        _check(L.mlp_create(in_dim, hidden, out_dim, init.ctypes.data, ctypes.byref(self.handle)))
        if L.mlp_param_count(self.handle) != init.size:
            raise ValueError("initial parameter vector has the wrong length")

    @property
    def n_params(self) -> int:
        return int(_mlp_lib().mlp_param_count(self.handle))

    def get_params(self):
        import numpy as np
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(_mlp_lib().mlp_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, params) -> None:
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        _check(_mlp_lib().mlp_set_params(self.handle, a.ctypes.data))

    def _device_rows(self, name, t, cols, rows=None):
        """t as a contiguous float32 tensor on the current GPU, checked to be
        rows x cols (rows taken from t when None): the C calls read rows*cols
        floats through a bare device pointer."""
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: torch tensor expected")
        dev = torch.cuda.current_device() if torch.cuda.is_available() else None
        if not t.is_cuda or t.device.index != dev:
            raise ValueError(f"{name} must live on the current GPU")
        mlp_rows_check(name, tuple(t.shape), cols, rows)
        return t.contiguous().float()

    @staticmethod
    def _after_torch():
        """The library's calls run on its own stream: wait for the work torch
        queued (e.g. the conversions above) before they read the tensors."""
        import torch
        torch.cuda.current_stream().synchronize()

    def set_data(self, X, T, M) -> None:
        X = self._device_rows("X", X, self.dims[0])
        T = self._device_rows("T", T, self.dims[2], X.shape[0])
        M = self._device_rows("M", M, self.dims[2], X.shape[0])
        self._data = (X, T, M)
        self._after_torch()
        _check(_mlp_lib().mlp_set_data(self.handle, X.shape[0], X.data_ptr(), T.data_ptr(),
                                       M.data_ptr()))

    def loss_grad(self):
        import numpy as np
        loss = ctypes.c_float()
        g = np.zeros(self.n_params, dtype=np.float32)
        _check(_mlp_lib().mlp_loss_grad(self.handle, ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def train(self, steps: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> float:
        loss = ctypes.c_float()
        _check(_mlp_lib().mlp_train(self.handle, steps, lr, beta1, beta2, eps, ctypes.byref(loss)))
        return loss.value

    def forward(self, X):
        import torch
        X = self._device_rows("X", X, self.dims[0])
        Y = torch.empty((X.shape[0], self.dims[2]), device=X.device, dtype=torch.float32)
        self._after_torch()
        _check(_mlp_lib().mlp_forward(self.handle, X.shape[0], X.data_ptr(), Y.data_ptr()))
        return Y

    def predict(self, X, M):
        import torch
        X = self._device_rows("X", X, self.dims[0])
        M = self._device_rows("M", M, self.dims[2], X.shape[0])
        idx = torch.empty((X.shape[0],), device=X.device, dtype=torch.int32)
        self._after_torch()
        _check(_mlp_lib().mlp_predict(self.handle, X.shape[0], X.data_ptr(), M.data_ptr(),
                                      idx.data_ptr()))
        return idx

    def save(self, path, table, mean, std) -> None:
        """Writes the network as a tile-configuration model file (mlp_save):
        ``table`` lists (dtype, configuration tuple) per output, ``mean`` and
        ``std`` the 6 feature scales."""
        if len(table) != self.dims[2]:
            raise ValueError("one (dtype, configuration) per output expected")
        dts = np.ascontiguousarray([d for d, _ in table], dtype=np.int32)
        cfgs = (Cfg * len(table))(*[Cfg(*c) for _, c in table])
        mu = np.ascontiguousarray(mean, dtype=np.float64)
        sd = np.ascontiguousarray(std, dtype=np.float64)
        if mu.shape != (6,) or sd.shape != (6,):
            raise ValueError("6 feature means and standard deviations expected")
        _check(_mlp_lib().mlp_save(self.handle, os.fsencode(path), dts.ctypes.data,
                                   ctypes.cast(cfgs, ctypes.c_void_p).value, mu.ctypes.data,
                                   sd.ctypes.data))

    def destroy(self) -> None:
        if self.handle:
            _mlp_lib().mlp_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
