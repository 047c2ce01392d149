"""Argument checks of the Python binding that run before any library call: the C
ABI takes bare device pointers, so tensors of the wrong element type or on the
host must be refused here."""
import pytest

torch = pytest.importorskip("torch")

import paper_1706_10086_amd as mg  # noqa: E402


def test_host_tensors_refused():
    A = torch.zeros((4, 3), dtype=torch.float64)
    B = torch.zeros((3, 5), dtype=torch.float64)
    C = torch.zeros((4, 5), dtype=torch.float64)
    with pytest.raises(ValueError, match="current GPU"):
        mg.gemm(A, B, C)
    with pytest.raises(ValueError, match="current GPU"):
        mg.gemm_batched([A], [B], [C])
    with pytest.raises(ValueError, match="current GPU"):
        mg.BatchedPlan([A], [B], [C])


def test_element_type_must_match_dtype():
    A32 = torch.zeros((4, 3), dtype=torch.float32)
    B32 = torch.zeros((3, 5), dtype=torch.float32)
    C32 = torch.zeros((4, 5), dtype=torch.float32)
    for dt in (mg.F64, mg.SPLIT_BF16, mg.SPLIT_INT8, mg.CRT_INT8):
        with pytest.raises(ValueError, match="takes torch.float64"):
            mg.gemm(A32, B32, C32, dtype=dt)
    C64 = torch.zeros((4, 5), dtype=torch.float64)
    with pytest.raises(ValueError, match="takes torch.float32"):
        mg.gemm(A32, B32, C64)
    with pytest.raises(ValueError, match="shape mismatch"):
        mg.gemm(A32, A32, C32)
    with pytest.raises(TypeError):
        mg.gemm_batched([A32], [B32], ["not a tensor"], dtype=mg.F32)


class _FakeLib:
    """Stands in for libmgemm.so: plan creation succeeds and hands out a handle
    without touching a device."""

    def gemm_batched_plan_create(self, *args):
        args[-1]._obj.value = 1234
        return 0

    def gemm_batched_plan_destroy(self, handle):
        return 0


def test_batched_plan_holds_its_tensors(monkeypatch):
    """A plan keeps raw addresses of A, B and C; the binding must hold the tensors
    until destroy(), or freed memory would be written by later executions."""
    import gc
    import weakref
    monkeypatch.setattr(mg, "lib", lambda: _FakeLib())
    monkeypatch.setattr(mg, "_check_operands", lambda *a, **k: None)
    As = [torch.zeros((4, 3), dtype=torch.float64)]
    Bs = [torch.zeros((3, 5), dtype=torch.float64)]
    Cs = [torch.zeros((4, 5), dtype=torch.float64)]
    refs = [weakref.ref(t) for t in As + Bs + Cs]
    plan = mg.BatchedPlan(As, Bs, Cs, stream=0)
    del As, Bs, Cs
    gc.collect()
    assert all(r() is not None for r in refs)
    plan.destroy()
    gc.collect()
    assert all(r() is None for r in refs)


def _mlp_without_device(dims=(6, 8, 5)):
    m = mg.MLP.__new__(mg.MLP)
    m.dims = dims
    m.handle = None
    return m


def test_mlp_refuses_host_or_misshapen_data():
    net = _mlp_without_device()
    X = torch.zeros((10, 6))
    T = torch.zeros((10, 5))
    with pytest.raises(ValueError, match="current GPU"):
        net.set_data(X, T, T)
    with pytest.raises(ValueError, match="current GPU"):
        net.forward(X)
    with pytest.raises(ValueError, match="current GPU"):
        net.predict(X, T)
    with pytest.raises(TypeError):
        net.set_data("X", T, T)


def test_mlp_shape_rules():
    mg.mlp_rows_check("X", (10, 6), 6)
    mg.mlp_rows_check("T", (10, 5), 5, 10)
    with pytest.raises(ValueError, match=r"expected \(rows, 6\)"):
        mg.mlp_rows_check("X", (10, 7), 6)
    with pytest.raises(ValueError, match=r"expected \(10, 5\)"):
        mg.mlp_rows_check("T", (9, 5), 5, 10)
    with pytest.raises(ValueError, match=r"expected \(10, 5\)"):
        mg.mlp_rows_check("M", (10, 4), 5, 10)
    with pytest.raises(ValueError):
        mg.mlp_rows_check("X", (60,), 6)
