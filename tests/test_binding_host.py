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
