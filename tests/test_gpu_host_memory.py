"""GEMM on operands that stay in host memory (pinned, mapped for the GPU: the
zero-copy counterpart of the paper's unified-memory runs, Sec. 3).  The kernels
read A and B and write C over the host link; the result must be bitwise equal to
the same configuration run on device memory and within the FP64 tolerance of the
oracle (normwise 1e-13)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mg.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def host_copy(X, np_dtype, coherent):
    """A HostBuffer holding X (row-major) and its numpy view."""
    hb = mg.HostBuffer(X.size * np.dtype(np_dtype).itemsize, coherent)
    v = hb.array(X.shape, np_dtype)
    v[...] = X
    return hb, v


def run_host(A, B, C, alpha, beta, dtype, cfg, coherent):
    npdt = np.float32 if dtype == mg.F32 else np.float64
    (ha, _), (hb, _), (hc, vc) = (host_copy(X, npdt, coherent) for X in (A, B, C))
    m, k = A.shape
    n = B.shape[1]
    s = torch.cuda.current_stream()
    mg._check(mg.gemm_ex_raw(m, n, k, alpha, ha.dev, k, hb.dev, n, beta, hc.dev, n, dtype, cfg,
                             s.cuda_stream))
    s.synchronize()
    out = vc.astype(np.float64)
    for h in (ha, hb, hc):
        h.free()
    return out


def run_device(dev, A, B, C, alpha, beta, dtype, cfg):
    tdt = torch.float32 if dtype == mg.F32 else torch.float64
    tA, tB, tC = (torch.from_numpy(np.ascontiguousarray(X)).to(dev, tdt) for X in (A, B, C))
    mg.gemm(tA, tB, tC, alpha, beta, dtype=dtype, cfg=cfg)
    torch.cuda.synchronize()
    return tC.cpu().double().numpy()


CASES = [
    # (m, n, k, dtype, cfg): the default choice, the three-stage direct-load kernel
    # (16-byte loads from host memory), FP32, and the int8 slice path
    (300, 257, 190, mg.F64, None),
    (512, 256, 96, mg.F64, (256, 128, 16, 8, 2, 2, 2)),
    (200, 130, 77, mg.F32, None),
    (128, 96, 200, mg.SPLIT_INT8, None),
]


@pytest.mark.parametrize("coherent", [True, False])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_host_mapped_operands(dev, orc, case, coherent):
    m, n, k, dtype, cfg = CASES[case]
    say(f"host memory: m={m} n={n} k={k} dtype={dtype} cfg={cfg} coherent={coherent}")
    seed = 9100 + 10 * case
    if dtype == mg.SPLIT_INT8:
        A, B = synth.wide_range((m, k), seed), synth.wide_range((k, n), seed + 1)
    else:
        A, B = synth.uniform_pm1((m, k), seed), synth.uniform_pm1((k, n), seed + 1)
    C = synth.uniform_pm1((m, n), seed + 2)
    if dtype == mg.F32:
        A, B, C = (X.astype(np.float32).astype(np.float64) for X in (A, B, C))
    alpha, beta = 1.5, 0.5
    got = run_host(A, B, C, alpha, beta, dtype, cfg, coherent)
    ref_dev = run_device(dev, A, B, C, alpha, beta, dtype, cfg)
    assert np.array_equal(got, ref_dev)
    ref = orc.gemm_f64(alpha, A, B, beta, C)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    tol = 1e-6 if dtype == mg.F32 else 1e-13
    say(f"  normwise error {err:.2e} (tol {tol:.0e})")
    assert err <= tol
