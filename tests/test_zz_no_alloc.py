"""gemm_ex_noalloc through the C ABI against gemm_ex: two calls in a row on the
same GPU (the second with a smaller problem, so the shared scratch array holds the
first call's partial products when it starts), each bitwise equal to gemm_ex on
the same inputs (same configuration and split of k) and within the oracle's
tolerance (FP64 normwise <= 1e-13; FP32 every element within gamma_{k+2})."""
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


def gamma(n, u):
    return n * u / (1 - n * u)


def call(fn, tA, tB, tC, alpha, beta, dtype, cfg=None):
    m, k = tA.shape
    n = tB.shape[1]
    rc = fn(m, n, k, alpha, tA.data_ptr(), tA.stride(0), tB.data_ptr(), tB.stride(0), beta,
            tC.data_ptr(), tC.stride(0), dtype, cfg, torch.cuda.current_stream().cuda_stream)
    assert rc == 0, mg.last_error()


# (m, n, k): the first two split k (on the three-stage tile in both dtypes, and
# on the two-stage tile in FP64), the third is too large to split, the fourth has
# odd rows and a short k (the measured configuration, run whole)
CASES = [(1024, 512, 4096), (384, 256, 3000), (2048, 2048, 512), (333, 271, 1517)]


@pytest.mark.parametrize("dtype", [mg.F64, mg.F32])
@pytest.mark.parametrize("first,second", [(0, 1), (2, 3), (0, 3)])
def test_noalloc_matches_gemm_ex_twice(dev, dtype, first, second):
    import oracle
    tdt = torch.float64 if dtype == mg.F64 else torch.float32
    for step, ci in enumerate((first, second)):
        m, n, k = CASES[ci]
        say(f"noalloc dtype={mg.DTYPE_NAMES[dtype]} call {step + 1}: {(m, n, k)}")
        A = synth.uniform_pm1((m, k), 300 + ci)
        B = synth.uniform_pm1((k, n), 310 + ci)
        C = synth.uniform_pm1((m, n), 320 + ci)
        if dtype == mg.F32:
            A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
        tA, tB, tC = (torch.from_numpy(x).to(dev, tdt) for x in (A, B, C))
        ref_c = tC.clone()
        call(mg.gemm_ex_noalloc_raw, tA, tB, tC, 1.25, -0.5, dtype)
        call(mg.gemm_ex_raw, tA, tB, ref_c, 1.25, -0.5, dtype)
        torch.cuda.synchronize()
        assert torch.equal(tC, ref_c), (m, n, k)
        got = tC.cpu().double().numpy()
        want = oracle.gemm_f64(1.25, A, B, -0.5, C, nthreads=oracle.num_procs())
        if dtype == mg.F64:
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            assert err <= 1e-13, err
        else:
            bound = (gamma(k + 2, 2.0 ** -24) + gamma(k + 2, 2.0 ** -53)) * \
                (1.25 * (np.abs(A) @ np.abs(B)) + 0.5 * np.abs(C))
            assert np.all(np.abs(got - want) <= bound)


def test_noalloc_explicit_config_and_quick_returns(dev):
    """A named configuration runs as in gemm_ex; alpha = 0 scales C; the emulated
    dtypes are refused with -12."""
    m, n, k = 200, 130, 77
    A = synth.uniform_pm1((m, k), 41)
    B = synth.uniform_pm1((k, n), 42)
    C = synth.uniform_pm1((m, n), 43)
    tA, tB, tC = (torch.from_numpy(x).to(dev) for x in (A, B, C))
    for cfg in mg.configs(mg.F64)[:6]:
        say(f"noalloc cfg={cfg}")
        c1, c2 = tC.clone(), tC.clone()
        call(mg.gemm_ex_noalloc_raw, tA, tB, c1, 1.0, 1.0, mg.F64, cfg)
        call(mg.gemm_ex_raw, tA, tB, c2, 1.0, 1.0, mg.F64, cfg)
        torch.cuda.synchronize()
        assert torch.equal(c1, c2), cfg
    c1 = tC.clone()
    call(mg.gemm_ex_noalloc_raw, tA, tB, c1, 0.0, 2.0, mg.F64)
    torch.cuda.synchronize()
    assert np.array_equal(c1.cpu().numpy(), 2.0 * C)
    rc = mg.gemm_ex_noalloc_raw(m, n, k, 1.0, tA.data_ptr(), k, tB.data_ptr(), n, 0.0,
                                c1.data_ptr(), n, mg.SPLIT_BF16)
    assert rc == -12
