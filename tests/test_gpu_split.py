"""GPU parity of the split-precision (Ozaki) emulated FP64 GEMM through the C ABI.

The GPU path sums the kept slice-pair products exactly and rounds once, like the
oracle's split model, so for k within one pass (131072 bf16 and FP8 / 16384 int8) the
results are compared BITWISE with the oracle on the same inputs; beyond that each
pass rounds once and the comparison is normwise.  Accuracy against the
double-double oracle: normwise relative error <= 1e-14 on the wide-range stress
inputs (entries u*2^e, e uniform in [-20, 20])."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402

FMT = {mg.SPLIT_BF16: (0, 6), mg.SPLIT_FP8: (1, 11), mg.SPLIT_INT8: (2, 8)}
DTYPES = [mg.SPLIT_BF16, mg.SPLIT_FP8, mg.SPLIT_INT8]


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


def gpu_split(dev, A, B, C, alpha, beta, dtype):
    tA = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    tB = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    tC = torch.from_numpy(np.ascontiguousarray(C)).to(dev)
    mg.gemm(tA, tB, tC, alpha, beta, dtype=dtype)
    torch.cuda.synchronize()
    return tC.cpu().numpy()


SHAPES = [(1, 1, 1), (3, 5, 7), (64, 128, 64), (65, 129, 65), (100, 77, 300), (257, 131, 1000),
          (31, 300, 17), (128, 256, 2048)]


@pytest.mark.parametrize("dtype", DTYPES)
def test_bitwise_equal_to_oracle_split_model(dev, orc, dtype):
    fmt, S = FMT[dtype]
    for (m, n, k) in SHAPES:
        say(f"split {mg.DTYPE_NAMES[dtype]} shape={(m, n, k)}")
        A = synth.wide_range((m, k), 100 + m)
        B = synth.wide_range((k, n), 200 + n)
        C = synth.uniform_pm1((m, n), 300 + k)
        got = gpu_split(dev, A, B, C, 1.5, 0.5, dtype)
        want = orc.split_gemm(1.5, A, B, 0.5, C, fmt=fmt, S=S, nthreads=8)
        bad = np.argwhere(got != want)
        assert bad.size == 0, (m, n, k, bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])


@pytest.mark.parametrize("dtype", DTYPES)
def test_wide_range_1024_meets_1e14(dev, orc, dtype):
    """The split-precision stress distribution at N = 1024 (alpha = 1, beta = 0):
    normwise error against the double-double oracle <= 1e-14, and bitwise equal
    to the oracle's split model."""
    fmt, S = FMT[dtype]
    n = 1024
    say(f"split {mg.DTYPE_NAMES[dtype]} wide-range n={n}")
    sa, sb, sc = synth.seeds_for(2, 10)
    A = synth.wide_range((n, n), sa)
    B = synth.wide_range((n, n), sb)
    got = gpu_split(dev, A, B, np.zeros((n, n)), 1.0, 0.0, dtype)
    ref = orc.gemm_dot2(1.0, A, B, nthreads=orc.num_procs())
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"  normwise err vs dot2 {err:.3e}")
    assert err <= 1e-14
    want = orc.split_gemm(1.0, A, B, fmt=fmt, S=S, nthreads=orc.num_procs())
    assert np.array_equal(got, want)


def test_fp8_level_flushes(dev, orc):
    """k = 10000: 157 FP8 chunks of 64, so the FP32 level sums are flushed into the
    exact FP64 sums twice before the final flush; bitwise equal to the oracle's
    split model."""
    m, n, k = 70, 90, 10000
    say(f"split fp8 flush periods k={k}")
    A = synth.wide_range((m, k), 4)
    B = synth.wide_range((k, n), 5)
    C = synth.uniform_pm1((m, n), 6)
    got = gpu_split(dev, A, B, C, 0.75, -1.25, mg.SPLIT_FP8)
    want = orc.split_gemm(0.75, A, B, -1.25, C, fmt=1, S=11, nthreads=orc.num_procs())
    assert np.array_equal(got, want)


def test_int8_multi_pass_k(dev, orc):
    """k = 20000 > 16384: two int8 passes, each rounded once."""
    m, n, k = 40, 48, 20000
    say(f"split int8 multi-pass k={k}")
    A = synth.wide_range((m, k), 1)
    B = synth.wide_range((k, n), 2)
    C = synth.uniform_pm1((m, n), 3)
    got = gpu_split(dev, A, B, C, 1.0, 0.25, mg.SPLIT_INT8)
    ref = orc.gemm_dot2(1.0, A, B, 0.25, C, nthreads=8)
    model = orc.split_gemm(1.0, A, B, 0.25, C, fmt=2, S=8, nthreads=8)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
    assert np.linalg.norm(got - model) <= 4e-16 * np.linalg.norm(model)


@pytest.mark.parametrize("dtype", DTYPES)
def test_nonfinite_inputs_rejected_and_C_untouched(dev, dtype):
    say(f"split {mg.DTYPE_NAMES[dtype]} non-finite")
    m, n, k = 50, 40, 30
    for where, val in (("A", np.nan), ("B", np.inf), ("A", -np.inf)):
        A = synth.uniform_pm1((m, k), 1)
        B = synth.uniform_pm1((k, n), 2)
        (A if where == "A" else B)[7, 3] = val
        tA = torch.from_numpy(A).to(dev)
        tB = torch.from_numpy(B).to(dev)
        tC = torch.full((m, n), 5.0, device=dev, dtype=torch.float64)
        with pytest.raises(mg.MgemmError) as ei:
            mg.gemm(tA, tB, tC, 1.0, 1.0, dtype=dtype)
        assert ei.value.code == mg.ERR_NONFINITE
        torch.cuda.synchronize()
        assert torch.all(tC == 5.0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_zero_rows_columns_and_quick_returns(dev, orc, dtype):
    fmt, S = FMT[dtype]
    say(f"split {mg.DTYPE_NAMES[dtype]} zeros / quick returns")
    m, n, k = 70, 90, 50
    A = synth.uniform_pm1((m, k), 4)
    B = synth.uniform_pm1((k, n), 5)
    A[3] = 0.0
    B[:, 11] = 0.0
    Cn = np.full((m, n), np.nan)
    got = gpu_split(dev, A, B, Cn, 2.0, 0.0, dtype)
    want = orc.split_gemm(2.0, A, B, fmt=fmt, S=S)
    assert np.array_equal(got, want)
    assert np.all(got[3] == 0.0) and np.all(got[:, 11] == 0.0)
    C = synth.uniform_pm1((m, n), 6)
    assert np.array_equal(gpu_split(dev, A, B, C, 0.0, 0.5, dtype), 0.5 * C)


def test_split_rejects_a_tile_configuration(dev):
    t = torch.zeros((4, 4), device=dev, dtype=torch.float64)
    with pytest.raises(mg.MgemmError) as ei:
        mg.gemm(t, t.clone(), t.clone(), 1.0, 0.0, dtype=mg.SPLIT_BF16, cfg=mg.configs(mg.F64)[0])
    assert ei.value.code == -13


@pytest.mark.parametrize("dtype", DTYPES)
def test_deterministic_and_workspace_release(dev, dtype):
    say(f"split {mg.DTYPE_NAMES[dtype]} determinism")
    n = 512
    A = torch.from_numpy(synth.wide_range((n, n), 8)).to(dev)
    B = torch.from_numpy(synth.wide_range((n, n), 9)).to(dev)
    C1 = torch.zeros((n, n), device=dev, dtype=torch.float64)
    C2 = torch.zeros((n, n), device=dev, dtype=torch.float64)
    mg.gemm(A, B, C1, 1.0, 0.0, dtype=dtype)
    mg.release_workspace()
    mg.gemm(A, B, C2, 1.0, 0.0, dtype=dtype)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("n", [4096, 8192])
@pytest.mark.parametrize("dtype", DTYPES)
def test_full_size_sampled_rows(dev, orc, dtype, n):
    """The split-precision workload sizes N = 4096 and 8192 (wide-range inputs):
    6 sampled rows recomputed by the oracle's split model, bitwise."""
    fmt, S = FMT[dtype]
    say(f"split {mg.DTYPE_NAMES[dtype]} n={n}: inputs")
    sa, sb, _ = synth.seeds_for(2, int(np.log2(n)))
    A = synth.wide_range((n, n), sa)
    B = synth.wide_range((n, n), sb)
    got = gpu_split(dev, A, B, np.zeros((n, n)), 1.0, 0.0, dtype)
    rows = np.array([0, 1, 777, n // 2, n - 1095, n - 1])
    say(f"  oracle split model on {len(rows)} rows")
    want = orc.split_gemm(1.0, A[rows], B, fmt=fmt, S=S, nthreads=orc.num_procs())
    assert np.array_equal(got[rows], want)


@pytest.mark.parametrize("dtype", DTYPES)
def test_extreme_exponents(dev, orc, dtype):
    """Products that underflow to subnormals or overflow: the one rounding of the
    exact level sum and the power-of-two scaling follow the oracle bit for bit."""
    fmt, S = FMT[dtype]
    m, n, k = 37, 45, 29
    base_a = synth.uniform_pm1((m, k), 51)
    base_b = synth.uniform_pm1((k, n), 52)
    for ea, eb in ((-1000, -60), (-520, -500), (-1040, -20), (600, 423), (1000, 22)):
        say(f"split {mg.DTYPE_NAMES[dtype]} exponents {(ea, eb)}")
        A = np.ldexp(base_a, ea)
        B = np.ldexp(base_b, eb)
        got = gpu_split(dev, A, B, np.zeros((m, n)), 1.0, 0.0, dtype)
        with np.errstate(over="ignore"):
            want = orc.split_gemm(1.0, A, B, fmt=fmt, S=S)
        bad = np.argwhere(got != want)
        assert bad.size == 0, (ea, eb, bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])


def test_bf16_operands_beyond_4gib(dev, orc):
    """bf16 slices of A beyond 4 GiB (m = 16384, k = 24576: 12 bytes per element)
    take the register-staged pair kernel with 64-bit addresses: sampled rows
    bitwise equal to the oracle's split model.  int8 slices beyond 4 GiB are
    refused with MGEMM_ERR_NOCONFIG before any operand is read, and so are FP8
    slices beyond 4 GiB."""
    m, n, k = 16384, 256, 24576
    say(f"split bf16 beyond 4 GiB: {(m, n, k)}, inputs on the device")
    g = torch.Generator(device=dev)
    g.manual_seed(61)
    u = torch.rand((m, k), device=dev, dtype=torch.float64, generator=g) * 2 - 1
    e = torch.randint(-20, 21, (m, k), device=dev, generator=g)
    tA = torch.ldexp(u, e)
    del u, e
    B = synth.wide_range((k, n), 62)
    tB = torch.from_numpy(B).to(dev)
    tC = torch.zeros((m, n), device=dev, dtype=torch.float64)
    mg.gemm(tA, tB, tC, 1.0, 0.0, dtype=mg.SPLIT_BF16)
    torch.cuda.synchronize()
    rows = torch.tensor([0, 1, 4095, 8191, 12000, m - 1], device=dev)
    got = tC[rows].cpu().numpy()
    say("  oracle split model on sampled rows")
    fmt, S = FMT[mg.SPLIT_BF16]
    want = orc.split_gemm(1.0, tA[rows].cpu().numpy(), B, fmt=fmt, S=S, nthreads=orc.num_procs())
    assert np.array_equal(got, want)
    del tA, tB, tC
    mg.release_workspace()
    torch.cuda.empty_cache()
    # int8: 16384 x 32768 x 8 slices = 2^32 bytes
    t = torch.empty((16384, 32768), device=dev, dtype=torch.float64)
    b = torch.zeros((32768, 8), device=dev, dtype=torch.float64)
    c = torch.zeros((16384, 8), device=dev, dtype=torch.float64)
    with pytest.raises(mg.MgemmError) as ei:
        mg.gemm(t, b, c, 1.0, 0.0, dtype=mg.SPLIT_INT8)
    assert ei.value.code == mg.ERR_NOCONFIG
    # FP8: 11 slices of one byte
    with pytest.raises(mg.MgemmError) as ei:
        mg.gemm(t, b, c, 1.0, 0.0, dtype=mg.SPLIT_FP8)
    assert ei.value.code == mg.ERR_NOCONFIG
    del t, b, c
    torch.cuda.empty_cache()
