"""GPU parity of the modular-integer (Ozaki scheme II) emulated FP64 GEMM through
the C ABI.

The GPU path recovers the exact product of the truncated operands from its
residues and rounds once, which is exactly the oracle's definition, so results
are compared BITWISE with the oracle on the same inputs (including k beyond
2^16, where the products run in passes whose residues are added modulo p).
Accuracy against the double-double oracle: normwise relative error <= 1e-14 on
the wide-range stress inputs."""
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


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def gpu_crt(dev, A, B, C, alpha, beta):
    tA, tB, tC = to_dev(A, dev), to_dev(B, dev), to_dev(C, dev)
    mg.gemm(tA, tB, tC, alpha, beta, dtype=mg.CRT_INT8)
    torch.cuda.synchronize()
    return tC.cpu().numpy()


def assert_bitwise(got, want, what):
    bad = np.argwhere(got != want)
    assert bad.size == 0, (what, bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])


SHAPES = [(1, 1, 1), (3, 5, 7), (64, 64, 64), (255, 257, 65), (256, 256, 256),
          (300, 200, 517), (5, 700, 2), (513, 130, 1000), (31, 300, 17)]


def test_bitwise_equal_to_oracle(dev, orc):
    for (m, n, k) in SHAPES:
        say(f"crt shape={(m, n, k)}")
        A = synth.wide_range((m, k), 100 + m)
        B = synth.wide_range((k, n), 200 + n)
        C = synth.uniform_pm1((m, n), 300 + k)
        got = gpu_crt(dev, A, B, C, 1.5, 0.5)
        want = orc.crt_gemm(1.5, A, B, 0.5, C, nthreads=8)
        assert_bitwise(got, want, (m, n, k))


def test_uniform_and_zero_rows_columns(dev, orc):
    m, n, k = 200, 300, 250
    say(f"crt uniform with zero rows/columns {(m, n, k)}")
    A = synth.uniform_pm1((m, k), 11)
    B = synth.uniform_pm1((k, n), 12)
    A[7, :] = 0.0
    B[:, 13] = 0.0
    C = synth.uniform_pm1((m, n), 13)
    got = gpu_crt(dev, A, B, C, 1.0, 0.0)
    assert_bitwise(got, orc.crt_gemm(1.0, A, B, 0.0, C, nthreads=8), "uniform")
    assert np.all(got[7] == 0.0) and np.all(got[:, 13] == 0.0)


def test_integer_inputs_exact(dev):
    m, n, k = 129, 70, 300
    say("crt integer inputs")
    A = synth.integer_valued((m, k), 21, 1 << 20)
    B = synth.integer_valued((k, n), 22, 1 << 20)
    C = synth.integer_valued((m, n), 23, 1000)
    want = 3 * (A.astype(np.int64) @ B.astype(np.int64)) - 2 * C.astype(np.int64)
    got = gpu_crt(dev, A, B, C, 3.0, -2.0)
    assert np.array_equal(got, want.astype(np.float64))


def test_k_beyond_reduction_period(dev, orc):
    """k = 70000 > 2^16: the product runs in two passes (int32 sums stay exact),
    the second adding its residues to the first's modulo p; the result is exact."""
    m, n, k = 40, 72, 70000
    say(f"crt long k {(m, n, k)}")
    A = synth.wide_range((m, k), 31)
    B = synth.wide_range((k, n), 32)
    C = synth.uniform_pm1((m, n), 33)
    got = gpu_crt(dev, A, B, C, 1.0, 1.0)
    assert_bitwise(got, orc.crt_gemm(1.0, A, B, 1.0, C, nthreads=orc.num_procs()), "long k")


def test_wide_range_1024_meets_1e14(dev, orc):
    n = 1024
    say(f"crt wide-range n={n}")
    sa, sb, _ = synth.seeds_for(2, 10)
    A = synth.wide_range((n, n), sa)
    B = synth.wide_range((n, n), sb)
    got = gpu_crt(dev, A, B, np.zeros((n, n)), 1.0, 0.0)
    ref = orc.gemm_dot2(1.0, A, B, nthreads=orc.num_procs())
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"  normwise error vs dot2 {err:.3e}")
    assert err <= 1e-14
    assert_bitwise(got, orc.crt_gemm(1.0, A, B, nthreads=orc.num_procs()), "n=1024")


def test_nonfinite_quick_returns_and_cfg(dev):
    say("crt non-finite / quick returns / cfg")
    A = synth.uniform_pm1((8, 9), 1)
    B = synth.uniform_pm1((9, 10), 2)
    C = synth.uniform_pm1((8, 10), 3)
    tA, tB, tC = to_dev(A, dev), to_dev(B, dev), to_dev(C, dev)
    bad = tA.clone()
    bad[2, 3] = float("inf")
    rc = mg.gemm_ex_raw(8, 10, 9, 1.0, bad.data_ptr(), 9, tB.data_ptr(), 10, 0.5, tC.data_ptr(),
                        10, mg.CRT_INT8)
    torch.cuda.synchronize()
    assert rc == 3 and np.array_equal(tC.cpu().numpy(), C)
    rc = mg.gemm_ex_raw(8, 10, 9, 0.0, tA.data_ptr(), 9, tB.data_ptr(), 10, 2.0, tC.data_ptr(),
                        10, mg.CRT_INT8)
    torch.cuda.synchronize()
    assert rc == 0 and np.array_equal(tC.cpu().numpy(), 2.0 * C)
    cfg = mg.configs(mg.F64)[0]
    rc = mg.gemm_ex_raw(8, 10, 9, 1.0, tA.data_ptr(), 9, tB.data_ptr(), 10, 0.0, tC.data_ptr(),
                        10, mg.CRT_INT8, cfg)
    assert rc == -13


def test_deterministic(dev):
    n = 700
    say("crt determinism")
    A = to_dev(synth.wide_range((n, n), 41), dev)
    B = to_dev(synth.wide_range((n, n), 42), dev)
    outs = []
    for _ in range(2):
        C = torch.zeros((n, n), dtype=torch.float64, device=dev)
        mg.gemm(A, B, C, 1.0, 0.0, dtype=mg.CRT_INT8)
        outs.append(C)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("n", [4096, 8192])
def test_full_size_sampled_rows(dev, orc, n):
    """N = 4096 and 8192 wide-range (the split-precision benchmark workload): sampled
    rows recomputed by the oracle, bitwise."""
    say(f"crt full size n={n}: generating inputs")
    sa, sb, _ = synth.seeds_for(3, int(np.log2(n)))
    A = synth.wide_range((n, n), sa)
    B = synth.wide_range((n, n), sb)
    tA, tB = to_dev(A, dev), to_dev(B, dev)
    tC = torch.zeros((n, n), dtype=torch.float64, device=dev)
    say("  gemm")
    mg.gemm(tA, tB, tC, 1.0, 0.0, dtype=mg.CRT_INT8)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([synth.log_uniform_int(14, 9, 1, n) - 1, [0, n - 1]]))
    got = tC[torch.from_numpy(rows).to(dev)].cpu().numpy()
    say(f"  oracle on {len(rows)} rows")
    # the row exponents of A are per row, the column exponents of B need all of B:
    # the oracle run on the sampled rows of A with the whole of B is the same product
    want = orc.crt_gemm(1.0, A[rows], B, nthreads=orc.num_procs())
    assert_bitwise(got, want, "n=8192 rows")


def test_extreme_exponents(dev, orc):
    """Products that underflow to subnormals and overflow to infinity: the single
    rounding and the power-of-two scaling follow the oracle bit for bit (the GPU
    keeps FP64 subnormals)."""
    m, n, k = 37, 45, 29
    say("crt extreme exponents")
    base_a = synth.uniform_pm1((m, k), 51)
    base_b = synth.uniform_pm1((k, n), 52)
    for ea, eb in ((-1000, -60), (-520, -500), (-1040, -20), (600, 423), (1000, 22)):
        A = np.ldexp(base_a, ea)
        B = np.ldexp(base_b, eb)
        got = gpu_crt(dev, A, B, np.zeros((m, n)), 1.0, 0.0)
        with np.errstate(over="ignore"):
            want = orc.crt_gemm(1.0, A, B)
        assert_bitwise(got, want, (ea, eb))
