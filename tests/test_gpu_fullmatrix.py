"""Full-matrix parity of the square workloads, through the C ABI, with the
default configuration choice (the kernels the sweep and the headline time).

* FP64, N = 1024, 2048, 4096, 8192, entries uniform[-1,1], alpha = beta = 1 (the
  square sweep's recipe): every element against the FP64 oracle (Eq. 1 written
  out); normwise relative error <= 1e-13 and every element within
  gamma_{k+2} (|A||B| + |C|) of the oracle, widened by the oracle's own bound
  (Higham, Sec. 3.5).
* FP32, N = 1024 and 4096, the same recipe on float inputs: every element within
  gamma_{k+2} with u = 2^-24 of the FP64 oracle on the same float values (plus
  the oracle's own FP64 bound).
* Squares whose tile the round-fill rule picks (FP64 N = 2048, every element; FP64
  and FP32 N = 6144, 256 rows), within the same gamma_{k+2} bounds.
* Emulated FP64 on the wide-range stress inputs (entries u * 2^e, e uniform in
  [-20, 20]): at N = 4096 every element, at N = 8192 256 sampled rows, against
  the double-double (Dot2) oracle, normwise <= 1e-14 for every emulation, and
  against the plain FP64 oracle (<= 1e-13, the plain path's tolerance: the
  plain oracle's own error is of the same size as the emulations')."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402

EMULATIONS = [mg.SPLIT_BF16, mg.SPLIT_FP8, mg.SPLIT_INT8, mg.CRT_INT8]


def say(*a):
    print(*a, flush=True)


def gamma(n, u):
    return n * u / (1 - n * u)


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


def nrm(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("n", [1024, 2048, 4096, 8192])
def test_fp64_square_full_matrix(dev, orc, n):
    say(f"full matrix fp64 n={n}: inputs")
    sa, sb, sc = synth.seeds_for(1, int(np.log2(n)))
    A, B, C = (synth.uniform_pm1((n, n), s) for s in (sa, sb, sc))
    tA, tB, tC = (torch.from_numpy(X).to(dev) for X in (A, B, C))
    mg.gemm(tA, tB, tC, 1.0, 1.0)
    torch.cuda.synchronize()
    got = tC.cpu().numpy()
    del tA, tB, tC
    say(f"  oracle, all {n} rows")
    ref = orc.gemm_f64(1.0, A, B, 1.0, C, nthreads=orc.num_procs())
    err = nrm(got, ref)
    say(f"  normwise error {err:.3e}")
    assert err <= 1e-13
    # both results lie within gamma_{k+2}(|A||B| + |C|) of the exact product
    mag = np.abs(A) @ np.abs(B)
    mag += np.abs(C)
    bound = 2 * gamma(n + 2, 2.0 ** -53) * mag
    worst = float(np.max(np.abs(got - ref) / bound))
    say(f"  worst element / bound {worst:.3e}")
    assert worst <= 1.0


@pytest.mark.parametrize("n", [1024, 4096])
def test_fp32_square_full_matrix(dev, orc, n):
    say(f"full matrix fp32 n={n}: inputs")
    sa, sb, sc = synth.seeds_for(1, int(np.log2(n)))
    A, B, C = (synth.uniform_pm1((n, n), s).astype(np.float32) for s in (sa, sb, sc))
    tA, tB, tC = (torch.from_numpy(X).to(dev) for X in (A, B, C))
    mg.gemm(tA, tB, tC, 1.0, 1.0)
    torch.cuda.synchronize()
    got = tC.cpu().double().numpy()
    del tA, tB, tC
    A, B, C = (X.astype(np.float64) for X in (A, B, C))
    say(f"  oracle, all {n} rows")
    ref = orc.gemm_f64(1.0, A, B, 1.0, C, nthreads=orc.num_procs())
    mag = np.abs(A) @ np.abs(B)
    mag += np.abs(C)
    bound = (gamma(n + 2, 2.0 ** -24) + gamma(n + 2, 2.0 ** -53)) * mag
    worst = float(np.max(np.abs(got - ref) / bound))
    say(f"  worst element / bound {worst:.3e}, normwise {nrm(got, ref):.3e}")
    assert worst <= 1.0


@pytest.fixture(scope="module")
def stress(orc):
    """Wide-range inputs at N = 4096 (all rows) and 8192 (256 sampled rows) with
    both oracles' results."""
    out = {}
    for n, count in ((4096, None), (8192, 256)):
        sa, sb, _ = synth.seeds_for(2, int(np.log2(n)))
        say(f"stress n={n}: inputs")
        A = synth.wide_range((n, n), sa)
        B = synth.wide_range((n, n), sb)
        # every row, or count rows spread evenly over the matrix (first and last included)
        rows = np.arange(n) if count is None else np.linspace(0, n - 1, count).astype(np.int64)
        say(f"  Dot2 and FP64 oracles on {len(rows)} rows")
        d2 = orc.gemm_dot2(1.0, A[rows], B, nthreads=orc.num_procs())
        f64 = orc.gemm_f64(1.0, A[rows], B, nthreads=orc.num_procs())
        out[n] = (A, B, rows, d2, f64)
    return out


@pytest.mark.parametrize("n", [4096, 8192])
@pytest.mark.parametrize("dtype", [mg.F64] + EMULATIONS)
def test_stress_inputs_against_both_oracles(dev, stress, dtype, n):
    A, B, rows, d2, f64 = stress[n]
    assert len(rows) == (n if n == 4096 else 256)
    tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    tC = torch.zeros((n, n), device=dev, dtype=torch.float64)
    say(f"stress {mg.DTYPE_NAMES[dtype]} n={n}")
    mg.gemm(tA, tB, tC, 1.0, 0.0, dtype=dtype)
    torch.cuda.synchronize()
    got = tC[torch.from_numpy(rows).to(dev)].cpu().numpy()
    del tA, tB, tC
    e2, e64 = nrm(got, d2), nrm(got, f64)
    say(f"  {len(rows)} rows: vs Dot2 {e2:.3e}, vs FP64 oracle {e64:.3e}, "
        f"FP64 oracle vs Dot2 {nrm(f64, d2):.3e}")
    assert e2 <= (1e-13 if dtype == mg.F64 else 1e-14)
    assert e64 <= 1e-13


@pytest.mark.parametrize("dtype,n", [(mg.F64, 2048), (mg.F64, 6144), (mg.F32, 6144)])
def test_round_fill_squares(dev, orc, dtype, n):
    """Squares whose tile the round-fill rule picks, in whole rounds (N = 2048 and
    6144: 128 x 128): at N = 2048 every element, at 6144 256 rows spread over the
    matrix, within gamma_{k+2}(|A||B| + |C|) of the FP64 oracle (plus the oracle's
    own bound), FP64 also normwise <= 1e-13.  (Squares that take a split tail are
    checked in test_gpu_gemm.py.)"""
    cfg, splits = mg.choice(n, n, n, dtype)
    assert splits == 1 and cfg.double_buffer == 2
    say(f"round-fill square {mg.DTYPE_NAMES[dtype]} n={n}: {cfg}")
    sa, sb, sc = synth.seeds_for(3, int(np.log2(n)) + (dtype == mg.F32))
    A, B, C = (synth.uniform_pm1((n, n), s) for s in (sa, sb, sc))
    tdt = torch.float64
    if dtype == mg.F32:
        A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
        tdt = torch.float32
    tA, tB, tC = (torch.from_numpy(X).to(dev, tdt) for X in (A, B, C))
    mg.gemm(tA, tB, tC, 1.0, 1.0, dtype=dtype)
    torch.cuda.synchronize()
    rows = np.arange(n) if n <= 4096 else np.linspace(0, n - 1, 256).astype(np.int64)
    got = tC[torch.from_numpy(rows).to(dev)].cpu().double().numpy()
    del tA, tB, tC
    ref = orc.gemm_f64(1.0, A[rows], B, 1.0, C[rows], nthreads=orc.num_procs())
    mag = np.abs(A[rows]) @ np.abs(B)
    mag += np.abs(C[rows])
    u = 2.0 ** -24 if dtype == mg.F32 else 2.0 ** -53
    bound = (gamma(n + 2, u) + gamma(n + 2, 2.0 ** -53)) * mag
    worst = float(np.max(np.abs(got - ref) / bound))
    say(f"  {len(rows)} rows: worst element / bound {worst:.3e}, normwise {nrm(got, ref):.3e}")
    assert worst <= 1.0
    if dtype == mg.F64:
        assert nrm(got, ref) <= 1e-13
