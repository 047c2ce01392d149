"""GPU parity of the tiled FP64 / FP32 GEMM against the CPU oracle, through the
C ABI.  Tolerances: FP64 normwise relative error <= 1e-13 against the FP64
oracle; every element within the componentwise bound gamma_{k+2} (u = 2^-53 for
FP64, 2^-24 for FP32; Higham, Sec. 3.5); integer-valued inputs whose products and
partial sums are exact give bitwise-equal results."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402


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


def to_dev(x, dev, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev, dtype)


def run_gemm(dev, A, B, C, alpha, beta, dtype=mg.F64, cfg=None):
    tdt = torch.float32 if dtype == mg.F32 else torch.float64
    tA, tB, tC = to_dev(A, dev, tdt), to_dev(B, dev, tdt), to_dev(C, dev, tdt)
    mg.gemm(tA, tB, tC, alpha, beta, dtype=dtype, cfg=cfg)
    torch.cuda.synchronize()
    return tC.cpu().double().numpy()


def test_mfma_fragment_layout(dev):
    say("probe: mfma layout f64/f32")
    A = synth.integer_valued((16, 4), 1, 7)
    B = synth.integer_valued((4, 16), 2, 7)
    for dt, tdt in ((mg.F64, torch.float64), (mg.F32, torch.float32)):
        tA, tB = to_dev(A, dev, tdt), to_dev(B, dev, tdt)
        tD = torch.full((16, 16), float("nan"), device=dev, dtype=tdt)
        mg.probe_mfma(dt, tA, tB, tD)
        torch.cuda.synchronize()
        assert np.array_equal(tD.cpu().double().numpy(), A @ B), dt
        # one-hot operands: each output element comes from exactly one product
        for (i, kk, j) in [(0, 0, 0), (15, 3, 15), (5, 2, 9), (12, 1, 3)]:
            Ao = np.zeros((16, 4)); Ao[i, kk] = 1.0
            Bo = np.zeros((4, 16)); Bo[kk, j] = 2.0
            tA, tB = to_dev(Ao, dev, tdt), to_dev(Bo, dev, tdt)
            mg.probe_mfma(dt, tA, tB, tD)
            torch.cuda.synchronize()
            want = np.zeros((16, 16)); want[i, j] = 2.0
            assert np.array_equal(tD.cpu().double().numpy(), want)


def test_parity_256_uniform_alpha_beta(dev, orc):
    """m = n = k = 256, entries uniform[-1,1], alpha = 1.5, beta = 0.5."""
    say("parity: 256^3 f64 alpha=1.5 beta=0.5")
    n = 256
    sa, sb, sc = synth.seeds_for(0, 8)
    A, B, C = synth.uniform_pm1((n, n), sa), synth.uniform_pm1((n, n), sb), synth.uniform_pm1((n, n), sc)
    got = run_gemm(dev, A, B, C, 1.5, 0.5)
    ref = orc.gemm_f64(1.5, A, B, 0.5, C)
    ref2 = orc.gemm_dot2(1.5, A, B, 0.5, C)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    err2 = np.linalg.norm(got - ref2) / np.linalg.norm(ref2)
    say(f"  normwise err vs f64 oracle {err:.3e}, vs dot2 {err2:.3e}")
    assert err <= 1e-13 and err2 <= 1e-13
    bound = gamma(n + 2, 2.0 ** -53) * (1.5 * np.abs(A) @ np.abs(B) + 0.5 * np.abs(C))
    assert np.all(np.abs(got - ref2) <= bound)


SHAPES = [(1, 1, 1), (1, 7, 3), (17, 33, 65), (64, 64, 64), (128, 128, 16), (129, 127, 17),
          (255, 257, 129), (127, 131, 137), (300, 200, 1000), (16, 1024, 8), (1000, 3, 5),
          # even n and k: the shapes the three-stage kernels take, with ragged edges
          (33, 2, 16), (129, 130, 48), (257, 254, 166), (5, 300, 2)]


@pytest.mark.parametrize("dtype", [mg.F64, mg.F32])
def test_integer_exact_all_configs(dev, dtype):
    """Integer-valued entries in [-8, 8]: every partial sum is an exact integer, so
    any summation order gives the same bits."""
    for cfg in mg.configs(dtype):
        for (m, n, k) in SHAPES:
            say(f"int-exact dtype={dtype} cfg={cfg} shape={(m, n, k)}")
            A = synth.integer_valued((m, k), m + 3, 8)
            B = synth.integer_valued((k, n), n + 5, 8)
            C = synth.integer_valued((m, n), k + 7, 50)
            want = 3 * (A.astype(np.int64) @ B.astype(np.int64)) - 2 * C.astype(np.int64)
            got = run_gemm(dev, A, B, C, 3.0, -2.0, dtype=dtype, cfg=cfg)
            assert np.array_equal(got, want.astype(np.float64)), (cfg, m, n, k)


@pytest.mark.parametrize("dtype", [mg.F64, mg.F32])
def test_leading_dims_padding_and_guard_bands(dev, dtype):
    """Sub-matrices of larger buffers: NaN in the padding of A and B must not leak,
    and C's padding columns and the rows around it must stay untouched."""
    tdt = torch.float32 if dtype == mg.F32 else torch.float64
    for (m, n, k, lda, ldb, ldc) in [(67, 45, 39, 41, 46, 50), (128, 128, 64, 65, 129, 131),
                                     (33, 17, 100, 101, 18, 18), (64, 64, 32, 34, 66, 64)]:
        say(f"padding dtype={dtype} shape={(m, n, k)} ld={(lda, ldb, ldc)}")
        A = synth.integer_valued((m, k), 1, 8)
        B = synth.integer_valued((k, n), 2, 8)
        C = synth.integer_valued((m, n), 3, 50)
        Abuf = torch.full((m, lda), float("nan"), device=dev, dtype=tdt)
        Bbuf = torch.full((k, ldb), float("nan"), device=dev, dtype=tdt)
        Cbuf = torch.full((m + 2, ldc), -777.0, device=dev, dtype=tdt)
        Abuf[:, :k] = to_dev(A, dev, tdt)
        Bbuf[:, :n] = to_dev(B, dev, tdt)
        Cbuf[1:m + 1, :n] = to_dev(C, dev, tdt)
        Cv = Cbuf[1:m + 1, :n]
        mg.gemm(Abuf[:, :k], Bbuf[:, :n], Cv, 1.0, 1.0, dtype=dtype)
        torch.cuda.synchronize()
        out = Cbuf.cpu().double().numpy()
        want = (A.astype(np.int64) @ B.astype(np.int64) + C.astype(np.int64)).astype(np.float64)
        assert np.array_equal(out[1:m + 1, :n], want)
        assert np.all(out[0] == -777.0) and np.all(out[m + 1] == -777.0)
        assert np.all(out[1:m + 1, n:] == -777.0)


def test_quick_returns_and_beta_zero(dev, orc):
    say("quick returns")
    m, n, k = 70, 50, 30
    A = synth.uniform_pm1((m, k), 1)
    B = synth.uniform_pm1((k, n), 2)
    C = synth.uniform_pm1((m, n), 3)
    # beta == 0: C may hold NaN, it is not read
    Cn = np.full((m, n), np.nan)
    got = run_gemm(dev, A, B, Cn, 1.25, 0.0)
    assert np.all(np.isfinite(got))
    ref = orc.gemm_f64(1.25, A, B)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
    # alpha == 0: A and B are not read
    An = np.full((m, k), np.nan)
    assert np.array_equal(run_gemm(dev, An, B, C, 0.0, 0.5), 0.5 * C)
    assert np.array_equal(run_gemm(dev, An, B, Cn, 0.0, 0.0), np.zeros((m, n)))
    # k == 0
    tA = torch.zeros((m, 0), device=dev, dtype=torch.float64)
    tB = torch.zeros((0, n), device=dev, dtype=torch.float64)
    tC = to_dev(C, dev)
    mg.gemm(tA, tB, tC, 1.0, 2.0)
    torch.cuda.synchronize()
    assert np.array_equal(tC.cpu().numpy(), 2.0 * C)


def test_fp32_within_gamma_bound(dev, orc):
    for (m, n, k) in [(256, 256, 256), (129, 77, 1000), (513, 257, 64)]:
        say(f"fp32 gamma bound shape={(m, n, k)}")
        A = synth.uniform_pm1((m, k), 11).astype(np.float32).astype(np.float64)
        B = synth.uniform_pm1((k, n), 12).astype(np.float32).astype(np.float64)
        C = synth.uniform_pm1((m, n), 13).astype(np.float32).astype(np.float64)
        got = run_gemm(dev, A, B, C, 1.5, 0.5, dtype=mg.F32)
        ref = orc.gemm_dot2(np.float32(1.5), A, B, np.float32(0.5), C)
        bound = gamma(k + 2, 2.0 ** -24) * (1.5 * np.abs(A) @ np.abs(B) + 0.5 * np.abs(C))
        assert np.all(np.abs(got - ref) <= bound)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(f"  fp32 normwise err {err:.3e}")
        assert err < 1e-6


# the first four take the three-stage 128 x 128 tile for the k ranges (the last
# with a ragged final range: 512 + 512 + 76), the others the 64 x 64 or 32 x 32 tile
# shapes the built-in choice runs with k cut (k >= 2048, or outside the measured
# range), and some it runs whole (the measured configuration) since k is short
SPLITK_SHAPES = [(1024, 512, 4096), (1000, 999, 3001), (300, 200, 6000), (511, 130, 2513),
                 (37, 45, 5000), (1, 1, 70000), (64, 1024, 2777), (1024, 1024, 1024),
                 (896, 1024, 1536), (300, 200, 600)]


# outputs whose 128 x 128 tiles leave a last round of few tiles: the rows that fill
# whole rounds run whole, the rest with k cut (FP64 3072^3: 21 + 3 tile rows, 3
# ranges; 3584 x 3584 x 2048: 27 + 1 tile rows; 4608 x 4608 x 1536 FP32)
SPLIT_TAIL_SHAPES = {mg.F64: [(3072, 3072, 3072), (3584, 3584, 2048)],
                     mg.F32: [(3584, 3584, 3584), (4608, 4608, 1536)]}


@pytest.mark.parametrize("dtype", [mg.F64, mg.F32])
def test_split_tail(dev, orc, dtype):
    """Split tail: 96 sampled rows (both sides of the boundary between the whole
    rows and the tail, the first and last rows among them) within gamma_{k+2} of
    the double-double oracle, FP64 normwise <= 1e-13; run-to-run identical; the
    no-allocation entry point gives the same bits; the whole rows equal the 128 x
    128 tile run whole (the same kernel), the tail rows do not (k cut)."""
    u = 2.0 ** -24 if dtype == mg.F32 else 2.0 ** -53
    tdt = torch.float32 if dtype == mg.F32 else torch.float64
    for (m, n, k) in SPLIT_TAIL_SHAPES[dtype]:
        cfg, S, main = mg.choice(m, n, k, dtype, rows=True)
        say(f"split tail {'f32' if dtype == mg.F32 else 'f64'} shape={(m, n, k)} cfg={cfg} "
            f"S={S} main rows={main}")
        assert S > 1 and 0 < main < m and (cfg.bm, cfg.bn, cfg.double_buffer) == (128, 128, 2)
        A = synth.uniform_pm1((m, k), 61 + m)
        B = synth.uniform_pm1((k, n), 62 + n)
        C = synth.uniform_pm1((m, n), 63 + k)
        if dtype == mg.F32:
            A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
        al, be = (np.float32(1.5), np.float32(-0.5)) if dtype == mg.F32 else (1.5, -0.5)
        got = run_gemm(dev, A, B, C, 1.5, -0.5, dtype=dtype)
        rows = np.unique(np.concatenate([[0, m - 1], np.arange(main - 8, main + 8),
                                         np.linspace(1, m - 2, 78).astype(np.int64)]))
        ref = orc.gemm_dot2(al, A[rows], B, be, C[rows], nthreads=orc.num_procs())
        mag = 1.5 * np.abs(A[rows]) @ np.abs(B) + 0.5 * np.abs(C[rows])
        assert np.all(np.abs(got[rows] - ref) <= gamma(k + 2, u) * mag), (m, n, k)
        if dtype == mg.F64:
            assert np.linalg.norm(got[rows] - ref) <= 1e-13 * np.linalg.norm(ref)
        assert np.array_equal(got, run_gemm(dev, A, B, C, 1.5, -0.5, dtype=dtype))
        tA, tB, tC = to_dev(A, dev, tdt), to_dev(B, dev, tdt), to_dev(C, dev, tdt)
        mg._check(mg.gemm_ex_noalloc_raw(m, n, k, 1.5, tA.data_ptr(), k, tB.data_ptr(), n, -0.5,
                                         tC.data_ptr(), n, dtype))
        torch.cuda.synchronize()
        assert np.array_equal(tC.cpu().double().numpy(), got)
        whole = run_gemm(dev, A, B, C, 1.5, -0.5, dtype=dtype, cfg=cfg)
        assert np.array_equal(got[:main], whole[:main])
        assert not np.array_equal(got[main:], whole[main:])


@pytest.mark.parametrize("dtype", [mg.F64, mg.F32])
def test_split_k_default_choice(dev, orc, dtype):
    """Outputs whose preferred tile leaves fewer than about four work-groups per
    compute unit, with k >= 2048 (or outside the measured range), run split-k
    under the built-in choice (k cut into ranges of 256j, partial products reduced
    in order; FP32 only on the three-stage tile, whose rows must be 16-byte
    aligned); shorter k runs the measured configuration whole: every element within
    gamma_{k+2} of the double-double oracle, FP64 normwise <= 1e-13, run-to-run
    identical, C not read when beta = 0."""
    u = 2.0 ** -24 if dtype == mg.F32 else 2.0 ** -53
    for (m, n, k) in SPLITK_SHAPES:
        say(f"split-k default choice {'f32' if dtype == mg.F32 else 'f64'} shape={(m, n, k)}")
        A = synth.uniform_pm1((m, k), 21 + m)
        B = synth.uniform_pm1((k, n), 22 + n)
        C = synth.uniform_pm1((m, n), 23 + k)
        if dtype == mg.F32:
            A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
        al, be = (np.float32(1.5), np.float32(-0.5)) if dtype == mg.F32 else (1.5, -0.5)
        got = run_gemm(dev, A, B, C, 1.5, -0.5, dtype=dtype)
        ref = orc.gemm_dot2(al, A, B, be, C, nthreads=orc.num_procs())
        bound = gamma(k + 2, u) * (1.5 * np.abs(A) @ np.abs(B) + 0.5 * np.abs(C))
        assert np.all(np.abs(got - ref) <= bound), (m, n, k)
        if dtype == mg.F64:
            assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
        again = run_gemm(dev, A, B, C, 1.5, -0.5, dtype=dtype)
        assert np.array_equal(got, again)
        nan_c = run_gemm(dev, A, B, np.full((m, n), np.nan), 1.5, 0.0, dtype=dtype)
        assert np.all(np.isfinite(nan_c))
    # the 1024 x 512 x 4096 product really took the split path: its summation order
    # differs from the same tile run whole (an explicit configuration never splits k)
    n, k = 1024, 4096
    A = synth.uniform_pm1((n, k), 31)
    B = synth.uniform_pm1((k, n // 2), 32)
    if dtype == mg.F32:
        A, B = (x.astype(np.float32).astype(np.float64) for x in (A, B))
    whole_cfg = [c for c in mg.configs(dtype) if (c.bm, c.bn, c.bk, c.waves) == (64, 64, 16, 4)][0]
    split = run_gemm(dev, A, B, np.zeros((n, n // 2)), 1.0, 0.0, dtype=dtype)
    whole = run_gemm(dev, A, B, np.zeros((n, n // 2)), 1.0, 0.0, dtype=dtype, cfg=whole_cfg)
    assert not np.array_equal(split, whole)
    assert np.linalg.norm(split - whole) <= 4 * k * u * np.linalg.norm(whole)
    if dtype == mg.F32:
        return
    # the same k ranges on the two-stage tile (an odd leading dimension of A rules
    # out the three-stage kernel): every tile sums a range in the same order, so
    # both splits agree bit for bit
    for k in (4096, 4100):
        A = synth.uniform_pm1((n, k), 33 + k)
        B = synth.uniform_pm1((k, n), 34 + k)
        tA, tB = to_dev(A, dev), to_dev(B, dev)
        tC1 = torch.zeros((n, n), device=dev, dtype=torch.float64)
        mg.gemm(tA, tB, tC1, 1.0, 0.0)
        pad = torch.full((n, k + 1), float("nan"), device=dev, dtype=torch.float64)
        pad[:, :k] = tA
        tC2 = torch.zeros((n, n), device=dev, dtype=torch.float64)
        mg.gemm(pad[:, :k], tB, tC2, 1.0, 0.0)
        torch.cuda.synchronize()
        assert torch.equal(tC1, tC2), k


def test_run_to_run_determinism(dev):
    say("determinism 1024^3")
    n = 1024
    A = to_dev(synth.uniform_pm1((n, n), 1), dev)
    B = to_dev(synth.uniform_pm1((n, n), 2), dev)
    outs = []
    for _ in range(3):
        C = torch.zeros((n, n), device=dev, dtype=torch.float64)
        mg.gemm(A, B, C, 1.0, 0.0)
        outs.append(C)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_all_configs_uniform_ragged(dev, orc):
    m, n, k = 333, 271, 517
    A = synth.uniform_pm1((m, k), 21)
    B = synth.uniform_pm1((k, n), 22)
    C = synth.uniform_pm1((m, n), 23)
    ref = orc.gemm_f64(1.5, A, B, 0.5, C)
    for cfg in mg.configs(mg.F64):
        say(f"ragged uniform cfg={cfg}")
        got = run_gemm(dev, A, B, C, 1.5, 0.5, cfg=cfg)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-13, (cfg, err)


def _twin(cfg, dtype):
    """A registered two-stage configuration of the same tile and k-step: the one
    with 16-byte loads per thread, two stages and no occupancy bound if there is
    one, else one stage or an occupancy bound (neither changes the sum order)."""
    ept = 2 if dtype == mg.F64 else 4
    cands = [c for c in mg.configs(dtype)
             if (c.bm, c.bn, c.bk, c.elems_per_thread) == (cfg.bm, cfg.bn, cfg.bk, ept)
             and c.double_buffer < 2]
    if not cands:
        raise AssertionError(f"no two-stage twin for {cfg}")
    return min(cands, key=lambda c: (c.double_buffer != 1, c.occupancy))


@pytest.mark.parametrize("dtype", [mg.F64, mg.F32])
@pytest.mark.parametrize("padded", [False, True])
def test_three_stage_matches_two_stage_bitwise(dev, orc, padded, dtype):
    """The direct-load three-stage kernels sum in the two-stage kernel's order, so
    on their own domain (n and leading dimensions multiples of the 16-byte load)
    the results agree bit for bit, including partial last k-steps, ragged edges
    and padded leading dimensions; FP64 is within 1e-13 of the oracle, FP32
    within 1e-5."""
    tdt = torch.float64 if dtype == mg.F64 else torch.float32
    epu = 2 if dtype == mg.F64 else 4
    pipes = [c for c in mg.configs(dtype) if c.double_buffer == 2]
    assert pipes
    for (m, n, k) in [(1, 4, 16), (64, 64, 64), (200, 260, 16), (257, 132, 333),
                      (300, 4, 1024), (513, 384, 47), (129, 1032, 8)]:
        A = synth.uniform_pm1((m, k), m + 31)
        B = synth.uniform_pm1((k, n), n + 37)
        C = synth.uniform_pm1((m, n), k + 41)
        ref = orc.gemm_f64(1.5, A, B, 0.5, C)
        lda, ldb = (-(-(k + 1) // epu) * epu, n + 2 * epu) if padded else (k, n)
        Abuf = torch.full((m, lda), float("nan"), device=dev, dtype=tdt)
        Bbuf = torch.full((k, ldb), float("nan"), device=dev, dtype=tdt)
        Abuf[:, :k] = to_dev(A, dev, tdt)
        Bbuf[:, :n] = to_dev(B, dev, tdt)
        for cfg in pipes:
            say(f"three-stage vs two-stage dtype={dtype} cfg={cfg} shape={(m, n, k)} "
                f"padded={padded}")
            outs = []
            for c in (cfg, _twin(cfg, dtype)):
                tC = to_dev(C, dev, tdt)
                mg.gemm(Abuf[:, :k], Bbuf[:, :n], tC, 1.5, 0.5, dtype=dtype, cfg=c)
                outs.append(tC)
            torch.cuda.synchronize()
            assert torch.equal(outs[0], outs[1]), (cfg, m, n, k)
            got = outs[0].cpu().double().numpy()
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert err <= (1e-13 if dtype == mg.F64 else 1e-5), (cfg, m, n, k, err)


@pytest.mark.parametrize("n", [8192, 16384])
def test_full_size_sampled_rows(dev, orc, n):
    """The square benchmark size and the sweep's largest with the default
    configuration: 64 sampled rows recomputed by the oracle; normwise error over the
    sample <= 1e-13."""
    say(f"full size n={n}: generating inputs")
    sa, sb, sc = synth.seeds_for(1, int(np.log2(n)))
    A = synth.uniform_pm1((n, n), sa)
    B = synth.uniform_pm1((n, n), sb)
    C = synth.uniform_pm1((n, n), sc)
    tA, tB, tC = to_dev(A, dev), to_dev(B, dev), to_dev(C, dev)
    say("  gemm")
    mg.gemm(tA, tB, tC, 1.0, 1.0)
    torch.cuda.synchronize()
    rows = np.unique(synth.log_uniform_int(64, 5, 1, n) - 1)
    rows = np.unique(np.concatenate([rows, [0, n - 1]]))
    got = tC[torch.from_numpy(rows).to(dev)].cpu().numpy()
    say(f"  oracle on {len(rows)} rows")
    ref = orc.gemm_f64(1.0, A[rows], B, 1.0, C[rows], nthreads=orc.num_procs())
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"  sampled normwise err {err:.3e}")
    assert err <= 1e-13


def test_full_size_fp32_sampled_rows(dev, orc):
    """FP32 at the square benchmark size, default configuration: 64 sampled rows
    against the FP64 oracle on the same float inputs, every element within
    gamma_{k+2} with u = 2^-24."""
    n = 8192
    say(f"full size fp32 n={n}: generating inputs")
    sa, sb, sc = synth.seeds_for(1, 13)
    A, B, C = (synth.uniform_pm1((n, n), s).astype(np.float32) for s in (sa, sb, sc))
    tA, tB, tC = (torch.from_numpy(X).to(dev) for X in (A, B, C))
    say("  gemm")
    mg.gemm(tA, tB, tC, 1.0, 1.0)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([synth.log_uniform_int(64, 6, 1, n) - 1, [0, n - 1]]))
    got = tC[torch.from_numpy(rows).to(dev)].cpu().double().numpy()
    A64, B64, C64 = A[rows].astype(np.float64), B.astype(np.float64), C[rows].astype(np.float64)
    say(f"  oracle on {len(rows)} rows")
    ref = orc.gemm_dot2(1.0, A64, B64, 1.0, C64, nthreads=orc.num_procs())
    bound = gamma(n + 2, 2.0 ** -24) * (np.abs(A64) @ np.abs(B64) + np.abs(C64))
    assert np.all(np.abs(got - ref) <= bound)
