"""GPU parity of the batched GEMM (persistent kernels in one captured HIP graph)
through the C ABI: bitwise equal to per-problem gemm_ex with the same tile
configurations, within the FP64 / FP32 tolerances of the oracle, stable across
graph replays."""
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


def make_batch(dev, count, lo, hi, seed, tdt, odd_ld_every=0):
    ms = synth.log_uniform_int(count, seed, lo, hi)
    ns = synth.log_uniform_int(count, seed + 1, lo, hi)
    ks = synth.log_uniform_int(count, seed + 2, lo, hi)
    As, Bs, Cs, host = [], [], [], []
    for i, (m, n, k) in enumerate(zip(ms, ns, ks)):
        A = synth.uniform_pm1((m, k), seed * 7919 + 3 * i)
        B = synth.uniform_pm1((k, n), seed * 7919 + 3 * i + 1)
        C = synth.uniform_pm1((m, n), seed * 7919 + 3 * i + 2)
        if tdt == torch.float32:
            A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
        host.append((A, B, C))
        if odd_ld_every and i % odd_ld_every == 0:
            # leading dimension k + 1 (odd/even mix) through a padded buffer
            buf = torch.full((m, k + 1), float("nan"), device=dev, dtype=tdt)
            buf[:, :k] = torch.from_numpy(A).to(dev, tdt)
            As.append(buf[:, :k])
        else:
            As.append(torch.from_numpy(A).to(dev, tdt))
        Bs.append(torch.from_numpy(B).to(dev, tdt))
        Cs.append(torch.from_numpy(C).to(dev, tdt))
    return As, Bs, Cs, host


@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_plan_bitwise_equals_per_problem_and_oracle(dev, orc, tdt):
    say(f"batched plan vs per-problem {tdt}")
    As, Bs, Cs, host = make_batch(dev, 96, 16, 300, 11, tdt, odd_ld_every=5)
    Cs_ref = [c.clone() for c in Cs]
    plan = mg.BatchedPlan(As, Bs, Cs, 1.5, 0.5)
    say(f"  plan {plan.info()}")
    plan.execute()
    mg.gemm_batched(As, Bs, Cs_ref, 1.5, 0.5)
    torch.cuda.synchronize()
    for i, (c, r) in enumerate(zip(Cs, Cs_ref)):
        assert torch.equal(c, r), i
    u = 2.0 ** -53 if tdt == torch.float64 else 2.0 ** -24
    for i in range(0, len(host), 7):
        A, B, C = host[i]
        ref = orc.gemm_dot2(1.5, A, B, 0.5, C)
        got = Cs[i].cpu().double().numpy()
        k = A.shape[1]
        bound = (k + 2) * u / (1 - (k + 2) * u) * (1.5 * np.abs(A) @ np.abs(B) + 0.5 * np.abs(C))
        assert np.all(np.abs(got - ref) <= bound), i
    plan.destroy()


def test_graph_replays_identical(dev):
    say("batched plan replays")
    As, Bs, Cs, _ = make_batch(dev, 64, 16, 256, 21, torch.float64)
    plan = mg.BatchedPlan(As, Bs, Cs, 1.0, 0.0)
    plan.execute()
    torch.cuda.synchronize()
    first = [c.clone() for c in Cs]
    for rep in range(3):
        for c in Cs:
            c.fill_(float("nan"))
        # some eager work between replays
        junk = torch.ones(1024, device=dev).sum()
        torch.cuda.synchronize()
        plan.execute()
        torch.cuda.synchronize()
        for i, (c, f) in enumerate(zip(Cs, first)):
            assert torch.equal(c, f), (rep, i)
        assert junk.item() == 1024.0
    plan.destroy()


def test_plan_with_explicit_configs(dev):
    say("batched plan explicit configs")
    As, Bs, Cs, _ = make_batch(dev, 40, 16, 200, 31, torch.float64)
    cfgs = mg.configs(mg.F64, mg.CFG_BATCHED)
    pick = [cfgs[i % len(cfgs)] for i in range(len(As))]
    Cref = [c.clone() for c in Cs]
    plan = mg.BatchedPlan(As, Bs, Cs, 1.0, 1.0, cfgs=pick)
    assert plan.info()["buckets"] >= min(len(cfgs), len(As)) // 2
    plan.execute()
    for a, b, c, cfg in zip(As, Bs, Cref, pick):
        mg.gemm(a, b, c, 1.0, 1.0, cfg=cfg)
    torch.cuda.synchronize()
    for i, (c, r) in enumerate(zip(Cs, Cref)):
        assert torch.equal(c, r), i
    plan.destroy()


def test_plan_rejects_bad_problems(dev):
    t = torch.zeros((8, 8), device=dev, dtype=torch.float64)
    with pytest.raises(mg.MgemmError) as ei:
        mg.BatchedPlan([t], [t.clone()], [t.clone()], 0.0, 1.0)
    assert ei.value.code == mg.ERR_PLAN
    with pytest.raises(mg.MgemmError):
        mg.BatchedPlan([t], [t.clone()], [t.clone()], 1.0, 0.0, dtype=mg.SPLIT_BF16)
    # empty problems are skipped
    e = torch.zeros((0, 8), device=dev, dtype=torch.float64)
    plan = mg.BatchedPlan([e], [t.clone()], [torch.zeros((0, 8), device=dev, dtype=torch.float64)])
    plan.execute()
    torch.cuda.synchronize()
    plan.destroy()


def test_uneven_batch_2048(dev, orc):
    """The batched workload: 2048 problems with m, n, k log-uniform in [16, 1024],
    alpha = 1, beta = 0; the plan (every problem on the 64 x 64 x 16 tile) bitwise
    against per-problem gemm_ex with that configuration; per-problem launches with
    the library's choice (which splits k for some small outputs) within 1e-13;
    sampled problems against the oracle."""
    say("batched 2048 uneven: building inputs on the device")
    cnt = 2048
    ms = synth.log_uniform_int(cnt, 4001, 16, 1024)
    ns = synth.log_uniform_int(cnt, 4002, 16, 1024)
    ks = synth.log_uniform_int(cnt, 4003, 16, 1024)
    g = torch.Generator(device=dev)
    g.manual_seed(4004)
    As = [torch.rand((int(m), int(k)), device=dev, dtype=torch.float64, generator=g) * 2 - 1
          for m, k in zip(ms, ks)]
    Bs = [torch.rand((int(k), int(n)), device=dev, dtype=torch.float64, generator=g) * 2 - 1
          for k, n in zip(ks, ns)]
    Cs = [torch.zeros((int(m), int(n)), device=dev, dtype=torch.float64) for m, n in zip(ms, ns)]
    Cr = [torch.zeros_like(c) for c in Cs]
    Cd = [torch.zeros_like(c) for c in Cs]
    plan = mg.BatchedPlan(As, Bs, Cs, 1.0, 0.0)
    say(f"  plan {plan.info()}")
    plan.execute()
    c64 = [c for c in mg.configs(mg.F64) if (c.bm, c.bn, c.bk, c.waves) == (64, 64, 16, 4)][0]
    for a, b, c in zip(As, Bs, Cr):
        mg.gemm(a, b, c, 1.0, 0.0, cfg=c64)
    mg.gemm_batched(As, Bs, Cd, 1.0, 0.0)
    torch.cuda.synchronize()
    for i in range(cnt):
        assert torch.equal(Cs[i], Cr[i]), i
        assert torch.linalg.norm(Cs[i] - Cd[i]) <= 1e-13 * torch.linalg.norm(Cs[i]), i
    for i in (0, 1, 777, 2047):
        A, B = As[i].cpu().numpy(), Bs[i].cpu().numpy()
        ref = orc.gemm_f64(1.0, A, B)
        err = np.linalg.norm(Cs[i].cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err <= 1e-13, (i, err)
    plan.destroy()


def test_uneven_batch_2048_fp32(dev, orc):
    """The FP32 variant of the batched workload: the plan bitwise against per-problem
    gemm_ex with the 64 x 64 x 16 configuration, and sampled problems within
    gamma_{k+2} (u = 2^-24) of the oracle on the same float inputs."""
    say("batched 2048 uneven fp32: building inputs on the device")
    cnt = 2048
    ms = synth.log_uniform_int(cnt, 4001, 16, 1024)
    ns = synth.log_uniform_int(cnt, 4002, 16, 1024)
    ks = synth.log_uniform_int(cnt, 4003, 16, 1024)
    g = torch.Generator(device=dev)
    g.manual_seed(4005)
    As = [torch.rand((int(m), int(k)), device=dev, dtype=torch.float32, generator=g) * 2 - 1
          for m, k in zip(ms, ks)]
    Bs = [torch.rand((int(k), int(n)), device=dev, dtype=torch.float32, generator=g) * 2 - 1
          for k, n in zip(ks, ns)]
    Cs = [torch.zeros((int(m), int(n)), device=dev, dtype=torch.float32) for m, n in zip(ms, ns)]
    Cr = [torch.zeros_like(c) for c in Cs]
    plan = mg.BatchedPlan(As, Bs, Cs, 1.0, 0.0)
    say(f"  plan {plan.info()}")
    plan.execute()
    c64 = [c for c in mg.configs(mg.F32) if (c.bm, c.bn, c.bk, c.waves) == (64, 64, 16, 4)][0]
    for a, b, c in zip(As, Bs, Cr):
        mg.gemm(a, b, c, 1.0, 0.0, cfg=c64)
    torch.cuda.synchronize()
    for i in range(cnt):
        assert torch.equal(Cs[i], Cr[i]), i
    u = 2.0 ** -24
    for i in (0, 1, 777, 2047):
        A, B = As[i].cpu().double().numpy(), Bs[i].cpu().double().numpy()
        ref = orc.gemm_dot2(1.0, A, B)
        k = A.shape[1]
        bound = (k + 2) * u / (1 - (k + 2) * u) * (np.abs(A) @ np.abs(B))
        assert np.all(np.abs(Cs[i].cpu().double().numpy() - ref) <= bound), i
    plan.destroy()


def test_plan_without_tile_map(dev, orc):
    """A problem with 2^20 + 1 tile rows (m = 2^25 + 5 with 32-row tiles) does not fit
    the tile map's fields, so the plan's kernels find each tile's problem by binary
    search over one list of tile numbers: still bitwise equal to per-problem gemm_ex
    with the same configurations, and sampled rows of the tall problem match the
    oracle."""
    cfgs = mg.configs(mg.F64, mg.CFG_BATCHED)
    c32 = [c for c in cfgs if c.bm == 32][0]
    c64 = [c for c in cfgs if (c.bm, c.bn, c.bk) == (64, 64, 16)][0]
    m_tall = (1 << 25) + 5
    say(f"batched plan without tile map: tall problem m={m_tall}, 32x32 tiles")
    g = torch.Generator(device=dev)
    g.manual_seed(91)
    shapes = [(m_tall, 3, 2, c32), (100, 70, 50, c32), (65, 130, 33, c64), (7, 5, 300, c64),
              (1, 1, 1, c32)]
    As = [torch.rand((m, k), device=dev, dtype=torch.float64, generator=g) * 2 - 1
          for m, n, k, _ in shapes]
    Bs = [torch.rand((k, n), device=dev, dtype=torch.float64, generator=g) * 2 - 1
          for m, n, k, _ in shapes]
    Cs = [torch.rand((m, n), device=dev, dtype=torch.float64, generator=g) for m, n, k, _ in shapes]
    Cr = [c.clone() for c in Cs]
    rows = torch.tensor([0, 31, 32, 1 << 20, (1 << 25) - 1, 1 << 25, m_tall - 1], device=dev)
    C0 = Cs[0][rows].cpu().numpy()
    pick = [s[3] for s in shapes]
    plan = mg.BatchedPlan(As, Bs, Cs, 1.25, -0.5, cfgs=pick)
    info = plan.info()
    say(f"  plan {info}")
    assert info["buckets"] == 2 and info["tiles"] > (1 << 20)
    plan.execute()
    for a, b, c, cfg in zip(As, Bs, Cr, pick):
        mg.gemm(a, b, c, 1.25, -0.5, cfg=cfg)
    torch.cuda.synchronize()
    for i, (c, r) in enumerate(zip(Cs, Cr)):
        assert torch.equal(c, r), i
    want = orc.gemm_f64(1.25, As[0][rows].cpu().numpy(), Bs[0].cpu().numpy(), -0.5, C0)
    got = Cs[0][rows].cpu().numpy()
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
    plan.destroy()
    del As, Bs, Cs, Cr
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_batch_tuner_choice(dev, orc, tdt):
    """The batch tuner times every candidate rule's plan and ranks them; the
    winning plan (beta = 0, as in the batched workload) gives the same bits as
    per-problem launches with the configurations it chose."""
    from paper_1706_10086_amd import tune
    dt = mg.F32 if tdt == torch.float32 else mg.F64
    say(f"batch tuner {tdt}")
    As, Bs, Cs, host = make_batch(dev, 64, 16, 400, 23, tdt)
    res = tune.tune_batch(As, Bs, Cs, 1.0, 0.0, dt, reps=2)
    assert len(res) == len(tune.batch_rules(dt))
    assert [r[1] for r in res] == sorted(r[1] for r in res)
    name, ms, nb, cfgs = res[0]
    say(f"  best {name}: {ms:.4f} ms, {nb} bucket(s)")
    assert nb == len(set(cfgs))
    plan = mg.BatchedPlan(As, Bs, Cs, 1.0, 0.0, cfgs=cfgs)
    plan.execute()
    Cs_ref = [torch.full_like(c, float("nan")) for c in Cs]
    for A, B, C, c in zip(As, Bs, Cs_ref, cfgs):
        mg.gemm(A, B, C, 1.0, 0.0, cfg=c)
    torch.cuda.synchronize()
    for i, (c, r) in enumerate(zip(Cs, Cs_ref)):
        assert torch.equal(c, r), i
    plan.destroy()
    u = 2.0 ** -53 if tdt == torch.float64 else 2.0 ** -24
    for i in range(0, len(host), 5):
        A, B, _ = host[i]
        ref = orc.gemm_dot2(1.0, A, B)
        k = A.shape[1]
        bound = (k + 2) * u / (1 - (k + 2) * u) * (np.abs(A) @ np.abs(B))
        assert np.all(np.abs(Cs[i].cpu().double().numpy() - ref) <= bound), i
