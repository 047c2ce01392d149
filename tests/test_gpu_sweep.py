"""The autotuner's sweep on the GPU, into a temporary database: every registered
configuration is timed on a few shapes (one shape record each); a second run of
the same sweep adds nothing (it resumes); the refinement pass re-times each
shape's fastest configurations (and resumes too); the exhaustive best is the
fastest configuration measured; re-timing that configuration reproduces its
refined time within 10 % (the sweep's own time of the winner is the fastest of
many noisy single runs, biased low by the choice itself); and it computes the
product within the oracle's error bound."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402
from paper_1706_10086_amd import tune  # noqa: E402

SHAPES = [(640, 896, 512), (1000, 333, 777), (1536, 1536, 1024)]


@pytest.mark.parametrize("dt", [mg.F64, mg.F32])
def test_sweep_resumes_and_finds_a_reproducible_best(dt, tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import synth
    path = str(tmp_path / "db.jsonl")
    db = tune.DB.load(path)
    log = lambda s: print(s, flush=True)  # noqa: E731
    cfgs = mg.configs(dt)
    assert tune.sweep(SHAPES, dt, db, reps=3, log=log) == len(SHAPES)
    db2 = tune.DB.load(path)
    assert db2.bad_lines == 0 and len(db2.records) == len(SHAPES) * len(cfgs)
    assert tune.sweep(SHAPES, dt, db2, reps=3, log=log) == 0
    assert tune.refine(SHAPES, dt, db2, top=8, log=log) == len(SHAPES)
    db2 = tune.DB.load(path)
    assert db2.bad_lines == 0 and tune.refine(SHAPES, dt, db2, top=8, log=log) == 0
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dt == mg.F64 else torch.float32
    winners = []
    for (m, n, k) in SHAPES:
        recs = db2.for_shape(dt, m, n, k)
        assert {tuple(r["cfg"]) for r in recs} == {c.as_tuple() for c in cfgs}
        cfg, tf = tune.exhaustive_best(db2, dt, m, n, k)
        assert tf == max(r["tflops"] for r in recs)
        assert tune.regret(db2, dt, m, n, k, cfg) == 0.0
        win = next(r for r in recs if tuple(r["cfg"]) == cfg)
        assert not win["abandoned"] and win["refined"]
        assert sum(1 for r in recs if r["refined"]) == 8
        winners.append((cfg, win["median_ms"]))
    # re-time every winner in one go, each after about 50 ms of untimed runs (the
    # GPU's clocks drop while it idles, and a cold run is slower)
    for (m, n, k), (cfg, ms) in zip(SHAPES, winners):
        ops = tune.Operands(m, n, k, dt)
        again = tune.time_config(ops, dt, mg.Cfg(*cfg), warmup=max(10, int(50.0 / ms)), reps=10)
        med = float(np.median(again))
        print(f"sweep dt={dt} {(m, n, k)} best {cfg}: {ms:.4f} ms, re-timed {med:.4f} ms",
              flush=True)
        assert abs(med - ms) <= 0.10 * ms
        del ops
    for i, ((m, n, k), (cfg, _)) in enumerate(zip(SHAPES, winners)):
        # the winner's product against the oracle
        A = synth.uniform_pm1((m, k), 9500 + i)
        B = synth.uniform_pm1((k, n), 9600 + i)
        if dt == mg.F32:
            A, B = (x.astype(np.float32).astype(np.float64) for x in (A, B))
        C = torch.zeros((m, n), device=dev, dtype=tdt)
        mg.gemm(torch.from_numpy(A).to(dev, tdt), torch.from_numpy(B).to(dev, tdt), C, 1.0, 0.0,
                cfg=mg.Cfg(*cfg))
        torch.cuda.synchronize()
        rows = np.array([0, m // 2, m - 1])
        ref = oracle.gemm_dot2(1.0, A[rows], B, nthreads=oracle.num_procs())
        got = C[torch.from_numpy(rows).to(dev)].cpu().double().numpy()
        u = 2.0 ** -24 if dt == mg.F32 else 2.0 ** -53
        bound = (k + 2) * u / (1 - (k + 2) * u) * (np.abs(A[rows]) @ np.abs(B))
        assert np.all(np.abs(got - ref) <= bound)


def test_added_configurations_sweep_refine_and_merge(tmp_path):
    """The path that brings configurations registered later into a database, with
    the tuner's command line: a sweep of those configurations alone (one shape
    record each, nothing else timed), a refinement of only the shapes where one of
    them ranks among the 4 fastest, and the merge, after which every shape has every
    configuration and the refined medians of the later pass."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dt = mg.F64
    base = str(tmp_path / "base.jsonl")
    shapes = tune.shape_set("aligned", count=3)
    allc = mg.configs(dt)
    added = [c for c in allc if (c.bm, c.bn, c.double_buffer) == (64, 64, 2)]
    assert added
    older = [c for c in allc if c.as_tuple() not in {a.as_tuple() for a in added}]
    # the earlier database: every other configuration swept
    assert tune.sweep(shapes, dt, tune.DB.load(base), cfgs=older, reps=2) == len(shapes)
    new = str(tmp_path / "new.jsonl")
    only = [",".join(str(v) for v in a.as_tuple()) for a in added]
    args = ["--set", "aligned", "--count", "3", "--dtype", "f64", "--db", new]
    tune.main(args + sum((["--only", o] for o in only), []))
    d = tune.DB.load(new)
    assert {tuple(r["cfg"]) for r in d.records} == {a.as_tuple() for a in added}
    assert len({(r["m"], r["n"], r["k"]) for r in d.records}) == len(shapes)
    # refine where an added configuration is among the 4 fastest
    comb = tune.DB("x", tune.prefer_refined(tune.DB.load(base).records + d.records))
    want = tune.shapes_with_top(comb, dt, shapes, [a.as_tuple() for a in added], 4)
    tune.main(args + ["--refine", "4", "--from", base] + sum((["--only", o] for o in only), []))
    refined = {(r["m"], r["n"], r["k"]) for r in tune.DB.load(new).records if r["refined"]}
    assert refined == set(want)
    out = str(tmp_path / "m.json.gz")
    tune.main(["--merge", out, "--from", base, "--update", new])
    m = tune.load_compact(out)
    per = {}
    for r in m.records:
        per.setdefault((r["m"], r["n"], r["k"]), set()).add(tuple(r["cfg"]))
    assert set(per) == set(shapes)
    assert all(v == {c.as_tuple() for c in allc} for v in per.values())
