"""The learned configuration predictor on the GPU: the MLP is trained by the
library's kernels on the shipped MI355X tuner database and evaluated on the 500
held-out shapes (FP64 and FP32) against the exhaustive best: geometric mean of
TFLOP/s(predicted) / TFLOP/s(best) >= 0.95, and better than the method without
the network (one tuned configuration per dtype)."""
import collections
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402
from paper_1706_10086_amd import learn, tune  # noqa: E402

DB_PATH = os.path.join(os.path.dirname(learn.__file__), "data", "tune_db.json.gz")


@pytest.fixture(scope="module")
def data():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    db = tune.load_compact(DB_PATH)
    table = learn.config_table()
    dtr, dho = learn.datasets(db, table)
    assert len(dtr.shapes) == 13600 and len(dho.shapes) == 1000, "database does not match registry"
    return table, dtr, dho


def test_mlp_regret_within_5_percent_and_beats_single_config(data):
    table, dtr, dho = data
    print("training the predictor", flush=True)
    pred = learn.train(dtr, table, **learn.TRAIN_SETTINGS)
    assert pred.history[-1][1] < pred.history[0][1]
    choice = learn.predict(pred, dho.shapes)
    mlp = learn.summarize(learn.achieved(dho, choice))
    base = learn.single_best_baseline(dtr, table)
    single = learn.summarize(learn.achieved(dho, [base[s[0]] for s in dho.shapes]))
    top3 = learn.summarize(learn.top_k_fallback(dho, pred, 3))
    print(f"  mlp {mlp}\n  single {single}\n  top3 {top3}", flush=True)
    # within 5 % of the exhaustive best over the 247 configurations, far above
    # the paper's one tuned configuration per dtype; measuring the three best
    # predictions comes within 3 %
    assert mlp["geomean"] >= 0.95
    assert mlp["geomean"] > single["geomean"] + 0.1
    assert top3["geomean"] >= max(mlp["geomean"], 0.97)
    for dt in (mg.F64, mg.F32):
        rows = [i for i, s in enumerate(dho.shapes) if s[0] == dt]
        assert learn.summarize(learn.achieved(dho, choice)[rows])["geomean"] >= 0.94
    # the shipped model file is this training run's result
    shipped = learn.Predictor.load(os.path.join(os.path.dirname(DB_PATH), "model.mlp"),
                                   check_table=table)
    assert np.array_equal(shipped.params, pred.params)


def test_predictions_are_valid_configurations(data):
    table, dtr, dho = data
    pred = learn.train(dtr, table, steps=500, lr=2e-3)
    choice = learn.predict(pred, dho.shapes[:50] + dho.shapes[-50:])
    for (dt, m, n, k), c in zip(dho.shapes[:50] + dho.shapes[-50:], choice):
        assert table[c][0] == dt
        cfg = mg.Cfg(*table[c][1])
        tdt = torch.float64 if dt == mg.F64 else torch.float32
        a = torch.ones((3, 5), device="cuda", dtype=tdt)
        b = torch.ones((5, 7), device="cuda", dtype=tdt)
        out = torch.zeros((3, 7), device="cuda", dtype=tdt)
        mg.gemm(a, b, out, 1.0, 0.0, cfg=cfg)
        torch.cuda.synchronize()
        assert torch.all(out == 5.0)


def test_chooser_database_then_model():
    """The run-time chooser: a swept shape takes its database best, an unseen
    shape the model's prediction (or, measuring the model's three best, the
    fastest of them); the product is correct every way."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import synth
    from paper_1706_10086_amd import choose
    ch = choose.ConfigChooser()
    chm = choose.ConfigChooser(measure_top=3)
    seen = tune.shape_set("heldout")[0]
    for i, ((m, n, k), want, c) in enumerate(((seen, "database", ch), ((333, 517, 271), "model", ch),
                                              ((333, 517, 271), "measured", chm))):
        print(f"chooser shape {(m, n, k)} {want}", flush=True)
        A = synth.uniform_pm1((m, k), 610 + 2 * i)
        B = synth.uniform_pm1((k, n), 611 + 2 * i)
        C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
        _, source = choose.tuned_gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C,
                                      chooser=c)
        torch.cuda.synchronize()
        assert source == want
        ref = oracle.gemm_f64(1.0, A, B, 0.0, None, nthreads=oracle.num_procs())
        got = C.cpu().numpy()
        assert float(np.linalg.norm(got - ref) / np.linalg.norm(ref)) <= 1e-13
        u = 2.0 ** -53
        assert np.all(np.abs(got - ref) <= 2 * (k + 2) * u / (1 - (k + 2) * u) * (np.abs(A) @ np.abs(B)))


def test_builtin_choice_runs_the_measured_configuration():
    """gemm without a configuration, on held-out shapes whose output is large enough
    that split-k does not apply: where the rows are not whole 16-byte loads, or the
    preference list names a two-stage configuration, it runs the configuration of
    the shape's cell in the library's measured table, bit for bit the same as naming
    that configuration, and within the FP64 / FP32 tolerances of the oracle on
    sampled rows."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import synth
    from paper_1706_10086_amd.csrc import gen_choice_table as gen
    import choice_rule as host
    db = tune.load_compact(DB_PATH)
    tables = gen.build_tables(db.records, gen.training_shapes())
    dev = torch.device("cuda:0")
    for dt in (mg.F64, mg.F32):
        picked = []
        for whole in (False, True):
            cand = []
            for s in tune.shape_set("heldout"):
                m, n, k = s
                if gen.three_stage_ineligible(dt, n, k) == whole or 2.0 * m * n * k >= 4e10:
                    continue
                if (-(-m // 128)) * (-(-n // 64)) < 256:
                    continue
                if whole and host.pref_choice(dt, m, n)[5] == 2:
                    continue
                if gen.cell_of(m, n, k) in tables[int(whole)][dt]:
                    cand.append(s)
            picked += cand[:4]
        assert len(picked) >= 6
        tdt = torch.float32 if dt == mg.F32 else torch.float64
        for i, (m, n, k) in enumerate(picked):
            cfg = host.library_choice(tables, dt, m, n, k)
            print(f"builtin choice dt={dt} shape={(m, n, k)} cfg={cfg}", flush=True)
            A = synth.uniform_pm1((m, k), 700 + i)
            B = synth.uniform_pm1((k, n), 800 + i)
            if dt == mg.F32:
                A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
            tA, tB = torch.from_numpy(A).to(dev, tdt), torch.from_numpy(B).to(dev, tdt)
            c1 = torch.full((m, n), float("nan"), device=dev, dtype=tdt)
            c2 = torch.full((m, n), float("nan"), device=dev, dtype=tdt)
            mg.gemm(tA, tB, c1, 1.0, 0.0)
            mg.gemm(tA, tB, c2, 1.0, 0.0, cfg=cfg)
            torch.cuda.synchronize()
            assert torch.equal(c1, c2), (m, n, k)
            rows = np.array([0, m // 2, m - 1])
            ref = oracle.gemm_dot2(1.0, A[rows], B, nthreads=oracle.num_procs())
            got = c1[torch.from_numpy(rows).to(dev)].cpu().double().numpy()
            u = 2.0 ** -24 if dt == mg.F32 else 2.0 ** -53
            bound = (k + 2) * u / (1 - (k + 2) * u) * (np.abs(A[rows]) @ np.abs(B))
            assert np.all(np.abs(got - ref) <= bound), (m, n, k)


def test_choice_c_abi_matches_the_rule():
    """mgemm_choice (what gemm with no configuration runs, for 16-byte aligned
    bases) agrees with the plan written out in tests/choice_rule.py -- its
    configuration, k ranges and rows run whole -- on squares, held-out and aligned
    shapes, long-k and out-of-range shapes and odd leading dimensions, both dtypes;
    every branch of the plan (split-k on the two-stage and three-stage tiles, split
    tail, round fill, preference list and measured table) is taken at least once."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1706_10086_amd.csrc import gen_choice_table as gen
    import choice_rule as host
    mg.model_load(None)
    db = tune.load_compact(DB_PATH)
    tables = gen.build_tables(db.records, gen.training_shapes())
    squares = (512, 1024, 1536, 2048, 2560, 3072, 3584, 4096, 4608, 5120, 6144, 7168, 8192,
               9216, 12288, 16384, 20480)
    shapes = [(n, n, n, n, n) for n in squares]
    shapes += [(m, n, k, k, n) for (m, n, k) in
               tune.shape_set("heldout")[:150] + tune.shape_set("aligned")[:100]]
    # long k and shapes outside the measured range (split-k first)
    shapes += [(m, n, k, k, n) for (m, n, k) in
               ((256, 256, 8192), (512, 512, 16384), (128, 256, 20000), (64, 64, 4096),
                (1000, 1000, 3000), (100, 100, 30000), (40, 3000, 5000), (3000, 48, 2500))]
    # leading dimensions that break or keep the 16-byte rows
    shapes += [(6144, 6144, 6144, 6145, 6144), (3072, 3072, 3072, 3072, 3073),
               (3072, 3072, 3072, 3076, 3072), (512, 512, 16384, 16385, 512)]
    branches = collections.Counter()
    for dt in (mg.F64, mg.F32):
        for (m, n, k, lda, ldb) in shapes:
            cfg, splits, whole = mg.choice(m, n, k, dt, lda=lda, ldb=ldb, rows=True)
            want = host.library_plan(tables, dt, m, n, k, lda, ldb)
            assert (cfg.as_tuple(), splits, whole) == want, (dt, m, n, k, lda, ldb)
            c = want[0]
            if splits > 1:
                branches["split tail" if whole else
                          "split-k, three-stage" if c[5] == 2 else "split-k, two-stage"] += 1
            elif c == host.pref_choice(dt, m, n):
                branches["preference list"] += 1
            elif c[5] == 2:
                branches["round fill"] += 1
            else:
                branches["measured table"] += 1
    print(f"  {sum(branches.values())} plans agree: {dict(branches)}", flush=True)
    assert sum(branches.values()) >= 500
    assert len(branches) == 6 and min(branches.values()) >= 2, branches
    # the plans stated for squares: FP64 N = 1024 64 x 64, 6144 128 x 128, 8192
    # 256 x 128, all whole; 3072 21 tile rows whole and the last 3 in 3 k ranges
    assert mg.choice(1024, 1024, 1024)[0].as_tuple()[:2] == (64, 64)
    assert mg.choice(6144, 6144, 6144)[0].as_tuple()[:2] == (128, 128)
    assert mg.choice(8192, 8192, 8192)[0].as_tuple()[:2] == (256, 128)
    c3, s3, r3 = mg.choice(3072, 3072, 3072, rows=True)
    assert (c3.as_tuple()[:2], s3, r3) == ((128, 128), 3, 2688)
    # an odd leading dimension of A breaks the 16-byte rows: the measured table's
    # cell for that row class decides
    c_odd, s_odd = mg.choice(6144, 6144, 6144, lda=6145)
    assert s_odd == 1 and c_odd.double_buffer != 2
