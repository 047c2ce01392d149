"""Host logic of the autotuner and the learned predictor (no GPU): shape sets,
the resumable JSONL database, the compact database, exhaustive best and regret,
dataset construction and the single-configuration baseline."""
import collections
import json
import os

import numpy as np
import pytest

import paper_1706_10086_amd as mg
from paper_1706_10086_amd import learn, tune


def test_shape_sets_are_log_uniform_disjoint_and_fixed():
    tr = tune.shape_set("train")
    ho = tune.shape_set("heldout")
    assert len(tr) == 3000 and len(ho) == 500
    assert not set(tr) & set(ho)
    allv = np.array(tr + ho)
    assert allv.min() >= 64 and allv.max() <= 16384
    # log-uniform: about half of the values below the geometric midpoint 1024
    assert abs(np.mean(allv < 1024) - 0.5) < 0.03
    assert tune.shape_set("train")[:5] == tr[:5]


def rec(dt, m, n, k, cfg, tf, device="dev", build="b"):
    return {"device": device, "build": build, "dtype": dt, "m": m, "n": n, "k": k,
            "cfg": list(cfg), "tflops": tf, "best_ms": 1.0, "median_ms": 1.0}


def test_db_resumes_and_skips_corrupt_lines(tmp_path):
    p = tmp_path / "db.jsonl"
    db = tune.DB.load(str(p))
    db.append(rec(0, 64, 64, 64, (1, 2, 3, 4, 5, 6, 7), 1.0))
    db.append(rec(0, 64, 64, 64, (1, 2, 3, 4, 5, 6, 8), 2.0))
    with open(p, "a") as f:
        f.write('{"truncated": \n')
        f.write("not json\n")
    db2 = tune.DB.load(str(p))
    assert db2.bad_lines == 2 and len(db2.records) == 2
    assert ("dev", "b", 0, 64, 64, 64, (1, 2, 3, 4, 5, 6, 8)) in db2.keys()


def test_shape_records_expand_and_resume(tmp_path):
    """A sweep writes one line per shape (every configuration with its times); the
    database reads it as per-configuration records, and knows which shapes a
    device has done."""
    p = tmp_path / "db.jsonl"
    db = tune.DB.load(str(p))
    db.append({"device": "gpu0", "build": "b", "dtype": 1, "m": 100, "n": 200, "k": 300,
               "reps": 2, "cfgs": [[1, 2, 3, 4, 5, 6, 7], [7, 6, 5, 4, 3, 2, 1]],
               "ms": [[0.5, 0.7], [2.0]], "ts": 1.0})
    with open(p, "a") as f:
        f.write('{"device": "gpu0", "cfgs": [[1]], "ms": [[]], "dtype": 1}\n')   # no times
    db2 = tune.DB.load(str(p))
    assert db2.bad_lines == 1 and len(db2.records) == 2
    r0, r1 = sorted(db2.records, key=lambda r: r["cfg"])
    assert r0["median_ms"] == 0.6 and r0["best_ms"] == 0.5 and not r0["abandoned"]
    assert r1["abandoned"] and r1["tflops"] == pytest.approx(2 * 100 * 200 * 300 / 2e-3 / 1e12)
    assert db2.shapes_done("gpu0") == {(1, 100, 200, 300)}
    assert db2.shapes_done("other") == set()
    assert tune.exhaustive_best(db2, 1, 100, 200, 300)[0] == (1, 2, 3, 4, 5, 6, 7)


def test_exhaustive_best_and_regret():
    db = tune.DB("x", [rec(0, 8, 8, 8, (1,), 10.0), rec(0, 8, 8, 8, (2,), 40.0),
                       rec(0, 8, 8, 8, (3,), 30.0), rec(1, 8, 8, 8, (1,), 99.0)])
    cfg, tf = tune.exhaustive_best(db, 0, 8, 8, 8)
    assert cfg == (2,) and tf == 40.0
    assert tune.regret(db, 0, 8, 8, 8, (3,)) == pytest.approx(0.25)
    assert tune.regret(db, 0, 8, 8, 8, (2,)) == 0.0
    with pytest.raises(KeyError):
        tune.regret(db, 0, 8, 8, 8, (9,))


def test_compact_roundtrip(tmp_path):
    recs = [rec(0, 64, 128, 256, (128, 128, 16, 4, 2, 1, 0), 12.5),
            rec(0, 64, 128, 256, (64, 64, 16, 4, 2, 1, 0), 20.25),
            rec(1, 99, 100, 101, (32, 32, 16, 1, 2, 1, 0), 3.0)]
    db = tune.DB("x", recs)
    path = str(tmp_path / "c.json.gz")
    tune.save_compact(db, path)
    back = tune.load_compact(path)
    got = {(r["dtype"], r["m"], r["n"], r["k"], tuple(r["cfg"])): r["tflops"] for r in back.records}
    want = {(r["dtype"], r["m"], r["n"], r["k"], tuple(r["cfg"])): r["tflops"] for r in recs}
    assert got == want


def test_features_flag_whole_16_byte_rows():
    """The last feature is 1 exactly where the three-stage kernels could load the
    rows of an unpadded product: n and k multiples of 2 (FP64) or 4 (FP32)."""
    f = learn.raw_features
    assert np.allclose(f(100, 66, 64, 0), [np.log2(100), np.log2(66), 6, 1, 0, 1])
    assert f(100, 65, 64, 0)[5] == 0 and f(100, 66, 63, 0)[5] == 0
    assert f(100, 66, 64, 1)[5] == 0 and f(7, 68, 60, 1)[5] == 1
    assert learn.rows_whole_loads(64, 64, 0, lda=65) is False
    assert learn.rows_whole_loads(64, 64, 1, ldb=66) is False


def test_dataset_targets_masks_and_single_best():
    table = [(0, (1,)), (0, (2,)), (1, (1,))]
    recs = []
    shapes = [(0, 64, 64, 64), (0, 128, 64, 64), (1, 64, 64, 64), (0, 999, 1, 1)]
    tfs = {(0, 64, 64, 64): {(1,): 10.0, (2,): 20.0},
           (0, 128, 64, 64): {(1,): 30.0, (2,): 15.0},
           (1, 64, 64, 64): {(1,): 7.0},
           (0, 999, 1, 1): {(1,): 1.0}}            # incomplete: dropped
    for (dt, m, n, k), d in tfs.items():
        for c, v in d.items():
            recs.append(rec(dt, m, n, k, c, v))
    ds = learn.build_dataset(tune.DB("x", recs), table, shapes)
    assert ds.shapes == shapes[:3]
    assert np.allclose(ds.T, [[0.5, 1.0, 0.0], [1.0, 0.5, 0.0], [0.0, 0.0, 1.0]])
    assert np.array_equal(ds.M, [[1, 1, 0], [1, 1, 0], [0, 0, 1]])
    assert np.allclose(ds.X[0], [6, 6, 6, 1, 0, 1]) and np.allclose(ds.X[2], [6, 6, 6, 0, 1, 1])
    base = learn.single_best_baseline(ds, table)
    # geometric means of (0.5, 1.0) and (1.0, 0.5) tie: the first slot wins
    assert base[0] == 0 and base[1] == 2
    assert np.allclose(learn.achieved(ds, [1, 0, 2]), [1.0, 1.0, 1.0])
    s = learn.summarize(np.array([1.0, 0.5, 1.0, 1.0]))
    assert s["median"] == 1.0 and s["share_ge_0.95"] == 0.75
    assert s["geomean"] == pytest.approx(0.5 ** 0.25)


def test_model_file_checks_its_table():
    table = [(0, (1, 2)), (1, (3, 4))]
    pred = learn.Predictor(table, np.zeros(6), np.ones(6), np.zeros(10, dtype=np.float32))
    s = pred.to_json()
    back = learn.Predictor.from_json(s, check_table=table)
    assert back.table == table
    with pytest.raises(ValueError):
        learn.Predictor.from_json(s, check_table=[(0, (9, 9))])
    bad = json.loads(s)
    bad["table"][0][1][0] = 77
    with pytest.raises(ValueError):
        learn.Predictor.from_json(json.dumps(bad))


def test_shipped_database_covers_the_registry():
    path = os.path.join(os.path.dirname(learn.__file__), "data", "tune_db.json.gz")
    if not os.path.exists(path):
        pytest.skip("no shipped database")
    db = tune.load_compact(path)
    dts = {r["dtype"] for r in db.records}
    assert dts == {0, 1}
    n_shapes = len({(r["dtype"], r["m"], r["n"], r["k"]) for r in db.records})
    assert n_shapes == 14600         # train, train2, held-out, aligned; both dtypes
    # every shape measured with every registered configuration of its dtype
    import paper_1706_10086_amd as mg
    per = collections.Counter((r["dtype"], r["m"], r["n"], r["k"]) for r in db.records)
    want = {dt: len(mg.configs(dt)) for dt in (0, 1)}
    assert all(c == want[key[0]] for key, c in per.items())


def test_raw_grid_and_validity_rules():
    g = tune.raw_grid()
    assert len(g) == 3072 and len(set(g)) == 3072
    f64, f32 = set(tune.valid_grid(0)), set(tune.valid_grid(1))
    # FP32 halves the LDS and accumulator footprint: every valid FP64 point is a
    # valid FP32 point
    assert f64 < f32
    # each rule on a point that breaks it
    assert tune.grid_violations(0, 32, 32, 32, 8, 4, 0, 2) == ["mfma", "loads"]
    assert tune.grid_violations(0, 64, 32, 32, 2, 16, 1, 1) == ["loads"]
    assert tune.grid_violations(0, 64, 64, 32, 8, 4, 0, 1) == ["occ"]
    assert tune.grid_violations(0, 256, 256, 64, 4, 4, 1, 1) == ["lds", "acc"]
    assert tune.grid_violations(1, 128, 128, 128, 4, 4, 1, 1) == ["lds"]
    assert tune.grid_violations(0, 256, 256, 32, 8, 4, 0, 2) == ["acc"]
    # the same tile at one and at two waves per SIMD: two work-groups must fit the
    # LDS, and all registers must fit 256 per lane
    assert tune.grid_violations(0, 64, 64, 32, 4, 4, 1, 1) == []
    assert tune.grid_violations(0, 64, 64, 32, 4, 4, 1, 2) == []
    assert tune.grid_violations(0, 128, 128, 64, 4, 4, 0, 1) == []
    assert tune.grid_violations(0, 128, 128, 32, 4, 4, 0, 2) == ["regs"]
    assert tune.grid_violations(0, 128, 128, 32, 4, 4, 1, 2) == ["lds", "regs"]
    # occupancy 2 with 8 waves: one work-group of two waves per SIMD
    assert tune.grid_violations(0, 128, 128, 32, 8, 4, 0, 2) == []


def test_wave_layout_and_footprints():
    assert tune.wave_layout(256, 128, 8) == (4, 2)
    assert tune.wave_layout(128, 64, 4) == (2, 2)
    assert tune.wave_layout(32, 32, 4) == (2, 2)
    assert tune.wave_layout(32, 32, 8) is None
    # LDS of the kernels' padded stages (two-stage) and 16-byte units (three-stage)
    assert tune.lds_bytes(0, 128, 128, 16, 1) == 2 * (128 * 18 + 16 * 136) * 8
    assert tune.lds_bytes(1, 128, 128, 32, 1) == 2 * (128 * 34 + 32 * 144) * 4
    assert tune.lds_bytes(0, 256, 128, 16, 2) == 3 * 16 * (256 * 9 + 16 * 68)
    acc, other = tune.reg_estimate(0, 128, 128, 16, 4, 2, 1)
    assert acc == 128 and other > 0


def test_registry_lies_in_the_valid_space():
    """Every compiled configuration runs as specified: it breaks no rule, and the
    two-stage ones are points of the extended grid (k-steps of 16, 2-element runs
    and occupancy 0 added)."""
    assert len(tune.extended_grid()) == 7680
    for dt in (mg.F64, mg.F32):
        ext = set(tune.valid_grid(dt, extended=True))
        for c in mg.configs(dt):
            assert tune.grid_violations(dt, c.bm, c.bn, c.bk, c.waves, c.elems_per_thread,
                                        c.double_buffer, c.occupancy) == [], c.as_tuple()
            if c.double_buffer < 2:
                assert c.as_tuple() in ext, c.as_tuple()


def test_batch_rules_map_every_shape_to_a_registered_configuration():
    shapes = [(16, 16, 16), (31, 1000, 17), (48, 48, 900), (300, 700, 64), (1024, 1024, 1024),
              (600, 20, 512)]
    for dt in (mg.F64, mg.F32):
        reg = {c.as_tuple() for c in mg.configs(dt)}
        rules = tune.batch_rules(dt)
        # one rule per registered two-stage configuration that batched plans take,
        # plus the mixtures
        singles = [r for r in rules if r.startswith("all ")]
        assert len(singles) == sum(1 for c in mg.configs(dt, mg.CFG_BATCHED)
                                   if c.double_buffer < 2)
        reg = {c.as_tuple() for c in mg.configs(dt, mg.CFG_BATCHED)}
        assert len(rules) > len(singles)
        for name, rule in rules.items():
            got = {rule(m, n, k) for m, n, k in shapes}
            assert got <= reg, name
            assert all(c[5] < 2 for c in got), name        # never a three-stage entry
            assert len(got) <= 2, name
        # a mixture gives thin problems the smallest tile and the rest the 64x64 one
        mix = next(r for n_, r in rules.items() if n_.startswith("min(m,n) <= 32"))
        assert mix(31, 1000, 17)[:2] == (32, 32) and mix(300, 700, 64)[:2] == (64, 64)


def test_aligned_shape_set():
    al = tune.shape_set("aligned")
    assert len(al) == 800 and len(set(al)) == 800
    assert all(x % 4 == 0 and 64 <= x <= 16384 for s in al for x in s)
    assert not set(al) & (set(tune.shape_set("train")) | set(tune.shape_set("heldout")))
    assert tune.shape_set("aligned")[:7] == al[:7]
    t2 = tune.shape_set("train2")
    assert len(t2) == 3000 and len(set(t2)) == 3000
    assert all(64 <= x <= 16384 for s in t2 for x in s)
    assert not set(t2) & (set(tune.shape_set("train")) | set(tune.shape_set("heldout")) | set(al))
    assert t2[:3] == [(4124, 1073, 2042), (1103, 4803, 73), (1575, 13872, 3795)]
    with pytest.raises(ValueError):
        tune.shape_set("other")


def test_refinement_records_replace_the_sweeps_measurements(tmp_path):
    """A refinement pass re-times a shape's fastest configurations with more runs:
    its medians replace the sweep's for those configurations (the others keep the
    sweep's), the shape still counts as swept, and the exhaustive best is taken
    over the merged measurements."""
    p = tmp_path / "db.jsonl"
    db = tune.DB.load(str(p))
    fl = tune.flops(100, 200, 300)
    sweep = {"device": "d", "build": "b", "dtype": 0, "m": 100, "n": 200, "k": 300, "reps": 2,
             "cfgs": [[1, 1, 1, 1, 1, 1, 1], [2, 2, 2, 2, 2, 2, 2], [3, 3, 3, 3, 3, 3, 3]],
             "ms": [[1.0, 1.0], [0.9, 1.1], [2.0]]}
    db.append(sweep)
    assert tune.exhaustive_best(db, 0, 100, 200, 300)[0] == (1, 1, 1, 1, 1, 1, 1)
    refined = dict(sweep, reps=5, refine=True, cfgs=sweep["cfgs"][:2],
                   ms=[[1.2] * 5, [0.95, 0.96, 0.97, 0.98, 0.99]])
    db.append(refined)
    for d in (db, tune.DB.load(str(p))):
        rs = d.for_shape(0, 100, 200, 300)
        assert len(rs) == 3
        by = {tuple(r["cfg"]): r for r in rs}
        assert by[(1, 1, 1, 1, 1, 1, 1)]["median_ms"] == 1.2 and by[(1, 1, 1, 1, 1, 1, 1)]["refined"]
        assert by[(3, 3, 3, 3, 3, 3, 3)]["median_ms"] == 2.0 and not by[(3, 3, 3, 3, 3, 3, 3)]["refined"]
        cfg, tf = tune.exhaustive_best(d, 0, 100, 200, 300)
        assert cfg == (2, 2, 2, 2, 2, 2, 2) and tf == pytest.approx(fl / (0.97e-3) / 1e12)
        assert d.shapes_done("d") == {(0, 100, 200, 300)}
        assert d.shapes_refined("d") == {(0, 100, 200, 300)}


def test_shipped_model_file_matches_the_registry():
    """The shipped model file parses (checksum, syntax), has one output per
    registered configuration in registry order, and standardises the six inputs."""
    path = os.path.join(os.path.dirname(tune.__file__), "data", "model.mlp")
    pred = learn.Predictor.load(path, check_table=learn.config_table())
    assert len(pred.mean) == 6 and len(pred.std) == 6 and pred.hidden == 64
    I, H, O = 6, 64, len(pred.table)
    assert pred.params.size == H * I + H + H * H + H + O * H + O
    assert np.all(np.isfinite(pred.params))


def _shape_line(dt, m, n, k, cfgs, ms, refine=False, device="dev"):
    r = {"device": device, "build": "b", "dtype": dt, "m": m, "n": n, "k": k, "reps": len(ms[0]),
         "cfgs": [list(c) for c in cfgs], "ms": ms, "ts": 1.0}
    if refine:
        r["refine"] = True
    return json.dumps(r) + "\n"


def test_top_n_selection_for_added_configurations():
    """Shapes are refined again only where an added configuration ranks among the
    N fastest."""
    A, B, C = (1,) * 7, (2,) * 7, (3,) * 7
    recs = []
    for (m, t) in ((64, {A: 1.0, B: 2.0, C: 3.0}), (128, {A: 3.0, B: 1.0, C: 2.0})):
        for c, v in t.items():
            r = rec(0, m, 64, 64, c, 1.0)
            r["median_ms"] = v
            recs.append(r)
    db = tune.DB("x", recs)
    shapes = [(64, 64, 64), (128, 64, 64), (256, 64, 64)]
    assert tune.shapes_with_top(db, 0, shapes, [C], 2) == [(128, 64, 64)]
    assert tune.shapes_with_top(db, 0, shapes, [C], 3) == [(64, 64, 64), (128, 64, 64)]
    assert tune.shapes_with_top(db, 1, shapes, [C], 3) == []


def test_merge_lets_later_refinements_replace_earlier_ones(tmp_path):
    """merge_databases: the update databases' refinement of a shape replaces the
    base databases' refinement of that shape (both passes timed the shape's fastest
    configurations; the later one includes the configurations added since), so a
    configuration the later pass left out falls back to its sweep measurement;
    shapes the update did not refine keep theirs; added configurations join."""
    A, B, N = (1,) * 7, (2,) * 7, (9,) * 7
    base = tmp_path / "base.jsonl"
    upd = tmp_path / "upd.jsonl"
    n = 1024
    f = 2.0 * n ** 3 / 1e9                     # TFLOP/s = f / ms for n^3
    with open(base, "w") as fh:
        fh.write(_shape_line(0, n, n, n, [A, B], [[4.0, 4.0], [2.0, 2.0]]))
        fh.write(_shape_line(0, n, n, n, [A, B], [[3.0] * 5, [1.0] * 5], refine=True))
        fh.write(_shape_line(0, 2 * n, n, n, [A, B], [[4.0, 4.0], [2.0, 2.0]]))
        fh.write(_shape_line(0, 2 * n, n, n, [B], [[1.5] * 5], refine=True))
    with open(upd, "w") as fh:
        fh.write(_shape_line(0, n, n, n, [N], [[0.5, 0.5]]))
        fh.write(_shape_line(0, n, n, n, [N, B], [[0.8] * 5, [1.6] * 5], refine=True))
        fh.write(_shape_line(0, 2 * n, n, n, [N], [[8.0, 8.0]]))
    out = tmp_path / "m.json.gz"
    tune.main(["--merge", str(out), "--from", str(base), "--update", str(upd)])
    db = tune.load_compact(str(out))
    tf = {(r["m"], tuple(r["cfg"])): r["tflops"] for r in db.records}
    # n^3: the update refined N and B; A falls back to its sweep (4.0 ms)
    assert tf[(n, N)] == pytest.approx(f / 0.8, rel=1e-4)
    assert tf[(n, B)] == pytest.approx(f / 1.6, rel=1e-4)
    assert tf[(n, A)] == pytest.approx(f / 4.0, rel=1e-4)
    # 2n x n x n: not refined by the update, so the base refinement of B stays
    assert tf[(2 * n, B)] == pytest.approx(2 * f / 1.5, rel=1e-4)
    assert tf[(2 * n, A)] == pytest.approx(2 * f / 4.0, rel=1e-4)
    assert tf[(2 * n, N)] == pytest.approx(2 * f / 8.0, rel=1e-4)
    with pytest.raises(SystemExit):
        tune.main(["--dtype", "f64"])
