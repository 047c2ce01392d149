"""The learned tile-configuration model through the C ABI on the GPU: a network
saved by mlp_save is byte for byte the file the Python writer makes of the same
parameters; after mgemm_model_load, mgemm_model_predict gives the prediction of
learn.predict (the same features, the same kernels) on held-out shapes; and gemm
with no configuration then runs the predicted configuration, bit for bit, within
the oracle's error bound."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402
from paper_1706_10086_amd import learn, tune  # noqa: E402


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    table = learn.config_table()
    H = 32
    rng = np.random.default_rng(77)
    P = H * 6 + H + H * H + H + len(table) * H + len(table)
    params = (rng.standard_normal(P) * 0.5).astype(np.float32)
    mean = np.array([11.0, 10.0, 10.5, 0.5, 0.5, 0.0])
    std = np.array([2.0, 2.25, 1.5, 0.5, 0.5, 1.0])
    path = tmp_path_factory.mktemp("model") / "net.mlp"
    net = mg.MLP(6, H, len(table), params)
    try:
        net.save(str(path), table, mean, std)
    finally:
        net.destroy()
    pred = learn.Predictor(table, mean, std, params, H)
    yield path, pred
    mg.model_load(None)


def test_saved_file_matches_python_writer(model):
    path, pred = model
    assert path.read_text() == learn.model_text(pred.table, pred.mean, pred.std, pred.hidden,
                                                pred.params)


def test_predict_matches_learn_predict(model):
    path, pred = model
    mg.model_load(str(path))
    try:
        shapes = [(dt, *s) for dt in (mg.F64, mg.F32) for s in tune.shape_set("heldout")[:150]]
        want = learn.predict(pred, shapes)
        for (dt, m, n, k), slot in zip(shapes, want):
            got = mg.model_predict(m, n, k, dt)
            assert got.as_tuple() == pred.table[slot][1], (dt, m, n, k)
    finally:
        mg.model_load(None)


def test_gemm_runs_the_predicted_configuration(model):
    import oracle
    import synth
    path, pred = model
    dev = torch.device("cuda:0")
    mg.model_load(str(path))
    try:
        # shapes the built-in choice does not cut k on (k < 512, or a first choice
        # of 128 x 64 tiles), so that the model's choice is the one that runs
        shapes = [(1500, 1100, 400), (999, 2049, 300), (2048, 1536, 512), (777, 1333, 480)]
        for dt in (mg.F64, mg.F32):
            tdt = torch.float64 if dt == mg.F64 else torch.float32
            for i, (m, n, k) in enumerate(shapes):
                cfg = mg.model_predict(m, n, k, dt)
                print(f"model choice dt={dt} shape={(m, n, k)} cfg={cfg}", flush=True)
                A = synth.uniform_pm1((m, k), 9300 + 2 * i)
                B = synth.uniform_pm1((k, n), 9301 + 2 * i)
                if dt == mg.F32:
                    A, B = (x.astype(np.float32).astype(np.float64) for x in (A, B))
                tA, tB = torch.from_numpy(A).to(dev, tdt), torch.from_numpy(B).to(dev, tdt)
                c1 = torch.full((m, n), float("nan"), device=dev, dtype=tdt)
                c2 = torch.full((m, n), float("nan"), device=dev, dtype=tdt)
                mg.gemm(tA, tB, c1, 1.0, 0.0)
                mg.gemm(tA, tB, c2, 1.0, 0.0, cfg=cfg)
                torch.cuda.synchronize()
                assert torch.equal(c1, c2), (dt, m, n, k)
                rows = np.array([0, m // 2, m - 1])
                ref = oracle.gemm_dot2(1.0, A[rows], B, nthreads=oracle.num_procs())
                got = c1[torch.from_numpy(rows).to(dev)].cpu().double().numpy()
                u = 2.0 ** -24 if dt == mg.F32 else 2.0 ** -53
                bound = (k + 2) * u / (1 - (k + 2) * u) * (np.abs(A[rows]) @ np.abs(B))
                assert np.all(np.abs(got - ref) <= bound), (dt, m, n, k)
    finally:
        mg.model_load(None)
