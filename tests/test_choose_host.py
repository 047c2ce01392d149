"""The run-time configuration chooser on the host: database hits give the
exhaustive best of the shipped sweep; shapes outside it fall back to the model
(GPU only) or to the library default."""
import pytest

import paper_1706_10086_amd as mg
from paper_1706_10086_amd import choose, tune


@pytest.fixture(scope="module")
def chooser():
    mg.lib()
    return choose.ConfigChooser()


def test_database_hit_is_the_exhaustive_best(chooser):
    db = tune.load_compact(choose.os.path.join(choose.DATA, "tune_db.json.gz"))
    for dt in (mg.F64, mg.F32):
        reg = {c.as_tuple() for c in mg.configs(dt)}
        for (m, n, k) in tune.shape_set("train")[:20]:
            cfg, source = chooser.choose(m, n, k, dt)
            assert source == "database"
            # the best measured configuration that is still registered
            best = max((r for r in db.records if r["dtype"] == dt and
                        (r["m"], r["n"], r["k"]) == (m, n, k) and tuple(r["cfg"]) in reg),
                       key=lambda r: r["tflops"])
            assert cfg.as_tuple() == tuple(best["cfg"])
            assert cfg.as_tuple() in {c.as_tuple() for c in mg.configs(dt)}


def test_unknown_shape_without_gpu_uses_the_default():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU evaluates the model instead")
    ch = choose.ConfigChooser()
    assert ch.choose(12345, 678, 91, mg.F64) == (None, "default")


def test_no_database_no_model():
    ch = choose.ConfigChooser(db_path=None, model_path=None)
    assert ch.choose(100, 100, 100, mg.F64) == (None, "default")
