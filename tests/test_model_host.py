"""The tile-configuration model file, on the host: the Python writer and the
library agree on the format (hexadecimal floats, FNV-1a checksum), and
mgemm_model_load accepts a valid file and rejects a corrupt one, one naming a
configuration the library does not register, and one of the wrong shape -- all
before any device work (the network is evaluated only by mgemm_model_predict)."""
import numpy as np
import pytest

import paper_1706_10086_amd as mg
from paper_1706_10086_amd import learn


@pytest.fixture(scope="module")
def L():
    try:
        return mg._mlp_lib()
    except mg.MgemmNotBuilt:
        pytest.skip("libmgemm.so not built")


def _table():
    return [(dt, c.as_tuple()) for dt in (mg.F64, mg.F32) for c in mg.configs(dt)[:3]]


def _text(table, hidden=4, seed=3):
    rng = np.random.default_rng(seed)
    P = hidden * 6 + hidden + hidden * hidden + hidden + len(table) * hidden + len(table)
    params = rng.standard_normal(P).astype(np.float32)
    mean = np.array([10.0, 10.5, 9.25, 0.5, 0.5, 0.0])
    std = np.array([2.0, 1.75, 2.5, 0.5, 0.5, 1.0])
    return learn.model_text(table, mean, std, hidden, params), (mean, std, params)


def test_hex_floats_are_glibc_style():
    assert learn.c_hex(1.5) == "0x1.8p+0"
    assert learn.c_hex(1.0) == "0x1p+0"
    assert learn.c_hex(0.0) == "0x0p+0"
    assert learn.c_hex(-0.125) == "-0x1p-3"
    assert learn.c_hex(float(np.float32(0.1))) == "0x1.99999ap-4"
    for x in (1e-300, 5e-324, -3.75, 2.0 ** 60):
        assert float.fromhex(learn.c_hex(x)) == x


def test_python_round_trip(L):
    table = _table()
    text, (mean, std, params) = _text(table)
    t2, m2, s2, h2, p2 = learn.parse_model_text(text)
    assert t2 == table and h2 == 4
    assert np.array_equal(m2, mean) and np.array_equal(s2, std) and np.array_equal(p2, params)
    with pytest.raises(ValueError, match="checksum"):
        learn.parse_model_text(text.replace("mean 0x1.4p+3", "mean 0x1.5p+3"))


def test_library_loads_valid_and_rejects_bad_files(L, tmp_path):
    table = _table()
    good, _ = _text(table)
    p = tmp_path / "m.mlp"
    p.write_text(good)
    assert L.mgemm_model_load(str(p).encode()) == 0
    # a model is loaded: a dtype without outputs is argument 4's error
    c = mg.Cfg()
    assert L.mgemm_model_predict(64, 64, 64, mg.SPLIT_BF16, c) == -4
    assert L.mgemm_model_predict(0, 64, 64, mg.F64, c) == -1
    assert L.mgemm_model_predict(64, 64, 64, mg.F64, None) == -5

    # one changed digit: checksum mismatch; the model loaded before stays loaded
    bad = tmp_path / "corrupt.mlp"
    bad.write_text(good.replace("std 0x1p+1", "std 0x1p+2"))
    assert L.mgemm_model_load(str(bad).encode()) == mg.ERR_MODEL
    assert "checksum" in mg.last_error()
    assert L.mgemm_model_predict(64, 64, 64, mg.SPLIT_BF16, c) == -4

    # a valid file naming a configuration that is not registered
    other = table[:-1] + [(mg.F32, (48, 48, 16, 4, 2, 1, 0))]
    q = tmp_path / "mismatch.mlp"
    q.write_text(_text(other)[0])
    assert L.mgemm_model_load(str(q).encode()) == mg.ERR_MODEL
    assert "does not register" in mg.last_error()

    # wrong input count, wrong parameter count, truncated file, missing file
    t5 = learn.model_text(table, np.zeros(5), np.ones(5), 4, np.zeros(10, np.float32))
    (tmp_path / "i5.mlp").write_text(t5)
    assert L.mgemm_model_load(str(tmp_path / "i5.mlp").encode()) == mg.ERR_MODEL
    tp = learn.model_text(table, np.zeros(6), np.ones(6), 4, np.zeros(10, np.float32))
    (tmp_path / "p.mlp").write_text(tp)
    assert L.mgemm_model_load(str(tmp_path / "p.mlp").encode()) == mg.ERR_MODEL
    assert "parameter count" in mg.last_error()
    # a file of the earlier format (its sixth feature flagged SPLIT_BF16, not the
    # row alignment)
    body = good[:good.index("checksum ")].replace("mgemm-mlp 2", "mgemm-mlp 1", 1)
    v1 = body + f"checksum {learn.fnv1a64(body.encode()):016x}\n"
    (tmp_path / "v1.mlp").write_text(v1)
    assert L.mgemm_model_load(str(tmp_path / "v1.mlp").encode()) == mg.ERR_MODEL
    assert "version 2" in mg.last_error()
    with pytest.raises(ValueError, match="version 2"):
        learn.parse_model_text(v1)
    (tmp_path / "cut.mlp").write_text(good[: len(good) // 2])
    assert L.mgemm_model_load(str(tmp_path / "cut.mlp").encode()) == mg.ERR_MODEL
    assert L.mgemm_model_load(str(tmp_path / "absent.mlp").encode()) == mg.ERR_MODEL

    # unload: no model any more
    assert L.mgemm_model_load(None) == 0
    assert L.mgemm_model_predict(64, 64, 64, mg.F64, c) == mg.ERR_MODEL


def test_zero_std_rejected(L, tmp_path):
    table = _table()
    text = learn.model_text(table, np.zeros(6), np.array([1, 1, 1, 1, 1, 0.0]), 4,
                            np.zeros(4 * 6 + 4 + 16 + 4 + len(table) * 4 + len(table), np.float32))
    (tmp_path / "z.mlp").write_text(text)
    assert L.mgemm_model_load(str(tmp_path / "z.mlp").encode()) == mg.ERR_MODEL
