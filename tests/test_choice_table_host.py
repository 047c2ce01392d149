"""The built-in configuration for rows the three-stage kernels cannot load
(csrc/choice_table.h): the committed table is what its generator derives from the
shipped tuner database, and on the database's held-out shapes it comes closer to the
exhaustive best than the preference list it replaces there."""
import collections
import math
import os

import numpy as np
import pytest

from paper_1706_10086_amd import tune
from paper_1706_10086_amd.csrc import gen_choice_table as gen

DATA = os.path.join(os.path.dirname(tune.__file__), "data", "tune_db.json.gz")

# the library's preference list (csrc/mgemm_api.hip), used where the table is not
PREF = {0: [((256, 128, 16, 8, 2, 2, 2), 512), ((128, 128, 16, 8, 2, 2, 2), 256),
            ((128, 64, 32, 4, 4, 0, 2), 256), ((64, 64, 16, 4, 2, 1, 0), 256),
            ((32, 32, 16, 1, 2, 1, 0), 0)],
        1: [((256, 128, 32, 8, 4, 2, 2), 512), ((128, 128, 32, 8, 4, 2, 2), 256),
            ((128, 64, 32, 4, 4, 1, 0), 256), ((64, 64, 16, 4, 2, 1, 0), 256),
            ((32, 32, 16, 1, 2, 1, 0), 0)]}


def pref_choice(dt, m, n):
    pl = PREF[dt]
    for i, (c, min_tiles) in enumerate(pl):
        if i + 1 < len(pl) and (-(-m // c[0])) * (-(-n // c[1])) < min_tiles:
            continue
        return c


@pytest.fixture(scope="module")
def db():
    if not os.path.exists(DATA):
        pytest.skip("no shipped database")
    return tune.load_compact(DATA)


def test_committed_table_matches_the_generator(db):
    text = gen.render(gen.build_table(db.records, set(tune.shape_set("train"))))
    with open(gen.OUT) as f:
        assert f.read() == text


def test_table_beats_the_preference_list_on_held_out_shapes(db):
    table = gen.build_table(db.records, set(tune.shape_set("train")))
    held = set(tune.shape_set("heldout"))
    per_shape = collections.defaultdict(dict)
    for r in db.records:
        per_shape[(r["dtype"], r["m"], r["n"], r["k"])][tuple(r["cfg"])] = r["tflops"]
    for dt in (0, 1):
        fp, ft = [], []
        for (d, m, n, k), v in per_shape.items():
            if d != dt or (m, n, k) not in held or not gen.three_stage_ineligible(dt, n, k):
                continue
            best = max(v.values())
            cp = pref_choice(dt, m, n)
            ct = table[dt].get(gen.cell_of(m, n, k), cp)
            fp.append(v[cp] / best)
            ft.append(v[ct] / best)
        g = lambda a: math.exp(float(np.mean(np.log(a))))
        assert len(ft) > 300
        assert g(ft) >= 0.95 and g(ft) > g(fp) + 0.05, (dt, g(fp), g(ft))


def test_cells_name_registered_configurations(db):
    import paper_1706_10086_amd as mg
    table = gen.build_table(db.records, set(tune.shape_set("train")))
    for dt in (0, 1):
        reg = {c.as_tuple() for c in mg.configs(dt)}
        assert set(table[dt].values()) <= reg
        for (lm, ln, lk) in table[dt]:
            assert all(gen.LO <= x <= gen.HI for x in (lm, ln, lk))
