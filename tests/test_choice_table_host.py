"""The library's measured configuration choice (csrc/choice_table.h): the committed
table is what its generator derives from the shipped tuner database, and on the
database's held-out shapes (both row classes) the library's rule comes closer to the
exhaustive best than the preference list alone."""
import collections
import math
import os

import numpy as np
import pytest

from paper_1706_10086_amd import tune
from paper_1706_10086_amd.csrc import gen_choice_table as gen
import choice_rule
from choice_rule import library_choice, pref_choice

DATA = os.path.join(os.path.dirname(tune.__file__), "data", "tune_db.json.gz")

@pytest.fixture(scope="module")
def db():
    if not os.path.exists(DATA):
        pytest.skip("no shipped database")
    return tune.load_compact(DATA)


def test_committed_table_matches_the_generator(db):
    text = gen.render(gen.build_tables(db.records, gen.training_shapes()))
    with open(gen.OUT) as f:
        assert f.read() == text


@pytest.mark.parametrize("whole,floor", [(False, 0.92), (True, 0.92)])
def test_table_beats_the_preference_list_on_held_out_shapes(db, whole, floor):
    tables = gen.build_tables(db.records, gen.training_shapes())
    held = set(tune.shape_set("heldout"))
    per_shape = collections.defaultdict(dict)
    for r in db.records:
        per_shape[(r["dtype"], r["m"], r["n"], r["k"])][tuple(r["cfg"])] = r["tflops"]
    g = lambda a: math.exp(float(np.mean(np.log(a))))
    for dt in (0, 1):
        fp, ft = [], []
        for (d, m, n, k), v in per_shape.items():
            if d != dt or (m, n, k) not in held or gen.three_stage_ineligible(dt, n, k) == whole:
                continue
            best = max(v.values())
            fp.append(v[pref_choice(dt, m, n)] / best)
            ft.append(v[library_choice(tables, dt, m, n, k)] / best)
        assert len(ft) >= 30
        assert g(ft) >= floor and g(ft) > g(fp) + 0.05, (dt, whole, g(fp), g(ft))


def test_cells_name_registered_configurations(db):
    import paper_1706_10086_amd as mg
    tables = gen.build_tables(db.records, gen.training_shapes())
    for w in (0, 1):
        for dt in (0, 1):
            reg = {c.as_tuple() for c in mg.configs(dt)}
            assert set(tables[w][dt].values()) <= reg
            for (lm, ln, lk) in tables[w][dt]:
                assert all(gen.LO <= x <= gen.HI for x in (lm, ln, lk))


def test_plan_rule_on_squares(db):
    """The written-out plan on FP64 / FP32 squares: the whole-tile choices and the
    N = 3072 split tail as the library's documentation states them, and for every
    square N = 1024 ... 16384 in steps of 256 whose plan is a split tail: the whole
    rows are whole 128-row tiles that fill whole rounds of the compute units (one
    more tile row would not), and S x the tail's tiles fit the compute units."""
    tables = gen.build_tables(db.records, gen.training_shapes())
    plan = lambda dt, n: choice_rule.library_plan(tables, dt, n, n, n)
    assert plan(0, 1024)[0][:2] == (64, 64) and plan(0, 1024)[1:] == (1, 1024)
    assert plan(0, 2048)[0][:2] == (128, 128) and plan(0, 2048)[1] == 1
    assert plan(0, 6144)[0][:2] == (128, 128) and plan(0, 6144)[1] == 1
    assert plan(0, 8192)[0][:2] == (256, 128) and plan(0, 8192)[1] == 1
    assert plan(0, 3072) == (choice_rule.PIPE128[0], 3, 21 * 128)
    # N = 7680: 128 x 128 tiles whole in 14.06 rounds; the tail (one tile row of 60
    # tiles in 4 k ranges) is estimated 4.7 % faster, over the 2 % a 128 x 128 best
    # tile asks for
    assert plan(0, 7680) == (choice_rule.PIPE128[0], 4, 59 * 128)
    cus = choice_rule.CUS
    tails = 0
    for dt in (0, 1):
        for n in range(1024, 16385, 256):
            c, s, whole = plan(dt, n)
            if s == 1:
                assert whole == n
                continue
            tails += 1
            assert c == choice_rule.PIPE128[dt] and 0 < whole < n and whole % 128 == 0
            tn = -(-n // 128)
            rows, full = whole // 128, (-(-n // 128)) * tn // cus
            assert rows * tn <= full * cus < (rows + 1) * tn
            assert s * (-(-n // 128) - rows) * tn <= cus
            # k ranges: multiples of 256, the last one possibly shorter
            kc = -(-(-(-n // s)) // 256) * 256
            assert -(-n // kc) == s
    assert tails >= 6


def test_written_out_rule_uses_the_library_constants():
    """tests/choice_rule.py restates the plan with the library's own constants:
    preference lists, three-stage rates, fill and tail thresholds, split-k limits,
    the measured range and the tiles registered with a two-stage split-k kernel,
    read here from the C sources (the GPU test then checks the plans themselves)."""
    import re
    csrc = os.path.join(os.path.dirname(gen.__file__))
    api = open(os.path.join(csrc, "mgemm_api.hip")).read()
    tiled = open(os.path.join(csrc, "gemm_tiled.hip")).read()
    table = open(os.path.join(csrc, "choice_table.h")).read()

    def const(name, text=api):
        return float(re.search(rf"constexpr \w+ {name} = ([0-9.e]+);", text).group(1))

    def block(name):
        return api[api.index(name):api.index("};", api.index(name))]

    cfg = r"\{\{?(\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+)\}, ([0-9.]+)\}"
    for dt, suffix in ((0, "F64"), (1, "F32")):
        pref = [(tuple(int(x) for x in g[:7]), int(g[7]))
                for g in re.findall(cfg, block(f"kPref{suffix}[]"))]
        assert pref == choice_rule.PREF[dt]
        rates = [(tuple(int(x) for x in g[:7]), float(g[7]))
                 for g in re.findall(cfg, block(f"kPipeRates{suffix}[]"))]
        assert rates == choice_rule.PIPE_RATES[dt]
    assert const("WAVE_FILL_MIN") == choice_rule.WAVE_FILL_MIN
    assert const("TAIL_RATE_FACTOR") == choice_rule.TAIL_RATE_FACTOR
    assert const("SUM_BYTES_PER_S") == choice_rule.SUM_BYTES_PER_S
    assert const("TAIL_GAIN") == choice_rule.TAIL_GAIN
    assert const("TAIL_GAIN_LARGE") == choice_rule.TAIL_GAIN_LARGE
    assert const("SPLITK_MIN_K") == choice_rule.SPLITK_MIN_K
    assert const("SPLITK_FIRST_K") == choice_rule.SPLITK_FIRST_K
    assert const("SPLITK_MAX") == choice_rule.SPLITK_MAX
    assert 2 ** const("CHOICE_LOG2_LO", table) == choice_rule.MEASURED_LO
    assert 2 ** const("CHOICE_LOG2_HI", table) == choice_rule.MEASURED_HI
    # two-stage split-k kernels: MGEMM_REG_SPLITK(T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC)
    regs = {0: set(), 1: set()}
    for t, *v in re.findall(r"^\s*MGEMM_REG_SPLITK\((\w+), (\d+), (\d+), (\d+), (\d+), (\d+), "
                            r"(\d+), (\d+), (\d+)\)", tiled, flags=re.M):
        bm, bn, bk, wgm, wgn, ept, dbuf, occ = (int(x) for x in v)
        regs[1 if t == "float" else 0].add((bm, bn, bk, wgm * wgn, ept, dbuf, occ))
    assert regs == choice_rule.TWO_STAGE_SPLITK
    assert choice_rule.CUS == 256
