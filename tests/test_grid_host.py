"""The tuning grid the library compiles (csrc/gen_grid.py): the committed kernel
files are what the generator writes; every grid point is valid; at least 100 per
dtype, together covering every value of every axis of the grid (tile M/N/K 32-256,
waves 1/2/4/8, elements per thread 4/8/16, one or two LDS stages, occupancy 1/2);
both occupancies of each tile that admits them; and the library registers exactly
these points, for single GEMMs only."""
import os

import pytest

import paper_1706_10086_amd as mg
from paper_1706_10086_amd import tune
from paper_1706_10086_amd.csrc import gen_grid


def test_committed_files_match_the_generator():
    for name, text in gen_grid.all_files().items():
        with open(os.path.join(gen_grid.HERE, name)) as f:
            assert f.read() == text, name


@pytest.mark.parametrize("dt", [mg.F64, mg.F32])
def test_selection_covers_every_axis_value(dt):
    pts = gen_grid.selection(dt)
    assert len(pts) >= 100 and len(set(pts)) == len(pts)
    for p in pts:
        assert tune.grid_violations(dt, *p) == [], p
        assert p in set(tune.raw_grid())
    axes = (tune.GRID_TILES, tune.GRID_TILES, tune.GRID_TILES, tune.GRID_WAVES, tune.GRID_EPT,
            tune.GRID_DBUF, tune.GRID_OCC)
    for i, values in enumerate(axes):
        assert {p[i] for p in pts} == set(values), i
    # occupancy pairs: every tile valid at both occupancies in FP64 is there at both
    both = set(tune.both_occupancy_tiles(mg.F64))
    hand = gen_grid.hand_configs(dt)
    for t in both:
        for o in tune.GRID_OCC:
            assert t + (o,) in pts or t + (o,) in hand
    assert len(both) >= 40


@pytest.mark.parametrize("dt", [mg.F64, mg.F32])
def test_library_registers_the_grid(dt):
    try:
        mg.lib()
    except mg.MgemmNotBuilt:
        pytest.skip("libmgemm.so not built")
    reg = [c.as_tuple() for c in mg.configs(dt)]
    assert set(gen_grid.selection(dt)) | gen_grid.hand_configs(dt) == set(reg)
    assert len(reg) == len(set(reg))
    batched = {c.as_tuple() for c in mg.configs(dt, mg.CFG_BATCHED)}
    assert batched == gen_grid.hand_configs(dt)
    for i, c in enumerate(mg.configs(dt)):
        f = mg.lib().mgemm_config_flags(dt, i)
        assert f & mg.CFG_GEMM
        if c.as_tuple() in set(gen_grid.selection(dt)):
            assert f == mg.CFG_GEMM
    assert mg.lib().mgemm_config_flags(dt, len(reg)) == -2
    assert mg.lib().mgemm_config_flags(17, 0) == -1
