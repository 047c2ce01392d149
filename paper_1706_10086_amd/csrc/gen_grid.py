"""Writes the tuning-grid kernel registry: grid_f64_*.hip, grid_f32_*.hip and
grid_registry.h (committed; a host test checks them against this script).

    python -m paper_1706_10086_amd.csrc.gen_grid

Which points of the tuning grid are compiled (each point is a kernel of its own):

* every tile (bm, bn, bk, waves, elements per thread, stages) that is valid in
  FP64 at occupancy 1 and at occupancy 2, at both occupancies (these are valid in
  FP32 too; comparing the two occupancies of one tile measures the occupancy
  axis, the paper's hardware threads per core, Sec. 3, Tab. 4);
* per dtype, a fixed list of points valid at one occupancy only: the axis values
  the first set lacks (k-steps of 256, 8 waves per work-group, which need two
  waves per SIMD) and the large tiles that large products need;
* minus points that are hand-registered already (gemm_tiled.hip).

Each point gets the two-stage kernel for aligned and for any rows; grid points
take no part in batched plans or split-k.  The points are dealt round-robin into
PARTS files per dtype so that they compile in parallel.
"""
from __future__ import annotations

import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1706_10086_amd import F32, F64, tune  # noqa: E402

PARTS = 4
NAMES = {F64: ("f64", "double"), F32: ("f32", "float")}

# (bm, bn, bk, waves, elems_per_thread, double_buffer, occupancy)
EXTRA = {
    F64: [
        (32, 32, 256, 4, 4, 0, 1), (32, 32, 256, 4, 8, 0, 1),
        (256, 64, 32, 8, 4, 0, 2), (64, 256, 32, 8, 4, 0, 2), (128, 128, 32, 8, 4, 0, 2),
        (128, 128, 32, 8, 4, 1, 2), (128, 128, 64, 8, 4, 0, 2), (128, 128, 32, 8, 8, 0, 2),
        (128, 128, 32, 4, 4, 0, 1), (128, 128, 32, 4, 4, 1, 1), (128, 128, 64, 4, 4, 0, 1),
        (256, 64, 32, 4, 4, 0, 1), (64, 256, 32, 4, 4, 0, 1), (128, 128, 32, 4, 8, 1, 1),
    ],
    F32: [
        (32, 32, 256, 4, 4, 0, 1), (64, 64, 256, 8, 8, 0, 2),
        (256, 128, 32, 8, 4, 0, 2), (256, 128, 32, 8, 4, 1, 2), (128, 256, 32, 8, 4, 0, 2),
        (128, 128, 64, 8, 4, 0, 2), (128, 128, 128, 8, 4, 0, 2), (256, 128, 64, 8, 4, 0, 2),
        (256, 64, 64, 8, 4, 0, 2),
        (256, 128, 32, 4, 4, 0, 1), (256, 128, 32, 4, 4, 1, 1), (128, 256, 64, 4, 4, 0, 1),
        (128, 128, 128, 4, 4, 0, 1), (256, 64, 64, 4, 4, 0, 1),
    ],
}


def hand_configs(dtype: int) -> set:
    """Configurations registered by hand in gemm_tiled.hip (its registry macros)."""
    text = open(os.path.join(HERE, "gemm_tiled.hip")).read()
    tname = NAMES[dtype][1]
    out = set()
    for kind, args in re.findall(r"^\s*(MGEMM_CFG|MGEMM_REG_SPLITK|MGEMM_PIPE_CFG)\(([^)]*)\)",
                                 text, flags=re.M):
        a = [x.strip() for x in args.split(",")]
        if a[0] != tname:
            continue
        v = [int(x) for x in a[1:]]
        if kind == "MGEMM_PIPE_CFG":
            bm, bn, bk, wgm, wgn = v[:5]
            es = 4 if dtype == F32 else 8
            out.add((bm, bn, bk, wgm * wgn, 16 // es, 2, wgm * wgn // 4))
        else:
            bm, bn, bk, wgm, wgn, ept, dbuf, occ = v
            out.add((bm, bn, bk, wgm * wgn, ept, dbuf, occ))
    return out


def selection(dtype: int) -> list:
    pts = [t + (o,) for t in tune.both_occupancy_tiles(F64) for o in tune.GRID_OCC]
    pts += EXTRA[dtype]
    hand = hand_configs(dtype)
    out = []
    for p in pts:
        if p in hand or p in out:
            continue
        bad = tune.grid_violations(dtype, *p)
        if bad:
            raise ValueError(f"grid point {p} breaks {bad} for dtype {dtype}")
        out.append(p)
    return out


def render(dtype: int) -> dict:
    """File name -> text of every generated file for dtype, and grid_registry.h."""
    short, tname = NAMES[dtype]
    pts = selection(dtype)
    files = {}
    for part in range(PARTS):
        mine = pts[part::PARTS]
        lines = [
            f"// Tuning-grid kernels ({short.upper()}), part {part} of {PARTS}: written by "
            "gen_grid.py, do not edit.",
            "// Each entry: (bm, bn, bk, waves along m, waves along n, elements per thread,",
            "// stages - 1, occupancy) with",
            "// the two-stage kernel for aligned and for any rows (tile_gemm.h).",
            '#include "tile_gemm.h"',
            "",
            "namespace mgemm {",
            "",
            f"#define MGEMM_GRID_CFG(BM, BN, BK, WGM, WGN, EPT, DBUF, OCC)                          \\",
            "    {{BM, BN, BK, WGM * WGN, EPT, DBUF, OCC},                                           \\",
            f"     &launch_tiled<{tname}, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, true>,                  \\",
            f"     &launch_tiled<{tname}, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, false>,                 \\",
            "     nullptr, nullptr, {nullptr, nullptr}}",
            "",
            "static const KernelEntry kGrid[] = {",
        ]
        for (bm, bn, bk, w, e, d, o) in mine:
            wgm, wgn = tune.wave_layout(bm, bn, w)
            lines.append(f"    MGEMM_GRID_CFG({bm}, {bn}, {bk}, {wgm}, {wgn}, {e}, {d}, {o}),")
        lines += [
            "};",
            "",
            f"const KernelEntry *grid_{short}_part{part}(int *count) {{",
            "    *count = (int)(sizeof(kGrid) / sizeof(kGrid[0]));",
            "    return kGrid;",
            "}",
            "",
            "}  // namespace mgemm",
            "",
        ]
        files[f"grid_{short}_{part}.hip"] = "\n".join(lines)
    return files


def render_header() -> str:
    lines = ["// Tuning-grid kernel registry parts: written by gen_grid.py, do not edit.",
             "#pragma once", "", '#include "mgemm_internal.h"', "", "namespace mgemm {", "",
             f"constexpr int GRID_PARTS = {PARTS};", ""]
    for dt in (F64, F32):
        short = NAMES[dt][0]
        for part in range(PARTS):
            lines.append(f"const KernelEntry *grid_{short}_part{part}(int *count);")
        lines.append("")
    for dt in (F64, F32):
        short = NAMES[dt][0]
        getters = ", ".join(f"&grid_{short}_part{p}" for p in range(PARTS))
        lines.append(f"static const GridPartFn kGrid{short.upper()}Parts[GRID_PARTS] = {{{getters}}};")
    lines += ["", "}  // namespace mgemm", ""]
    return "\n".join(lines)


def all_files() -> dict:
    files = {"grid_registry.h": render_header()}
    for dt in (F64, F32):
        files.update(render(dt))
    return files


def main() -> int:
    for name, text in all_files().items():
        with open(os.path.join(HERE, name), "w") as f:
            f.write(text)
    for dt in (F64, F32):
        print(f"{NAMES[dt][0]}: {len(selection(dt))} grid points", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
