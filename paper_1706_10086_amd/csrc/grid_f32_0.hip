// Tuning-grid kernels (F32), part 0 of 4: written by gen_grid.py, do not edit.
// Each entry: (bm, bn, bk, waves along m, waves along n, elements per thread,
// stages - 1, occupancy) with
// the two-stage kernel for aligned and for any rows (tile_gemm.h).
#include "tile_gemm.h"

namespace mgemm {

#define MGEMM_GRID_CFG(BM, BN, BK, WGM, WGN, EPT, DBUF, OCC)                          \
    {{BM, BN, BK, WGM * WGN, EPT, DBUF, OCC},                                           \
     &launch_tiled<float, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, true>,                  \
     &launch_tiled<float, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, false>,                 \
     nullptr, nullptr, {nullptr, nullptr}}

static const KernelEntry kGrid[] = {
    MGEMM_GRID_CFG(32, 32, 32, 1, 1, 4, 0, 1),
    MGEMM_GRID_CFG(32, 32, 32, 1, 1, 16, 0, 1),
    MGEMM_GRID_CFG(32, 32, 32, 1, 2, 4, 1, 1),
    MGEMM_GRID_CFG(32, 32, 32, 1, 2, 8, 1, 1),
    MGEMM_GRID_CFG(32, 32, 32, 2, 2, 4, 1, 1),
    MGEMM_GRID_CFG(32, 32, 64, 1, 2, 8, 0, 1),
    MGEMM_GRID_CFG(32, 32, 64, 2, 2, 4, 0, 1),
    MGEMM_GRID_CFG(32, 32, 64, 2, 2, 8, 0, 1),
    MGEMM_GRID_CFG(32, 32, 128, 2, 2, 4, 0, 1),
    MGEMM_GRID_CFG(32, 32, 128, 2, 2, 16, 0, 1),
    MGEMM_GRID_CFG(32, 64, 32, 1, 2, 8, 0, 1),
    MGEMM_GRID_CFG(32, 64, 32, 1, 4, 4, 1, 1),
    MGEMM_GRID_CFG(32, 64, 64, 1, 4, 8, 0, 1),
    MGEMM_GRID_CFG(32, 256, 32, 1, 4, 4, 0, 1),
    MGEMM_GRID_CFG(64, 32, 32, 2, 1, 8, 0, 1),
    MGEMM_GRID_CFG(64, 32, 32, 2, 2, 4, 1, 1),
    MGEMM_GRID_CFG(64, 32, 64, 2, 2, 8, 0, 1),
    MGEMM_GRID_CFG(64, 64, 32, 1, 2, 8, 0, 1),
    MGEMM_GRID_CFG(64, 64, 32, 2, 2, 4, 0, 1),
    MGEMM_GRID_CFG(64, 64, 32, 2, 2, 8, 0, 1),
    MGEMM_GRID_CFG(64, 64, 64, 2, 2, 4, 0, 1),
    MGEMM_GRID_CFG(64, 64, 64, 2, 2, 16, 0, 1),
    MGEMM_GRID_CFG(64, 128, 32, 1, 4, 8, 0, 1),
    MGEMM_GRID_CFG(128, 64, 32, 2, 2, 4, 0, 1),
    MGEMM_GRID_CFG(256, 32, 32, 4, 1, 4, 0, 1),
    MGEMM_GRID_CFG(256, 128, 32, 4, 2, 4, 0, 2),
    MGEMM_GRID_CFG(128, 128, 128, 2, 4, 4, 0, 2),
    MGEMM_GRID_CFG(256, 128, 32, 2, 2, 4, 1, 1),
};

const KernelEntry *grid_f32_part0(int *count) {
    *count = (int)(sizeof(kGrid) / sizeof(kGrid[0]));
    return kGrid;
}

}  // namespace mgemm
