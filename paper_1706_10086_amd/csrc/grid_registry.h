// Tuning-grid kernel registry parts: written by gen_grid.py, do not edit.
#pragma once

#include "mgemm_internal.h"

namespace mgemm {

constexpr int GRID_PARTS = 4;

const KernelEntry *grid_f64_part0(int *count);
const KernelEntry *grid_f64_part1(int *count);
const KernelEntry *grid_f64_part2(int *count);
const KernelEntry *grid_f64_part3(int *count);

const KernelEntry *grid_f32_part0(int *count);
const KernelEntry *grid_f32_part1(int *count);
const KernelEntry *grid_f32_part2(int *count);
const KernelEntry *grid_f32_part3(int *count);

static const GridPartFn kGridF64Parts[GRID_PARTS] = {&grid_f64_part0, &grid_f64_part1, &grid_f64_part2, &grid_f64_part3};
static const GridPartFn kGridF32Parts[GRID_PARTS] = {&grid_f32_part0, &grid_f32_part1, &grid_f32_part2, &grid_f32_part3};

}  // namespace mgemm
