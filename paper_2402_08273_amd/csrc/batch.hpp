// Batched (multi-frame) launches: a plan kernel builds the tile queue of a batch on the
// device, then one persistent launch drains it.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "ramlt.h"

namespace ramlt {

// Tile counts per frame for each operation (frames whose radius differs from
// radius_sel get no tiles for the filter operations; radius_sel < 0 selects all).
constexpr int kStatsTilePixels = 256;
constexpr int kFilterTileW = 32;
constexpr int kFilterTileH = 8;
constexpr int kLossTilePixels = 1024;

// Enqueue the plan kernel: fills plan (order by cost, tile prefix sums, zeroed counter).
hipError_t launch_plan(const ramlt_frame *frames_dev, int n, int op, int radius_sel, BatchPlan *plan,
                       hipStream_t st);

// Number of workgroups that keeps every CU of the current device fully occupied with
// `kernel` at `block` threads (cached per kernel).
int persistent_grid(const void *kernel, int block);

// Distinct radii of a batch, ascending; returns their count (<= RAMLT_MAX_RADIUS + 1).
int distinct_radii(const ramlt_frame *fh, int n, int *radii);

}  // namespace ramlt
