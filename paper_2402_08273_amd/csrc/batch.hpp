// Batched (multi-frame) launches: a plan kernel orders the frames of a batch and numbers
// their tiles on the device, then one launch covers every planned tile.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "ramlt.h"

namespace ramlt {

// Work units of the batched launches (the planner gives frames whose radius differs from
// its radius_sel no filter tiles; radius_sel < 0 selects all).
constexpr int kStatsTilePixels = 256;
constexpr int kFilterTileW = 32;
constexpr int kFilterTileH = 8;
constexpr int kLossTilePixels = 1024;

// 256-pixel statistics tiles per batched work unit: enough that a unit reads >= 64
// samples per pixel slot (1 for S >= 64, at most 16).
__host__ __device__ inline int stats_unit_tiles(int S) {
  const int m = S >= 64 ? 1 : (64 + S - 1) / (S > 0 ? S : 1);
  return m > 16 ? 16 : m;
}

// Filter tiling, shared by the filter kernels and the batch planner. Output tiles are at
// most kFilterTileW x kFilterTileH; when regions are >= 16 px wide and >= 4 px tall the
// tiles are laid out inside each region column / row (some may be empty).

// First coordinate (of n) whose cell floor((2c + 1) N / (2n)) is >= k. Every region is
// at most ceil(n / N) wide. 32-bit arithmetic: n <= 65536 and N <= 4096 (validated).
__host__ __device__ inline int region_start(int k, int n, int N) {
  if (k <= 0) return 0;
  if (k >= N) return n;
  // (2c + 1) N >= 2 k n  <=>  c >= (2 k n - N) / (2 N)
  const int num = 2 * k * n - N;
  const int c = num <= 0 ? 0 : (int)(((unsigned)num + 2u * (unsigned)N - 1u) / (2u * (unsigned)N));
  return c > n ? n : c;
}

__host__ __device__ inline bool aligned_tiling(const ramlt_frame &f) {
  return f.W >= 16 * f.n_regions && f.H >= 4 * f.n_regions;
}

// Tiles per region along an axis when aligned.
__host__ __device__ inline int tiles_per_region(int n, int N, int T) { return ((n + N - 1) / N + T - 1) / T; }

__host__ __device__ inline int tiles_along(int n, int N, int T, bool aligned) {
  return aligned ? N * tiles_per_region(n, N, T) : (n + T - 1) / T;
}

// (0 for an invalid frame, so workspace queries on unvalidated descriptors are safe)
__host__ __device__ inline long long filter_tile_count(const ramlt_frame &f) {
  if (f.W < 1 || f.H < 1 || f.n_regions < 1 || f.W > RAMLT_MAX_SIDE || f.H > RAMLT_MAX_SIDE ||
      f.n_regions > RAMLT_MAX_REGIONS)
    return 0;
  const bool al = aligned_tiling(f);
  return (long long)tiles_along(f.W, f.n_regions, kFilterTileW, al) * tiles_along(f.H, f.n_regions, kFilterTileH, al);
}

// Enqueue the plan kernel: fills plan (order by cost, tile prefix sums).
hipError_t launch_plan(const ramlt_frame *frames_dev, int n, int op, int radius_sel, BatchPlan *plan,
                       hipStream_t st);

// Distinct radii of a batch, ascending; returns their count (<= RAMLT_MAX_RADIUS + 1).
int distinct_radii(const ramlt_frame *fh, int n, int *radii);

}  // namespace ramlt
