// Batched (multi-frame) launches: a plan kernel orders the frames of a batch and numbers
// their tiles on the device, then one launch covers every planned tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "ramlt.h"

namespace ramlt {

// Work units of the batched launches (the planner gives frames whose filter_group differs
// from its group_sel no filter tiles; group_sel < 0 selects all).
constexpr int kStatsTilePixels = 256;

// Filter output tiles, by RAMLT_TILE_* kind (the default is 32 x 8).
struct TileWH {
  int w, h;
};
constexpr TileWH kTileShapes[4] = {{32, 8}, {32, 8}, {32, 16}, {64, 8}};

__host__ __device__ constexpr int tile_kind(int32_t flags) {
  return (flags & RAMLT_TILE_MASK) == RAMLT_TILE_DEFAULT ? RAMLT_TILE_32X8 : (flags & RAMLT_TILE_MASK);
}
__host__ __device__ constexpr int tile_w(int kind) { return kind == RAMLT_TILE_64X8 ? 64 : 32; }
__host__ __device__ constexpr int tile_h(int kind) { return kind == RAMLT_TILE_32X16 ? 16 : 8; }
static_assert(tile_w(RAMLT_TILE_64X8) == kTileShapes[RAMLT_TILE_64X8].w &&
                  tile_h(RAMLT_TILE_32X16) == kTileShapes[RAMLT_TILE_32X16].h &&
                  tile_w(RAMLT_TILE_32X8) == kTileShapes[RAMLT_TILE_32X8].w &&
                  tile_h(RAMLT_TILE_32X8) == kTileShapes[RAMLT_TILE_32X8].h,
              "tile table and accessors agree");

// Batched filter launches group frames by (radius, tile kind, loss in the forward pass).
__host__ __device__ constexpr int filter_group(const ramlt_frame &f) {
  return f.radius + 16 * tile_kind(f.flags) + ((f.flags & RAMLT_LOSS_IN_FORWARD) ? 64 : 0);
}
__host__ __device__ constexpr int group_radius(int group) { return group % 16; }
__host__ __device__ constexpr int group_kind(int group) { return (group / 16) % 4; }
__host__ __device__ constexpr bool group_loss_in_forward(int group) { return group >= 64; }
constexpr int kLossTilePixels = 1024;

// 256-pixel statistics tiles per batched work unit: enough that a unit reads >= 64
// samples per pixel slot (1 for S >= 64, at most 16).
__host__ __device__ inline int stats_unit_tiles(int S) {
  const int m = S >= 64 ? 1 : (64 + S - 1) / (S > 0 ? S : 1);
  return m > 16 ? 16 : m;
}

// Filter tiling, shared by the filter kernels and the batch planner. Output tiles are at
// most tile_w x tile_h of the frame's tile kind; when regions are >= 16 px wide and >= 4 px
// tall the tiles are laid out inside each region column / row (some may be empty).

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
  const int kind = tile_kind(f.flags);
  return (long long)tiles_along(f.W, f.n_regions, tile_w(kind), al) *
         tiles_along(f.H, f.n_regions, tile_h(kind), al);
}

// Division by a per-frame constant with one multiply: for 1 <= d < 2^31 and
// 0 <= n < 2^31, n / d == (n * m) >> s with s = 31 + ceil(log2 d), m = ceil(2^s / d)
// (Granlund and Montgomery, "Division by invariant integers using multiplication", PLDI
// 1994): with e = m d - 2^s in [0, d), n m / 2^s = n / d + n e / (d 2^s), and the excess
// is below 1 / d because n e < 2^31 2^ceil(log2 d) = 2^s, so the floor is exact.
struct FastDiv {
  uint32_t m, s;
};

constexpr __host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while (l < 31 && (1u << l) < d) ++l;
  const uint32_t s = 31 + l;
  return FastDiv{(uint32_t)((((uint64_t)1 << s) + d - 1) / d), s};
}

constexpr __host__ __device__ __forceinline__ uint32_t fast_div(uint32_t n, FastDiv D) {
  return (uint32_t)(((uint64_t)n * D.m) >> D.s);
}

// Compile-time check against plain division: every divisor up to 1024 and the powers of
// two and their neighbours up to 2^30, on numerators around multiples of the divisor and
// at the top of the range.
constexpr bool fastdiv_check_one(uint32_t d) {
  const FastDiv D = make_fastdiv(d);
  const uint32_t top = 0x7FFFFFFFu;
  const uint32_t ns[] = {0u, 1u, d - 1u, d, d + 1u, 2u * d - 1u, 2u * d, 1000u * d - 1u, top, top - 1u, top - d,
                         top / d * d, top / d * d - 1u};
  for (uint32_t n : ns)
    if (n <= top && fast_div(n, D) != n / d) return false;
  return true;
}

constexpr bool fastdiv_check() {
  for (uint32_t d = 1; d <= 1024; ++d)
    if (!fastdiv_check_one(d)) return false;
  for (uint32_t p = 1; p <= 30; ++p) {
    const uint32_t b = 1u << p;
    if (!fastdiv_check_one(b) || !fastdiv_check_one(b - 1) || !fastdiv_check_one(b + 1)) return false;
  }
  // divisors of the largest frames: 2W, 2H, 2N
  return fastdiv_check_one(131072u) && fastdiv_check_one(2u * 3840u) && fastdiv_check_one(2u * 2160u) &&
         fastdiv_check_one(2u * 1080u) && fastdiv_check_one(8192u) && fastdiv_check_one(40u);
}
static_assert(fastdiv_check(), "FastDiv disagrees with division");

// Filter tiling of one frame in a form the kernels decode without divide instructions.
// All numerators stay below 2^31: (2c + 1) N < 2^17 * 2^12, 2 k n < 2^30, tile indices
// < 2^31 (W, H <= 65536, W H <= 2^30, N <= 4096 are validated).
struct TileGeom {
  int32_t W, H, N, aligned;
  int32_t ntx, tpx, tpy, pad;
  FastDiv d_ntx, d_tpx, d_tpy, d_2N, d_2W, d_2H;
};

__host__ __device__ inline TileGeom make_geom(const ramlt_frame &f) {
  TileGeom g{};
  g.W = f.W;
  g.H = f.H;
  g.N = f.n_regions;
  g.aligned = aligned_tiling(f) ? 1 : 0;
  const int kind = tile_kind(f.flags);
  g.ntx = tiles_along(f.W, f.n_regions, tile_w(kind), g.aligned);
  g.tpx = g.aligned ? tiles_per_region(f.W, f.n_regions, tile_w(kind)) : 1;
  g.tpy = g.aligned ? tiles_per_region(f.H, f.n_regions, tile_h(kind)) : 1;
  g.d_ntx = make_fastdiv((uint32_t)g.ntx);
  g.d_tpx = make_fastdiv((uint32_t)g.tpx);
  g.d_tpy = make_fastdiv((uint32_t)g.tpy);
  g.d_2N = make_fastdiv(2u * (uint32_t)f.n_regions);
  g.d_2W = make_fastdiv(2u * (uint32_t)f.W);
  g.d_2H = make_fastdiv(2u * (uint32_t)f.H);
  return g;
}

static_assert(sizeof(TileGeom) == kPlanFrameBytes, "per-frame plan data is the tile geometry");

__host__ __device__ inline TileGeom *plan_geom(BatchPlan *p, int n_frames) {
  return (TileGeom *)plan_frame_data(p, n_frames);
}

// Enqueue the plan kernel: fills plan (order by cost, tile prefix sums, tile geometry).
hipError_t launch_plan(const ramlt_frame *frames_dev, int n, int op, int group_sel, BatchPlan *plan,
                       hipStream_t st);

// Distinct filter_group values of a batch, ascending; returns their count (at most
// kMaxFilterGroups).
constexpr int kMaxFilterGroups = 16 * 4 * 2;
int distinct_groups(const ramlt_frame *fh, int n, int *groups);

}  // namespace ramlt
