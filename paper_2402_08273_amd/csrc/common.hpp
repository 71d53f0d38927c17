// Shared device-side helpers for the ramlt kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ramlt.h"

namespace ramlt {

constexpr int kWave = 64;

// Screen-grid region of a pixel centre: cell floor(N * (x + 1/2) / W) per axis, computed
// in integers (Sec. 5.2 state-dependent parameters over the Sec. 6.1 uniform grid).
// 32-bit unsigned arithmetic is exact: W, H <= 65536 and N <= 4096 are validated.
__device__ __forceinline__ int cell_of(int c, int n, int N) {
  return (int)(((unsigned)(2 * c + 1) * (unsigned)N) / (2u * (unsigned)n));
}
__device__ __forceinline__ int region_of(int x, int y, int W, int H, int N) {
  return cell_of(y, H, N) * N + cell_of(x, W, N);
}

// lambda clamped below at lambda_min; a NaN lambda stays NaN (fmaxf would return the bound).
__device__ __forceinline__ float clamp_lambda(float lam, float lambda_min) {
  return lam < lambda_min ? lambda_min : lam;
}

// 1/(2 sigma^2) for the region parameter lambda = log sigma^2 (Sec. 5.3), with lambda
// clamped below at lambda_min (NaN propagates).
__device__ __forceinline__ float half_inv_var(float lam, float lambda_min) {
  return 0.5f * expf(-clamp_lambda(lam, lambda_min));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Batched-launch bookkeeping kept in the caller's workspace. The plan kernel fills it at
// the start of every batched launch (stream-ordered, so it is safe under graph capture).
struct BatchPlan {
  unsigned long long reserved0;
  unsigned long long total_tiles;
  int n_frames;
  int pad1[11];
  // followed by: int order[n_frames]; long long prefix[n_frames + 1]; per-frame data
  // (kPlanFrameBytes each, by frame index)
};

// Bytes per frame of per-frame data the plan kernel stores after the prefix sums (the
// filter's tile geometry), 16-byte aligned.
constexpr size_t kPlanFrameBytes = 80;

__host__ __device__ inline size_t plan_frames_offset(int n_frames) {
  size_t b = sizeof(BatchPlan) + sizeof(int) * (size_t)n_frames;
  b = (b + 7) & ~(size_t)7;
  b += sizeof(long long) * (size_t)(n_frames + 1);
  return (b + 15) & ~(size_t)15;
}

__host__ __device__ inline size_t plan_bytes(int n_frames) {
  const size_t b = plan_frames_offset(n_frames) + kPlanFrameBytes * (size_t)n_frames;
  return (b + 255) & ~(size_t)255;
}

__host__ __device__ inline void *plan_frame_data(BatchPlan *p, int n_frames) {
  return (char *)p + plan_frames_offset(n_frames);
}

__host__ __device__ inline int *plan_order(BatchPlan *p) { return (int *)(p + 1); }
__host__ __device__ inline long long *plan_prefix(BatchPlan *p, int n_frames) {
  size_t b = sizeof(BatchPlan) + sizeof(int) * (size_t)n_frames;
  b = (b + 7) & ~(size_t)7;
  return (long long *)((char *)p + b);
}

// Locate the frame and frame-local tile (or unit) of planned position t.
__device__ __forceinline__ void plan_lookup(BatchPlan *plan, unsigned long long t, int *frame,
                                            long long *local) {
  const int n = plan->n_frames;
  const long long *pre = plan_prefix(plan, n);
  int lo = 0, hi = n;  // largest q with pre[q] <= t
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((unsigned long long)pre[mid] <= t) lo = mid; else hi = mid;
  }
  *frame = plan_order(plan)[lo];
  *local = (long long)t - pre[lo];
}

}  // namespace ramlt
