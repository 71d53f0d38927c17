// Device-side planning of batched launches.
//
// For a batch of frames the plan kernel computes each frame's tile (or work-unit) count,
// orders frames by per-tile cost (samples per pixel for the statistics pass; uniform
// otherwise), largest first, so that the costliest workgroups are dispatched first and
// the tail of the launch is made of cheap ones (longest-processing-time-first), and
// writes the exclusive prefix of tile counts in that order. A batched launch then runs
// one workgroup per planned tile, which finds its frame by binary search of the prefix.
// Everything stays on the device and in stream order, so a batch can be captured in a
// graph.
#include <utility>

#include "batch.hpp"

namespace ramlt {

namespace {

constexpr int kPlanBlock = 256;

__device__ long long tiles_of(const ramlt_frame &f, int op, int group_sel) {
  const long long P = (long long)f.W * f.H;
  switch (op) {
    case RAMLT_OP_STATS: {
      const long long unit = (long long)kStatsTilePixels * stats_unit_tiles(f.S);
      return (P + unit - 1) / unit;
    }
    case RAMLT_OP_LOSS_SEED:
      return (P + kLossTilePixels - 1) / kLossTilePixels;
    default:
      if (group_sel >= 0 && filter_group(f) != group_sel) return 0;
      return filter_tile_count(f);
  }
}

__device__ long long cost_of(const ramlt_frame &f, int op) { return op == RAMLT_OP_STATS ? f.S : 1; }

__global__ __launch_bounds__(kPlanBlock) void plan_kernel(const ramlt_frame *__restrict__ frames, int n, int op,
                                                          int group_sel, BatchPlan *plan) {
  int *order = plan_order(plan);
  long long *prefix = plan_prefix(plan, n);
  // rank = number of frames that go before frame i (higher cost, or equal cost and
  // lower index)
  if (op == RAMLT_OP_FILTER_FORWARD || op == RAMLT_OP_FILTER_BACKWARD) {  // validated filter frames
    TileGeom *geom = plan_geom(plan, n);
    for (int i = threadIdx.x; i < n; i += kPlanBlock) geom[i] = make_geom(frames[i]);
  }
  for (int i = threadIdx.x; i < n; i += kPlanBlock) {
    const long long ci = cost_of(frames[i], op);
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const long long cj = cost_of(frames[j], op);
      rank += (cj > ci) || (cj == ci && j < i);
    }
    order[rank] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = 0;
    for (int q = 0; q < n; ++q) {
      prefix[q] = acc;
      acc += tiles_of(frames[order[q]], op, group_sel);
    }
    prefix[n] = acc;
    plan->n_frames = n;
    plan->total_tiles = (unsigned long long)acc;
    plan->reserved0 = 0ULL;
  }
}

}  // namespace

hipError_t launch_plan(const ramlt_frame *frames_dev, int n, int op, int group_sel, BatchPlan *plan,
                       hipStream_t st) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanBlock), 0, st, frames_dev, n, op, group_sel, plan);
  return hipGetLastError();
}

int distinct_groups(const ramlt_frame *fh, int n, int *groups) {
  bool seen[kMaxFilterGroups] = {};
  for (int i = 0; i < n; ++i) {
    const int g = filter_group(fh[i]);
    if (g >= 0 && g < kMaxFilterGroups) seen[g] = true;
  }
  int k = 0;
  for (int g = 0; g < kMaxFilterGroups; ++g)
    if (seen[g]) groups[k++] = g;
  return k;
}

}  // namespace ramlt
