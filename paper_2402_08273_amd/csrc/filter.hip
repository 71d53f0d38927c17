// Launches of the regional reconstruction filter, its adjoint and the MSE loss seed, for
// one frame or a batch (kernels: filter_kernels.hpp); the adjoint's fixed-order finalize
// and the standalone loss-seed kernels.
#include "filter_kernels.hpp"
#include "launch.hpp"

namespace ramlt {

namespace {

using namespace filt;

// Adds the per-tile partials in a fixed order. blockIdx.y = frame (its position q in a
// batch plan, or the single frame); block x < kFinalizeLamBlocks(N) sums regions, one wave
// per region (lane l takes the region's l-th, (l+64)-th, ... tile, then a butterfly sum);
// the block after those sums the frame's loss partials. One atomic add per region and per
// frame lands the result in grad_lambda / *loss.
constexpr int kFinalizeWaves = kFinalizeBlock / kWave;

__host__ __device__ inline int finalize_lam_blocks(int N) { return (N * N + kFinalizeWaves - 1) / kFinalizeWaves; }

// after_forward: the partials of the forward pass with the loss (RAMLT_LOSS_IN_FORWARD
// frames only), else those of the adjoint (the other frames).
__global__ __launch_bounds__(kFinalizeBlock) void backward_finalize_kernel(const ramlt_frame single,
                                                                        const ramlt_frame *__restrict__ frames,
                                                                        BatchPlan *plan, const float *lam_part,
                                                                        const double *loss_part, int after_forward) {
  __shared__ double red[kFinalizeWaves];
  ramlt_frame f;
  long long base = 0;
  if (plan) {
    const int q = blockIdx.y;
    f = frames[plan_order(plan)[q]];
    const long long *pre = plan_prefix(plan, plan->n_frames);
    if (pre[q + 1] == pre[q]) return;  // frame of another launch group: not in this plan
    base = pre[q];
  } else {
    f = single;
  }
  const bool lif = (f.flags & RAMLT_LOSS_IN_FORWARD) != 0;
  if (lif != (after_forward != 0)) return;
  const int N = f.n_regions;
  const bool al = aligned_tiling(f);
  const int tw = tile_w(tile_kind(f.flags)), th = tile_h(tile_kind(f.flags));
  const int ntx = tiles_along(f.W, N, tw, al), nty = tiles_along(f.H, N, th, al);
  const int nlb = finalize_lam_blocks(N);
  if ((int)blockIdx.x < nlb) {
    if (!f.grad_lambda || !al) return;
    const int k = blockIdx.x * kFinalizeWaves + threadIdx.x / kWave;
    if (k >= N * N) return;  // wave-uniform
    const int lane = threadIdx.x & (kWave - 1);
    const int tpx = tiles_per_region(f.W, N, tw), tpy = tiles_per_region(f.H, N, th);
    const int ky = k / N, kx = k - ky * N;
    float v = 0.f;
    for (int l = lane; l < tpx * tpy; l += kWave) {
      const int j = l / tpx, i = l - j * tpx;
      v += lam_part[base + (long long)(ky * tpy + j) * ntx + (kx * tpx + i)];
    }
    v = wave_sum(v);
    if (lane == 0 && v != 0.f) unsafeAtomicAdd(f.grad_lambda + k, v);
    return;
  }
  if ((int)blockIdx.x != nlb || !f.loss || (!lif && f.grad_out != nullptr)) return;
  const long long nt = (long long)ntx * nty;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  long long t = threadIdx.x;
  for (; t + 3 * kFinalizeBlock < nt; t += 4 * kFinalizeBlock) {
    acc0 += loss_part[base + t];
    acc1 += loss_part[base + t + kFinalizeBlock];
    acc2 += loss_part[base + t + 2 * kFinalizeBlock];
    acc3 += loss_part[base + t + 3 * kFinalizeBlock];
  }
  for (; t < nt; t += kFinalizeBlock) acc0 += loss_part[base + t];
  const double s = block_sum((acc0 + acc1) + (acc2 + acc3), red);
  if (threadIdx.x == 0) unsafeAtomicAdd(f.loss, s / (3.0 * (double)f.W * (double)f.H));
}

__global__ __launch_bounds__(kLossBlock) void loss_seed_kernel(const ramlt_frame f) {
  __shared__ double red[kLossBlock / kWave];
  const long long P = (long long)f.W * f.H;
  const long long per = (P + gridDim.x - 1) / gridDim.x;
  const long long p0 = (long long)blockIdx.x * per;
  if (p0 >= P) return;
  loss_range(f, p0, min(per, P - p0), red);
}

__global__ __launch_bounds__(kLossBlock) void loss_seed_batched_kernel(const ramlt_frame *__restrict__ frames,
                                                                       BatchPlan *plan) {
  __shared__ double red[kLossBlock / kWave];
  const unsigned long long total = plan->total_tiles;
  for (unsigned long long t = blockIdx.x; t < total; t += gridDim.x) {
    int fi;
    long long local;
    plan_lookup(plan, t, &fi, &local);
    const ramlt_frame f = frames[fi];
    const long long P = (long long)f.W * f.H;
    const long long p0 = local * kLossTilePixels;
    loss_range(f, p0, min((long long)kLossTilePixels, P - p0), red);  // ends with a barrier
  }
}

KindKernels kernels_of(int kind) {
  switch (kind) {
    case RAMLT_TILE_32X16: return kernels_32x16();
    case RAMLT_TILE_64X8: return kernels_64x8();
    default: return kernels_32x8();
  }
}

long long filter_tiles(const ramlt_frame &f) { return filter_tile_count(f); }

// Workspace of filter operations on a batch: per launch group (radius, tile kind) one
// plan, then (backward) the per-tile partials: lam float[T], loss double[T], T = tiles of
// all frames.
size_t partials_bytes(const ramlt_frame *fh, int n) {
  long long T = 0;
  for (int i = 0; i < n; ++i) T += filter_tiles(fh[i]);
  const size_t b = (size_t)T * (sizeof(float) + sizeof(double));
  return (b + 255) & ~(size_t)255;
}

// One workgroup per tile, in launches of at most kMaxTileGrid workgroups (a multiple of 8
// for the XCD-aware order).
constexpr long long kMaxTileGrid = 1LL << 22;

template <typename K, typename... Args>
hipError_t launch_tiles(K kernel, int block, long long tiles, hipStream_t st, const ramlt_frame &single,
                        const TileGeom &g, const ramlt_frame *fd, BatchPlan *plan, long long ntiles, Args... rest) {
  for (long long t0 = 0; t0 < tiles; t0 += kMaxTileGrid) {
    const unsigned grid = (unsigned)(((min(tiles - t0, kMaxTileGrid) + 7) / 8) * 8);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, st, single, g, fd, plan, ntiles, t0, rest...);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Partial-sum slots (dL/dlambda float[nt], loss double[nt]) at the start of ws.
void partial_slots(void *ws, long long nt, float **lam_part, double **loss_part) {
  *lam_part = (float *)ws;
  *loss_part = (double *)((char *)ws + (((size_t)nt * sizeof(float) + 7) & ~(size_t)7));
}

hipError_t launch_finalize(const ramlt_frame &single, const ramlt_frame *fd, BatchPlan *plan, int n, int nmax,
                           float *lam_part, double *loss_part, bool after_forward, hipStream_t st) {
  hipLaunchKernelGGL(backward_finalize_kernel, dim3(finalize_lam_blocks(nmax) + 1, n), dim3(kFinalizeBlock), 0, st,
                     single, fd, plan, lam_part, loss_part, after_forward ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_filter(bool bwd, const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws,
                         hipStream_t st) {
  if (n == 1) {
    const ramlt_frame &f = fh[0];
    const KindKernels K = kernels_of(tile_kind(f.flags));
    const TileGeom g = make_geom(f);
    const long long nt = filter_tiles(f);
    const bool lif = (f.flags & RAMLT_LOSS_IN_FORWARD) != 0;
    if (!bwd && !lif)
      return launch_tiles(K.forward[f.radius], K.fwd_block, nt, st, f, g, (const ramlt_frame *)nullptr,
                          (BatchPlan *)nullptr, nt, (float *)nullptr, (double *)nullptr);
    float *lam_part;
    double *loss_part;
    partial_slots(ws, nt, &lam_part, &loss_part);
    if (bwd && lif)  // the radiance adjoint alone: no partial sums
      return launch_tiles(K.radiance[f.radius], K.fwd_block, nt, st, f, g, (const ramlt_frame *)nullptr,
                          (BatchPlan *)nullptr, nt, (float *)nullptr, (double *)nullptr);
    hipError_t e = launch_tiles(bwd ? K.backward[f.radius] : K.forward_loss[f.radius], bwd ? K.block : K.fwd_block,
                                nt, st, f, g, (const ramlt_frame *)nullptr, (BatchPlan *)nullptr, nt, lam_part,
                                loss_part);
    if (e != hipSuccess) return e;
    return launch_finalize(f, nullptr, nullptr, 1, f.n_regions, lam_part, loss_part, !bwd, st);
  }
  int groups[kMaxFilterGroups];
  const int ng = distinct_groups(fh, n, groups);
  const size_t pb = plan_bytes(n);
  bool any_lif = false;
  for (int i = 0; i < n; ++i) any_lif |= (fh[i].flags & RAMLT_LOSS_IN_FORWARD) != 0;
  const bool parts = bwd || any_lif;
  const size_t part = parts ? partials_bytes(fh, n) : 0;
  long long T = 0;
  for (int i = 0; i < n; ++i) T += filter_tiles(fh[i]);
  int nmax = 1;
  for (int i = 0; i < n; ++i) nmax = max(nmax, fh[i].n_regions);
  const ramlt_frame none{};
  const TileGeom none_g{};
  for (int q = 0; q < ng; ++q) {
    const int radius = group_radius(groups[q]);
    const bool lif = group_loss_in_forward(groups[q]);
    const KindKernels K = kernels_of(group_kind(groups[q]));
    char *base = (char *)ws + (size_t)q * (pb + part);
    BatchPlan *plan = (BatchPlan *)base;
    float *lam_part = nullptr;
    double *loss_part = nullptr;
    if (parts) partial_slots(base + pb, T, &lam_part, &loss_part);
    hipError_t e = launch_plan(fd, n, bwd ? RAMLT_OP_FILTER_BACKWARD : RAMLT_OP_FILTER_FORWARD, groups[q], plan, st);
    if (e != hipSuccess) return e;
    long long tiles = 0;  // the planner counts the same tiles on the device
    for (int i = 0; i < n; ++i)
      if (filter_group(fh[i]) == groups[q]) tiles += filter_tiles(fh[i]);
    if (tiles == 0) continue;
    if (!bwd && !lif) {
      e = launch_tiles(K.forward_batched[radius], K.fwd_block, tiles, st, none, none_g, fd, plan, 0LL,
                       (float *)nullptr, (double *)nullptr);
      if (e != hipSuccess) return e;
      continue;
    }
    if (bwd && lif) {  // the radiance adjoint alone: no partial sums
      e = launch_tiles(K.radiance_batched[radius], K.fwd_block, tiles, st, none, none_g, fd, plan, 0LL,
                       (float *)nullptr, (double *)nullptr);
      if (e != hipSuccess) return e;
      continue;
    }
    e = launch_tiles(bwd ? K.backward_batched[radius] : K.forward_loss_batched[radius],
                     bwd ? K.block : K.fwd_block, tiles, st, none, none_g, fd, plan, 0LL, lam_part, loss_part);
    if (e != hipSuccess) return e;
    e = launch_finalize(none, fd, plan, n, nmax, lam_part, loss_part, !bwd, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_filter_forward(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws,
                                 hipStream_t st) {
  return launch_filter(false, fh, fd, n, ws, st);
}

hipError_t launch_filter_backward(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws,
                                  hipStream_t st) {
  return launch_filter(true, fh, fd, n, ws, st);
}

hipError_t launch_loss_seed(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws, hipStream_t st) {
  if (n == 1) {
    const long long P = (long long)fh[0].W * fh[0].H;
    long long blocks = (P + kLossTilePixels - 1) / kLossTilePixels;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(loss_seed_kernel, dim3((unsigned)blocks), dim3(kLossBlock), 0, st, fh[0]);
    return hipGetLastError();
  }
  BatchPlan *plan = (BatchPlan *)ws;
  hipError_t e = launch_plan(fd, n, RAMLT_OP_LOSS_SEED, -1, plan, st);
  if (e != hipSuccess) return e;
  long long tiles = 0;  // as counted by the planner
  for (int i = 0; i < n; ++i) tiles += ((long long)fh[i].W * fh[i].H + kLossTilePixels - 1) / kLossTilePixels;
  hipLaunchKernelGGL(loss_seed_batched_kernel, dim3((unsigned)min(tiles, kMaxBatchGrid)), dim3(kLossBlock), 0, st,
                     fd, plan);
  return hipGetLastError();
}

size_t workspace_bytes(const ramlt_frame *fh, int n, int op) {
  bool any_lif = false;
  for (int i = 0; i < n; ++i) any_lif |= (fh[i].flags & RAMLT_LOSS_IN_FORWARD) != 0;
  if (op == RAMLT_OP_FILTER_BACKWARD || (op == RAMLT_OP_FILTER_FORWARD && any_lif)) {
    if (n == 1) {
      const long long nt = filter_tiles(fh[0]);
      const size_t b = (((size_t)nt * sizeof(float) + 7) & ~(size_t)7) + (size_t)nt * sizeof(double);
      return (b + 255) & ~(size_t)255;
    }
    int groups[kMaxFilterGroups];
    return (size_t)distinct_groups(fh, n, groups) * (plan_bytes(n) + partials_bytes(fh, n));
  }
  if (n <= 1) return 0;
  if (op == RAMLT_OP_FILTER_FORWARD) {
    int groups[kMaxFilterGroups];
    return (size_t)distinct_groups(fh, n, groups) * plan_bytes(n);
  }
  return plan_bytes(n);
}

}  // namespace ramlt
