// Host-side launchers of the ramlt kernels. Arguments are already validated by the
// C-ABI layer (abi.hip); these only size grids and enqueue on the given stream.
#pragma once

#include <hip/hip_runtime.h>

#include "ramlt.h"

namespace ramlt {

// fh: host descriptors; fd: device copy (may be null when n == 1); ws: workspace.
hipError_t launch_stats(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws, hipStream_t st);
hipError_t launch_filter_forward(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws,
                                 hipStream_t st);
hipError_t launch_loss_seed(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws, hipStream_t st);
hipError_t launch_filter_backward(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws,
                                  hipStream_t st);
size_t workspace_bytes(const ramlt_frame *fh, int n, int op);

// The whole step of one validated frame (flags with RAMLT_LOSS_IN_FORWARD): statistics,
// forward with the loss, radiance adjoint, in that order on st (step.hip).
hipError_t launch_step(const ramlt_frame &f, void *ws, hipStream_t st);

// The library's own device workspace of filter_backward_noalloc (noalloc.hip): this many
// bytes per GPU; *ptr = the current device's copy (resolved once per device).
constexpr size_t kNoallocWorkspaceBytes = RAMLT_NOALLOC_WORKSPACE_BYTES;
hipError_t noalloc_workspace(void **ptr);

// Regional adaptation (adapt.hip): n proposals, validated parameters and state.
hipError_t launch_region_adapt(const ramlt_adapt_params &p, const ramlt_region_state &s, const int32_t *region,
                               const float *alpha, long long n, void *ws, hipStream_t st);
size_t adapt_workspace_bytes(long long n, int m);

// Quadtree partitions (quadtree.hip): validated tree descriptor and arguments.
hipError_t launch_quadtree_init(const ramlt_quadtree &t, hipStream_t st);
hipError_t launch_quadtree_lookup(const ramlt_quadtree &t, const int32_t *root, const float *x, const float *y,
                                  int32_t *leaf, long long n, int count, hipStream_t st);
hipError_t launch_quadtree_refine(const ramlt_quadtree &t, int m_split, const ramlt_region_state *s, void *ws,
                                  hipStream_t st);
size_t quadtree_workspace_bytes(int capacity);

// Direction perturbation (perturb.hip): validated arguments.
hipError_t launch_perturb(const double *lambda, int m, const int32_t *region, const float *omega, const float *uv,
                          float *omega_out, float *theta_out, long long n, void *ws, hipStream_t st);
size_t perturb_workspace_bytes(int m);
// Lens-perturbation chain step (perturb.hip): validated arguments; ty = tx H / W; the
// workspace is perturb_workspace_bytes(N * N).
hipError_t launch_lens_step(const float *lum, int W, int H, float tx, float ty, const double *lambda, int N,
                            float *omega, float *density, int32_t *pixel, const float *noise, int32_t *region,
                            float *alpha, float *omega_prop, long long n, void *ws, hipStream_t st);

// Reorder of lens chains by screen tile (chains.hip): validated arguments; ty as for the
// step. Tiles are 2^lens_sort_tile_shift(W, H) pixels on a side.
int lens_sort_tile_shift(int W, int H);
size_t lens_sort_workspace_bytes(long long n);
hipError_t launch_lens_sort(int W, int H, float tx, float ty, const float *omega, const float *density, long long n,
                            float *omega_out, float *density_out, int32_t *perm, void *ws, hipStream_t st);

// rRMSE (rrmse.hip): validated arguments; P = W H pixels.
hipError_t launch_rrmse(const float *image, const float *reference, long long P, double eps, float *map,
                        double *out, void *ws, hipStream_t st);
size_t rrmse_workspace_bytes(long long P);

}  // namespace ramlt
