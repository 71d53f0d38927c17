// rRMSE of an image against a reference (Sec. 8.2): per pixel, the mean over the three
// channels of (I - R)^2 / (R^2 + eps) (fp64), its square root as the map (fp32), and the
// square root of the mean over pixels as the image value.
//
// One pass streams both images (24 B per pixel) and writes the map (4 B per pixel); every
// workgroup leaves the fp64 sum of its pixels in the workspace, and one workgroup adds the
// partials in a fixed order, so the image value does not depend on scheduling.
#include "launch.hpp"

#include <math.h>
#include <stdint.h>

namespace ramlt {

namespace {

constexpr int kErrBlock = 256;
constexpr int kErrPerThread = 8;
constexpr int kErrTile = kErrBlock * kErrPerThread;   // pixels per workgroup
constexpr int kErrWaves = kErrBlock / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over the workgroup: lanes, then waves in index order.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kErrWaves; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(kErrBlock) void rel_error_kernel(const float *__restrict__ image,
                                                              const float *__restrict__ reference, long long P,
                                                              double eps, float *__restrict__ map,
                                                              double *__restrict__ partial) {
  __shared__ double red[kErrWaves];
  const long long base = (long long)blockIdx.x * kErrTile;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < kErrPerThread; ++j) {
    const long long p = base + (long long)j * kErrBlock + threadIdx.x;
    if (p < P) {
      double e = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double r = reference[c * P + p];
        const double d = (double)image[c * P + p] - r;
        e += d * d / (r * r + eps);
      }
      e *= 1.0 / 3.0;
      if (map) map[p] = (float)sqrt(e);
      acc += e;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kErrBlock) void rel_error_finalize_kernel(const double *__restrict__ partial,
                                                                       int nparts, long long P,
                                                                       double *__restrict__ out) {
  __shared__ double red[kErrWaves];
  // four independent chains per thread keep four loads in flight; the order of every
  // addition is fixed by the thread and chain index
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b0 = 0; b0 < nparts; b0 += 4 * kErrBlock) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + q * kErrBlock + threadIdx.x;
      if (b < nparts) acc[q] += partial[b];
    }
  }
  const double s = block_sum((acc[0] + acc[1]) + (acc[2] + acc[3]), red);
  if (threadIdx.x == 0) *out = sqrt(s / (double)P);
}

}  // namespace

size_t rrmse_workspace_bytes(long long P) {
  const long long parts = (P + kErrTile - 1) / kErrTile;
  return ((size_t)parts * sizeof(double) + 255) / 256 * 256;
}

hipError_t launch_rrmse(const float *image, const float *reference, long long P, double eps, float *map,
                        double *out, void *ws, hipStream_t st) {
  const long long parts = (P + kErrTile - 1) / kErrTile;
  double *partial = (double *)ws;
  rel_error_kernel<<<(unsigned)parts, kErrBlock, 0, st>>>(image, reference, P, eps, map, partial);
  if (out) rel_error_finalize_kernel<<<1, kErrBlock, 0, st>>>(partial, (int)parts, P, out);
  return hipGetLastError();
}

}  // namespace ramlt
