// Reorder of screen-space lens chains by where they are on the screen, for the locality of
// the chain step's luminance reads.
//
// The chains of the lens perturbation (Sec. 3.3 "Lens Perturbation", Sec. 6.1 "2d Partition
// for the Lens Perturbation") are independent; their order in memory is free. In index order
// their pixels are scattered over the whole image, so every luminance read of a step fetches a
// cache line of its own. Grouped by screen tile, the chains of a workgroup read a few KB of
// the image, which stay in cache, and a chain moves a few pixels per accepted step, so the
// grouping lasts for many steps.
//
// The key of chain i is the T x T pixel tile of its current pixel (the step's raster map,
// raster.hpp), tiles numbered row-major, and the number of tiles for a chain outside the
// frame or NaN; T is the smallest power of two >= 16 that leaves at most 63 tiles (256 px at
// 1920 x 1080: a tile's luminance, 256 KB, stays in one XCD's L2), so keys fit 6 bits and one
// pass of a stable radix sort groups them:
//   1. per workgroup of kChainTile chains, a histogram of the keys (LDS atomics);
//   2. an exclusive scan of the histograms, digit-major (a workgroup per digit row, then
//      one over the row totals): the first destination of every (digit, workgroup) run;
//   3. per workgroup, each chain's rank among the chains of its digit in index order (one
//      ballot per key bit and per-wave running counts in LDS), the ranked positions placed
//      in LDS in key order, and the chains written out run by run: omega, density and the
//      chain's old index. A chain keeps its place among the chains of its tile.
// Few keys and large workgroups make long runs (about 100 chains of each tile per workgroup
// at 1080p), so the output lines are written whole: with 510 tiles of 64 px and 2048 chains
// per workgroup, runs of 4 chains wrote every line in pieces from different XCDs and the
// scatter took 0.5 ms for 16 M chains.
#include "launch.hpp"
#include "raster.hpp"

#include <stdint.h>

namespace ramlt {

namespace {

constexpr int kChainBlock = 256;
constexpr int kChainItems = 16;
constexpr int kChainTile = kChainBlock * kChainItems;  // chains per workgroup
constexpr int kKeyBits = 6;
constexpr int kKeys = 1 << kKeyBits;  // tiles 0 .. ntiles - 1, ntiles = outside the frame
constexpr int kWaves = kChainBlock / 64;
constexpr int kWaveChunk = kChainTile / kWaves;  // chains per wave, ranked 64 per round
constexpr int kRounds = kWaveChunk / 64;
constexpr int kScanBlock = 1024;
static_assert(kChainTile <= 65536, "positions inside a workgroup's tile fit 16 bits");

struct SortGeom {
  int W, H, shift, ntx, ntiles;
  float tx, ty;
};

__device__ __forceinline__ uint32_t chain_key(const float *__restrict__ omega, long long i, const SortGeom &g) {
  const Raster c = raster_of(omega[3 * i], omega[3 * i + 1], omega[3 * i + 2], g.tx, g.ty, g.W, g.H);
  return c.inside ? (uint32_t)((c.iy >> g.shift) * g.ntx + (c.ix >> g.shift)) : (uint32_t)g.ntiles;
}

// hist[d * nblocks + b] = chains of workgroup b's tile whose key is d.
__global__ __launch_bounds__(kChainBlock) void chain_hist_kernel(const float *__restrict__ omega, long long n,
                                                                 SortGeom g, uint32_t *__restrict__ hist,
                                                                 int nblocks) {
  __shared__ uint32_t h[kKeys];
  for (int d = threadIdx.x; d < kKeys; d += kChainBlock) h[d] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kChainTile;
#pragma unroll
  for (int j = 0; j < kChainItems; ++j) {
    const long long pos = base + (long long)j * kChainBlock + threadIdx.x;
    if (pos < n) atomicAdd(&h[chain_key(omega, pos, g)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kKeys; d += kChainBlock) hist[(long long)d * nblocks + blockIdx.x] = h[d];
}

// Exclusive scan of v[0 .. kScanBlock) over the workgroup, one entry per thread; returns the
// thread's exclusive prefix and leaves the total in *total.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t x, uint32_t *wave_tot, uint32_t *total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wave_tot[wave] = incl;
  __syncthreads();
  uint32_t run = incl - x, all = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) run += wave_tot[w];
    all += wave_tot[w];
  }
  *total = all;
  return run;
}

// Row d of the digit-major histogram (the counts of key d in workgroup order) becomes its
// exclusive prefix in place; totals[d] = the row's sum.
__global__ __launch_bounds__(kScanBlock) void chain_scan_rows_kernel(uint32_t *__restrict__ hist, int nblocks,
                                                                     uint32_t *__restrict__ totals) {
  __shared__ uint32_t wave_tot[kScanBlock / 64];
  uint32_t *v = hist + (long long)blockIdx.x * nblocks;
  const int chunk = (nblocks + kScanBlock - 1) / kScanBlock;
  const int b = min(nblocks, (int)threadIdx.x * chunk);
  const int e = min(nblocks, b + chunk);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += v[i];
  uint32_t total;
  uint32_t run = block_exclusive(s, wave_tot, &total);
  for (int i = b; i < e; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// totals[d] becomes the first sorted position of key d.
__global__ __launch_bounds__(kKeys) void chain_scan_keys_kernel(uint32_t *__restrict__ totals) {
  __shared__ uint32_t wave_tot[kKeys / 64];
  uint32_t total;
  const uint32_t x = totals[threadIdx.x];
  const uint32_t run = block_exclusive(x, wave_tot, &total);
  totals[threadIdx.x] = run;
}

// Ranks, LDS placement in key order, and the write-out of workgroup b's chains.
__global__ __launch_bounds__(kChainBlock) void chain_scatter_kernel(
    const float *__restrict__ omega, const float *__restrict__ density, long long n, SortGeom g,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ key_base, int nblocks,
    float *__restrict__ omega_out, float *__restrict__ density_out, int32_t *__restrict__ perm) {
  __shared__ uint16_t lpos[kChainTile];        // by slot: position in the tile
  __shared__ uint16_t lkey[kChainTile];        // by slot: key
  __shared__ uint32_t wcount[kWaves][kKeys];   // running counts, then wave offsets
  __shared__ uint32_t lstart[kKeys];           // first slot of each key in this tile
  __shared__ uint32_t gbase[kKeys];            // first destination of each key from this tile
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const long long tile = (long long)blockIdx.x * kChainTile;
  const int count = (int)min((long long)kChainTile, n - tile);
  for (int i = threadIdx.x; i < kWaves * kKeys; i += kChainBlock) (&wcount[0][0])[i] = 0;
  __syncthreads();
  uint32_t key[kRounds], rank[kRounds];
  uint32_t *wc = wcount[wave];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int i = wave * kWaveChunk + r * 64 + lane;  // position in the tile, in index order
    const bool valid = i < count;
    const uint32_t d = valid ? chain_key(omega, tile + i, g) : 0u;
    // lanes of this wave with the same key: the AND over the key bits of the lanes that
    // agree on that bit
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kKeyBits; ++bit) {
      const unsigned long long ones = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? ones : ~ones;
    }
    const uint32_t below = (uint32_t)__popcll(peers & __lanemask_lt());
    // every lane of the key reads the count before the key's first lane advances it (one
    // wave, program order on one LDS address)
    const uint32_t c0 = valid ? wc[d] : 0u;
    rank[r] = c0 + below;
    key[r] = d;
    if (valid && below == 0) wc[d] = c0 + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per key: the waves' offsets in wave order, the tile's count, and its first destination
  for (int d = threadIdx.x; d < kKeys; d += kChainBlock) {
    uint32_t acc = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcount[w][d];
      wcount[w][d] = acc;
      acc += c;
    }
    lstart[d] = acc;
    gbase[d] = key_base[d] + hist[(long long)d * nblocks + blockIdx.x];
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // lstart: the tile's counts -> first slots, by the first wave
    static_assert(kKeys == 64, "one key per lane of the first wave");
    const uint32_t c = lstart[threadIdx.x];
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o, 64);
      if ((int)threadIdx.x >= o) incl += u;
    }
    lstart[threadIdx.x] = incl - c;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int i = wave * kWaveChunk + r * 64 + lane;
    if (i < count) {
      const uint32_t d = key[r];
      const uint32_t slot = lstart[d] + wc[d] + rank[r];
      if ((int)slot < count) {  // always true: the counts are this tile's
        lpos[slot] = (uint16_t)i;
        lkey[slot] = (uint16_t)d;
      }
    }
  }
  __syncthreads();
  // write-out in slot order: runs of one key go to consecutive destinations
  for (int s = threadIdx.x; s < count; s += kChainBlock) {
    const uint32_t d = lkey[s];
    const long long out = (long long)gbase[d] + (s - (int)lstart[d]);
    const long long src = tile + lpos[s];
    if (out < n) {  // always true for consistent histograms
      omega_out[3 * out] = omega[3 * src];
      omega_out[3 * out + 1] = omega[3 * src + 1];
      omega_out[3 * out + 2] = omega[3 * src + 2];
      if (density) density_out[out] = density[src];
      if (perm) perm[out] = (int32_t)src;
    }
  }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int lens_sort_tile_shift(int W, int H) {
  int s = 4;
  while ((long long)((W + (1 << s) - 1) >> s) * ((H + (1 << s) - 1) >> s) > kKeys - 1) ++s;
  return s;
}

size_t lens_sort_workspace_bytes(long long n) {
  if (n <= 0) return 0;
  const long long nblocks = (n + kChainTile - 1) / kChainTile;
  return align256((size_t)kKeys * (size_t)nblocks * sizeof(uint32_t)) + align256(kKeys * sizeof(uint32_t));
}

hipError_t launch_lens_sort(int W, int H, float tx, float ty, const float *omega, const float *density, long long n,
                            float *omega_out, float *density_out, int32_t *perm, void *ws, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  SortGeom g;
  g.W = W;
  g.H = H;
  g.tx = tx;
  g.ty = ty;
  g.shift = lens_sort_tile_shift(W, H);
  g.ntx = (W + (1 << g.shift) - 1) >> g.shift;
  g.ntiles = g.ntx * ((H + (1 << g.shift) - 1) >> g.shift);
  const int nblocks = (int)((n + kChainTile - 1) / kChainTile);
  uint32_t *hist = (uint32_t *)ws;
  uint32_t *totals = (uint32_t *)((char *)ws + align256((size_t)kKeys * (size_t)nblocks * sizeof(uint32_t)));
  hipLaunchKernelGGL(chain_hist_kernel, dim3(nblocks), dim3(kChainBlock), 0, st, omega, n, g, hist, nblocks);
  hipLaunchKernelGGL(chain_scan_rows_kernel, dim3(kKeys), dim3(kScanBlock), 0, st, hist, nblocks, totals);
  hipLaunchKernelGGL(chain_scan_keys_kernel, dim3(1), dim3(kKeys), 0, st, totals);
  hipLaunchKernelGGL(chain_scatter_kernel, dim3(nblocks), dim3(kChainBlock), 0, st, omega, density, n, g, hist,
                     totals, nblocks, omega_out, density_out, perm);
  return hipGetLastError();
}

}  // namespace ramlt
