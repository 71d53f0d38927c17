// Per-pixel chain statistics of Monte Carlo sample planes (Appendix A of the paper):
// estimator mean, sample variance, lag autocorrelations rho_k and the truncated
// autocorrelation time tau = 1 + 2 sum_{k <= K_L} rho_k; mean and variance of features.
//
// Design (HBM-bound: every sample is read exactly once, 40 B per sample with fp32
// features):
//  * one thread per pixel, 256 pixels per workgroup; consecutive lanes read consecutive
//    x of one sample plane, so each wave load is a contiguous 256 B (fp32) run. Loads are
//    non-temporal: the planes are streamed once;
//  * channels are processed one after another and samples are streamed in register chunks
//    (16 samples of radiance, 8 of an fp32 feature, 16 of an fp16 one), so the working set
//    per thread stays small and several waves per SIMD keep loads in flight;
//  * accumulation is fp64 about a shift K0 = the pixel's first sample, d_s = g_s - K0
//    (exact for fp32 inputs). On CDNA4 fp64 FMA issues at the fp32 (non-packed) rate,
//    so this costs registers, not time, and makes the one-pass formulas
//       M2  = sum d^2 - (sum d)^2 / S,
//       C_k = sum d_s d_{s-k} - m (T - head_k) - m (T - tail_k) + (S - k) m^2
//    (m = T / S, T = sum d, head_k / tail_k = sums of the first / last k of d) accurate to
//    ~1e-13 relative to M2 even with a firefly as the first sample, where an fp32
//    one-pass shifted sum loses most digits;
//  * lag products are formed against a register ring of the last KT deviations; KT is a
//    compile-time bucket >= K_L and lags beyond K_L are computed but not written;
//  * the 23 per-pixel results are parked in LDS and written after the pixel's last load,
//    with the "sc1" store policy. Stores share the in-order outstanding-operation counter
//    with loads, and measured mixed read/write streams on MI355X run fastest this way;
//  * a frame is covered by a series of launches of kStatsWgPerCu workgroups per compute
//    unit each: every workgroup of a launch is resident from its start, so the launch's
//    waves move through the sample planes together and read each plane over one
//    contiguous span at a time. One launch over the whole frame lets resident workgroups
//    drift apart by whole channels, and the same bytes took 9 % longer on MI355X.
#include <algorithm>
#include <atomic>

#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace ramlt {

namespace {

constexpr int kStatsBlock = 256;
static_assert(kStatsBlock == kStatsTilePixels, "one thread per pixel of a planned tile");
constexpr int kParked = 9 + 14;  // radiance mean/var/tau x 3, feature mean/var x 7
constexpr int kStoreSC1 = 16;    // buffer cache-policy operand: sc1
// Workgroups per compute unit in one launch of the statistics pass. Measured on MI355X at
// 1080p, 64 spp (one box): 3, 4, 5, 8 per CU took 0.888, 0.864, 0.891, 0.891 ms, and one
// launch of the frame 0.95 ms; launches whose size is not a whole number per CU,
// 0.91-0.95 ms. With 16-sample chunks for the fp32 features as well, 3 per CU was best
// (0.879 ms).
constexpr int kStatsWgPerCu = 4;
// A single frame of fewer 256-pixel tiles than this (under 262 144 pixels) gets a workgroup per
// (tile, channel) instead of per tile, and one launch whatever the launch size asks for.
constexpr long long kChannelSplitTiles = 1024;
constexpr int kMaxDevices = 64;

// Workgroups (tiles, or batched units) per launch on the current device for the launch
// size field of a frame's flags: v per compute unit (kStatsWgPerCu for 0), or no limit
// for RAMLT_STATS_ONE_LAUNCH. The CU count is read once per device.
long long stats_launch_size(int32_t flags) {
  int v = (flags & RAMLT_STATS_WG_MASK) >> RAMLT_STATS_WG_SHIFT;
  if (v == RAMLT_STATS_ONE_LAUNCH) return 1LL << 40;
  if (v == 0) v = kStatsWgPerCu;
  static std::atomic<int> cached[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256LL * v;
  int cus = cached[dev].load(std::memory_order_relaxed);
  if (cus <= 0) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cached[dev].store(cus, std::memory_order_relaxed);
  }
  return (long long)cus * v;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)0xFFFFFFFF, 0x00020000);
}
__device__ __forceinline__ void store_result(float *base, uint32_t idx, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), plane_rsrc(base), idx * 4u, 0,
                                        kStoreSC1);
}

template <typename T>
__device__ __forceinline__ float load_sample(const T *p);
template <>
__device__ __forceinline__ float load_sample<float>(const float *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ float load_sample<_Float16>(const _Float16 *p) {
  return (float)__builtin_nontemporal_load(p);
}

// All Appendix A statistics of one radiance channel of one pixel. Results go to park[0],
// park[kStatsBlock], park[2 * kStatsBlock] (mean, var, tau); lag correlations, if
// requested, straight to lag_o[k * plane_elems].
template <int KT, int B>
__device__ __forceinline__ void radiance_channel(const float *__restrict__ plane0, int64_t stride_s, uint32_t off,
                                                 int S, int K_L, float *park, float *__restrict__ lag_o,
                                                 int64_t plane_elems) {
  double K0 = 0.0;
  double T = 0.0, Q = 0.0;
  double P[KT > 0 ? KT : 1];
  double ring[KT > 0 ? KT : 1];
  float head[KT > 0 ? KT : 1];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    P[k] = 0.0;
    ring[k] = 0.0;
    head[k] = 0.0f;
  }

  auto consume = [&](float g) {
    const double d = (double)g - K0;
    T += d;
    Q = fma(d, d, Q);
#pragma unroll
    for (int k = 0; k < KT; ++k) P[k] = fma(d, ring[k], P[k]);
#pragma unroll
    for (int k = KT - 1; k > 0; --k) ring[k] = ring[k - 1];
    if (KT > 0) ring[0] = d;
  };

  int s0 = 0;
  if (S >= B) {
    // first chunk peeled: it fixes the shift K0 and the head samples
    float x[B];
#pragma unroll
    for (int i = 0; i < B; ++i) x[i] = load_sample(plane0 + (int64_t)i * stride_s + off);
    K0 = (double)x[0];
#pragma unroll
    for (int i = 0; i < KT && i < B; ++i) head[i] = x[i];
#pragma unroll
    for (int i = 0; i < B; ++i) consume(x[i]);
    for (s0 = B; s0 + B <= S; s0 += B) {
#pragma unroll
      for (int i = 0; i < B; ++i) x[i] = load_sample(plane0 + (int64_t)(s0 + i) * stride_s + off);
#pragma unroll
      for (int i = 0; i < B; ++i) consume(x[i]);
    }
  }
  // ragged tail (and S < B), one sample at a time
#pragma unroll 1
  for (; s0 < S; ++s0) {
    const float g = load_sample(plane0 + (int64_t)s0 * stride_s + off);
    if (s0 == 0) K0 = (double)g;
    if (s0 < KT) {
#pragma unroll
      for (int k = 0; k < KT; ++k)
        if (s0 == k) head[k] = g;
    }
    consume(g);
  }

  const double Sd = (double)S;
  const double m = T / Sd;
  double M2 = fma(-T, m, Q);
  M2 = M2 > 0.0 ? M2 : 0.0;
  park[0] = (float)(K0 + m);
  park[kStatsBlock] = S >= 2 ? (float)(M2 / (Sd - 1.0)) : 0.0f;

  double tau = 1.0;
  if (KT > 0 && M2 > 0.0) {
    const double inv = 1.0 / M2;
    const double m2 = m * m;
    const double twoT = T + T;
    const double Sm2 = Sd * m2;
    double head_k = 0.0, tail_k = 0.0;
#pragma unroll
    for (int k = 1; k <= KT; ++k) {
      head_k += (double)head[k - 1] - K0;  // sum of the first k deviations
      tail_k += ring[k - 1];               // sum of the last k deviations
      if (k <= K_L) {
        // C_k = P_k - m (T - head_k) - m (T - tail_k) + (S - k) m^2
        const double C = P[k - 1] - m * (twoT - head_k - tail_k) + (Sm2 - (double)k * m2);
        const double rho = C * inv;
        tau += 2.0 * rho;
        if (lag_o) lag_o[(int64_t)(k - 1) * plane_elems] = (float)rho;
      }
    }
  } else if (lag_o) {
    for (int k = 0; k < K_L; ++k) lag_o[(int64_t)k * plane_elems] = 0.0f;
  }
  park[2 * kStatsBlock] = (float)tau;
}

// Mean and variance of one feature channel of one pixel: park[0] and park[7 * kStatsBlock].
template <typename T, int B>
__device__ __forceinline__ void feature_channel(const T *__restrict__ plane0, int64_t stride_s, uint32_t off,
                                                int S, float *park) {
  double K0 = 0.0, Ts = 0.0, Q = 0.0;
  int s0 = 0;
  for (; s0 + B <= S; s0 += B) {
    float x[B];
#pragma unroll
    for (int i = 0; i < B; ++i) x[i] = load_sample(plane0 + (int64_t)(s0 + i) * stride_s + off);
    if (s0 == 0) K0 = (double)x[0];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const double d = (double)x[i] - K0;
      Ts += d;
      Q = fma(d, d, Q);
    }
  }
  for (; s0 < S; ++s0) {
    const float g = load_sample(plane0 + (int64_t)s0 * stride_s + off);
    if (s0 == 0) K0 = (double)g;
    const double d = (double)g - K0;
    Ts += d;
    Q = fma(d, d, Q);
  }
  const double Sd = (double)S;
  const double m = Ts / Sd;
  double M2 = fma(-Ts, m, Q);
  M2 = M2 > 0.0 ? M2 : 0.0;
  park[0] = (float)(K0 + m);
  park[RAMLT_N_FEATURES * kStatsBlock] = S >= 2 ? (float)(M2 / (Sd - 1.0)) : 0.0f;
}

// One 256-pixel tile (pixels pix0 .. pix0 + 255 of the frame, row-major).
template <int KT, int B>
__device__ __forceinline__ void stats_tile(const ramlt_frame &f, long long pix0, float *park_all) {
  const long long P = (long long)f.W * f.H;
  const int t = threadIdx.x;
  const long long pix = pix0 + t;
  if (pix >= P) return;
  float *park = park_all + t;
  // W * H <= 2^30 (validated), so 32-bit division is exact
  const int y = (int)((unsigned)pix / (unsigned)f.W);
  const int x = (int)pix - y * f.W;
  const int K_L = min(f.max_lag, f.S - 1);
  const uint32_t roff = (uint32_t)((long long)y * f.rad_stride_y + x);
#pragma unroll 1
  for (int c = 0; c < RAMLT_N_RADIANCE; ++c) {
    radiance_channel<KT, B>(f.radiance + c * f.rad_stride_c, f.rad_stride_s, roff, f.S, K_L,
                            park + 3 * c * kStatsBlock,
                            f.lag_corr ? f.lag_corr + (long long)c * K_L * P + pix : nullptr, P);
  }
  const bool feat = f.features != nullptr;
  if (feat) {
    const uint32_t foff = (uint32_t)((long long)y * f.feat_stride_y + x);
    float *fpark = park + 9 * kStatsBlock;
    if (f.feat_dtype == RAMLT_F16) {
      const _Float16 *fb = (const _Float16 *)f.features;
#pragma unroll 1
      for (int c = 0; c < RAMLT_N_FEATURES; ++c)
        feature_channel<_Float16, 16>(fb + c * f.feat_stride_c, f.feat_stride_s, foff, f.S,
                                      fpark + c * kStatsBlock);
    } else {
      const float *fb = (const float *)f.features;
#pragma unroll 1
      for (int c = 0; c < RAMLT_N_FEATURES; ++c)
        feature_channel<float, 8>(fb + c * f.feat_stride_c, f.feat_stride_s, foff, f.S, fpark + c * kStatsBlock);
    }
  }
  // deferred result stores
  const uint32_t o = (uint32_t)pix;
#pragma unroll
  for (int c = 0; c < RAMLT_N_RADIANCE; ++c) {
    store_result(f.mean + c * P, o, park[(3 * c + 0) * kStatsBlock]);
    store_result(f.var + c * P, o, park[(3 * c + 1) * kStatsBlock]);
    store_result(f.tau + c * P, o, park[(3 * c + 2) * kStatsBlock]);
  }
  if (feat) {
#pragma unroll
    for (int c = 0; c < RAMLT_N_FEATURES; ++c) {
      store_result(f.feat_mean + c * P, o, park[(9 + c) * kStatsBlock]);
      store_result(f.feat_var + c * P, o, park[(16 + c) * kStatsBlock]);
    }
  }
}

// One (256-pixel tile, channel) per workgroup, for frames of few tiles: blockIdx.x = tile,
// blockIdx.y = channel (radiance 0-2, then the features). A workgroup per tile would leave most
// compute units idle there while each workgroup walks its channels one after another. The
// channel functions, their order of operations and the result slots are those of stats_tile,
// so the results are bit for bit the same.
template <int KT, int B>
__global__ __launch_bounds__(kStatsBlock) void stats_channel_kernel(const ramlt_frame f) {
  __shared__ float park_all[kParked * kStatsBlock];
  const long long P = (long long)f.W * f.H;
  const int t = threadIdx.x;
  const long long pix = (long long)blockIdx.x * kStatsBlock + t;
  if (pix >= P) return;
  float *park = park_all + t;
  const int y = (int)((unsigned)pix / (unsigned)f.W);
  const int x = (int)pix - y * f.W;
  const uint32_t o = (uint32_t)pix;
  const int c = blockIdx.y;
  if (c < RAMLT_N_RADIANCE) {
    const int K_L = min(f.max_lag, f.S - 1);
    const uint32_t roff = (uint32_t)((long long)y * f.rad_stride_y + x);
    float *pk = park + 3 * c * kStatsBlock;
    radiance_channel<KT, B>(f.radiance + c * f.rad_stride_c, f.rad_stride_s, roff, f.S, K_L, pk,
                            f.lag_corr ? f.lag_corr + (long long)c * K_L * P + pix : nullptr, P);
    store_result(f.mean + c * P, o, pk[0]);
    store_result(f.var + c * P, o, pk[kStatsBlock]);
    store_result(f.tau + c * P, o, pk[2 * kStatsBlock]);
    return;
  }
  const int fc = c - RAMLT_N_RADIANCE;
  const uint32_t foff = (uint32_t)((long long)y * f.feat_stride_y + x);
  float *fpark = park + (9 + fc) * kStatsBlock;
  if (f.feat_dtype == RAMLT_F16)
    feature_channel<_Float16, 16>((const _Float16 *)f.features + fc * f.feat_stride_c, f.feat_stride_s, foff, f.S,
                                  fpark);
  else
    feature_channel<float, 8>((const float *)f.features + fc * f.feat_stride_c, f.feat_stride_s, foff, f.S, fpark);
  store_result(f.feat_mean + fc * P, o, fpark[0]);
  store_result(f.feat_var + fc * P, o, fpark[RAMLT_N_FEATURES * kStatsBlock]);
}

// Tiles tile0 .. tile0 + gridDim.x - 1 of the frame.
template <int KT, int B>
__global__ __launch_bounds__(kStatsBlock) void stats_kernel(const ramlt_frame f, long long tile0) {
  __shared__ float park[kParked * kStatsBlock];
  stats_tile<KT, B>(f, (tile0 + blockIdx.x) * kStatsBlock, park);
}

// Batched form: one workgroup per planned work unit, frames in the plan's order (most
// samples per pixel first, so the longest units are dispatched first). A unit is
// stats_unit_tiles(S) consecutive 256-pixel tiles, so frames with few samples per pixel
// still give each workgroup a useful amount of data. (A persistent form popping units
// from an atomic queue measured 6 % slower than this plain grid on a 32-frame batch.)
// Units unit0 .. unit0 + gridDim.x - 1 of the plan.
template <int KT, int B>
__global__ __launch_bounds__(kStatsBlock) void stats_batched_kernel(const ramlt_frame *__restrict__ frames,
                                                                    BatchPlan *plan, long long unit0) {
  __shared__ float park[kParked * kStatsBlock];
  const unsigned long long t = (unsigned long long)unit0 + blockIdx.x;
  if (t >= plan->total_tiles) return;
  int fi;
  long long local;
  plan_lookup(plan, t, &fi, &local);
  const ramlt_frame f = frames[fi];
  const long long P = (long long)f.W * f.H;
  const int m = stats_unit_tiles(f.S);
  for (int j = 0; j < m; ++j) {  // park entries are per thread: no barrier between tiles
    const long long p0 = (local * m + j) * kStatsBlock;
    if (p0 >= P) break;
    stats_tile<KT, B>(f, p0, park);
  }
}

int lag_bucket(int k) {
  if (k <= 0) return 0;
  if (k <= 1) return 1;
  if (k <= 2) return 2;
  if (k <= 4) return 4;
  if (k <= 8) return 8;
  if (k <= 16) return 16;
  return 32;
}

template <int KT, int B>
hipError_t launch_stats_kt(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws, hipStream_t st) {
  // (at most 2^22 workgroups per launch: 2^30 work-items)
  const long long per_launch = std::min(stats_launch_size(fh[0].flags), 1LL << 22);
  if (n == 1) {
    const long long P = (long long)fh[0].W * fh[0].H;
    const long long tiles = (P + kStatsBlock - 1) / kStatsBlock;
    if (tiles < kChannelSplitTiles) {
      const int nch = RAMLT_N_RADIANCE + (fh[0].features ? RAMLT_N_FEATURES : 0);
      hipLaunchKernelGGL((stats_channel_kernel<KT, B>), dim3((unsigned)tiles, (unsigned)nch), dim3(kStatsBlock), 0,
                         st, fh[0]);
      return hipGetLastError();
    }
    for (long long t0 = 0; t0 < tiles; t0 += per_launch) {
      const unsigned grid = (unsigned)(tiles - t0 < per_launch ? tiles - t0 : per_launch);
      hipLaunchKernelGGL((stats_kernel<KT, B>), dim3(grid), dim3(kStatsBlock), 0, st, fh[0], t0);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  BatchPlan *plan = (BatchPlan *)ws;
  hipError_t e = launch_plan(fd, n, RAMLT_OP_STATS, -1, plan, st);
  if (e != hipSuccess) return e;
  long long units = 0;  // as counted by the planner
  for (int i = 0; i < n; ++i) {
    const long long unit = (long long)kStatsTilePixels * stats_unit_tiles(fh[i].S);
    units += ((long long)fh[i].W * fh[i].H + unit - 1) / unit;
  }
  for (long long u0 = 0; u0 < units; u0 += per_launch) {
    const unsigned grid = (unsigned)(units - u0 < per_launch ? units - u0 : per_launch);
    hipLaunchKernelGGL((stats_batched_kernel<KT, B>), dim3(grid), dim3(kStatsBlock), 0, st, fd, plan, u0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_stats(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws, hipStream_t st) {
  int kl = 0;
  for (int i = 0; i < n; ++i) kl = max(kl, min(fh[i].max_lag, fh[i].S - 1));
  switch (lag_bucket(kl)) {
    case 0: return launch_stats_kt<0, 16>(fh, fd, n, ws, st);
    case 1: return launch_stats_kt<1, 16>(fh, fd, n, ws, st);
    case 2: return launch_stats_kt<2, 16>(fh, fd, n, ws, st);
    case 4: return launch_stats_kt<4, 16>(fh, fd, n, ws, st);
    case 8: return launch_stats_kt<8, 16>(fh, fd, n, ws, st);
    case 16: return launch_stats_kt<16, 16>(fh, fd, n, ws, st);
    default: return launch_stats_kt<32, 32>(fh, fd, n, ws, st);
  }
}

}  // namespace ramlt
