// Per-pixel chain statistics of Monte Carlo sample planes (Appendix A of the paper):
// estimator mean, sample variance, lag autocorrelations rho_k and the truncated
// autocorrelation time tau = 1 + 2 sum_{k <= K_L} rho_k; mean and variance of features.
//
// Design (HBM-bound: every sample is read exactly once, 40 B per sample with fp32
// features):
//  * one thread per pixel, 256 pixels per workgroup; consecutive lanes read consecutive
//    x of one sample plane, so each wave load is a contiguous 256 B (fp32) run;
//  * channels are processed one after another and samples are streamed in chunks of B
//    registers, so the working set per thread stays small and many waves per CU keep
//    enough loads in flight;
//  * accumulation is fp64 about a shift K0 = the pixel's first sample, d_s = g_s - K0
//    (exact for fp32 inputs). On CDNA4 fp64 FMA issues at the fp32 (non-packed) rate,
//    so this costs registers, not time, and makes the one-pass formulas
//       M2  = sum d^2 - (sum d)^2 / S,
//       C_k = sum d_s d_{s-k} - m (T - head_k) - m (T - tail_k) + (S - k) m^2
//    (m = T / S, T = sum d, head_k / tail_k = sums of the first / last k of d) accurate to
//    ~1e-13 relative to M2 even with a firefly as the first sample, where an fp32
//    one-pass shifted sum loses most digits;
//  * lag products are formed against a register ring of the last KT deviations; KT is a
//    compile-time bucket >= K_L and lags beyond K_L are computed but not written.
#include "common.hpp"
#include "launch.hpp"

namespace ramlt {

namespace {

constexpr int kStatsBlock = 256;

template <typename T>
__device__ __forceinline__ float load_sample(const T *p);
template <>
__device__ __forceinline__ float load_sample<float>(const float *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ float load_sample<_Float16>(const _Float16 *p) {
  return (float)__builtin_nontemporal_load(p);
}

// Radiance channel: all Appendix A statistics of one pixel's sequence.
template <int KT, int B>
__device__ __forceinline__ void radiance_channel(const float *__restrict__ plane0, int64_t stride_s,
                                                 uint32_t off, int S, int K_L, float *__restrict__ mean_o,
                                                 float *__restrict__ var_o, float *__restrict__ tau_o,
                                                 float *__restrict__ lag_o, int64_t plane_elems,
                                                 uint32_t out_off) {
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
  for (; s0 + B <= S; s0 += B) {
    float x[B];
#pragma unroll
    for (int i = 0; i < B; ++i) x[i] = load_sample(plane0 + (int64_t)(s0 + i) * stride_s + off);
    if (s0 == 0) {
      K0 = (double)x[0];
#pragma unroll
      for (int i = 0; i < KT && i < B; ++i) head[i] = x[i];
    }
#pragma unroll
    for (int i = 0; i < B; ++i) consume(x[i]);
  }
  if (s0 < S) {
    const int n = S - s0;
    float x[B];
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (i < n) x[i] = load_sample(plane0 + (int64_t)(s0 + i) * stride_s + off);
    if (s0 == 0) {
      K0 = (double)x[0];
#pragma unroll
      for (int i = 0; i < KT && i < B; ++i) head[i] = i < n ? x[i] : x[0];
    }
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (i < n) consume(x[i]);
  }

  const double Sd = (double)S;
  const double m = T / Sd;
  double M2 = fma(-T, m, Q);
  M2 = M2 > 0.0 ? M2 : 0.0;
  mean_o[out_off] = (float)(K0 + m);
  var_o[out_off] = S >= 2 ? (float)(M2 / (Sd - 1.0)) : 0.0f;

  double tau = 1.0;
  if (KT > 0 && M2 > 0.0) {
    const double inv = 1.0 / M2;
    double head_k = 0.0, tail_k = 0.0;
#pragma unroll
    for (int k = 1; k <= KT; ++k) {
      // head_k = sum_{s<k} d_s, tail_k = sum of the last k deviations
      head_k += (double)head[k - 1] - K0;
      tail_k += ring[k - 1];
      if (k <= K_L) {
        const double C = P[k - 1] - m * (T - head_k) - m * (T - tail_k) + (Sd - k) * m * m;
        const double rho = C * inv;
        tau += 2.0 * rho;
        if (lag_o) lag_o[(int64_t)(k - 1) * plane_elems + out_off] = (float)rho;
      }
    }
  } else if (lag_o) {
    for (int k = 0; k < K_L; ++k) lag_o[(int64_t)k * plane_elems + out_off] = 0.0f;
  }
  tau_o[out_off] = (float)tau;
}

// Feature channel: mean and variance only.
template <typename T, int B>
__device__ __forceinline__ void feature_channel(const T *__restrict__ plane0, int64_t stride_s, uint32_t off,
                                                int S, float *__restrict__ mean_o,
                                                float *__restrict__ var_o, uint32_t out_off) {
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
  mean_o[out_off] = (float)(K0 + m);
  var_o[out_off] = S >= 2 ? (float)(M2 / (Sd - 1.0)) : 0.0f;
}

template <int KT, int B>
__device__ __forceinline__ void stats_pixels(const ramlt_frame &f, long long pix) {
  const long long P = (long long)f.W * f.H;
  if (pix >= P) return;
  const int y = (int)(pix / f.W);
  const int x = (int)(pix - (long long)y * f.W);
  const uint32_t out_off = (uint32_t)pix;
  const int K_L = min(f.max_lag, f.S - 1);
  const uint32_t roff = (uint32_t)((long long)y * f.rad_stride_y + x);
#pragma unroll 1
  for (int c = 0; c < RAMLT_N_RADIANCE; ++c) {
    radiance_channel<KT, B>(f.radiance + c * f.rad_stride_c, f.rad_stride_s, roff, f.S, K_L,
                            f.mean + c * P, f.var + c * P, f.tau + c * P,
                            f.lag_corr ? f.lag_corr + (long long)c * K_L * P : nullptr, P, out_off);
  }
  if (f.features) {
    const uint32_t foff = (uint32_t)((long long)y * f.feat_stride_y + x);
    if (f.feat_dtype == RAMLT_F16) {
      const _Float16 *fb = (const _Float16 *)f.features;
#pragma unroll 1
      for (int c = 0; c < RAMLT_N_FEATURES; ++c)
        feature_channel<_Float16, 16>(fb + c * f.feat_stride_c, f.feat_stride_s, foff, f.S,
                                      f.feat_mean + c * P, f.feat_var + c * P, out_off);
    } else {
      const float *fb = (const float *)f.features;
#pragma unroll 1
      for (int c = 0; c < RAMLT_N_FEATURES; ++c)
        feature_channel<float, 16>(fb + c * f.feat_stride_c, f.feat_stride_s, foff, f.S,
                                   f.feat_mean + c * P, f.feat_var + c * P, out_off);
    }
  }
}

template <int KT, int B>
__global__ __launch_bounds__(kStatsBlock) void stats_kernel(const ramlt_frame f) {
  stats_pixels<KT, B>(f, (long long)blockIdx.x * kStatsBlock + threadIdx.x);
}

}  // namespace

template <int KT, int B>
static hipError_t launch_stats_single(const ramlt_frame &f, hipStream_t st) {
  const long long P = (long long)f.W * f.H;
  const unsigned grid = (unsigned)((P + kStatsBlock - 1) / kStatsBlock);
  hipLaunchKernelGGL((stats_kernel<KT, B>), dim3(grid), dim3(kStatsBlock), 0, st, f);
  return hipGetLastError();
}

static int lag_bucket(int k) {
  if (k <= 0) return 0;
  if (k <= 1) return 1;
  if (k <= 2) return 2;
  if (k <= 4) return 4;
  if (k <= 8) return 8;
  if (k <= 16) return 16;
  return 32;
}

hipError_t launch_stats(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws, hipStream_t st) {
  (void)fd;
  (void)ws;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const ramlt_frame &f = fh[i];
    const int KT = lag_bucket(min(f.max_lag, f.S - 1));
    switch (KT) {
      case 0: e = launch_stats_single<0, 16>(f, st); break;
      case 1: e = launch_stats_single<1, 16>(f, st); break;
      case 2: e = launch_stats_single<2, 16>(f, st); break;
      case 4: e = launch_stats_single<4, 16>(f, st); break;
      case 8: e = launch_stats_single<8, 16>(f, st); break;
      case 16: e = launch_stats_single<16, 16>(f, st); break;
      default: e = launch_stats_single<32, 32>(f, st); break;
    }
  }
  return e;
}

}  // namespace ramlt
