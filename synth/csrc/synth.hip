// GPU implementation of the synthetic render-buffer recipe of synth/recipe.py and
// synth/numpy_gen.py (the NumPy version is the definition; this one is checked against it).
// It produces inputs only; none of the statistics/filter arithmetic lives here.
//
// All floating point is float64 with contraction disabled, so that every value matches
// the NumPy recipe operation for operation before the single final rounding to the
// storage type (transcendentals may differ in the last float64 ulp).
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kSamplePixel = (1ULL << 20) - 1;
constexpr double kInv24 = 1.0 / 16777216.0;
constexpr double kPi = 3.141592653589793;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t frame_key(uint64_t seed, uint64_t frame) {
  return mix64(mix64((seed + 1) * kGamma) + (frame + 1) * kGamma);
}

__device__ __forceinline__ uint64_t sample_key(uint64_t fk, uint64_t pixel, uint64_t s) {
  return mix64(fk + ((pixel << 20) | s) * kGamma + kGamma);
}

__device__ __forceinline__ uint64_t draw(uint64_t sk, uint64_t d) { return mix64(sk + (d + 1) * kGamma); }

__device__ __forceinline__ void uniform_pair(uint64_t h, double &ua, double &ub) {
  ua = (double)(h >> 40) * kInv24;
  ub = (double)((h >> 16) & 0xFFFFFFULL) * kInv24;
}

__device__ __forceinline__ void box_muller(double u1, double u2, double &z0, double &z1) {
  const double r = sqrt(-2.0 * log(1.0 - u1));
  const double t = 2.0 * kPi * u2;
  z0 = r * cos(t);
  z1 = r * sin(t);
}

struct Sample {
  double g[3];
  double feat[7];
};

__device__ __forceinline__ double pixel_sigma(uint64_t fk, uint64_t pix, int noise, double sigma) {
  if (noise == 0) return sigma;
  double ua, ub;
  uniform_pair(draw(sample_key(fk, pix, kSamplePixel), 0), ua, ub);
  return 0.02 + 0.48 * ua;
}

__device__ __forceinline__ Sample sample_at(uint64_t fk, int x, int y, uint64_t pix, uint64_t s, int W, int H,
                                            double sig, double firefly_p) {
  const uint64_t sk = sample_key(fk, pix, s);
  double xi_x, xi_y, u1, u2, u3, u4, uf, unused;
  uniform_pair(draw(sk, 0), xi_x, xi_y);
  uniform_pair(draw(sk, 1), u1, u2);
  uniform_pair(draw(sk, 2), u3, u4);
  uniform_pair(draw(sk, 3), uf, unused);
  const double u = ((double)x + xi_x) / (double)W;
  const double v = ((double)y + xi_y) / (double)H;
  const bool edge = (u + 0.37 * v) < 0.62;
  const double du = u - 0.7, dv = v - 0.35;
  const bool disc = (du * du + dv * dv) < 0.0225;
  const double att = edge ? 1.0 : 0.3;
  double L[3], alb[3], nrm[3], depth;
  if (disc) {
    L[0] = 0.95; L[1] = 0.85; L[2] = 0.15;
    alb[0] = 0.95; alb[1] = 0.85; alb[2] = 0.15;
    nrm[0] = 0.0; nrm[1] = 0.0; nrm[2] = 1.0;
    depth = 0.5;
  } else {
    L[0] = (0.2 + 0.6 * u) * att;
    L[1] = (0.2 + 0.6 * v) * att;
    L[2] = (0.8 - 0.6 * u) * att;
    if (edge) { alb[0] = 0.8; alb[1] = 0.8; alb[2] = 0.8; }
    else { alb[0] = 0.3; alb[1] = 0.5; alb[2] = 0.7; }
    const double nx = 0.5 - u, ny = 0.5 - v;
    const double inv = 1.0 / sqrt(nx * nx + ny * ny + 1.0);
    nrm[0] = nx * inv; nrm[1] = ny * inv; nrm[2] = inv;
    depth = 1.0 + u;
  }
  double z0, z1, z2, z3;
  box_muller(u1, u2, z0, z1);
  box_muller(u3, u4, z2, z3);
  Sample o;
  o.g[0] = L[0] + sig * z0;
  o.g[1] = L[1] + sig * z1;
  o.g[2] = L[2] + sig * z2;
  if (uf < firefly_p) {
    const double yff = exp(3.0 + z3);
    o.g[0] = o.g[0] + yff;
    o.g[1] = o.g[1] + yff;
    o.g[2] = o.g[2] + yff;
  }
  o.feat[0] = alb[0]; o.feat[1] = alb[1]; o.feat[2] = alb[2];
  o.feat[3] = nrm[0]; o.feat[4] = nrm[1]; o.feat[5] = nrm[2];
  o.feat[6] = depth;
  return o;
}

__global__ void frame_kernel(float *rad, void *feat, int feat_f16, int W, int H, int S, uint64_t seed,
                             uint64_t frame, int noise, double sigma, double firefly_p) {
  const long long P = (long long)W * H;
  const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (pix >= P) return;
  const int y = (int)(pix / W), x = (int)(pix - (long long)y * W);
  const uint64_t fk = frame_key(seed, frame);
  const double sig = pixel_sigma(fk, (uint64_t)pix, noise, sigma);
  const Sample o = sample_at(fk, x, y, (uint64_t)pix, (uint64_t)s, W, H, sig, firefly_p);
  const long long plane = (long long)S * P;
  const long long off = (long long)s * P + pix;
  for (int c = 0; c < 3; ++c) rad[c * plane + off] = (float)o.g[c];
  if (feat) {
    if (feat_f16) {
      _Float16 *fh = (_Float16 *)feat;
      for (int c = 0; c < 7; ++c) fh[c * plane + off] = (_Float16)(float)o.feat[c];
    } else {
      float *ff = (float *)feat;
      for (int c = 0; c < 7; ++c) ff[c * plane + off] = (float)o.feat[c];
    }
  }
}

__global__ void reference_kernel(float *ref, int W, int H, int spp, uint64_t seed, uint64_t frame, int noise,
                                 double sigma, double firefly_p) {
  const long long P = (long long)W * H;
  const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= P) return;
  const int y = (int)(pix / W), x = (int)(pix - (long long)y * W);
  const uint64_t fk = frame_key(seed, frame);
  const double sig = pixel_sigma(fk, (uint64_t)pix, noise, sigma);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < spp; ++s) {
    const Sample o = sample_at(fk, x, y, (uint64_t)pix, (uint64_t)s, W, H, sig, firefly_p);
    for (int c = 0; c < 3; ++c) acc[c] = acc[c] + (double)(float)o.g[c];
  }
  for (int c = 0; c < 3; ++c) ref[c * P + pix] = (float)(acc[c] / (double)spp);
}

}  // namespace

extern "C" {

// radiance: dense [3][S][H][W] fp32; features: dense [7][S][H][W] (fp32, or fp16 if
// feat_f16) or NULL. Returns a hipError_t value.
int synth_frame(float *radiance, void *features, int feat_f16, int W, int H, int S, uint64_t seed, uint64_t frame,
                int noise, double sigma, double firefly_p, void *stream) {
  if (W < 1 || H < 1 || S < 1 || S >= (int)kSamplePixel || radiance == nullptr) return (int)hipErrorInvalidValue;
  const long long P = (long long)W * H;
  dim3 grid((unsigned)((P + 255) / 256), (unsigned)S);
  hipLaunchKernelGGL(frame_kernel, grid, dim3(256), 0, (hipStream_t)stream, radiance, features, feat_f16, W, H, S,
                     seed, frame, noise, sigma, firefly_p);
  return (int)hipGetLastError();
}

// ref: dense [3][H][W] fp32, the float64 mean of spp float32-rounded radiance samples.
int synth_reference(float *ref, int W, int H, int spp, uint64_t seed, uint64_t frame, int noise, double sigma,
                    double firefly_p, void *stream) {
  if (W < 1 || H < 1 || spp < 1 || spp >= (int)kSamplePixel || ref == nullptr) return (int)hipErrorInvalidValue;
  const long long P = (long long)W * H;
  hipLaunchKernelGGL(reference_kernel, dim3((unsigned)((P + 127) / 128)), dim3(128), 0, (hipStream_t)stream, ref, W,
                     H, spp, seed, frame, noise, sigma, firefly_p);
  return (int)hipGetLastError();
}

}  // extern "C"
