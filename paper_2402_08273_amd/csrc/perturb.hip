// Direction perturbation (Sec. 3.3 "Perturbing Ray Directions"; sigma_k = sqrt(exp(lambda_k)),
// Sec. 5.3): a thread per region turns lambda into the terms that depend on sigma only
// (sigma, erf and erfc of pi / (sigma sqrt 2)) in the workspace, then a thread per proposal
// reads its region's terms (for many regions each proposal computes them itself).
//
// theta' is the inverse CDF of N(0, sigma^2) truncated to [-pi, pi] at u, evaluated in fp64
// through erf: with e = erf(a / sqrt 2), a = pi / sigma, 2p - 1 = (2u - 1) e, so
// |Phi^-1(p)| = sqrt 2 erfinv(y), y = |2u - 1| e, whose complement 1 - y =
// 2 min(u, 1 - u) e + erfc(a / sqrt 2) is formed without cancellation. erfinv comes from
// polynomials in log(1 - y^2) and its square root (erfinv_poly.hpp, relative error below
// 1e-9, a fraction of the float32 rounding of theta'). phi' = 2 pi v. The new direction is
// sin theta' (cos phi' t + sin phi' b) + cos theta' omega in the Duff et al. (2017) basis
// (t, b) of omega, in fp32.
#include "batch.hpp"
#include "erfinv_poly.hpp"
#include "launch.hpp"
#include "raster.hpp"

#include <math.h>
#include <stdint.h>

namespace ramlt {

namespace {

constexpr int kPerturbBlock = 256;
// Up to this many regions the sigma terms go through a table (1.5 MB, cache-resident);
// beyond, gathering 24 B per proposal from a table costs more than recomputing them.
constexpr int kMaxTableRegions = 65536;
constexpr double kPi = 3.141592653589793;
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kInvSqrt2 = 0.7071067811865476;

// The terms of a region's truncated normal that depend on sigma only.
struct Scale {
  double sigma;   // sqrt(exp(lambda))
  double e;       // erf(a / sqrt 2), a = pi / sigma: the mass of [-pi, pi] in units of sigma
  double ec;      // erfc(a / sqrt 2) = 1 - e
};

__device__ __forceinline__ Scale scale_of(double lam) {
  const double sigma = sqrt(exp(lam));
  const double h = (kPi / sigma) * kInvSqrt2;
  return Scale{sigma, erf(h), erfc(h)};
}

template <int N>
__device__ __forceinline__ double horner(const double (&c)[N], double t) {
  double p = c[0];
#pragma unroll
  for (int k = 1; k < N; ++k) p = fma(p, t, c[k]);
  return p;
}

// Natural logarithm of v in [0, 1] (v = x (2 - x) below) in fp64, from the series of
// atanh: v = m 2^e with m in [sqrt(1/2), sqrt(2)), log v = e ln 2 + 2 atanh(f),
// f = (m - 1) / (m + 1), |f| <= 3 - 2 sqrt(2) < 0.1716, and 2 atanh(f) = 2 f (1 + f^2/3 + f^4/5
// + ...) cut after f^14/15: the first term left out is below 2 f^16/17 < 3.6e-14 relative
// to 2 f, so the result is within ~1e-13 relative of log v (a few ulp of rounding besides),
// far inside what the inverse CDF built on it needs (1e-9). Eight fused steps and one
// division replace the library's double-double logarithm, ~50 instructions fewer per
// proposal. log 0 = -inf; NaN gives NaN.
__device__ __forceinline__ double log_unit(double v) {
  constexpr double kSqrtHalf = 0.70710678118654752440;
  constexpr double kLn2 = 0.69314718055994530942;
  int e;
  double m = frexp(v, &e);  // m in [1/2, 1) for v > 0
  const bool lo = m < kSqrtHalf;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double f = (m - 1.0) / (m + 1.0);
  const double f2 = f * f;
  double p = 1.0 / 15.0;
  p = fma(p, f2, 1.0 / 13.0);
  p = fma(p, f2, 1.0 / 11.0);
  p = fma(p, f2, 1.0 / 9.0);
  p = fma(p, f2, 1.0 / 7.0);
  p = fma(p, f2, 1.0 / 5.0);
  p = fma(p, f2, 1.0 / 3.0);
  p = fma(p, f2, 1.0);
  const double r = fma((double)e, kLn2, 2.0 * f * p);
  return v == 0.0 ? -__builtin_huge_val() : r;
}

// erfinv(y) for y in [0, 1], given y and its complement x = 1 - y, each to full relative
// precision: y P(w) with w = -log(x (2 - x)) = -log(1 - y^2) (Giles, GPU Computing Gems Jade
// Edition, 2011), P a polynomial in w below w = 6.25 and in sqrt(w) on three intervals up to
// sqrt(w) = 10.2 (x ~ 2^-148, the smallest complement a float32 u in (0, 1) can give). Below
// that (x = 0, or NaN) the library's erfcinv answers. Almost every lane of a wave takes the
// first form: the tail needs x < 0.001 (w >= 6.25).
__device__ __forceinline__ double erfinv_from_complement(double y, double x) {
  namespace ep = erfinv_poly;
  const double w = -log_unit(x * (2.0 - x));
  if (w < ep::kCentralHi) return y * horner(ep::kCentral, fma(w, ep::kCentralScale, ep::kCentralShift));
  const double s = sqrt(w);
  if (s < ep::kTail1Hi) return y * horner(ep::kTail1, fma(s, ep::kTail1Scale, ep::kTail1Shift));
  if (s < ep::kTail2Hi) return y * horner(ep::kTail2, fma(s, ep::kTail2Scale, ep::kTail2Shift));
  if (s <= ep::kTail3Hi) return y * horner(ep::kTail3, fma(s, ep::kTail3Scale, ep::kTail3Shift));
  return erfcinv(x);
}

// theta' = sgn(2u - 1) sigma sqrt 2 erfinv(y), y = |2u - 1| e.
__device__ __forceinline__ double theta_of(double u, const Scale &sc) {
  const double y = fabs(2.0 * u - 1.0) * sc.e;
  const double x = 2.0 * fmin(u, 1.0 - u) * sc.e + sc.ec;
  const double z = kSqrt2 * erfinv_from_complement(y, x);
  const double sgn = u > 0.5 ? 1.0 : (u < 0.5 ? -1.0 : 0.0);
  const double t = sgn * sc.sigma * z;
  return t < -kPi ? -kPi : (t > kPi ? kPi : t);   // the support; NaN passes through
}

// omega' = sin th (cos phi t + sin phi b) + cos th omega, phi = 2 pi v, in the Duff et al.
// (2017) basis of omega: s = sign(z), a = -1 / (s + z), c = x y a,
// t = (1 + s x^2 a, s c, -s x), b = (c, s + y^2 a, -y).
__device__ __forceinline__ void propose(float wx, float wy, float wz, float th, float v, float &ox, float &oy,
                                        float &oz) {
  float st, ct, sp, cp;
  sincosf(th, &st, &ct);
  sincospif(2.0f * v, &sp, &cp);   // phi' = 2 pi v (2v is exact)
  const float s = copysignf(1.0f, wz);
  const float aa = -1.0f / (s + wz);
  const float bb = wx * wy * aa;
  const float tx = 1.0f + s * wx * wx * aa, ty = s * bb, tz = -s * wx;
  const float bx = bb, by = s + wy * wy * aa, bz = -wy;
  const float c1 = st * cp, c2 = st * sp;
  ox = c1 * tx + c2 * bx + ct * wx;
  oy = c1 * ty + c2 * by + ct * wy;
  oz = c1 * tz + c2 * bz + ct * wz;
}

__global__ __launch_bounds__(kPerturbBlock) void scale_kernel(const double *__restrict__ lambda, int m,
                                                              Scale *__restrict__ table) {
  const int j = blockIdx.x * kPerturbBlock + threadIdx.x;
  if (j < m) table[j] = scale_of(lambda[j]);
}

template <bool kTable>
__global__ __launch_bounds__(kPerturbBlock) void perturb_kernel(const Scale *__restrict__ table,
                                                                const double *__restrict__ lambda, int m,
                                                                const int32_t *__restrict__ region,
                                                                const float *__restrict__ omega,
                                                                const float2 *__restrict__ uv,
                                                                float *__restrict__ omega_out,
                                                                float *__restrict__ theta_out, long long n) {
  const long long i = (long long)blockIdx.x * kPerturbBlock + threadIdx.x;
  if (i >= n) return;
  const int k = region[i];
  const float wx = omega[3 * i], wy = omega[3 * i + 1], wz = omega[3 * i + 2];
  const float2 r = uv[i];
  float ox, oy, oz, th;
  if (k < 0 || k >= m) {
    ox = oy = oz = th = __builtin_nanf("");
  } else {
    th = (float)theta_of((double)r.x, kTable ? table[k] : scale_of(lambda[k]));
    propose(wx, wy, wz, th, r.y, ox, oy, oz);
  }
  omega_out[3 * i] = ox;
  omega_out[3 * i + 1] = oy;
  omega_out[3 * i + 2] = oz;
  if (theta_out) theta_out[i] = th;
}

// ------------------------------------------------------------------------ lens chains
// One Metropolis step per chain (Alg. 1 lines 8-13 with the lens perturbation of Sec. 3.3):
// region k of the current state's pixel on the N x N screen grid (Sec. 6.1, the filter's
// map), proposal by the direction perturbation with sigma_k, alpha = min(1, L' / L) from
// the luminance at both pixels (0 outside the frame), move iff the uniform is below alpha.
// With `density`, each chain carries the luminance of its current pixel between steps (an
// entry below 0 or NaN is read from the image), so a step reads the image once per chain,
// at the proposal, instead of twice. With `pixel`, each chain carries its current pixel
// (iy W + ix, -1 outside the frame; an entry below -1 or past the image is taken from the
// raster map of omega), so a step skips the raster map of its current state (four correctly
// rounded divisions and the compares, 8 % of the step's instructions).
template <bool kTable>
__global__ __launch_bounds__(kPerturbBlock) void lens_step_kernel(
    const Scale *__restrict__ table, const double *__restrict__ lambda, int N, FastDiv d2W, FastDiv d2H, FastDiv dW,
    const float *__restrict__ lum, int W, int H, float tx, float ty, float *__restrict__ omega,
    float *__restrict__ density, int32_t *__restrict__ pixel, const float *__restrict__ noise,
    int32_t *__restrict__ region, float *__restrict__ alpha, float *__restrict__ omega_prop, long long n) {
  const long long i = (long long)blockIdx.x * kPerturbBlock + threadIdx.x;
  if (i >= n) return;
  const float wx = omega[3 * i], wy = omega[3 * i + 1], wz = omega[3 * i + 2];
  const float u = noise[3 * i], v = noise[3 * i + 1], ua = noise[3 * i + 2];
  // every load of the chain's own state up front: issued together, one round trip
  const float carried = density ? density[i] : -1.0f;
  const int carried_pix = pixel ? pixel[i] : -2;
  const bool known = carried_pix >= -1 && carried_pix < W * H;  // W H <= 2^30
  Raster c;
  if (known) {
    c.inside = carried_pix >= 0;
    c.iy = c.inside ? (int)fast_div((uint32_t)carried_pix, dW) : 0;
    c.ix = c.inside ? carried_pix - c.iy * W : 0;
  } else {
    c = raster_of(wx, wy, wz, tx, ty, W, H);
  }
  int k = -1;
  float a = __builtin_nanf(""), ox = a, oy = a, oz = a, dens = -1.0f;
  int new_pix = -1;
  if (c.inside) {
    // (2 i + 1) N < 2^17 2^12: exact by FastDiv
    const int kx = (int)fast_div((uint32_t)(2 * c.ix + 1) * (uint32_t)N, d2W);
    const int ky = (int)fast_div((uint32_t)(2 * c.iy + 1) * (uint32_t)N, d2H);
    k = ky * N + kx;
    const float th = (float)theta_of((double)u, kTable ? table[k] : scale_of(lambda[k]));
    propose(wx, wy, wz, th, v, ox, oy, oz);
    const Raster p = raster_of(ox, oy, oz, tx, ty, W, H);
    const float lc = carried >= 0.0f ? carried : lum[(long long)c.iy * W + c.ix];
    float lp = 0.0f;
    if (p.inside) {
      lp = lum[(long long)p.iy * W + p.ix];
      a = lp >= lc ? 1.0f : __fdiv_rn(lp, lc);
    } else {
      a = 0.0f;
    }
    dens = lc;
    new_pix = c.iy * W + c.ix;
    if (ua < a) {
      omega[3 * i] = ox;
      omega[3 * i + 1] = oy;
      omega[3 * i + 2] = oz;
      dens = lp;
      new_pix = p.iy * W + p.ix;  // a = 0 outside the frame: p is inside here
    }
  }
  region[i] = k;
  alpha[i] = a;
  if (density) density[i] = dens;
  if (pixel && new_pix != carried_pix) pixel[i] = new_pix;
  if (omega_prop) {
    omega_prop[3 * i] = ox;
    omega_prop[3 * i + 1] = oy;
    omega_prop[3 * i + 2] = oz;
  }
}

}  // namespace

size_t perturb_workspace_bytes(int m) {
  return m <= kMaxTableRegions ? ((size_t)m * sizeof(Scale) + 255) / 256 * 256 : 0;
}

hipError_t launch_perturb(const double *lambda, int m, const int32_t *region, const float *omega, const float *uv,
                          float *omega_out, float *theta_out, long long n, void *ws, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + kPerturbBlock - 1) / kPerturbBlock;
  if (m <= kMaxTableRegions) {
    Scale *table = (Scale *)ws;
    scale_kernel<<<(m + kPerturbBlock - 1) / kPerturbBlock, kPerturbBlock, 0, st>>>(lambda, m, table);
    perturb_kernel<true><<<(unsigned)blocks, kPerturbBlock, 0, st>>>(table, lambda, m, region, omega,
                                                                     (const float2 *)uv, omega_out, theta_out, n);
  } else {
    perturb_kernel<false><<<(unsigned)blocks, kPerturbBlock, 0, st>>>(nullptr, lambda, m, region, omega,
                                                                      (const float2 *)uv, omega_out, theta_out, n);
  }
  return hipGetLastError();
}

hipError_t launch_lens_step(const float *lum, int W, int H, float tx, float ty, const double *lambda, int N,
                            float *omega, float *density, int32_t *pixel, const float *noise, int32_t *region,
                            float *alpha, float *omega_prop, long long n, void *ws, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int m = N * N;
  const long long blocks = (n + kPerturbBlock - 1) / kPerturbBlock;
  const FastDiv d2W = make_fastdiv(2u * (uint32_t)W), d2H = make_fastdiv(2u * (uint32_t)H);
  const FastDiv dW = make_fastdiv((uint32_t)W);
  if (m <= kMaxTableRegions) {
    Scale *table = (Scale *)ws;
    scale_kernel<<<(m + kPerturbBlock - 1) / kPerturbBlock, kPerturbBlock, 0, st>>>(lambda, m, table);
    lens_step_kernel<true><<<(unsigned)blocks, kPerturbBlock, 0, st>>>(
        table, lambda, N, d2W, d2H, dW, lum, W, H, tx, ty, omega, density, pixel, noise, region, alpha, omega_prop, n);
  } else {
    lens_step_kernel<false><<<(unsigned)blocks, kPerturbBlock, 0, st>>>(
        nullptr, lambda, N, d2W, d2H, dW, lum, W, H, tx, ty, omega, density, pixel, noise, region, alpha, omega_prop,
        n);
  }
  return hipGetLastError();
}

}  // namespace ramlt
