// Direction perturbation (Sec. 3.3 "Perturbing Ray Directions"; sigma_k = sqrt(exp(lambda_k)),
// Sec. 5.3): a thread per region turns lambda into the terms that depend on sigma only
// (sigma, erf and erfc of pi / (sigma sqrt 2)) in the workspace, then a thread per proposal
// reads its region's terms (for many regions each proposal computes them itself).
//
// theta' is the inverse CDF of N(0, sigma^2) truncated to [-pi, pi] at u, evaluated in fp64
// through erf: with e = erf(a / sqrt 2), a = pi / sigma, 2p - 1 = (2u - 1) e, so
// |Phi^-1(p)| = sqrt 2 erfinv(|2u - 1| e) = sqrt 2 erfcinv(2 min(u, 1 - u) e + erfc(a / sqrt 2))
// (the complement formed without cancellation). phi' = 2 pi v. The new direction is
// sin theta' (cos phi' t + sin phi' b) + cos theta' omega in the Duff et al. (2017) basis
// (t, b) of omega, in fp32.
#include "launch.hpp"

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

// theta' = sgn(2u - 1) sigma sqrt 2 erfinv(y), y = |2u - 1| e = |2p - 1|. Evaluated as
// sqrt 2 erfcinv(x) with x = 1 - y = 2 min(u, 1 - u) e + ec formed from the complements
// (no cancellation at either tail); below y = 2^-20, where x = 1 - y would keep too few
// digits of y, as erfinv(y). Every lane of a wave takes the erfcinv form unless sigma is
// beyond ~10^6 or u = 1/2, so the waves do not diverge.
__device__ __forceinline__ double theta_of(double u, const Scale &sc) {
  const double y = fabs(2.0 * u - 1.0) * sc.e;
  double z;
  if (y >= 0x1p-20) {
    z = kSqrt2 * erfcinv(2.0 * fmin(u, 1.0 - u) * sc.e + sc.ec);
  } else {
    z = kSqrt2 * erfinv(y);
  }
  const double sgn = u > 0.5 ? 1.0 : (u < 0.5 ? -1.0 : 0.0);
  const double t = sgn * sc.sigma * z;
  return t < -kPi ? -kPi : (t > kPi ? kPi : t);   // the support; NaN passes through
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
    const double theta = theta_of((double)r.x, kTable ? table[k] : scale_of(lambda[k]));
    th = (float)theta;
    float st, ct, sp, cp;
    sincosf(th, &st, &ct);
    sincospif(2.0f * r.y, &sp, &cp);   // phi' = 2 pi v (2v is exact)
    // Duff et al. 2017: s = sign(z), a = -1 / (s + z), b = x y a,
    // t = (1 + s x^2 a, s b, -s x), b' = (b, s + y^2 a, -y)
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
  omega_out[3 * i] = ox;
  omega_out[3 * i + 1] = oy;
  omega_out[3 * i + 2] = oz;
  if (theta_out) theta_out[i] = th;
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

}  // namespace ramlt
