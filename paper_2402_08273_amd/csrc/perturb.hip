// Direction perturbation (Sec. 3.3 "Perturbing Ray Directions"; sigma_k = sqrt(exp(lambda_k)),
// Sec. 5.3): one thread per proposal.
//
// theta' is the inverse CDF of N(0, sigma^2) truncated to [-pi, pi] at u, evaluated in fp64
// through erf: with e = erf(a / sqrt 2), a = pi / sigma, 2p - 1 = (2u - 1) e, so
// |Phi^-1(p)| = sqrt 2 erfinv(|2u - 1| e) when that argument is below 1/2, and
// sqrt 2 erfcinv(2 min(u, 1 - u) e + erfc(a / sqrt 2)) above (the complement formed without
// cancellation). phi' = 2 pi v. The new direction is sin theta' (cos phi' t + sin phi' b) +
// cos theta' omega in the Duff et al. (2017) basis (t, b) of omega, in fp32.
#include "launch.hpp"

#include <math.h>
#include <stdint.h>

namespace ramlt {

namespace {

constexpr int kPerturbBlock = 256;
constexpr double kPi = 3.141592653589793;
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kInvSqrt2 = 0.7071067811865476;

__device__ __forceinline__ double theta_of(double u, double sigma) {
  const double a = kPi / sigma;
  const double e = erf(a * kInvSqrt2);
  const double ec = erfc(a * kInvSqrt2);
  const double y = fabs(2.0 * u - 1.0) * e;
  double z;
  if (y < 0.5) {
    z = kSqrt2 * erfinv(y);
  } else {
    const double x = 2.0 * fmin(u, 1.0 - u) * e + ec;
    z = kSqrt2 * erfcinv(x);
  }
  const double sgn = u > 0.5 ? 1.0 : (u < 0.5 ? -1.0 : 0.0);
  const double t = sgn * sigma * z;
  return t < -kPi ? -kPi : (t > kPi ? kPi : t);   // the support; NaN passes through
}

__global__ __launch_bounds__(kPerturbBlock) void perturb_kernel(const double *__restrict__ lambda, int m,
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
    const double sigma = sqrt(exp(lambda[k]));
    const double theta = theta_of((double)r.x, sigma);
    th = (float)theta;
    const float phi = (float)(2.0 * kPi * (double)r.y);
    float st, ct, sp, cp;
    sincosf(th, &st, &ct);
    sincosf(phi, &sp, &cp);
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

hipError_t launch_perturb(const double *lambda, int m, const int32_t *region, const float *omega, const float *uv,
                          float *omega_out, float *theta_out, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + kPerturbBlock - 1) / kPerturbBlock;
  perturb_kernel<<<(unsigned)blocks, kPerturbBlock, 0, st>>>(lambda, m, region, omega, (const float2 *)uv,
                                                             omega_out, theta_out, n);
  return hipGetLastError();
}

}  // namespace ramlt
