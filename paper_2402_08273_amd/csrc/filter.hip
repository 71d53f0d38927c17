// Regional reconstruction filter (forward), MSE loss seed, and the filter's adjoint.
//
// The filter is the pixel reconstruction filter h_j of the path integral (Sec. 3.1),
// read as a normalised Gaussian over the (2R+1)^2 window clipped at the image border,
// whose width sigma_k = sqrt(exp(lambda_k)) (Sec. 5.3) comes from the screen-grid region
// of the output pixel (Sec. 5.2, Sec. 6.1).
//
// Design: 32 x 8 output tiles, one thread per output pixel. The tile plus an R-pixel
// halo of per-pixel values is staged in LDS as float4 (one 16-byte LDS read per tap).
// Out-of-image halo entries are zero, so clipped taps contribute nothing and the
// normaliser D_j = (sum of in-image 1-D weights along x) * (same along y) is formed in
// closed form. Taps are summed row by row, then the row sums are combined, which keeps
// the fp32 rounding error near 2(2R+1) ulp. The radius R is a template parameter so the
// window loops unroll and the 1-D weights stay in registers.
#include "common.hpp"
#include "launch.hpp"

namespace ramlt {

namespace {

constexpr int kTX = 32;
constexpr int kTY = 8;
constexpr int kFilterBlock = kTX * kTY;
constexpr float kLog2e = 1.4426950408889634f;

template <int R>
__device__ __forceinline__ void gauss_weights(float beta, float (&w)[R + 1]) {
  w[0] = 1.0f;
#pragma unroll
  for (int d = 1; d <= R; ++d) w[d] = expf(-(float)(d * d) * beta);
}

// Sum over the in-image offsets d in [-R, R] around coordinate c (0 <= c < n) of
// w[|d|] (MOM = 0) or w[|d|] d^2 (MOM = 2).
template <int R, int MOM>
__device__ __forceinline__ float clipped_sum(const float (&w)[R + 1], int c, int n) {
  float s = 0.0f;
#pragma unroll
  for (int d = -R; d <= R; ++d) {
    const int a = d < 0 ? -d : d;
    const float t = MOM == 0 ? w[a] : w[a] * (float)(a * a);
    s += (c + d >= 0 && c + d < n) ? t : 0.0f;
  }
  return s;
}

__device__ __forceinline__ int tiles_x(int W) { return (W + kTX - 1) / kTX; }
__device__ __forceinline__ int tiles_y(int H) { return (H + kTY - 1) / kTY; }

// ------------------------------------------------------------------------ forward
template <int R>
__device__ __forceinline__ void forward_tile(const ramlt_frame &f, int x0, int y0, float4 *lds) {
  constexpr int HX = kTX + 2 * R;
  constexpr int HY = kTY + 2 * R;
  const int W = f.W, H = f.H;
  const long long P = (long long)W * H;
  const float *__restrict__ mean = f.mean;
  for (int i = threadIdx.x; i < HX * HY; i += kFilterBlock) {
    const int hy = i / HX;
    const int hx = i - hy * HX;
    const int gx = x0 - R + hx;
    const int gy = y0 - R + hy;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      const long long o = (long long)gy * W + gx;
      v.x = mean[o];
      v.y = mean[P + o];
      v.z = mean[2 * P + o];
    }
    lds[i] = v;
  }
  __syncthreads();
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;
  const int x = x0 + tx;
  const int y = y0 + ty;
  if (x < W && y < H) {
    const int k = region_of(x, y, W, H, f.n_regions);
    const float beta = half_inv_var(f.lambda[k], f.lambda_min);
    float w[R + 1];
    gauss_weights<R>(beta, w);
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
      const float4 *row = lds + (ty + R + dy) * HX + tx + R;
      float rx = 0.f, ry = 0.f, rz = 0.f;
#pragma unroll
      for (int dx = -R; dx <= R; ++dx) {
        const float4 m = row[dx];
        const float ww = w[dx < 0 ? -dx : dx];
        rx = fmaf(ww, m.x, rx);
        ry = fmaf(ww, m.y, ry);
        rz = fmaf(ww, m.z, rz);
      }
      const float wy = w[dy < 0 ? -dy : dy];
      ax = fmaf(wy, rx, ax);
      ay = fmaf(wy, ry, ay);
      az = fmaf(wy, rz, az);
    }
    const float D = clipped_sum<R, 0>(w, x, W) * clipped_sum<R, 0>(w, y, H);
    const long long o = (long long)y * W + x;
    f.out[o] = ax / D;
    f.out[P + o] = ay / D;
    f.out[2 * P + o] = az / D;
  }
}

template <int R>
__global__ __launch_bounds__(kFilterBlock) void forward_kernel(const ramlt_frame f) {
  __shared__ float4 lds[(kTX + 2 * R) * (kTY + 2 * R)];
  const int ntx = tiles_x(f.W);
  const int t = blockIdx.x;
  forward_tile<R>(f, (t % ntx) * kTX, (t / ntx) * kTY, lds);
}

// ------------------------------------------------------------------------ loss seed
constexpr int kLossBlock = 256;

__global__ __launch_bounds__(kLossBlock) void loss_seed_kernel(const ramlt_frame f) {
  const long long n = 3LL * f.W * f.H;
  const float scale = (float)(2.0 / (double)n);
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kLossBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kLossBlock) {
    const float d = f.out[i] - f.reference[i];
    f.grad_out[i] = d * scale;
    acc = fma((double)d, (double)d, acc);
  }
  if (f.loss) {
    __shared__ double part[kLossBlock / kWave];
    acc = wave_sum(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < kLossBlock / kWave; ++i) s += part[i];
      unsafeAtomicAdd(f.loss, s / (double)n);
    }
  }
}

// ------------------------------------------------------------------------ backward
// Per tile: stage a_j = U_j / (S D_j) with beta_j * log2(e) (float4) and mean_j (float4)
// over tile + halo; then for each pixel p of the tile
//   G_p = sum_{e in window} a_{p+e} exp2(-|e|^2 beta'_{p+e})        (transpose gather)
// and for each output pixel j of the tile
//   dL/dlam_k(j) += beta_j sum_c U_jc (N2_jc - out_jc H2_j) / D_j,
//   N2 = sum_p h_jp d^2 mean_p,  H2 = sum_p h_jp d^2  (h' = h d^2 beta).
template <int R>
__device__ __forceinline__ void backward_tile(const ramlt_frame &f, int x0, int y0, float4 *la,
                                              float4 *lm) {
  constexpr int HX = kTX + 2 * R;
  constexpr int HY = kTY + 2 * R;
  const int W = f.W, H = f.H, N = f.n_regions;
  const long long P = (long long)W * H;
  const float invS = 1.0f / (float)f.S;
  for (int i = threadIdx.x; i < HX * HY; i += kFilterBlock) {
    const int hy = i / HX;
    const int hx = i - hy * HX;
    const int gx = x0 - R + hx;
    const int gy = y0 - R + hy;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      const long long o = (long long)gy * W + gx;
      const int k = region_of(gx, gy, W, H, N);
      const float beta = half_inv_var(f.lambda[k], f.lambda_min);
      float w[R + 1];
      gauss_weights<R>(beta, w);
      const float D = clipped_sum<R, 0>(w, gx, W) * clipped_sum<R, 0>(w, gy, H);
      const float s = invS / D;
      a = make_float4(f.grad_out[o] * s, f.grad_out[P + o] * s, f.grad_out[2 * P + o] * s, beta * kLog2e);
      m = make_float4(f.mean[o], f.mean[P + o], f.mean[2 * P + o], 0.f);
    }
    la[i] = a;
    lm[i] = m;
  }
  __syncthreads();
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;
  const int x = x0 + tx;
  const int y = y0 + ty;
  const bool inside = x < W && y < H;
  int key = -1;
  float contrib = 0.f;
  if (inside) {
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
      const float4 *row = la + (ty + R + dy) * HX + tx + R;
#pragma unroll
      for (int dx = -R; dx <= R; ++dx) {
        const float4 a = row[dx];
        const float h = __builtin_amdgcn_exp2f(-(float)(dx * dx + dy * dy) * a.w);
        gx = fmaf(h, a.x, gx);
        gy = fmaf(h, a.y, gy);
        gz = fmaf(h, a.z, gz);
      }
    }
    const long long o = (long long)y * W + x;
    f.grad_radiance[o] = gx;
    f.grad_radiance[P + o] = gy;
    f.grad_radiance[2 * P + o] = gz;

    if (f.grad_lambda) {
      const int k = region_of(x, y, W, H, N);
      const float lam = f.lambda[k];
      key = k;
      if (lam >= f.lambda_min) {
        const float beta = half_inv_var(lam, f.lambda_min);
        float w[R + 1], wd2[R + 1];
        gauss_weights<R>(beta, w);
#pragma unroll
        for (int d = 0; d <= R; ++d) wd2[d] = w[d] * (float)(d * d);
        float nx = 0.f, ny = 0.f, nz = 0.f;
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
          const float4 *row = lm + (ty + R + dy) * HX + tx + R;
          float r1x = 0.f, r1y = 0.f, r1z = 0.f, r2x = 0.f, r2y = 0.f, r2z = 0.f;
#pragma unroll
          for (int dx = -R; dx <= R; ++dx) {
            const float4 m = row[dx];
            const int ax = dx < 0 ? -dx : dx;
            r1x = fmaf(w[ax], m.x, r1x);
            r1y = fmaf(w[ax], m.y, r1y);
            r1z = fmaf(w[ax], m.z, r1z);
            r2x = fmaf(wd2[ax], m.x, r2x);
            r2y = fmaf(wd2[ax], m.y, r2y);
            r2z = fmaf(wd2[ax], m.z, r2z);
          }
          const int ay = dy < 0 ? -dy : dy;
          nx = fmaf(w[ay], r2x, fmaf(wd2[ay], r1x, nx));
          ny = fmaf(w[ay], r2y, fmaf(wd2[ay], r1y, ny));
          nz = fmaf(w[ay], r2z, fmaf(wd2[ay], r1z, nz));
        }
        const float sx0 = clipped_sum<R, 0>(w, x, W), sy0 = clipped_sum<R, 0>(w, y, H);
        const float sx2 = clipped_sum<R, 2>(w, x, W), sy2 = clipped_sum<R, 2>(w, y, H);
        const float H2 = sx2 * sy0 + sx0 * sy2;
        const float D = sx0 * sy0;
        const float t = f.grad_out[o] * (nx - f.out[o] * H2) + f.grad_out[P + o] * (ny - f.out[P + o] * H2) +
                        f.grad_out[2 * P + o] * (nz - f.out[2 * P + o] * H2);
        contrib = beta * t / D;
      }
    }
  }
  if (f.grad_lambda) {
    // Segmented wave reduction keyed by region, then one float atomic per (wave, region).
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
      const unsigned long long pending = __ballot(key >= 0);
      if (pending == 0ULL) break;
      const int lead = __ffsll((long long)pending) - 1;
      const int kk = __shfl(key, lead, kWave);
      float v = (key == kk) ? contrib : 0.f;
      v = wave_sum(v);
      if (lane == lead) unsafeAtomicAdd(f.grad_lambda + kk, v);
      if (key == kk) key = -1;
    }
  }
}

template <int R>
__global__ __launch_bounds__(kFilterBlock) void backward_kernel(const ramlt_frame f) {
  __shared__ float4 la[(kTX + 2 * R) * (kTY + 2 * R)];
  __shared__ float4 lm[(kTX + 2 * R) * (kTY + 2 * R)];
  const int ntx = tiles_x(f.W);
  const int t = blockIdx.x;
  backward_tile<R>(f, (t % ntx) * kTX, (t / ntx) * kTY, la, lm);
}

using FrameKernel = void (*)(const ramlt_frame);

template <int... Rs>
struct KernelTables {
  static constexpr int kCount = sizeof...(Rs);
  static constexpr FrameKernel forward[kCount] = {forward_kernel<Rs>...};
  static constexpr FrameKernel backward[kCount] = {backward_kernel<Rs>...};
};

using Tables = KernelTables<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15>;

unsigned filter_grid(const ramlt_frame &f) {
  return (unsigned)(((f.W + kTX - 1) / kTX) * ((f.H + kTY - 1) / kTY));
}

}  // namespace

hipError_t launch_filter_forward(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws,
                                 hipStream_t st) {
  (void)fd;
  (void)ws;
  for (int i = 0; i < n; ++i) {
    const ramlt_frame &f = fh[i];
    hipLaunchKernelGGL(Tables::forward[f.radius], dim3(filter_grid(f)), dim3(kFilterBlock), 0, st, f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_filter_backward(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws,
                                  hipStream_t st) {
  (void)fd;
  (void)ws;
  for (int i = 0; i < n; ++i) {
    const ramlt_frame &f = fh[i];
    hipLaunchKernelGGL(Tables::backward[f.radius], dim3(filter_grid(f)), dim3(kFilterBlock), 0, st, f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_loss_seed(const ramlt_frame *fh, const ramlt_frame *fd, int n, void *ws, hipStream_t st) {
  (void)fd;
  (void)ws;
  for (int i = 0; i < n; ++i) {
    const ramlt_frame &f = fh[i];
    const long long elems = 3LL * f.W * f.H;
    long long blocks = (elems + kLossBlock - 1) / kLossBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(loss_seed_kernel, dim3((unsigned)blocks), dim3(kLossBlock), 0, st, f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ramlt
