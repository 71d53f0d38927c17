// Filter kernels (forward and adjoint), templated on the window radius R and the output
// tile shape SH. Each tile shape is instantiated in its own translation unit
// (filter_tiles_*.hip) so the three compile in parallel; filter.hip launches them.
//
// The filter is the pixel reconstruction filter h_j of the path integral (Sec. 3.1),
// read as a normalised Gaussian over the (2R+1)^2 window clipped at the image border,
// whose width sigma_k = sqrt(exp(lambda_k)) (Sec. 5.3) comes from the screen-grid region
// of the output pixel (Sec. 5.2, Sec. 6.1).
//
// Tiling. Output tiles are at most 32 x 8 pixels and, when the regions are large enough
// (>= 16 px wide and >= 4 px tall), never straddle a region boundary: tile columns and
// rows are laid out inside each region column / row. Every output pixel of such a tile
// shares one sigma, so the forward filter and the lambda gather are separable (a pass
// over rows, then over columns) and the 1-D weights w(d) = exp(-d^2 / (2 sigma^2)) are
// computed once per thread. Smaller regions use plain 32 x 8 tiles and a direct (2R+1)^2
// gather with per-pixel weights.
//
// The tile plus an R-pixel halo of per-pixel values is staged in LDS as float4 (one
// 16-byte LDS read per tap). Out-of-image halo entries are zero, so clipped taps
// contribute nothing and the normaliser D_j = (sum of in-image 1-D weights along x) *
// (same along y) is formed in closed form. Sums are formed row by row, then over rows,
// which keeps the fp32 rounding error near 2(2R+1) ulp.
//
// Adjoint. G_p = (1/S) sum_j U_j h_jp / D_j weights each SOURCE j with its own sigma.
// Sources of a tile's window lie in at most three region columns (the tile's and its two
// neighbours); G is accumulated as a sum over those columns of separable convolutions of
// the masked field a_j = U_j / (S D_j), with row weights taken from each source row's
// region. With the fused loss seed (reference given, grad_out NULL), U_j = 2 (out_j - R_j)
// / (3P) is formed on the fly and the loss is accumulated per tile in fp64.
#pragma once

#include <type_traits>

#include "batch.hpp"
#include "common.hpp"

namespace ramlt {
namespace filt {

// Output tile shape of a filter kernel (one thread per output pixel of a tile).
template <int TX_, int TY_>
struct Shape {
  static constexpr int TX = TX_;
  static constexpr int TY = TY_;
  static constexpr int BLOCK = TX_ * TY_;
};
using Shape32x8 = Shape<32, 8>;
using Shape32x16 = Shape<32, 16>;
using Shape64x8 = Shape<64, 8>;
static_assert(Shape32x8::TX == kTileShapes[RAMLT_TILE_32X8].w && Shape32x8::TY == kTileShapes[RAMLT_TILE_32X8].h &&
                  Shape32x16::TX == kTileShapes[RAMLT_TILE_32X16].w &&
                  Shape32x16::TY == kTileShapes[RAMLT_TILE_32X16].h &&
                  Shape64x8::TX == kTileShapes[RAMLT_TILE_64X8].w && Shape64x8::TY == kTileShapes[RAMLT_TILE_64X8].h,
              "kernel shapes match the planner's table");

constexpr int kFinalizeBlock = 256;
constexpr float kLog2e = 1.4426950408889634f;
constexpr long long kMaxBatchGrid = 1LL << 22;  // workgroups of one loss-seed launch

// ------------------------------------------------------------------------ tiling
// All index arithmetic below divides by per-frame constants through FastDiv (TileGeom);
// a divide instruction sequence per division was the largest share of these kernels'
// scalar work.
struct Rect {
  int x0, y0, x1, y1;  // outputs [x0, x1) x [y0, y1)
  int kx, ky;          // the tile's region (aligned tiling), else -1
};

__device__ __forceinline__ int cell_x(int x, const TileGeom &g) {
  return (int)fast_div((uint32_t)(2 * x + 1) * (uint32_t)g.N, g.d_2W);
}
__device__ __forceinline__ int cell_y(int y, const TileGeom &g) {
  return (int)fast_div((uint32_t)(2 * y + 1) * (uint32_t)g.N, g.d_2H);
}
__device__ __forceinline__ int region_at(const TileGeom &g, int x, int y) { return cell_y(y, g) * g.N + cell_x(x, g); }

// First coordinate (of n) in region column / row k (the same as region_start).
__device__ __forceinline__ int region_begin(const TileGeom &g, int k, int n) {
  if (k <= 0) return 0;
  if (k >= g.N) return n;
  const int num = 2 * k * n - g.N;
  return num <= 0 ? 0 : min((int)fast_div((uint32_t)num + 2u * (uint32_t)g.N - 1u, g.d_2N), n);
}

// Output rectangle of tile t (possibly empty when aligned). Tile t < 2^31.
template <class SH>
__device__ __forceinline__ Rect tile_rect(const TileGeom &g, long long t) {
  constexpr int kTX = SH::TX, kTY = SH::TY;
  const uint32_t tt = (uint32_t)t;
  const uint32_t tr = fast_div(tt, g.d_ntx);
  const uint32_t tc = tt - tr * (uint32_t)g.ntx;
  Rect r;
  if (g.aligned) {
    const int kx = (int)fast_div(tc, g.d_tpx), i = (int)tc - kx * g.tpx;
    const int ky = (int)fast_div(tr, g.d_tpy), j = (int)tr - ky * g.tpy;
    const int bx = region_begin(g, kx + 1, g.W), by = region_begin(g, ky + 1, g.H);
    r.x0 = min(region_begin(g, kx, g.W) + i * kTX, bx);
    r.x1 = min(bx, r.x0 + kTX);
    r.y0 = min(region_begin(g, ky, g.H) + j * kTY, by);
    r.y1 = min(by, r.y0 + kTY);
    r.kx = kx;
    r.ky = ky;
  } else {
    r.x0 = (int)tc * kTX;
    r.x1 = min(g.W, r.x0 + kTX);
    r.y0 = (int)tr * kTY;
    r.y1 = min(g.H, r.y0 + kTY);
    r.kx = r.ky = -1;
  }
  return r;
}

// Region of the tile's first pixel (clamped into the image: an empty tile of an aligned
// tiling may start at x0 == W or y0 == H), and whether all its pixels share it.
__device__ __forceinline__ int tile_region(const TileGeom &g, const Rect &r) {
  if (r.kx >= 0) return r.ky * g.N + r.kx;
  return region_at(g, min(r.x0, g.W - 1), min(r.y0, g.H - 1));
}

__device__ __forceinline__ bool tile_uniform(const TileGeom &g, const Rect &r) {
  return r.kx >= 0 || region_at(g, r.x0, r.y0) == region_at(g, r.x1 - 1, r.y1 - 1);
}

// ------------------------------------------------------------------------ weights
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

// Halo items per thread: the (TX + 2R) x (TY + 2R) halo tile over the workgroup.
template <int R, class SH>
constexpr int halo_iters() {
  return ((SH::TX + 2 * R) * (SH::TY + 2 * R) + SH::BLOCK - 1) / SH::BLOCK;
}

// Stage a float4 per halo pixel of the tile at (x0, y0): value(q) at the pixel's offset q
// inside the image, zero outside. All of a thread's loads are issued before the first LDS
// store (addresses are clamped into the image, so every load is in bounds), so the
// workgroup waits for one memory round trip instead of one per item.
template <int R, class SH, typename F>
__device__ __forceinline__ void stage_halo(const ramlt_frame &f, int x0, int y0, float4 *lds, F value) {
  constexpr int kTX = SH::TX, kTY = SH::TY, kFilterBlock = SH::BLOCK;
  constexpr int HX = kTX + 2 * R;
  constexpr int HY = kTY + 2 * R;
  constexpr int NIT = halo_iters<R, SH>();
  float4 v[NIT];
  bool ok[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFilterBlock;
    const int hy = i / HX;
    const int hx = i - hy * HX;
    const int gx = x0 - R + hx;
    const int gy = y0 - R + hy;
    ok[it] = i < HX * HY && gx >= 0 && gx < f.W && gy >= 0 && gy < f.H;
    const int cx = min(max(gx, 0), f.W - 1);
    const int cy = min(max(gy, 0), f.H - 1);
    v[it] = value((long long)cy * f.W + cx);
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFilterBlock;
    if (i < HX * HY) lds[i] = ok[it] ? v[it] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__device__ __forceinline__ float4 load3(const float *p, long long P, long long o) {
  return make_float4(p[o], p[P + o], p[2 * P + o], 0.f);
}

// ------------------------------------------------------------------------ forward
// 1-D normaliser along an axis: the full window sum Z = sum_{|d|<=R} w(|d|) away from the
// border, the clipped sum within R of it.
template <int R, int MOM>
__device__ __forceinline__ float axis_sum(const float (&w)[R + 1], float full, int c, int n) {
  return (c >= R && c + R < n) ? full : clipped_sum<R, MOM>(w, c, n);
}

template <int R>
__device__ __forceinline__ float window_sum(const float (&w)[R + 1]) {
  float z = 0.f;
#pragma unroll
  for (int d = R; d >= 1; --d) z += w[d];
  return 1.0f + 2.0f * z;
}

template <int R>
__device__ __forceinline__ float window_moment2(const float (&w)[R + 1]) {
  float z = 0.f;
#pragma unroll
  for (int d = R; d >= 1; --d) z += w[d] * (float)(d * d);
  return 2.0f * z;
}

// ------------------------------------------------------------------------ loss seed
constexpr int kLossBlock = 256;

__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += red[i];
  __syncthreads();
  return s;
}

// grad_out and the loss for pixels [p0, p0 + npix) of a frame (all three planes).
__device__ __forceinline__ void loss_range(const ramlt_frame &f, long long p0, long long npix, double *red) {
  const long long P = (long long)f.W * f.H;
  const float scale = (float)(2.0 / (3.0 * (double)P));
  double acc = 0.0;
  for (long long i = threadIdx.x; i < npix; i += kLossBlock) {
    const long long o = p0 + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float d = f.out[c * P + o] - f.reference[c * P + o];
      f.grad_out[c * P + o] = d * scale;
      acc = fma((double)d, (double)d, acc);
    }
  }
  if (f.loss) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) unsafeAtomicAdd(f.loss, s / (3.0 * (double)P));
  }
}

// ------------------------------------------------------------------------ backward
// Segmented wave reduction keyed by region, then one float atomic per (wave, region).
__device__ __forceinline__ void reduce_lambda(float *grad_lambda, int key, float contrib) {
  const int lane = threadIdx.x & (kWave - 1);
  for (;;) {
    const unsigned long long pending = __ballot(key >= 0);
    if (pending == 0ULL) break;
    const int lead = __ffsll((long long)pending) - 1;
    const int kk = __shfl(key, lead, kWave);
    float v = (key == kk) ? contrib : 0.f;
    v = wave_sum(v);
    if (lane == lead) unsafeAtomicAdd(grad_lambda + kk, v);
    if (key == kk) key = -1;
  }
}

template <int R, class SH>
struct BwdLds {
  static constexpr int HX = SH::TX + 2 * R;
  static constexpr int HY = SH::TY + 2 * R;
  static constexpr int RS = R > 0 ? R : 1;                                  // strip width
  static constexpr int HB2 = HY * (SH::TX > 4 * RS ? SH::TX : 4 * RS);      // hb2 also holds the strips
  float4 stage[HX * HY];
  float4 hb1[HY * SH::TX];
  float4 hb2[HB2];
  float tab[9 * (R + 1)];
  float ztab[9];
  int rows[HY];  // region row of each halo row, relative to the first (separable path)
  int cols[HX];  // same for halo columns
  double red[SH::BLOCK / kWave];
};

// Per-tile adjoint.
//
// Transpose gather (separable path, region-aligned tiles): the tile's outputs lie in one
// region column [rs, re). Sources of the window lie in that column ("own"), or within R
// columns to its left or right (the neighbouring region columns). G is
//   own pass:  rows-then-columns convolution of the own sources (neighbour sources zeroed),
//              with each source row's weights (its region row may differ from the tile's);
//   strips:    the <= R neighbour columns on each side, for the <= R output columns they
//              reach, with the neighbour region's weights.
// Lambda gather (all tiles of a region share sigma): rows-then-columns sums of mean and
// mean * dx^2. Per-tile partial sums of dL/dlambda and of the loss go to lam_part /
// loss_part[slot] when given (a fixed-order finalize kernel adds them up), else atomics.
template <int R, class SH>
__device__ __forceinline__ void backward_tile(const ramlt_frame &f, const TileGeom &g, const Rect &r, long long slot,
                                              float *lam_part,
                                              double *loss_part, BwdLds<R, SH> &L) {
  constexpr int kTX = SH::TX, kTY = SH::TY, kFilterBlock = SH::BLOCK;
  constexpr int HX = BwdLds<R, SH>::HX;
  constexpr int HY = BwdLds<R, SH>::HY;
  constexpr int RS = BwdLds<R, SH>::RS;
  float4 *stage = L.stage, *hb1 = L.hb1, *hb2 = L.hb2;
  float *tab = L.tab, *ztab = L.ztab;
  int *rows = L.rows, *cols = L.cols;
  const int W = f.W, H = f.H, N = f.n_regions;
  const long long P = (long long)W * H;
  const bool fused = f.grad_out == nullptr;
  const float useed = (float)(2.0 / (3.0 * (double)P));
  const float invS = 1.0f / (float)f.S;
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;
  const int x = r.x0 + tx;
  const int y = r.y0 + ty;
  const bool inside = x < r.x1 && y < r.y1;
  const long long o = (long long)y * W + x;

  // Region columns / rows reachable from the tile's window.
  const int gx_lo = max(r.x0 - R, 0), gx_hi = min(r.x1 + R, W) - 1;
  const int gy_lo = max(r.y0 - R, 0), gy_hi = min(r.y1 + R, H) - 1;
  const int kx_lo = cell_x(gx_lo, g), kx_hi = cell_x(gx_hi, g);
  const int ky_lo = cell_y(gy_lo, g), nsy = cell_y(gy_hi, g) - ky_lo + 1;
  const int kx_own = r.kx >= 0 ? r.kx : cell_x(r.x0, g);
  const int k0 = tile_region(g, r);
  const bool uniform = tile_uniform(g, r);
  const bool direct = (f.flags & RAMLT_SCHED_DIRECT) != 0;  // schedule: no separable passes
  // block-uniform: separable gather when the outputs share a region column and only one
  // neighbour column lies within R on each side
  const bool sep = uniform && !direct && kx_lo >= kx_own - 1 && kx_hi <= kx_own + 1 && nsy <= 3;
  const int so = kx_own - kx_lo;  // own slot among the (<= 3) region columns
  const int rs = region_begin(g, kx_own, W), re = region_begin(g, kx_own + 1, W);
  const int nL = sep ? rs - gx_lo : 0;          // left strip width (<= R)
  const int nR = sep ? gx_hi + 1 - re : 0;      // right strip width (<= R)
  const int mL = nL > 0 ? min(r.x1, rs + R) - r.x0 : 0;  // outputs the left strip reaches
  const int xR0 = max(r.x0, re - R);                      // first output the right strip reaches
  const int mR = nR > 0 ? r.x1 - xR0 : 0;
  float4 *lst = hb2, *rst = hb2 + HY * RS, *hbl = hb2 + 2 * HY * RS, *hbr = hb2 + 3 * HY * RS;

  // U_j of an in-image pixel (given, or from the fused MSE seed)
  auto U_at = [&](long long q) -> float4 {
    if (fused) {
      return make_float4(useed * (f.out[q] - f.reference[q]), useed * (f.out[P + q] - f.reference[P + q]),
                         useed * (f.out[2 * P + q] - f.reference[2 * P + q]), 0.f);
    }
    return load3(f.grad_out, P, q);
  };

  // all loads of U first (clamped, in-bounds addresses; in flight while the tables are
  // built), then the per-item arithmetic
  constexpr int NIT = halo_iters<R, SH>();
  float4 uv[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFilterBlock;
    const int hy = i / HX;
    const int hx = i - hy * HX;
    const int cx = min(max(r.x0 - R + hx, 0), W - 1);
    const int cy = min(max(r.y0 - R + hy, 0), H - 1);
    uv[it] = U_at((long long)cy * W + cx);
  }
  if (sep) {
    // weights and window sums of the (<= 3 x 3) regions around the tile; row slots
    if (threadIdx.x < 9) {
      const int sx = threadIdx.x % 3, sy = threadIdx.x / 3;
      const int kx = min(kx_lo + sx, N - 1), ky = min(ky_lo + sy, N - 1);
      const float beta = half_inv_var(f.lambda[ky * N + kx], f.lambda_min);
      float w[R + 1];
      gauss_weights<R>(beta, w);
#pragma unroll
      for (int d = 0; d <= R; ++d) tab[threadIdx.x * (R + 1) + d] = w[d];
      ztab[threadIdx.x] = window_sum<R>(w);
    }
    for (int i = threadIdx.x; i < HY; i += kFilterBlock) {
      const int gy = min(max(r.y0 - R + i, 0), H - 1);
      rows[i] = cell_y(gy, g) - ky_lo;
    }
    for (int i = threadIdx.x; i < HX; i += kFilterBlock) {
      const int gx = min(max(r.x0 - R + i, 0), W - 1);
      cols[i] = cell_x(gx, g) - kx_lo;
    }
    __syncthreads();
  }

  // ---- stage a_j = U_j / (S D_j) over tile + halo: own-column sources in `stage`
  // (others zero), neighbour columns in the strips; the direct path keeps every source with
  // beta' = beta log2(e) in .w
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFilterBlock;
    if (i >= HX * HY) break;
    const int hy = i / HX;
    const int hx = i - hy * HX;
    const int gx = r.x0 - R + hx;
    const int gy = r.y0 - R + hy;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      float D, tag = 0.f;
      if (sep) {
        const int sl = rows[hy] * 3 + cols[hx];
        const float z = ztab[sl];
        float Dx = z, Dy = z;
        if (gx < R || gx + R >= W || gy < R || gy + R >= H) {
          float w[R + 1];
#pragma unroll
          for (int d = 0; d <= R; ++d) w[d] = tab[sl * (R + 1) + d];
          Dx = axis_sum<R, 0>(w, z, gx, W);
          Dy = axis_sum<R, 0>(w, z, gy, H);
        }
        D = Dx * Dy;
      } else {
        const float beta = half_inv_var(f.lambda[region_at(g, gx, gy)], f.lambda_min);
        float w[R + 1];
        gauss_weights<R>(beta, w);
        D = clipped_sum<R, 0>(w, gx, W) * clipped_sum<R, 0>(w, gy, H);
        tag = beta * kLog2e;
      }
      const float s = invS / D;
      const float4 u = uv[it];
      a = make_float4(u.x * s, u.y * s, u.z * s, tag);
    }
    if (sep) {  // every strip entry is written, zero for rows outside the image
      if (gx < rs) {
        if (gx >= rs - nL) lst[hy * RS + (gx - (rs - nL))] = a;
        a = make_float4(0.f, 0.f, 0.f, 0.f);
      } else if (gx >= re) {
        if (gx < re + nR) rst[hy * RS + (gx - re)] = a;
        a = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    stage[i] = a;
  }
  __syncthreads();

  // ---- G_p = sum_e a_{p+e} h(e; sigma of p+e)
  float gx_ = 0.f, gy_ = 0.f, gz_ = 0.f;
  if (sep) {
    // rows: own sources with the own column's weights for each source row
    for (int i = threadIdx.x; i < HY * kTX; i += kFilterBlock) {
      const int hy = i / kTX;
      const int hx = i - hy * kTX;
      const float *wt = tab + (rows[hy] * 3 + so) * (R + 1);
      float w[R + 1];
#pragma unroll
      for (int d = 0; d <= R; ++d) w[d] = wt[d];
      const float4 *src = stage + hy * HX + hx + R;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int dx = -R; dx <= R; ++dx) {
        const float4 v = src[dx];
        const float ww = w[dx < 0 ? -dx : dx];
        acc.x = fmaf(ww, v.x, acc.x);
        acc.y = fmaf(ww, v.y, acc.y);
        acc.z = fmaf(ww, v.z, acc.z);
      }
      hb1[i] = acc;
    }
    // rows: the strips, for the output columns they reach
    const int nLitems = HY * mL, nRitems = HY * mR;
    for (int i = threadIdx.x; i < nLitems + nRitems; i += kFilterBlock) {
      const bool left = i < nLitems;
      const int ii = left ? i : i - nLitems;
      const int m = left ? mL : mR;
      const int hy = ii / m;
      const int c = ii - hy * m;
      const float *wt = tab + (rows[hy] * 3 + (left ? so - 1 : so + 1)) * (R + 1);
      const int xo = left ? r.x0 + c : xR0 + c;       // output column
      const int s0 = left ? rs - nL : re;             // first strip column
      const int ns = left ? nL : nR;
      const float4 *strip = (left ? lst : rst) + hy * RS;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int j = 0; j < RS; ++j) {
        const int d = abs(s0 + j - xo);
        if (j < ns && d <= R) {
          const float4 v = strip[j];
          const float ww = wt[d];
          acc.x = fmaf(ww, v.x, acc.x);
          acc.y = fmaf(ww, v.y, acc.y);
          acc.z = fmaf(ww, v.z, acc.z);
        }
      }
      (left ? hbl : hbr)[hy * RS + c] = acc;
    }
    __syncthreads();
    if (inside) {
#pragma unroll
      for (int dy = -R; dy <= R; ++dy) {
        const int hy = ty + R + dy;
        const int ay = dy < 0 ? -dy : dy;
        const int rb = rows[hy] * 3;
        const float wy = tab[(rb + so) * (R + 1) + ay];
        const float4 h = hb1[hy * kTX + tx];
        gx_ = fmaf(wy, h.x, gx_);
        gy_ = fmaf(wy, h.y, gy_);
        gz_ = fmaf(wy, h.z, gz_);
        if (x - r.x0 < mL) {
          const float wl = tab[(rb + so - 1) * (R + 1) + ay];
          const float4 hl = hbl[hy * RS + (x - r.x0)];
          gx_ = fmaf(wl, hl.x, gx_);
          gy_ = fmaf(wl, hl.y, gy_);
          gz_ = fmaf(wl, hl.z, gz_);
        }
        if (mR > 0 && x >= xR0) {
          const float wr = tab[(rb + so + 1) * (R + 1) + ay];
          const float4 hr = hbr[hy * RS + (x - xR0)];
          gx_ = fmaf(wr, hr.x, gx_);
          gy_ = fmaf(wr, hr.y, gy_);
          gz_ = fmaf(wr, hr.z, gz_);
        }
      }
    }
  } else if (inside) {
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
      const float4 *row = stage + (ty + R + dy) * HX + tx + R;
#pragma unroll
      for (int dx = -R; dx <= R; ++dx) {
        const float4 a = row[dx];
        const float h = __builtin_amdgcn_exp2f(-(float)(dx * dx + dy * dy) * a.w);
        gx_ = fmaf(h, a.x, gx_);
        gy_ = fmaf(h, a.y, gy_);
        gz_ = fmaf(h, a.z, gz_);
      }
    }
  }
  if (inside) {
    f.grad_radiance[o] = gx_;
    f.grad_radiance[P + o] = gy_;
    f.grad_radiance[2 * P + o] = gz_;
  }

  // ---- loss value of the tile's pixels (fused seed)
  if (fused && f.loss) {
    double acc = 0.0;
    if (inside) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float d = f.out[c * P + o] - f.reference[c * P + o];
        acc = fma((double)d, (double)d, acc);
      }
    }
    const double s = block_sum(acc, L.red);
    if (threadIdx.x == 0) {
      if (loss_part)
        loss_part[slot] = s;
      else
        unsafeAtomicAdd(f.loss, s / (3.0 * (double)P));
    }
  }

  // ---- dL/dlambda_k(j) += beta_j sum_c U_jc (N2_jc - out_jc H2_j) / D_j
  if (!f.grad_lambda) return;
  __syncthreads();  // stage and hb2 are reused below
  float4 *smu = stage;
  stage_halo<R, SH>(f, r.x0, r.y0, smu, [&](long long q) { return load3(f.mean, P, q); });
  __syncthreads();
  const int k_own = inside ? region_at(g, x, y) : k0;
  const float lam = f.lambda[k_own];
  // the gradient passes the clamp for lambda >= lambda_min; a NaN lambda counts as live, so
  // its NaN reaches dL/dlambda as it reaches out and G
  const bool live = !(lam < f.lambda_min);
  const float beta = half_inv_var(lam, f.lambda_min);
  float w[R + 1], wd2[R + 1];
  if (sep) {
    const int sl = (cell_y(r.y0, g) - ky_lo) * 3 + so;
#pragma unroll
    for (int d = 0; d <= R; ++d) w[d] = tab[sl * (R + 1) + d];
  } else {
    gauss_weights<R>(beta, w);
  }
#pragma unroll
  for (int d = 0; d <= R; ++d) wd2[d] = w[d] * (float)(d * d);
  float nx = 0.f, ny = 0.f, nz = 0.f;
  if (uniform && !direct) {  // separable lambda gather
    if (live) {
      for (int i = threadIdx.x; i < HY * kTX; i += kFilterBlock) {
        const int hy = i / kTX;
        const int hx = i - hy * kTX;
        const float4 *row = smu + hy * HX + hx + R;
        float4 a1 = make_float4(0.f, 0.f, 0.f, 0.f), a2 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
          const float4 m = row[dx];
          const int ax = dx < 0 ? -dx : dx;
          a1.x = fmaf(w[ax], m.x, a1.x);
          a1.y = fmaf(w[ax], m.y, a1.y);
          a1.z = fmaf(w[ax], m.z, a1.z);
          a2.x = fmaf(wd2[ax], m.x, a2.x);
          a2.y = fmaf(wd2[ax], m.y, a2.y);
          a2.z = fmaf(wd2[ax], m.z, a2.z);
        }
        hb1[i] = a1;
        hb2[i] = a2;
      }
    }
    __syncthreads();
    if (inside && live) {
#pragma unroll
      for (int dy = -R; dy <= R; ++dy) {
        const int ay = dy < 0 ? -dy : dy;
        const float4 h1 = hb1[(ty + R + dy) * kTX + tx];
        const float4 h2 = hb2[(ty + R + dy) * kTX + tx];
        nx = fmaf(w[ay], h2.x, fmaf(wd2[ay], h1.x, nx));
        ny = fmaf(w[ay], h2.y, fmaf(wd2[ay], h1.y, ny));
        nz = fmaf(w[ay], h2.z, fmaf(wd2[ay], h1.z, nz));
      }
    }
  } else if (inside && live) {
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
      const float4 *row = smu + (ty + R + dy) * HX + tx + R;
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
  }
  float contrib = 0.f;
  if (inside && live) {
    const float Z0 = window_sum<R>(w), Z2 = window_moment2<R>(w);
    const float sx0 = axis_sum<R, 0>(w, Z0, x, W), sy0 = axis_sum<R, 0>(w, Z0, y, H);
    const float sx2 = axis_sum<R, 2>(w, Z2, x, W), sy2 = axis_sum<R, 2>(w, Z2, y, H);
    const float H2 = sx2 * sy0 + sx0 * sy2;
    const float D = sx0 * sy0;
    const float4 u = U_at(o);
    const float t = u.x * (nx - f.out[o] * H2) + u.y * (ny - f.out[P + o] * H2) + u.z * (nz - f.out[2 * P + o] * H2);
    contrib = beta * t / D;
  }
  if (uniform) {
    // one region for the whole tile: block reduction, one partial (or atomic)
    const double s = block_sum((double)contrib, L.red);
    if (threadIdx.x == 0) {
      if (lam_part && g.aligned)  // the finalize kernel reads region-aligned partials
        lam_part[slot] = live ? (float)s : 0.f;
      else if (live)
        unsafeAtomicAdd(f.grad_lambda + k0, (float)s);
    }
  } else {
    reduce_lambda(f.grad_lambda, inside ? k_own : -1, contrib);
  }
}

// ------------------------------------------------------------------------ kernels
// XCD-aware order for single-frame grids: consecutive workgroup ids land on different
// XCDs, so give each XCD a contiguous band of tiles (its halos overlap in that XCD's L2).
__device__ __forceinline__ long long xcd_tile(unsigned b, unsigned nblocks) {
  const unsigned per = (nblocks + 7) / 8;
  return (long long)(b & 7) * per + (b >> 3);
}

// Frame, tiling and output rectangle of tile t: the single frame's tile t, or the planned
// tile t of a batch.
template <class SH, bool BATCH>
__device__ __forceinline__ void fetch_tile(const ramlt_frame &single, const TileGeom &single_g,
                                           const ramlt_frame *frames, BatchPlan *plan, long long t, ramlt_frame &f,
                                           TileGeom &g, Rect &r) {
  if constexpr (BATCH) {
    int fi;
    long long local;
    plan_lookup(plan, (unsigned long long)t, &fi, &local);
    f = frames[fi];
    g = plan_geom(plan, plan->n_frames)[fi];
    r = tile_rect<SH>(g, local);
  } else {
    f = single;
    g = single_g;
    r = tile_rect<SH>(g, t);
  }
}

// ------------------------------------------------------------------------ forward
// The forward tile, register-blocked. kFwdBlock threads per tile; thread u owns output
// column u % TX and V consecutive output rows, so the column pass reads each row sum once for
// V outputs, and a row-pass item covers 4 consecutive columns, so it reads each staged mean
// once for 4 outputs. The mean halo is held in LDS channel by channel (structure of arrays,
// rows padded to a multiple of 4 floats), so a row-pass item reads 4 columns of a channel
// with one 16-byte LDS read and lanes read consecutive words; the passes run one channel at
// a time, so only one channel's row sums take LDS space.
// The plain sums are taken in the same order as a per-pixel gather: along x from -R to R,
// then along y from -R to R; with the loss, the taps at -d and +d are added first (the
// plain and d^2-weighted sums share those pairs).
//
// With LOSS (RAMLT_LOSS_IN_FORWARD) the tile also forms the MSE seed U_j = 2 (out_j - R_j)
// / (3P) and the parameter adjoint
//   dL/dlambda_k(j) += beta_j sum_c U_jc (N2_jc - out_jc H2_j) / D_j,
//   N2_jc = sum_p h_jp d^2 mean_pc, H2_j = sum_p h_jp d^2, beta = 1 / (2 sigma^2),
// with d^2 = dx^2 + dy^2 split over the two passes: the row pass carries sum w(dx) dx^2 mean
// beside sum w(dx) mean, and N2 = sum_dy w(dy) (row d^2 sum) + w(dy) dy^2 (row sum).
// Per-tile partials of the loss and of dL/dlambda go to the same slots as the adjoint's.
constexpr int kFwdBlock = 256;

template <int R, class SH>
struct FwdGeom {
  static constexpr int TX = SH::TX, TY = SH::TY;
  static constexpr int HX = TX + 2 * R, HY = TY + 2 * R;
  static constexpr int HXP = (HX + 3) & ~3;  // LDS row stride (16-byte rows)
  static constexpr int PLANE = HY * HXP;      // one channel of the staged halo
  static constexpr int RPLANE = HY * TX;      // one channel of the row sums
  static constexpr int V = TX * TY / kFwdBlock;  // output rows per thread
  static constexpr int NQ = (4 + 2 * R + 3) / 4;  // 16-byte reads per row-pass item and channel
  static_assert(V >= 1 && TX * TY == V * kFwdBlock && TY % V == 0, "one column unit per thread");
  static_assert(TX % 4 == 0, "row-pass items of 4 columns");
  static_assert(4 * NQ <= HXP, "row-pass reads stay inside an LDS row");
};

template <int R, class SH, bool LOSS>
struct FwdLds {
  using G = FwdGeom<R, SH>;
  alignas(16) float stage[3 * G::PLANE];
  alignas(16) float rows[(LOSS ? 2 : 1) * G::RPLANE];  // row sums of one channel: plain, then d^2-weighted
  float wtab[R + 1];
  // a tile in one region: the in-image sums of w (and w d^2) along x for each output column
  // and along y for each output row, so D = cx0 ry0 and H2 = cx2 ry0 + cx0 ry2
  float cx0[G::TX], cx2[G::TX], ry0[G::TY], ry2[G::TY];
  double red[kFwdBlock / kWave];
};

// Stage the mean over tile + halo, channel planes, zero outside the image: the first hy_n
// (<= HY) halo rows. All loads are issued before the first LDS store (addresses clamped
// into the image).
template <int R, class SH>
__device__ __forceinline__ void stage_mean_soa(const ramlt_frame &f, int x0, int y0, int hy_n, float *stage) {
  using G = FwdGeom<R, SH>;
  constexpr int NIT = (G::HX * G::HY + kFwdBlock - 1) / kFwdBlock;
  const long long P = (long long)f.W * f.H;
  const int n = G::HX * hy_n;
  float4 v[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFwdBlock;
    const int hy = i / G::HX;
    const int hx = i - hy * G::HX;
    const int cx = min(max(x0 - R + hx, 0), f.W - 1);
    const int cy = min(max(y0 - R + hy, 0), f.H - 1);
    if (i < n) v[it] = load3(f.mean, P, (long long)cy * f.W + cx);
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFwdBlock;
    if (i < n) {
      const int hy = i / G::HX;
      const int hx = i - hy * G::HX;
      const int gx = x0 - R + hx, gy = y0 - R + hy;
      const bool in = gx >= 0 && gx < f.W && gy >= 0 && gy < f.H;
      const int o = hy * G::HXP + hx;
      stage[o] = in ? v[it].x : 0.f;
      stage[G::PLANE + o] = in ? v[it].y : 0.f;
      stage[2 * G::PLANE + o] = in ? v[it].z : 0.f;
    }
  }
}

// Row pass of channel c of a tile in one region, halo rows 0 .. hy_n - 1: rows[0][hy][x] =
// sum_dx w(|dx|) mean_c(hy, x + dx) and, with LOSS, rows[1][hy][x] = sum_dx w(|dx|) dx^2
// mean_c(hy, x + dx).
template <int R, class SH, bool LOSS>
__device__ __forceinline__ void forward_rows(const float *stage, float *rows, const float (&w)[R + 1],
                                             const float (&wd2)[R + 1], int c, int hy_n) {
  using G = FwdGeom<R, SH>;
  constexpr int NG = G::TX / 4;
  for (int u = threadIdx.x; u < hy_n * NG; u += kFwdBlock) {
    const int hy = u / NG;
    const int x0 = 4 * (u - hy * NG);
    const float4 *src = (const float4 *)(stage + c * G::PLANE + hy * G::HXP + x0);
    float m[4 * G::NQ];
#pragma unroll
    for (int q = 0; q < G::NQ; ++q) {
      const float4 t = src[q];
      m[4 * q] = t.x;
      m[4 * q + 1] = t.y;
      m[4 * q + 2] = t.z;
      m[4 * q + 3] = t.w;
    }
    float a1[4] = {0.f, 0.f, 0.f, 0.f}, a2[4] = {0.f, 0.f, 0.f, 0.f};
    if (LOSS) {
      // the two sums share the tap pairs m(x - d) + m(x + d) (w and w d^2 are even in d)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a1[k] = w[0] * m[k + R];
#pragma unroll
        for (int d = 1; d <= R; ++d) {
          const float pr = m[k + R - d] + m[k + R + d];
          a1[k] = fmaf(w[d], pr, a1[k]);
          a2[k] = fmaf(wd2[d], pr, a2[k]);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4 + 2 * R; ++j) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int d = j - k - R;  // tap offset of output x0 + k
          if (d >= -R && d <= R) a1[k] = fmaf(w[d < 0 ? -d : d], m[j], a1[k]);
        }
      }
    }
    *(float4 *)(rows + hy * G::TX + x0) = make_float4(a1[0], a1[1], a1[2], a1[3]);
    if (LOSS) *(float4 *)(rows + G::RPLANE + hy * G::TX + x0) = make_float4(a2[0], a2[1], a2[2], a2[3]);
  }
}

// Column pass of channel c for the thread's column tx and rows ty0 .. ty0 + V - 1: a[k] +=
// sum_dy w(|dy|) rows[0] and, with LOSS, n[k] += sum_dy w(|dy|) rows[1] + w(|dy|) dy^2 rows[0].
template <int R, class SH, bool LOSS>
__device__ __forceinline__ void forward_columns(const float *rows, int tx, int ty0, const float (&w)[R + 1],
                                                const float (&wd2)[R + 1], float (&a)[FwdGeom<R, SH>::V][3],
                                                float (&n)[FwdGeom<R, SH>::V][3], int c) {
  using G = FwdGeom<R, SH>;
  constexpr int V = G::V;
  if (LOSS) {
    // tap pairs of rows ty0 + k + R -+ d share w(d) and w(d) d^2
    float h1[V + 2 * R], h2[V + 2 * R];
#pragma unroll
    for (int j = 0; j < V + 2 * R; ++j) {
      h1[j] = rows[(ty0 + j) * G::TX + tx];
      h2[j] = rows[G::RPLANE + (ty0 + j) * G::TX + tx];
    }
#pragma unroll
    for (int k = 0; k < V; ++k) {
      float ak = w[0] * h1[k + R], nk = w[0] * h2[k + R];
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        const float p1 = h1[k + R - d] + h1[k + R + d];
        const float p2 = h2[k + R - d] + h2[k + R + d];
        ak = fmaf(w[d], p1, ak);
        nk = fmaf(w[d], p2, fmaf(wd2[d], p1, nk));
      }
      a[k][c] = ak;
      n[k][c] = nk;
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < V + 2 * R; ++j) {
    const float h1 = rows[(ty0 + j) * G::TX + tx];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int d = j - k - R;
      if (d >= -R && d <= R) a[k][c] = fmaf(w[d < 0 ? -d : d], h1, a[k][c]);
    }
  }
}

// Direct (2R+1)^2 gather for output (tx, ty) with its own weights w (and wd2 for N2).
template <int R, class SH, bool LOSS>
__device__ __forceinline__ void forward_direct(const float *stage, int tx, int ty, const float (&w)[R + 1],
                                               const float (&wd2)[R + 1], float (&a)[3], float (&n)[3]) {
  using G = FwdGeom<R, SH>;
#pragma unroll
  for (int dy = -R; dy <= R; ++dy) {
    const int ay = dy < 0 ? -dy : dy;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float *row = stage + c * G::PLANE + (ty + R + dy) * G::HXP + tx + R;
      float r1 = 0.f, r2 = 0.f;
#pragma unroll
      for (int dx = -R; dx <= R; ++dx) {
        const int ax = dx < 0 ? -dx : dx;
        const float m = row[dx];
        r1 = fmaf(w[ax], m, r1);
        if (LOSS) r2 = fmaf(wd2[ax], m, r2);
      }
      a[c] = fmaf(w[ay], r1, a[c]);
      if (LOSS) n[c] = fmaf(w[ay], r2, fmaf(wd2[ay], r1, n[c]));
    }
  }
}

// Forward filter of one tile per workgroup: tile t0 + (the XCD-aware order of the workgroup)
// of the single frame, or of a batch's plan. With LOSS, per-tile partials go to slot t.
// (A loop over several tiles per workgroup kept more values live and cost occupancy; large
// launches are split by the host.)
template <int R, class SH, bool BATCH, bool LOSS>
__global__ __launch_bounds__(kFwdBlock) void forward_kernel(const ramlt_frame single, const TileGeom single_g,
                                                            const ramlt_frame *__restrict__ frames, BatchPlan *plan,
                                                            long long ntiles, long long t0, float *lam_part,
                                                            double *loss_part) {
  using G = FwdGeom<R, SH>;
  constexpr int V = G::V;
  __shared__ FwdLds<R, SH, LOSS> L;
  const long long total = BATCH ? (long long)plan->total_tiles : ntiles;
  const long long t = t0 + xcd_tile(blockIdx.x, gridDim.x);
  if (t >= total) return;
  ramlt_frame f;
  TileGeom g;
  Rect r;
  fetch_tile<SH, BATCH>(single, single_g, frames, plan, t, f, g, r);
  if (r.x0 >= r.x1 || r.y0 >= r.y1) {  // block-uniform
    if (LOSS && threadIdx.x == 0) {
      if (lam_part) lam_part[t] = 0.f;
      if (loss_part) loss_part[t] = 0.0;
    }
    return;
  }
  const long long P = (long long)f.W * f.H;
  // one region for the whole tile: one sigma, separable passes (unless the schedule asks for
  // the direct gather) and one partial sum of dL/dlambda
  const bool one_region = tile_uniform(g, r);
  const bool uniform = one_region && !(f.flags & RAMLT_SCHED_DIRECT);
  const int tx = threadIdx.x % G::TX;
  const int ty0 = (threadIdx.x / G::TX) * V;
  const int x = r.x0 + tx;
  // a tile clipped at a region edge has fewer rows: only the halo rows its row groups read
  // are staged and filtered, and row groups past its last row skip the column pass
  const int nrows = r.y1 - r.y0;
  const int hy_n = min(G::HY, (nrows + V - 1) / V * V + 2 * R);
  stage_mean_soa<R, SH>(f, r.x0, r.y0, hy_n, L.stage);
  // the tile's region, and (one region) its weights and per-column / per-row axis sums
  const int k_tile = tile_region(g, r);
  const float lam_tile = f.lambda[k_tile];
  const float beta_tile = half_inv_var(lam_tile, f.lambda_min);
  if (one_region) {
    const int tt = threadIdx.x;
    if (tt <= R) L.wtab[tt] = tt == 0 ? 1.0f : expf(-(float)(tt * tt) * beta_tile);
    if (tt < G::TX + G::TY) {
      float w[R + 1];
      gauss_weights<R>(beta_tile, w);
      const bool col = tt < G::TX;
      const int c = col ? r.x0 + tt : r.y0 + (tt - G::TX);
      const int n = col ? f.W : f.H;
      const float s0 = axis_sum<R, 0>(w, window_sum<R>(w), c, n);
      const float s2 = axis_sum<R, 2>(w, window_moment2<R>(w), c, n);
      if (col) {
        L.cx0[tt] = s0;
        L.cx2[tt] = s2;
      } else {
        L.ry0[tt - G::TX] = s0;
        L.ry2[tt - G::TX] = s2;
      }
    }
  }
  // the own pixels' reference values, in flight during the passes
  float ref[V][3];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const int y = r.y0 + ty0 + k;
    const bool in = x < r.x1 && y < r.y1;
#pragma unroll
    for (int c = 0; c < 3; ++c) ref[k][c] = (LOSS && in) ? f.reference[c * P + (long long)y * f.W + x] : 0.f;
  }
  __syncthreads();
  float a[V][3], n[V][3];
#pragma unroll
  for (int k = 0; k < V; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) a[k][c] = n[k][c] = 0.f;
  float w[R + 1], wd2[R + 1];
  if (uniform) {
#pragma unroll
    for (int d = 0; d <= R; ++d) w[d] = L.wtab[d];
#pragma unroll
    for (int d = 0; d <= R; ++d) wd2[d] = w[d] * (float)(d * d);
    // channel by channel, so the row sums of one channel fit in LDS (more resident tiles)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c > 0) __syncthreads();  // the previous channel's column pass is done with rows
      forward_rows<R, SH, LOSS>(L.stage, L.rows, w, wd2, c, hy_n);
      __syncthreads();
      if (ty0 < nrows) forward_columns<R, SH, LOSS>(L.rows, tx, ty0, w, wd2, a, n, c);
    }
  }
  double lacc = 0.0;
  float contrib = 0.f;
  const bool live_tile = !(lam_tile < f.lambda_min);  // NaN counts as live: it reaches dL/dlambda
  if (one_region && !uniform) {  // the direct schedule on a tile in one region: its weights
#pragma unroll
    for (int d = 0; d <= R; ++d) w[d] = L.wtab[d];
#pragma unroll
    for (int d = 0; d <= R; ++d) wd2[d] = w[d] * (float)(d * d);
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const int ty = ty0 + k;
    const int y = r.y0 + ty;
    const bool inside = x < r.x1 && y < r.y1;
    int kr = k_tile;
    bool live = live_tile;
    float beta = beta_tile;
    if (!one_region) {  // per-pixel region, weights and window sums
      kr = inside ? region_at(g, x, y) : k_tile;
      const float lam = f.lambda[kr];
      live = !(lam < f.lambda_min);
      beta = half_inv_var(lam, f.lambda_min);
      gauss_weights<R>(beta, w);
#pragma unroll
      for (int d = 0; d <= R; ++d) wd2[d] = w[d] * (float)(d * d);
    }
    if (!uniform && inside) forward_direct<R, SH, LOSS>(L.stage, tx, ty, w, wd2, a[k], n[k]);
    float ck = 0.f;
    if (inside) {
      // out is rounded on its own before out - R is formed (no fused multiply-add across
      // them): U and the loss come from the value written to out
#pragma clang fp contract(off)
      float sx0, sy0;
      if (one_region) {
        sx0 = L.cx0[tx];
        sy0 = L.ry0[ty];
      } else {
        sx0 = clipped_sum<R, 0>(w, x, f.W);
        sy0 = clipped_sum<R, 0>(w, y, f.H);
      }
      const float D = sx0 * sy0;
      const float invD = 1.0f / D;
      const long long o = (long long)y * f.W + x;
      float out[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        out[c] = a[k][c] * invD;
        f.out[c * P + o] = out[c];
      }
      if (LOSS) {
        const float useed = (float)(2.0 / (3.0 * (double)P));
        float u[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float dd = out[c] - ref[k][c];
          u[c] = useed * dd;
          f.grad_out[c * P + o] = u[c];
          lacc = fma((double)dd, (double)dd, lacc);
        }
        if (live) {
          float sx2, sy2;
          if (one_region) {
            sx2 = L.cx2[tx];
            sy2 = L.ry2[ty];
          } else {
            sx2 = clipped_sum<R, 2>(w, x, f.W);
            sy2 = clipped_sum<R, 2>(w, y, f.H);
          }
          const float H2 = sx2 * sy0 + sx0 * sy2;
          const float tt = u[0] * (n[k][0] - out[0] * H2) + u[1] * (n[k][1] - out[1] * H2) +
                           u[2] * (n[k][2] - out[2] * H2);
          ck = beta * tt * invD;
        }
      }
    }
    if (LOSS && !one_region && f.grad_lambda) reduce_lambda(f.grad_lambda, inside && live ? kr : -1, ck);
    contrib += ck;
  }
  if (!LOSS) return;
  if (f.loss) {
    const double s = block_sum(lacc, L.red);
    if (threadIdx.x == 0) {
      if (loss_part)
        loss_part[t] = s;
      else
        unsafeAtomicAdd(f.loss, s / (3.0 * (double)P));
    }
  }
  if (f.grad_lambda && one_region) {
    // one region for the whole tile: block reduction, one partial (or atomic)
    const double s = block_sum((double)contrib, L.red);
    if (threadIdx.x == 0) {
      if (lam_part && g.aligned)  // the finalize kernel reads region-aligned partials
        lam_part[t] = live_tile ? (float)s : 0.f;
      else if (live_tile)
        unsafeAtomicAdd(f.grad_lambda + k_tile, (float)s);
    }
  }
}

// ------------------------------------------------------------------------ radiance adjoint
// The radiance half of the adjoint on its own (RAMLT_LOSS_IN_FORWARD: the forward pass has
// formed U, the loss and dL/dlambda), register-blocked like the forward: kFwdBlock threads,
// V output rows per thread, 4 columns per row-pass item, channel planes in LDS.
//   G_p = sum_{j : p in window(j)} a_j h_j(p - j),  a_j = U_j / (S D_j),
// each source j with its own sigma. A region-aligned tile's outputs lie in one region column;
// its window's sources lie in that column ("own") or in the <= R columns of a neighbouring
// region column on either side ("strips"), in at most three region rows. G is the own
// sources' separable sum (row pass with each source row's weights, then the column pass with
// the same source row's weights) plus the strips' (row sums over the <= R strip columns for
// the <= R output columns they reach, then the same column pass). Other tiles gather the
// window directly, each source with its own weight.
template <int R, class SH>
struct AdjLds {
  using G = FwdGeom<R, SH>;
  static constexpr int RS = R > 0 ? R : 1;   // strip width
  static constexpr int SPLANE = G::HY * RS;   // one channel of one strip
  // the own row sums and the strip row sums (separable tiles), or the sources' beta log2(e)
  // (direct gather): never both
  static constexpr int SEPAUX = 3 * G::RPLANE + 2 * 3 * SPLANE;
  static constexpr int AUX = SEPAUX > G::PLANE ? SEPAUX : G::PLANE;
  alignas(16) float stage[3 * G::PLANE];     // a_j by channel
  alignas(16) float aux[AUX];
  float strip[2 * 3 * SPLANE];               // left / right strip sources, by channel
  float tab[9 * (R + 1)];                    // weights of the (<= 3 x 3) regions around the tile
  float ztab[9];                             // their full window sums
  float inv_zz[9];                           // 1 / (S z^2): a_j / U_j of a source away from the border
  float wrow[3 * G::HY * (R + 1)];           // by halo row: the weights of its own / left / right region
  int rowslot[G::HY];                        // region row of each halo row, from the first
  int colslot[G::HX];                        // same for halo columns
};

template <int R, class SH, bool BATCH>
__global__ __launch_bounds__(kFwdBlock) void radiance_adjoint_kernel(const ramlt_frame single,
                                                                     const TileGeom single_g,
                                                                     const ramlt_frame *__restrict__ frames,
                                                                     BatchPlan *plan, long long ntiles, long long t0,
                                                                     float *, double *) {
  using G = FwdGeom<R, SH>;
  using A = AdjLds<R, SH>;
  constexpr int V = G::V, TX = G::TX, HX = G::HX, HY = G::HY, HXP = G::HXP;
  constexpr int PLANE = G::PLANE, RS = A::RS, SPLANE = A::SPLANE;
  __shared__ A L;
  float *rows = L.aux;                  // own row sums by channel (separable)
  float *srow = L.aux + 3 * G::RPLANE;  // left / right strip row sums by channel
  float *tagp = L.aux;                  // beta log2(e) of every source (direct)
  const long long total = BATCH ? (long long)plan->total_tiles : ntiles;
  const long long t = t0 + xcd_tile(blockIdx.x, gridDim.x);
  if (t >= total) return;
  ramlt_frame f;
  TileGeom g;
  Rect r;
  fetch_tile<SH, BATCH>(single, single_g, frames, plan, t, f, g, r);
  if (r.x0 >= r.x1 || r.y0 >= r.y1) return;  // block-uniform
  const int W = f.W, H = f.H, N = f.n_regions;
  const long long P = (long long)W * H;
  const float invS = 1.0f / (float)f.S;

  // region columns / rows reachable from the tile's window
  const int gx_lo = max(r.x0 - R, 0), gx_hi = min(r.x1 + R, W) - 1;
  const int gy_lo = max(r.y0 - R, 0), gy_hi = min(r.y1 + R, H) - 1;
  const int kx_lo = cell_x(gx_lo, g), kx_hi = cell_x(gx_hi, g);
  const int ky_lo = cell_y(gy_lo, g), nsy = cell_y(gy_hi, g) - ky_lo + 1;
  const int kx_own = r.kx >= 0 ? r.kx : cell_x(r.x0, g);
  const bool direct = (f.flags & RAMLT_SCHED_DIRECT) != 0;
  // block-uniform: separable when the outputs share a region column and only one neighbour
  // column lies within R on each side
  const bool sep = tile_uniform(g, r) && !direct && kx_lo >= kx_own - 1 && kx_hi <= kx_own + 1 && nsy <= 3;
  const int so = kx_own - kx_lo;  // own slot among the (<= 3) region columns
  const int rs = region_begin(g, kx_own, W), re = region_begin(g, kx_own + 1, W);
  const int nL = sep ? rs - gx_lo : 0;                    // left strip width (<= R)
  const int nR = sep ? gx_hi + 1 - re : 0;                // right strip width (<= R)
  const int mL = nL > 0 ? min(r.x1, rs + R) - r.x0 : 0;  // outputs the left strip reaches
  const int xR0 = max(r.x0, re - R);                      // first output the right strip reaches
  const int mR = nR > 0 ? r.x1 - xR0 : 0;
  // a tile clipped at a region edge has fewer rows: only the halo rows its row groups read
  // are staged and summed, and row groups past its last row skip the column pass
  const int nrows = r.y1 - r.y0;
  const int hy_n = min(HY, (nrows + V - 1) / V * V + 2 * R);
  const int nstage = HX * hy_n;

  // U over tile + halo: every load first (clamped, in-bounds addresses)
  constexpr int NIT = (HX * HY + kFwdBlock - 1) / kFwdBlock;
  float4 uv[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFwdBlock;
    const int hy = i / HX;
    const int hx = i - hy * HX;
    const int cx = min(max(r.x0 - R + hx, 0), W - 1);
    const int cy = min(max(r.y0 - R + hy, 0), H - 1);
    if (i < nstage) uv[it] = load3(f.grad_out, P, (long long)cy * W + cx);
  }
  if (sep) {
    if (threadIdx.x < 9) {
      const int sx = threadIdx.x % 3, sy = threadIdx.x / 3;
      const int kx = min(kx_lo + sx, N - 1), ky = min(ky_lo + sy, N - 1);
      const float beta = half_inv_var(f.lambda[ky * N + kx], f.lambda_min);
      float w[R + 1];
      gauss_weights<R>(beta, w);
#pragma unroll
      for (int d = 0; d <= R; ++d) L.tab[threadIdx.x * (R + 1) + d] = w[d];
      const float z = window_sum<R>(w);
      L.ztab[threadIdx.x] = z;
      L.inv_zz[threadIdx.x] = invS / (z * z);
    }
    for (int i = threadIdx.x; i < HY; i += kFwdBlock)
      L.rowslot[i] = cell_y(min(max(r.y0 - R + i, 0), H - 1), g) - ky_lo;
    for (int i = threadIdx.x; i < HX; i += kFwdBlock)
      L.colslot[i] = cell_x(min(max(r.x0 - R + i, 0), W - 1), g) - kx_lo;
    __syncthreads();
  }

  // stage a_j = U_j / (S D_j): own-column sources in `stage` (others zero), neighbour
  // columns in the strips; the direct path keeps every source, with beta log2(e)
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * kFwdBlock;
    if (i < nstage) {
      const int hy = i / HX;
      const int hx = i - hy * HX;
      const int gx = r.x0 - R + hx;
      const int gy = r.y0 - R + hy;
      float a[3] = {0.f, 0.f, 0.f};
      float tag = 0.f;
      if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
        float sc;  // 1 / (S D_j)
        if (sep) {
          const int sl = L.rowslot[hy] * 3 + L.colslot[hx];
          if (gx < R || gx + R >= W || gy < R || gy + R >= H) {
            const float z = L.ztab[sl];
            float w[R + 1];
#pragma unroll
            for (int d = 0; d <= R; ++d) w[d] = L.tab[sl * (R + 1) + d];
            sc = invS / (axis_sum<R, 0>(w, z, gx, W) * axis_sum<R, 0>(w, z, gy, H));
          } else {
            sc = L.inv_zz[sl];  // the full window: D = z^2
          }
        } else {
          const float beta = half_inv_var(f.lambda[region_at(g, gx, gy)], f.lambda_min);
          float w[R + 1];
          gauss_weights<R>(beta, w);
          sc = invS / (clipped_sum<R, 0>(w, gx, W) * clipped_sum<R, 0>(w, gy, H));
          tag = beta * kLog2e;
        }
        a[0] = uv[it].x * sc;
        a[1] = uv[it].y * sc;
        a[2] = uv[it].z * sc;
      }
      if (sep) {  // every strip entry is written, zero for rows outside the image
        int side = -1, col = 0;
        if (gx < rs) {
          if (gx >= rs - nL) side = 0, col = gx - (rs - nL);
        } else if (gx >= re) {
          if (gx < re + nR) side = 1, col = gx - re;
        }
        if (gx < rs || gx >= re) {
          if (side >= 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) L.strip[(side * 3 + c) * SPLANE + hy * RS + col] = a[c];
          }
          a[0] = a[1] = a[2] = 0.f;
        }
      }
      const int o = hy * HXP + hx;
#pragma unroll
      for (int c = 0; c < 3; ++c) L.stage[c * PLANE + o] = a[c];
      if (!sep) tagp[o] = tag;
    }
  }
  if (sep) {  // each halo row's weights for the own column and the two strips
    for (int i = threadIdx.x; i < 3 * HY * (R + 1); i += kFwdBlock) {
      const int side = i / (HY * (R + 1));  // 0 own, 1 left, 2 right
      const int rest = i - side * HY * (R + 1);
      const int hy = rest / (R + 1);
      const int d = rest - hy * (R + 1);
      const int col = side == 0 ? so : (side == 1 ? so - 1 : so + 1);
      L.wrow[i] = (col >= 0 && col < 3) ? L.tab[(L.rowslot[hy] * 3 + col) * (R + 1) + d] : 0.f;
    }
  }
  __syncthreads();

  const int tx = threadIdx.x % TX;
  const int ty0 = (threadIdx.x / TX) * V;
  const int x = r.x0 + tx;
  float gacc[V][3];
#pragma unroll
  for (int k = 0; k < V; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) gacc[k][c] = 0.f;
  if (sep) {
    // own row pass, 4 columns per item, each source row with its own region's weights
    constexpr int NG = TX / 4;
    for (int u = threadIdx.x; u < hy_n * NG; u += kFwdBlock) {
      const int hy = u / NG;
      const int x0 = 4 * (u - hy * NG);
      const float *wt = L.tab + (L.rowslot[hy] * 3 + so) * (R + 1);
      float w[R + 1];
#pragma unroll
      for (int d = 0; d <= R; ++d) w[d] = wt[d];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float4 *src = (const float4 *)(L.stage + c * PLANE + hy * HXP + x0);
        float m[4 * G::NQ];
#pragma unroll
        for (int q = 0; q < G::NQ; ++q) {
          const float4 v4 = src[q];
          m[4 * q] = v4.x;
          m[4 * q + 1] = v4.y;
          m[4 * q + 2] = v4.z;
          m[4 * q + 3] = v4.w;
        }
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4 + 2 * R; ++j) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int d = j - k - R;
            if (d >= -R && d <= R) acc[k] = fmaf(w[d < 0 ? -d : d], m[j], acc[k]);
          }
        }
        *(float4 *)(rows + c * G::RPLANE + hy * TX + x0) = make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
    }
    // strip row sums at the output columns each strip reaches
    const int nLitems = hy_n * mL, nRitems = hy_n * mR;
    for (int i = threadIdx.x; i < nLitems + nRitems; i += kFwdBlock) {
      const bool left = i < nLitems;
      const int ii = left ? i : i - nLitems;
      const int m = left ? mL : mR;
      const int hy = ii / m;
      const int cc = ii - hy * m;
      const float *wt = L.tab + (L.rowslot[hy] * 3 + (left ? so - 1 : so + 1)) * (R + 1);
      const int xo = left ? r.x0 + cc : xR0 + cc;  // output column
      const int s0 = left ? rs - nL : re;          // first strip column
      const int ns = left ? nL : nR;
      const int side = left ? 0 : 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float *sp = L.strip + (side * 3 + c) * SPLANE + hy * RS;
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < RS; ++j) {
          const int d = abs(s0 + j - xo);
          if (j < ns && d <= R) acc = fmaf(wt[d], sp[j], acc);
        }
        srow[(side * 3 + c) * SPLANE + hy * RS + cc] = acc;
      }
    }
    __syncthreads();
    // column pass: V outputs per thread, each source row with its region's weights (from the
    // per-row tables: with j and k unrolled every LDS address is the thread's base plus a
    // constant); the strips only in waves with a lane they reach
    const bool active = ty0 < nrows;
    const bool lreach = active && x - r.x0 < mL;       // (mL <= the tile's width)
    const bool rreach = active && mR > 0 && x >= xR0 && x < r.x1;
    constexpr int NJ = V + 2 * R;
    if (active) {
      float wj[NJ][V];  // own-column weight of source row ty0 + j for output row ty0 + k
      const float *wb = L.wrow + ty0 * (R + 1);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const int d = j - k - R;
          wj[j][k] = (d >= -R && d <= R) ? wb[j * (R + 1) + (d < 0 ? -d : d)] : 0.f;
        }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float *hb = rows + c * G::RPLANE + ty0 * TX + tx;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const float h = hb[j * TX];
#pragma unroll
          for (int k = 0; k < V; ++k) {
            const int d = j - k - R;
            if (d >= -R && d <= R) gacc[k][c] = fmaf(wj[j][k], h, gacc[k][c]);
          }
        }
      }
    }
#pragma unroll
    for (int side = 1; side <= 2; ++side) {
      const bool reach = side == 1 ? lreach : rreach;
      if (__ballot(reach) == 0ULL) continue;  // wave-uniform
      const float *wb = L.wrow + (side * HY + ty0) * (R + 1);
      const int col = side == 1 ? x - r.x0 : x - xR0;
      const float *hb = srow + (side - 1) * 3 * SPLANE + ty0 * RS + (reach ? col : 0);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        float h[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) h[c] = reach ? hb[c * SPLANE + j * RS] : 0.f;
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const int d = j - k - R;
          if (d >= -R && d <= R) {
            // zero weight where the strip does not reach (a NaN weight times 0 is NaN)
            const float wgt = reach ? wb[j * (R + 1) + (d < 0 ? -d : d)] : 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) gacc[k][c] = fmaf(wgt, h[c], gacc[k][c]);
          }
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int ty = ty0 + k;
      if (x < r.x1 && r.y0 + ty < r.y1) {
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
          const int base = (ty + R + dy) * HXP + tx + R;
#pragma unroll
          for (int dx = -R; dx <= R; ++dx) {
            const float h = __builtin_amdgcn_exp2f(-(float)(dx * dx + dy * dy) * tagp[base + dx]);
#pragma unroll
            for (int c = 0; c < 3; ++c) gacc[k][c] = fmaf(h, L.stage[c * PLANE + base + dx], gacc[k][c]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const int y = r.y0 + ty0 + k;
    if (x < r.x1 && y < r.y1) {
      const long long o = (long long)y * W + x;
#pragma unroll
      for (int c = 0; c < 3; ++c) f.grad_radiance[c * P + o] = gacc[k][c];
    }
  }
}

__device__ __forceinline__ void empty_tile_partials(long long slot, float *lam_part, double *loss_part) {
  if (threadIdx.x == 0) {
    if (lam_part) lam_part[slot] = 0.f;
    if (loss_part) loss_part[slot] = 0.0;
  }
}

// Adjoint, one tile per workgroup; per-tile partials go to slot t.
template <int R, class SH, bool BATCH>
__global__ __launch_bounds__(SH::BLOCK) void backward_kernel(const ramlt_frame single, const TileGeom single_g,
                                                                const ramlt_frame *__restrict__ frames,
                                                                BatchPlan *plan, long long ntiles, long long t0,
                                                                float *lam_part, double *loss_part) {
  __shared__ BwdLds<R, SH> s;
  const long long total = BATCH ? (long long)plan->total_tiles : ntiles;
  const long long t = t0 + xcd_tile(blockIdx.x, gridDim.x);
  if (t >= total) return;
  ramlt_frame f;
  TileGeom g;
  Rect r;
  fetch_tile<SH, BATCH>(single, single_g, frames, plan, t, f, g, r);
  if (r.x0 < r.x1 && r.y0 < r.y1)  // block-uniform
    backward_tile<R, SH>(f, g, r, t, lam_part, loss_part, s);
  else
    empty_tile_partials(t, lam_part, loss_part);
}

using BwdKernel = void (*)(const ramlt_frame, const TileGeom, const ramlt_frame *, BatchPlan *, long long, long long,
                           float *, double *);
using FwdKernel = BwdKernel;  // the forward takes the partial-sum slots too (used with the loss)
using FwdLossKernel = BwdKernel;

template <class SH, int... Rs>
struct KernelTables {
  static constexpr int kCount = sizeof...(Rs);
  static constexpr FwdKernel forward[kCount] = {forward_kernel<Rs, SH, false, false>...};
  static constexpr FwdKernel forward_batched[kCount] = {forward_kernel<Rs, SH, true, false>...};
  static constexpr FwdLossKernel forward_loss[kCount] = {forward_kernel<Rs, SH, false, true>...};
  static constexpr FwdLossKernel forward_loss_batched[kCount] = {forward_kernel<Rs, SH, true, true>...};
  static constexpr BwdKernel backward[kCount] = {backward_kernel<Rs, SH, false>...};
  static constexpr BwdKernel backward_batched[kCount] = {backward_kernel<Rs, SH, true>...};
  static constexpr BwdKernel radiance[kCount] = {radiance_adjoint_kernel<Rs, SH, false>...};
  static constexpr BwdKernel radiance_batched[kCount] = {radiance_adjoint_kernel<Rs, SH, true>...};
};

template <class SH>
using TablesFor = KernelTables<SH, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15>;

// Kernels of one tile kind: forward/backward, single frame/batch, by radius.
struct KindKernels {
  const FwdKernel *forward, *forward_batched;
  const FwdLossKernel *forward_loss, *forward_loss_batched;
  const BwdKernel *backward, *backward_batched;
  const BwdKernel *radiance, *radiance_batched;  // the radiance adjoint alone (loss in the forward pass)
  int block;      // threads per workgroup of the adjoint
  int fwd_block;  // of the forward
};

template <class SH>
KindKernels kind_kernels() {
  using T = TablesFor<SH>;
  return KindKernels{T::forward,  T::forward_batched,  T::forward_loss, T::forward_loss_batched,
                     T::backward, T::backward_batched, T::radiance,     T::radiance_batched,
                     SH::BLOCK,   kFwdBlock};
}

// The kernel tables of each tile kind, one per translation unit.
KindKernels kernels_32x8();
KindKernels kernels_32x16();
KindKernels kernels_64x8();

}  // namespace filt
}  // namespace ramlt
