// Regional adaptation of the scaling parameters lambda_k (Algorithm 1 with eqs.
// est_exp_acc, update_lambda and step_size_n) for a batch of proposals.
//
// The sequential algorithm visits the proposals in order and updates the state of the
// region each one falls in. Regions are independent, so the batch is regrouped by region,
// stably (a proposal keeps its place among the proposals of its region), and every region
// then replays its own sub-sequence:
//
//   1. stable LSD radix sort of (region, alpha) by region, 8 (or 9) bits per pass: per-tile digit
//      histograms -> an exclusive scan (digit-major) -> a stable scatter that ranks equal
//      digits by ballots (one per digit bit) and per-wave running counts in LDS;
//   2. region boundaries: the first sorted position of every region;
//   3. one thread per region (a workgroup for regions closing more than 64 windows) sums
//      each window of L visits it closes (fp64, in proposal order, the region's first
//      window continuing the carried A_k), forms sgn(alpha_hat - alpha*) and the update
//      gamma(n_k + w) sgn_w, folds the updates with the clamp at lambda_min in window order,
//      and the visits after the last closed window become the pending sum.
//
// Keys of at most 9 bits (m < 512, e.g. the 2-D grid) sort in one pass, and the batch then
// takes a shorter path: the pass writes only the sorted alphas (the digit bases of its scan
// are the regions' first positions), one thread per closed window (windows numbered region
// by region) sums it and forms its update, workgroups compose the updates of chunks of a
// region's windows, and one thread per region applies its chunks in order. The window sums,
// signs and updates are the same operations in the same order on both paths; the fold of
// a region's updates into lambda_k is associated differently (within the same rounding
// bound of the sequential fold).
//
// Proposals with a region outside [0, m) get the key m and are sorted past every region;
// step 3 never reads them.
#include "launch.hpp"

#include <stdint.h>

namespace ramlt {

namespace {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;                        // per thread
constexpr int kSortTile = kSortBlock * kSortItems;    // proposals per workgroup and pass
constexpr int kMaxDigitBits = 9;  // digits of a pass: 8 or 9 bits (see sort_plan)
constexpr int kScanBlock = 1024;
constexpr int kWavesPerBlock = kSortBlock / 64;

// Pending visits i_k of a region, 0 <= i_k < L by the state invariant (a state outside it
// is read as L - 1, the same way by every kernel).
__device__ __forceinline__ int pending_visits(int v, int L) { return (v >= 0 && v < L) ? v : L - 1; }

__device__ __forceinline__ uint32_t input_key(const int32_t *region, long long pos, int m) {
  const int32_t k = region[pos];
  return (k < 0 || k >= m) ? (uint32_t)m : (uint32_t)k;
}

// Pass p of the sort, histogram: hist[d * nblocks + b] = proposals of tile b whose digit p
// is d. Pass 0 reads the regions (and maps invalid ones to m), later passes the keys.
template <int BITS>
__global__ __launch_bounds__(kSortBlock) void sort_hist_kernel(const int32_t *__restrict__ region,
                                                               const uint32_t *__restrict__ keys, long long n, int m,
                                                               int shift, uint32_t *__restrict__ hist,
                                                               int nblocks) {
  constexpr int kDigits = 1 << BITS;
  __shared__ uint32_t h[kDigits];
  for (int d = threadIdx.x; d < kDigits; d += kSortBlock) h[d] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kSortTile;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const long long pos = base + (long long)j * kSortBlock + threadIdx.x;
    if (pos < n) {
      const uint32_t key = keys ? keys[pos] : input_key(region, pos, m);
      atomicAdd(&h[(key >> shift) & (kDigits - 1)], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kDigits; d += kSortBlock) hist[(long long)d * nblocks + blockIdx.x] = h[d];
}

// Exclusive scan of the digit-major histogram in two steps: every workgroup scans the row
// of one digit (the counts of that digit in tile order) in place and writes the row total;
// one workgroup then scans the 256 totals into digit bases, which the scatter adds.
__global__ __launch_bounds__(kScanBlock) void scan_rows_kernel(uint32_t *__restrict__ hist, int nblocks,
                                                               uint32_t *__restrict__ totals) {
  __shared__ uint32_t part[kScanBlock];
  uint32_t *v = hist + (long long)blockIdx.x * nblocks;
  const int chunk = (nblocks + kScanBlock - 1) / kScanBlock;
  const int b = threadIdx.x * chunk;
  const int e = min(nblocks, b + chunk);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {  // Hillis-Steele, inclusive
    const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int i = b; i < e; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  if (threadIdx.x == kScanBlock - 1) totals[blockIdx.x] = part[kScanBlock - 1];
}

// With start (a single pass over keys 0..m, m < 2^BITS): the digit bases are the regions'
// first sorted positions, start[k] for k = 0..m, and start[m + 1] = n.
template <int BITS>
__global__ __launch_bounds__(1 << BITS) void scan_digits_kernel(uint32_t *__restrict__ totals,
                                                                uint32_t *__restrict__ start, int m, long long n) {
  constexpr int kDigits = 1 << BITS;
  __shared__ uint32_t t[kDigits];
  t[threadIdx.x] = totals[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int d = 0; d < kDigits; ++d) {
      const uint32_t x = t[d];
      t[d] = run;
      run += x;
    }
  }
  __syncthreads();
  totals[threadIdx.x] = t[threadIdx.x];
  if (start) {
    if ((int)threadIdx.x <= m) start[threadIdx.x] = t[threadIdx.x];
    if (threadIdx.x == 0) start[m + 1] = (uint32_t)n;
  }
}

// Exclusive scan of v[0..kDigits) in place over the workgroup (each thread takes
// kDigits / kSortBlock consecutive entries); the order of the additions is fixed.
template <int kDigits>
__device__ __forceinline__ void block_exclusive_scan(uint32_t *v) {
  constexpr int kPer = kDigits / kSortBlock;
  static_assert(kPer * kSortBlock == kDigits, "digits a multiple of the block");
  __shared__ uint32_t wave_tot[kWavesPerBlock];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t own[kPer];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    own[j] = v[threadIdx.x * kPer + j];
    sum += own[j];
  }
  uint32_t incl = sum;  // inclusive scan of the per-thread sums inside the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wave_tot[wave] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int w = 0; w < wave; ++w) run += wave_tot[w];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    v[threadIdx.x * kPer + j] = run;
    run += own[j];
  }
  __syncthreads();
}

// Pass p of the sort, stable scatter of (key, alpha). Wave w of the workgroup ranks the
// proposals [w kWaveChunk, (w + 1) kWaveChunk) of the tile, 64 per round in index order:
// a proposal's rank within its wave is the wave's running count of its digit (kept in
// LDS, advanced by the digit's first lane) plus its place among the lanes with the same
// digit (one ballot per digit bit), so the work per round does not grow with the number
// of digits. The waves' counts then become per-digit offsets in wave order, and the
// ranked proposals are placed in LDS in digit order and written out run by run, so
// consecutive threads write consecutive addresses of one digit's destination range.
// KEYS false: only the values are written (the single pass of the small-grid path).
template <int BITS, bool KEYS>
__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(
    const int32_t *__restrict__ region, const float *__restrict__ alpha, const uint32_t *__restrict__ keys_in,
    const float *__restrict__ val_in, long long n, int m, int shift, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ digit_base, int nblocks, uint32_t *__restrict__ keys_out,
    float *__restrict__ val_out) {
  constexpr int kDigits = 1 << BITS;
  constexpr int kWaveChunk = kSortTile / kWavesPerBlock;   // proposals per wave
  constexpr int kRounds = kWaveChunk / 64;
  __shared__ uint32_t lkey[kSortTile];
  __shared__ float lval[kSortTile];
  __shared__ uint32_t wcount[kWavesPerBlock][kDigits];  // running counts, then wave offsets
  __shared__ uint32_t lstart[kDigits];                  // first LDS slot of each digit in this tile
  __shared__ uint32_t gbase[kDigits];                   // first destination of each digit from this tile
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const long long tile = (long long)blockIdx.x * kSortTile;
  const int count = (int)min((long long)kSortTile, n - tile);
  for (int i = threadIdx.x; i < kWavesPerBlock * kDigits; i += kSortBlock) (&wcount[0][0])[i] = 0;
  __syncthreads();
  uint32_t key[kRounds];
  float val[kRounds];
  uint32_t rank[kRounds];
  uint32_t *wc = wcount[wave];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int i = wave * kWaveChunk + r * 64 + lane;  // slot in the tile, in index order
    const bool valid = i < count;
    key[r] = 0;
    val[r] = 0.f;
    if (valid) {
      key[r] = keys_in ? keys_in[tile + i] : input_key(region, tile + i, m);
      val[r] = val_in ? val_in[tile + i] : alpha[tile + i];
    }
    const int d = valid ? (int)((key[r] >> shift) & (kDigits - 1)) : 0;
    // lanes of this wave with the same digit: the AND over the digit's bits of the lanes
    // that agree on that bit
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
      const unsigned long long ones = __ballot((d >> bit) & 1);
      peers &= ((d >> bit) & 1) ? ones : ~ones;
    }
    const uint32_t below = (uint32_t)__popcll(peers & __lanemask_lt());
    // every lane of the digit reads the count before the digit's first lane advances it
    // (one wave, program order on one LDS address)
    const uint32_t base = valid ? wc[d] : 0u;
    rank[r] = base + below;
    if (valid && below == 0) wc[d] = base + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: the waves' offsets, and the tile's count of the digit
  for (int d = threadIdx.x; d < kDigits; d += kSortBlock) {
    uint32_t acc = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
      const uint32_t c = wcount[w][d];
      wcount[w][d] = acc;
      acc += c;
    }
    lstart[d] = acc;
    gbase[d] = digit_base[d] + hist[(long long)d * nblocks + blockIdx.x];
  }
  __syncthreads();
  block_exclusive_scan<kDigits>(lstart);
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int i = wave * kWaveChunk + r * 64 + lane;
    if (i < count) {
      const int d = (int)((key[r] >> shift) & (kDigits - 1));
      const uint32_t slot = lstart[d] + wc[d] + rank[r];
      if ((int)slot < count) {  // always true: the counts above are this tile's
        lkey[slot] = key[r];
        lval[slot] = val[r];
      }
    }
  }
  __syncthreads();
  // write out in slot order: runs of equal digits go to consecutive destinations
  for (int i = threadIdx.x; i < count; i += kSortBlock) {
    const uint32_t k = lkey[i];
    const int d = (int)((k >> shift) & (kDigits - 1));
    const long long out = (long long)gbase[d] + (i - (int)lstart[d]);
    if (out < n) {  // always true for consistent histograms
      if (KEYS) keys_out[out] = k;
      val_out[out] = lval[i];
    }
  }
}

// start[k] = first sorted position with key >= k, for k = 0..m+1 (start[m+1] = n).
__global__ void region_starts_kernel(const uint32_t *__restrict__ keys, long long n, int m,
                                     uint32_t *__restrict__ start, uint32_t *__restrict__ n_big) {
  const long long pos = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos == 0) *n_big = 0;  // the list of large regions is rebuilt by region_update_kernel
  if (pos >= n) return;
  // keys are <= m by construction; the clamps keep every write inside start[0 .. m+1]
  const long long cur = min((long long)keys[pos], (long long)m);
  const long long prev = pos ? min((long long)keys[pos - 1], (long long)m) : -1;
  for (long long k = prev + 1; k <= cur; ++k) start[k] = (uint32_t)pos;
  if (pos == n - 1)
    for (long long k = cur + 1; k <= (long long)m + 1; ++k) start[k] = (uint32_t)n;
}

// The update of window w of region k (eq. step_size_n, eq. update_lambda): gamma(n_k + w)
// sgn_w, with n_k the region's update count at the start of the batch.
__device__ __forceinline__ double window_delta(const ramlt_adapt_params &p, int n_k, long long w, int8_t sgn) {
  const double gamma = fmin(p.gamma_max, p.gamma_scale / sqrt((double)((long long)n_k + w)));
  return gamma * (double)sgn;
}

// Region k's share of the sorted batch and the pending-window bookkeeping.
struct RegionSpan {
  long long lo, hi, need0;  // sorted positions [lo, hi); visits that close the pending window
  int i0;
};

__device__ __forceinline__ RegionSpan region_span(const uint32_t *start, long long n, int k, const ramlt_adapt_params &p,
                                                  const ramlt_region_state &s) {
  RegionSpan r;
  r.hi = min((long long)start[k + 1], n);
  r.lo = min((long long)start[k], r.hi);
  r.i0 = pending_visits(s.visits[k], p.L);
  r.need0 = p.L - r.i0;
  return r;
}

// The update of closed window w of region k: the window's acceptance sum in proposal order
// (fp64; the region's first window continues the carried A_k), alpha_hat = sum / L, and
// gamma(n_k + w) sgn(alpha_hat - alpha*).
__device__ __forceinline__ double closed_window_update(const ramlt_adapt_params &p, const ramlt_region_state &s,
                                                       const float *__restrict__ alpha_sorted, const RegionSpan &r,
                                                       int k, int n_k, long long w) {
  const int L = p.L;
  double a;
  long long b, e;
  if (w == 0) {
    a = s.acc[k];
    b = r.lo;
    e = r.lo + r.need0;
  } else {
    a = 0.0;
    b = r.lo + r.need0 + (w - 1) * L;
    e = b + L;
  }
#pragma unroll 8
  for (long long q = b; q < e; ++q) a += (double)alpha_sorted[q];  // loads issue ahead of the adds
  const double ahat = a / (double)L;
  const int8_t sgn = (int8_t)((ahat > p.alpha_target) - (ahat < p.alpha_target));
  return window_delta(p, n_k, w, sgn);
}

constexpr int kSmallWindows = 64;  // regions closing more windows go to the wave kernel

// One thread per region. A region whose batch closes at most kSmallWindows windows is
// finished here: its window updates lambda <- max(lambda + delta_w, lambda_min) applied in
// order, the visits after the last closed window summed (in proposal order) into the new
// A_k / i_k. Larger regions are listed for region_update_wave_kernel (a workgroup each).
__global__ __launch_bounds__(kSortBlock) void region_update_kernel(const uint32_t *__restrict__ start,
                                                                   const float *__restrict__ alpha_sorted,
                                                                   long long n, const ramlt_adapt_params p,
                                                                   const ramlt_region_state s,
                                                                   uint32_t *__restrict__ big,
                                                                   uint32_t *__restrict__ n_big) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.n_regions) return;
  const RegionSpan r = region_span(start, n, k, p, s);
  const long long c = r.hi - r.lo;
  double lam = s.lambda[k];
  if (c < r.need0) {  // no window closes: only the pending sum grows
    if (c > 0) {
      double a = s.acc[k];
      for (long long t = r.lo; t < r.hi; ++t) a += (double)alpha_sorted[t];
      s.acc[k] = a;
      s.visits[k] = r.i0 + (int)c;
    }
    if (s.lambda_f32) s.lambda_f32[k] = (float)lam;
    return;
  }
  const int L = p.L;
  const long long nw = 1 + (c - r.need0) / L;
  if (nw > kSmallWindows) {
    big[atomicAdd(n_big, 1u)] = (uint32_t)k;  // order of the list is irrelevant
    return;
  }
  const long long rem = (c - r.need0) % L;
  const int n_k = s.updates[k];
  for (long long w = 0; w < nw; ++w)
    lam = fmax(lam + closed_window_update(p, s, alpha_sorted, r, k, n_k, w), p.lambda_min);
  double a = 0.0;
  for (long long t = r.hi - rem; t < r.hi; ++t) a += (double)alpha_sorted[t];
  s.acc[k] = a;
  s.visits[k] = (int)rem;
  s.lambda[k] = lam;
  s.updates[k] = s.updates[k] + (int)nw;
  if (s.lambda_f32) s.lambda_f32[k] = (float)lam;
}

// One workgroup per listed region (grid-stride over the list): the window updates are
// maps lambda -> max(lambda + A, C); maps compose to the same form (A = A1 + A2,
// C = max(C1 + A2, C2)), so each thread composes a contiguous block of windows and thread
// 0 applies the 256 block maps in thread order.
__global__ __launch_bounds__(kSortBlock) void region_update_wave_kernel(const uint32_t *__restrict__ start,
                                                                        const float *__restrict__ alpha_sorted,
                                                                        long long n, const ramlt_adapt_params p,
                                                                        const ramlt_region_state s,
                                                                        const uint32_t *__restrict__ big,
                                                                        const uint32_t *__restrict__ n_big) {
  __shared__ double mA[kSortBlock], mC[kSortBlock];
  const uint32_t count = *n_big;
  for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {  // block-uniform
    const int k = (int)big[i];
    const RegionSpan r = region_span(start, n, k, p, s);
    const int L = p.L;
    const long long c = r.hi - r.lo;
    const long long nw = 1 + (c - r.need0) / L;  // > kSmallWindows
    const long long rem = (c - r.need0) % L;
    const long long per = (nw + kSortBlock - 1) / kSortBlock;
    double A = 0.0, C = -INFINITY;
    const long long w1 = min(nw, (long long)threadIdx.x * per), w2 = min(nw, w1 + per);
    const int n_k = s.updates[k];
    for (long long w = w1; w < w2; ++w) {
      const double d = closed_window_update(p, s, alpha_sorted, r, k, n_k, w);
      A += d;
      C = fmax(C + d, p.lambda_min);
    }
    mA[threadIdx.x] = A;
    mC[threadIdx.x] = C;
    __syncthreads();
    if (threadIdx.x == 0) {
      double lam = s.lambda[k];
      const int used = (int)((nw + per - 1) / per);  // threads holding a block of windows
      for (int j = 0; j < used; ++j) lam = fmax(lam + mA[j], mC[j]);
      double a = 0.0;
      for (long long t = r.hi - rem; t < r.hi; ++t) a += (double)alpha_sorted[t];
      s.acc[k] = a;
      s.visits[k] = (int)rem;
      s.lambda[k] = lam;
      s.updates[k] = s.updates[k] + (int)nw;
      if (s.lambda_f32) s.lambda_f32[k] = (float)lam;
    }
    __syncthreads();  // mA / mC are reused for the next listed region
  }
}

// ---------------------------------------------------------------- small-grid path (m < 512)
constexpr int kSmallGrid = 1 << kMaxDigitBits;  // regions of the single-pass path: m < kSmallGrid
constexpr int kPlanBlock = kSmallGrid;

// Windows closed by region k's visits in this batch (0 if the pending window stays open).
__device__ __forceinline__ long long closed_windows(const RegionSpan &r, int L) {
  const long long c = r.hi - r.lo;
  return c < r.need0 ? 0 : 1 + (c - r.need0) / L;
}

// A window update is the map lambda -> max(lambda + A, C) (A = delta_w, C = lambda_min);
// maps compose to the same form, (A1, C1) then (A2, C2) = (A1 + A2, max(C1 + A2, C2)), with
// the identity (0, -inf). A region's closed windows are folded in chunks of kFoldChunk.
constexpr int kFoldPer = 8;                         // windows per thread of a chunk
constexpr int kFoldChunk = kSortBlock * kFoldPer;   // windows per chunk (one workgroup)

struct WinMap {
  double A, C;
};
__device__ __forceinline__ WinMap then(WinMap f, WinMap g) { return WinMap{f.A + g.A, fmax(f.C + g.A, g.C)}; }

// wbase[k] = closed windows of the regions before k, wbase[m] = all of them; cbase the same
// for the regions' chunks of windows (one workgroup, a thread per region; one scan of both
// counts packed in 64 bits).
__global__ __launch_bounds__(kPlanBlock) void window_plan_kernel(const uint32_t *__restrict__ start, long long n,
                                                                 const ramlt_adapt_params p,
                                                                 const ramlt_region_state s,
                                                                 uint32_t *__restrict__ wbase,
                                                                 uint32_t *__restrict__ cbase) {
  __shared__ unsigned long long v[kPlanBlock];
  const int k = threadIdx.x;
  const int m = p.n_regions;
  const unsigned long long nw = k < m ? (unsigned long long)closed_windows(region_span(start, n, k, p, s), p.L) : 0ull;
  const unsigned long long own = (nw << 32) | ((nw + kFoldChunk - 1) / kFoldChunk);
  v[k] = own;
  __syncthreads();
  for (int off = 1; off < kPlanBlock; off <<= 1) {  // inclusive scan
    const unsigned long long add = k >= off ? v[k - off] : 0ull;
    __syncthreads();
    v[k] += add;
    __syncthreads();
  }
  const unsigned long long ex = v[k] - own;
  if (k < m) {
    wbase[k] = (uint32_t)(ex >> 32);
    cbase[k] = (uint32_t)ex;
  }
  if (k == m - 1) {
    wbase[m] = (uint32_t)(v[k] >> 32);
    cbase[m] = (uint32_t)v[k];
  }
}

// One thread per closed window g (windows numbered region by region): its region k and
// ordinal w from wbase, and the window's update into delta[g].
__global__ __launch_bounds__(kSortBlock) void window_sums_kernel(const uint32_t *__restrict__ start,
                                                                 const uint32_t *__restrict__ wbase,
                                                                 const float *__restrict__ alpha_sorted, long long n,
                                                                 const ramlt_adapt_params p,
                                                                 const ramlt_region_state s,
                                                                 double *__restrict__ delta) {
  __shared__ uint32_t wb[kSmallGrid + 1];
  const int m = p.n_regions;
  for (int i = threadIdx.x; i <= m; i += kSortBlock) wb[i] = wbase[i];
  __syncthreads();
  const uint32_t g = blockIdx.x * kSortBlock + threadIdx.x;
  if (g >= wb[m]) return;
  int lo = 0, hi = m - 1;  // the last region whose first window is <= g (it closes window g)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wb[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  const int k = lo;
  const RegionSpan r = region_span(start, n, k, p, s);
  delta[g] = closed_window_update(p, s, alpha_sorted, r, k, s.updates[k], (long long)(g - wb[k]));
}

// One workgroup per chunk of a region's closed windows: each thread composes kFoldPer
// consecutive windows in order, then the threads' maps are combined pairwise in a fixed
// tree (neighbours first), and the chunk's map goes to chunk_map[c].
__global__ __launch_bounds__(kSortBlock) void fold_chunks_kernel(const uint32_t *__restrict__ wbase,
                                                                 const uint32_t *__restrict__ cbase,
                                                                 const double *__restrict__ delta,
                                                                 const ramlt_adapt_params p,
                                                                 WinMap *__restrict__ chunk_map) {
  __shared__ uint32_t cb[kSmallGrid + 1];
  __shared__ WinMap red[kSortBlock];
  const int m = p.n_regions;
  for (int i = threadIdx.x; i <= m; i += kSortBlock) cb[i] = cbase[i];
  __syncthreads();
  const uint32_t c = blockIdx.x;
  if (c >= cb[m]) return;  // block-uniform
  int lo = 0, hi = m - 1;  // the region of chunk c
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cb[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const int k = lo;
  const long long w0 = (long long)(c - cb[k]) * kFoldChunk;
  const long long nw = (long long)wbase[k + 1] - wbase[k];
  const double *d = delta + wbase[k];
  WinMap f{0.0, -INFINITY};
  const long long b = w0 + (long long)threadIdx.x * kFoldPer;
#pragma unroll
  for (int j = 0; j < kFoldPer; ++j) {
    if (b + j < nw) {
      const double x = d[b + j];
      f.A += x;
      f.C = fmax(f.C + x, p.lambda_min);
    }
  }
  red[threadIdx.x] = f;
  __syncthreads();
  for (int h = 1; h < kSortBlock; h <<= 1) {
    if ((threadIdx.x & (2 * h - 1)) == 0) red[threadIdx.x] = then(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) chunk_map[c] = red[0];
}

// One thread per region: the chunk maps applied to lambda in order, the visits after the
// last closed window summed into the new A_k / i_k (or, when no window closes, the visits
// added to the pending A_k).
__global__ __launch_bounds__(kSortBlock) void region_fold_kernel(const uint32_t *__restrict__ start,
                                                                 const uint32_t *__restrict__ wbase,
                                                                 const uint32_t *__restrict__ cbase,
                                                                 const float *__restrict__ alpha_sorted, long long n,
                                                                 const WinMap *__restrict__ chunk_map,
                                                                 const ramlt_adapt_params p,
                                                                 const ramlt_region_state s) {
  const int k = blockIdx.x * kSortBlock + threadIdx.x;
  if (k >= p.n_regions) return;
  const RegionSpan r = region_span(start, n, k, p, s);
  const long long c = r.hi - r.lo;
  if (c < r.need0) {  // no window closes: only the pending sum grows
    if (c > 0) {
      double a = s.acc[k];
      for (long long t = r.lo; t < r.hi; ++t) a += (double)alpha_sorted[t];
      s.acc[k] = a;
      s.visits[k] = r.i0 + (int)c;
    }
    if (s.lambda_f32) s.lambda_f32[k] = (float)s.lambda[k];
    return;
  }
  const int L = p.L;
  const long long nw = (long long)wbase[k + 1] - wbase[k];
  const long long rem = (c - r.need0) % L;
  double lam = s.lambda[k];
  for (uint32_t j = cbase[k]; j < cbase[k + 1]; ++j) lam = fmax(lam + chunk_map[j].A, chunk_map[j].C);
  double a = 0.0;
  for (long long t = r.hi - rem; t < r.hi; ++t) a += (double)alpha_sorted[t];
  s.acc[k] = a;
  s.visits[k] = (int)rem;
  s.lambda[k] = lam;
  s.updates[k] = s.updates[k] + (int)nw;
  if (s.lambda_f32) s.lambda_f32[k] = (float)lam;
}

// Passes and digit width of the sort for keys 0..m (m marks invalid proposals): 8-bit
// digits, except that keys of exactly 9 bits (256 <= m < 512, e.g. a 20 x 20 grid) sort
// in one 9-bit pass. A pass reads and writes the stream once, but wider digits cost
// histogram bins, per-tile tables and LDS occupancy: measured on 16 M proposals, one
// 9-bit pass (~230 us) beats two 8-bit passes, while 10-bit passes (~340 us each) lose to
// the 8-bit passes they would save.
struct SortPlan {
  int passes, bits;
};

SortPlan sort_plan(int m) {
  int bits = 1;
  while (bits < 31 && ((long long)1 << bits) <= (long long)m) ++bits;
  if (bits == kMaxDigitBits) return SortPlan{1, kMaxDigitBits};
  return SortPlan{(bits + 7) / 8, 8};
}

// One pass of the sort; start non-null: the single pass of the small-grid path (values only,
// region starts from the digit scan).
template <int BITS>
void launch_sort_pass(const int32_t *region, const float *alpha, const uint32_t *kin, const float *vin, long long n,
                      int m, int shift, uint32_t *hist, uint32_t *totals, int nblocks, uint32_t *kout, float *vout,
                      uint32_t *start, hipStream_t st) {
  hipLaunchKernelGGL(sort_hist_kernel<BITS>, dim3(nblocks), dim3(kSortBlock), 0, st, region, kin, n, m, shift, hist,
                     nblocks);
  hipLaunchKernelGGL(scan_rows_kernel, dim3(1 << BITS), dim3(kScanBlock), 0, st, hist, nblocks, totals);
  hipLaunchKernelGGL(scan_digits_kernel<BITS>, dim3(1), dim3(1 << BITS), 0, st, totals, start, m, n);
  if (start)
    hipLaunchKernelGGL((sort_scatter_kernel<BITS, false>), dim3(nblocks), dim3(kSortBlock), 0, st, region, alpha, kin,
                       vin, n, m, shift, hist, totals, nblocks, kout, vout);
  else
    hipLaunchKernelGGL((sort_scatter_kernel<BITS, true>), dim3(nblocks), dim3(kSortBlock), 0, st, region, alpha, kin,
                       vin, n, m, shift, hist, totals, nblocks, kout, vout);
}

struct AdaptWorkspace {
  uint32_t *keys[2], *hist, *totals, *start, *big, *n_big, *wbase, *cbase;
  float *vals[2];
  double *delta;   // small-grid path: the update of each closed window, by window number
  WinMap *chunk_map;  // small-grid path: the map of each chunk of a region's windows
  size_t bytes;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

AdaptWorkspace carve(void *ws, long long n, int m) {
  const long long nblocks = (n + kSortTile - 1) / kSortTile;
  AdaptWorkspace w{};
  char *p = (char *)ws;
  size_t off = 0;
  auto take = [&](size_t b) {
    char *q = p ? p + off : nullptr;
    off += align256(b);
    return (uint32_t *)q;
  };
  w.keys[0] = take((size_t)n * 4);
  w.keys[1] = take((size_t)n * 4);
  w.vals[0] = (float *)take((size_t)n * 4);
  w.vals[1] = (float *)take((size_t)n * 4);
  const size_t digits = (size_t)1 << sort_plan(m).bits;
  w.hist = take(digits * (size_t)nblocks * 4);
  w.totals = take(digits * 4);
  w.start = take(((size_t)m + 2) * 4);
  w.big = take((size_t)m * 4);
  w.n_big = take(4);
  if (m < kSmallGrid) {
    // closed windows <= n / L + m <= n + m; chunks <= (n + m) / kFoldChunk + m
    w.wbase = take(((size_t)m + 1) * 4);
    w.cbase = take(((size_t)m + 1) * 4);
    w.delta = (double *)take(((size_t)n + (size_t)m) * 8);
    w.chunk_map = (WinMap *)take((((size_t)n + (size_t)m) / kFoldChunk + (size_t)m + 1) * sizeof(WinMap));
  }
  w.bytes = off;
  return w;
}

}  // namespace

size_t adapt_workspace_bytes(long long n, int m) {
  if (n <= 0 || m < 1) return 0;
  return carve(nullptr, n, m).bytes;
}

hipError_t launch_region_adapt(const ramlt_adapt_params &p, const ramlt_region_state &s, const int32_t *region,
                               const float *alpha, long long n, void *ws, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int m = p.n_regions;
  const AdaptWorkspace w = carve(ws, n, m);
  const int nblocks = (int)((n + kSortTile - 1) / kSortTile);
  const SortPlan plan = sort_plan(m);
  if (m < kSmallGrid) {  // keys of at most 9 bits: one pass
    if (plan.passes != 1) return hipErrorInvalidValue;  // (sort_plan gives one pass here)
    if (plan.bits == 8)
      launch_sort_pass<8>(region, alpha, nullptr, nullptr, n, m, 0, w.hist, w.totals, nblocks, nullptr, w.vals[0],
                          w.start, st);
    else
      launch_sort_pass<9>(region, alpha, nullptr, nullptr, n, m, 0, w.hist, w.totals, nblocks, nullptr, w.vals[0],
                          w.start, st);
    hipLaunchKernelGGL(window_plan_kernel, dim3(1), dim3(kPlanBlock), 0, st, w.start, n, p, s, w.wbase, w.cbase);
    // closed windows <= n / L + m, their chunks <= wmax / kFoldChunk + m
    const long long wmax = n / p.L + m;
    hipLaunchKernelGGL(window_sums_kernel, dim3((unsigned)((wmax + kSortBlock - 1) / kSortBlock)), dim3(kSortBlock),
                       0, st, w.start, w.wbase, w.vals[0], n, p, s, w.delta);
    hipLaunchKernelGGL(fold_chunks_kernel, dim3((unsigned)(wmax / kFoldChunk + m)), dim3(kSortBlock), 0, st, w.wbase,
                       w.cbase, w.delta, p, w.chunk_map);
    hipLaunchKernelGGL(region_fold_kernel, dim3((unsigned)((m + kSortBlock - 1) / kSortBlock)), dim3(kSortBlock), 0,
                       st, w.start, w.wbase, w.cbase, w.vals[0], n, w.chunk_map, p, s);
    return hipGetLastError();
  }
  int cur = 0;  // buffers holding the keys of the previous pass (none before pass 0)
  for (int q = 0; q < plan.passes; ++q) {
    const uint32_t *kin = q ? w.keys[cur] : nullptr;
    const float *vin = q ? w.vals[cur] : nullptr;
    const int out = q ? cur ^ 1 : 0;
    const int shift = q * plan.bits;
    if (plan.bits == 8)
      launch_sort_pass<8>(region, alpha, kin, vin, n, m, shift, w.hist, w.totals, nblocks, w.keys[out], w.vals[out],
                          nullptr, st);
    else
      launch_sort_pass<9>(region, alpha, kin, vin, n, m, shift, w.hist, w.totals, nblocks, w.keys[out], w.vals[out],
                          nullptr, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur = out;
  }
  hipLaunchKernelGGL(region_starts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w.keys[cur], n, m,
                     w.start, w.n_big);
  hipLaunchKernelGGL(region_update_kernel, dim3((unsigned)((m + kSortBlock - 1) / kSortBlock)), dim3(kSortBlock), 0,
                     st, w.start, w.vals[cur], n, p, s, w.big, w.n_big);
  // large regions: at most n / (L kSmallWindows) of them; a fixed grid strides the list
  hipLaunchKernelGGL(region_update_wave_kernel, dim3(256), dim3(kSortBlock), 0, st, w.start, w.vals[cur], n, p, s,
                     w.big, w.n_big);
  return hipGetLastError();
}

}  // namespace ramlt
