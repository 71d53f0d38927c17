// Quadtree partitions (Sec. 6.1-6.3): a forest of quadtrees stored as flat arrays, leaf lookup
// by descent, and a deterministic refinement pass.
//
// Layout: node i has child[i] (first of its four consecutive children, -1 for a leaf) and
// depth[i]; squares are implicit (a descent follows the bits of the point's coordinates).
// The lookup keeps the first kCacheNodes entries of child[] in LDS (nodes are numbered in
// creation order, so the low indices are the upper levels every descent passes through;
// the forests of the paper's settings, a few thousand nodes, fit whole), adds a jump table
// over the top levels of forests of few trees, and counts the visits of the first
// kBinNodes nodes in LDS, one global atomic per counter and workgroup (global atomics on
// the same few thousand counters run at a fraction of LDS speed).
//
// Refinement (one pass, split leaves numbered in node order):
//   1. count the leaves to split per tile of kRefineBlock nodes;
//   2. one workgroup scans the tile counts, caps the number of splits at the free storage
//      and publishes the new node count;
//   3. every leaf that splits takes rank r among the splitting leaves (tile offset + its
//      place inside the tile) and writes its children at n_nodes_old + 4 r; every visit
//      counter restarts from 0.
#include "launch.hpp"

#include <stdint.h>

#include <algorithm>

namespace ramlt {

namespace {

constexpr int kMaxDepth = RAMLT_QT_MAX_DEPTH;
constexpr int kLookupBlock = 1024;
constexpr int kLookupBatch = 4;      // points per thread in flight
constexpr int kCacheNodes = 9712;    // child[] of the first nodes (+1 slot), 38 KB of LDS
constexpr int kBinNodes = 9728;      // visit counters of the first nodes, 38 KB
constexpr int kJumpEntries = 1024;   // jump table, 4 KB: 80 KB in all, two workgroups per CU
constexpr int kRefineBlock = 1024;   // nodes per tile, one per thread
constexpr int kRefineWaves = kRefineBlock / 64;
constexpr int kInitBlock = 256;

struct RefineHeader {
  int32_t old_nodes;   // node count before the pass
  int32_t splits;      // splits made in the pass
};

constexpr size_t kHeaderBytes = 256;

__device__ __forceinline__ int clamp_nodes(int n, int capacity) { return n < 0 ? 0 : (n > capacity ? capacity : n); }

__global__ __launch_bounds__(kInitBlock) void init_kernel(int32_t *__restrict__ child, int32_t *__restrict__ depth,
                                                          int32_t *__restrict__ visits, int32_t *__restrict__ n_nodes,
                                                          int n_roots) {
  const int i = blockIdx.x * kInitBlock + threadIdx.x;
  if (i < n_roots) {
    child[i] = -1;
    depth[i] = 0;
    visits[i] = 0;
  }
  if (i == 0) *n_nodes = n_roots;
}

// Range test of a first-child index c >= 0: valid iff n_roots <= c <= nn - 4, done as one
// unsigned compare (c - lo) <= span. With no valid index (nn < n_roots + 4), lo = INT_MIN
// puts every c >= 0 out of range.
struct ChildRange {
  uint32_t lo, span;
};

__device__ __forceinline__ ChildRange child_range(int nn, int n_roots) {
  const int span = nn - 4 - n_roots;
  return span >= 0 ? ChildRange{(uint32_t)n_roots, (uint32_t)span} : ChildRange{0x80000000u, 0u};
}

// The quadrant tests run on integers: with X = floor(x 2^20) (x 2^20 is exact in float32),
// limited to 2^20 - 1 so that x = 1 lies right of every split, the test x >= x0 + s/2 at
// depth d (a threshold that is an integer multiple of 2^-20 for d < 20) is bit 19 - d of X,
// given that the descent so far followed X's higher bits. That is the same decision as
// the floating-point test.
__device__ __forceinline__ uint32_t grid_coord(float v) { return min((uint32_t)(v * 1048576.f), 0xFFFFFu); }

__device__ __forceinline__ bool point_valid(int r, int n_roots, int nn, float x, float y) {
  return r >= 0 && r < n_roots && r < nn && x >= 0.f && x <= 1.f && y >= 0.f && y <= 1.f;
}

// Forest held whole in LDS (n_nodes <= kCacheNodes). Entry of node i, as a byte address
// plus a quadrant mask: 4 c + 3 for an inner node with first child c, 4 i for a leaf (a
// step from a leaf stays there), 4 kc for an inner node whose link is inconsistent, where
// slot kc is a leaf that stands for "no region". One step from entry E with quadrant q is
// then (E & ~3) + 4 (q & E): no per-lane branch, so the lanes of a wave step together and
// the only branch is the loop exit, taken every two levels once every lane sits at a leaf
// (the descent is bound by instruction issue). At most 20 steps; a lane still at an inner
// node then (a node at depth 20 with children) gets -1.
__device__ __forceinline__ uint32_t encode_entry(int i, int c, ChildRange cr, int kc) {
  if (c < 0) return 4u * (uint32_t)i;
  return (uint32_t)c - cr.lo <= cr.span ? 4u * (uint32_t)c + 3u : 4u * (uint32_t)kc;
}

// Jump table: for every tree of a forest with few trees, the table address reached after
// the first J levels (J even) for each of the 4^J cells of the top J bits of X and Y -- the
// leaf the descent stopped at if it was reached earlier (leaves loop to themselves).
// Descents then start at depth J.
__device__ __forceinline__ int jump_levels(int n_roots) {
  return n_roots * 256 <= kJumpEntries ? 4 : (n_roots * 16 <= kJumpEntries ? 2 : 0);
}

__device__ __forceinline__ uint32_t jump_cell(uint32_t X, uint32_t Y, int J) {
  return (X >> (20 - J)) | ((Y >> (20 - J)) << J);
}

__device__ void build_jump_table(const uint32_t *__restrict__ table, uint32_t *__restrict__ jump, int J, int n_roots,
                                 int nn, int kc) {
  const int cells = 1 << (2 * J);
  const char *base = (const char *)table;
  for (int i = threadIdx.x; i < n_roots * cells; i += kLookupBlock) {
    const int r = i >> (2 * J);
    const uint32_t c = (uint32_t)(i & (cells - 1));
    uint32_t a = 4u * (uint32_t)(r < nn ? r : kc);
    for (int t = J - 1; t >= 0; --t) {   // the cell's bits, most significant first
      const uint32_t q = ((c >> t) & 1u) | (((c >> (J + t)) & 1u) << 1);
      const uint32_t E = *(const uint32_t *)(base + a);
      a = (E & ~3u) + ((q & E) << 2);
    }
    jump[i] = a;
  }
}

template <int J>
__device__ __forceinline__ int descend_lds(const uint32_t *__restrict__ table, const uint32_t *__restrict__ jump,
                                           int kc, int n_roots, int nn, int r, float x, float y) {
  const bool ok = point_valid(r, n_roots, nn, x, y);
  const uint32_t X = ok ? grid_coord(x) : 0u;
  const uint32_t Y = ok ? grid_coord(y) : 0u;
  const char *base = (const char *)table;
  uint32_t a = !ok ? 4u * (uint32_t)kc
                   : (J > 0 ? jump[((uint32_t)r << (2 * J)) | jump_cell(X, Y, J)] : 4u * (uint32_t)r);
  uint32_t E = *(const uint32_t *)(base + a);
  // two levels per pass; J is even, so s stays odd and s - 1 >= 0
  for (int s = kMaxDepth - 1 - J; s >= 0 && __ballot(E & 3u) != 0; s -= 2) {
    uint32_t q = ((X >> s) & 1u) | (((Y >> s) & 1u) << 1);
    a = (E & ~3u) + ((q & E) << 2);
    E = *(const uint32_t *)(base + a);
    q = ((X >> (s - 1)) & 1u) | (((Y >> (s - 1)) & 1u) << 1);
    a = (E & ~3u) + ((q & E) << 2);
    E = *(const uint32_t *)(base + a);
  }
  const int leaf = (int)(a >> 2);
  return ((E & 3u) != 0 || leaf == kc) ? -1 : leaf;
}

// Forest larger than the LDS table: `cache` holds child[0..kc) as stored. A child is
// always numbered after its parent, so a descent reads LDS while its node is below kc and
// global memory from the first node at or above it on. A leaf's entry is negative, so one
// unsigned compare of c - lo with span stops a lane at a leaf or at an inconsistent link;
// the latter, and children below the depth limit, give -1. Every lane counts its depth.
__device__ __forceinline__ int descend_mixed(const int32_t *__restrict__ cache, int kc,
                                             const int32_t *__restrict__ child, ChildRange cr, int nn, int n_roots,
                                             int r, float x, float y) {
  bool live = point_valid(r, n_roots, nn, x, y);
  uint32_t X = live ? grid_coord(x) << 12 : 0u;
  uint32_t Y = live ? grid_coord(y) << 12 : 0u;
  int node = live ? r : 0;
  bool bad = !live;
  int d = 0;
  while (__ballot(live && node < kc) != 0) {
    const bool act = live && node < kc;
    const int c = cache[act ? node : 0];
    const bool stop = (uint32_t)c - cr.lo > cr.span || d == kMaxDepth;
    bad = bad || (act && stop && c >= 0);
    live = live && !(act && stop);
    const bool go = act && !stop;
    node = go ? c + (int)(X >> 31) + 2 * (int)(Y >> 31) : node;
    X = go ? X << 1 : X;
    Y = go ? Y << 1 : Y;
    d += go ? 1 : 0;
  }
  while (__ballot(live) != 0) {
    const int c = child[live ? node : 0];
    const bool stop = (uint32_t)c - cr.lo > cr.span || d == kMaxDepth;
    bad = bad || (live && stop && c >= 0);
    const bool go = live && !stop;
    live = go;
    node = go ? c + (int)(X >> 31) + 2 * (int)(Y >> 31) : node;
    X <<= 1;
    Y <<= 1;
    d += 1;
  }
  return bad ? -1 : node;
}

// kJump < 0: the forest is not held whole in LDS; else the LDS descent with kJump levels
// taken from the jump table.
template <int kJump>
__device__ __forceinline__ int descend(const int32_t *__restrict__ cache, const uint32_t *__restrict__ jump, int kc,
                                       const int32_t *__restrict__ child, ChildRange cr, int nn, int n_roots, int r,
                                       float x, float y) {
  if (kJump >= 0) return descend_lds<(kJump >= 0 ? kJump : 0)>((const uint32_t *)cache, jump, kc, n_roots, nn, r, x, y);
  return descend_mixed(cache, kc, child, cr, nn, n_roots, r, x, y);
}

// Grid-stride over points; a thread takes its points kLookupBatch at a time (p, p + stride,
// ... at the same lane of consecutive grid passes, so every load is coalesced), and loads
// the next batch before it descends the current one: a chain of LDS reads per point
// leaves the loads exposed otherwise. Visits of nodes below kBinNodes are counted in LDS
// and added to the global counters once per workgroup; the others take a global atomic.
struct PointBatch {
  float x[kLookupBatch], y[kLookupBatch];
  int r[kLookupBatch];
};

__device__ __forceinline__ void load_batch(PointBatch &b, const int32_t *__restrict__ root,
                                           const float *__restrict__ xs, const float *__restrict__ ys, uint32_t p,
                                           uint32_t stride, uint32_t n) {
#pragma unroll
  for (int j = 0; j < kLookupBatch; ++j) {
    const uint32_t i = p + j * stride;
    const bool in = i < n;
    b.x[j] = in ? xs[i] : 0.f;
    b.y[j] = in ? ys[i] : 0.f;
    b.r[j] = (in && root) ? root[i] : 0;
  }
}

template <int kJump>
__device__ __forceinline__ void lookup_loop(const int32_t *__restrict__ cache, const uint32_t *__restrict__ jump,
                                            int kc, int32_t *__restrict__ bins,
                                            int kb, const int32_t *__restrict__ child, int32_t *__restrict__ visits,
                                            const int32_t *__restrict__ root, const float *__restrict__ xs,
                                            const float *__restrict__ ys, int32_t *__restrict__ leaf, uint32_t n,
                                            int nn, int n_roots, int count) {
  // n <= 2^30 and the grid is at most 2^19 threads, so no index below wraps
  const ChildRange cr = child_range(nn, n_roots);
  const uint32_t stride = gridDim.x * kLookupBlock;
  uint32_t p = blockIdx.x * kLookupBlock + threadIdx.x;
  if (p >= n) return;
  PointBatch cur, nxt;
  load_batch(cur, root, xs, ys, p, stride, n);
  while (true) {
    const uint32_t q = p + kLookupBatch * stride;
    if (q < n) load_batch(nxt, root, xs, ys, q, stride, n);
#pragma unroll
    for (int j = 0; j < kLookupBatch; ++j) {
      const uint32_t i = p + j * stride;
      if (i < n) {
        const int l = descend<kJump>(cache, jump, kc, child, cr, nn, n_roots, cur.r[j], cur.x[j], cur.y[j]);
        leaf[i] = l;
        if (count && l >= 0) {
          if (l < kb)
            atomicAdd(&bins[l], 1);
          else
            atomicAdd(&visits[l], 1);
        }
      }
    }
    if (q >= n) break;
    p = q;
    cur = nxt;
  }
}

__global__ __launch_bounds__(kLookupBlock) void lookup_kernel(const int32_t *__restrict__ child,
                                                              const int32_t *__restrict__ n_nodes,
                                                              int32_t *__restrict__ visits,
                                                              const int32_t *__restrict__ root,
                                                              const float *__restrict__ xs,
                                                              const float *__restrict__ ys, int32_t *__restrict__ leaf,
                                                              long long n, int n_roots, int capacity, int count) {
  __shared__ int32_t cache[kCacheNodes + 1];
  __shared__ int32_t bins[kBinNodes];
  __shared__ uint32_t jump[kJumpEntries];
  const int nn = clamp_nodes(*n_nodes, capacity);
  const int kc = min(nn, kCacheNodes);
  const int kb = count ? min(nn, kBinNodes) : 0;
  const bool all = kc == nn;
  const int J = all ? jump_levels(n_roots) : 0;
  if (all) {
    const ChildRange cr = child_range(nn, n_roots);
    for (int i = threadIdx.x; i <= kc; i += kLookupBlock)
      cache[i] = (int32_t)(i < kc ? encode_entry(i, child[i], cr, kc) : 4u * (uint32_t)kc);
  } else {
    for (int i = threadIdx.x; i < kc; i += kLookupBlock) cache[i] = child[i];
  }
  for (int i = threadIdx.x; i < kb; i += kLookupBlock) bins[i] = 0;
  __syncthreads();
  if (J > 0) {
    build_jump_table((const uint32_t *)cache, jump, J, n_roots, nn, kc);
    __syncthreads();
  }
#define RAMLT_LOOKUP(JJ) \
  lookup_loop<JJ>(cache, jump, kc, bins, kb, child, visits, root, xs, ys, leaf, (uint32_t)n, nn, n_roots, count)
  if (!all)
    RAMLT_LOOKUP(-1);
  else if (J == 4)
    RAMLT_LOOKUP(4);
  else if (J == 2)
    RAMLT_LOOKUP(2);
  else
    RAMLT_LOOKUP(0);
#undef RAMLT_LOOKUP
  if (kb > 0) {
    __syncthreads();
    for (int i = threadIdx.x; i < kb; i += kLookupBlock) {
      const int c = bins[i];
      if (c != 0) atomicAdd(&visits[i], c);
    }
  }
}

__device__ __forceinline__ bool splits_now(const int32_t *__restrict__ child, const int32_t *__restrict__ depth,
                                           const int32_t *__restrict__ visits, int i, int m_split) {
  return child[i] < 0 && visits[i] > m_split && depth[i] < kMaxDepth;
}

// Exclusive prefix of `flag` over the workgroup (node order = thread order); also returns
// the workgroup's total in *total.
__device__ __forceinline__ int block_rank(bool flag, int *total) {
  __shared__ int wave_count[kRefineWaves];
  const unsigned long long b = __ballot(flag);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (lane == 0) wave_count[wave] = __popcll(b);
  __syncthreads();
  int before = 0, all = 0;
  for (int w = 0; w < kRefineWaves; ++w) {
    const int c = wave_count[w];
    before += w < wave ? c : 0;
    all += c;
  }
  *total = all;
  return before + __popcll(b & __lanemask_lt());
}

__global__ __launch_bounds__(kRefineBlock) void refine_count_kernel(const int32_t *__restrict__ child,
                                                                    const int32_t *__restrict__ depth,
                                                                    const int32_t *__restrict__ visits,
                                                                    const int32_t *__restrict__ n_nodes, int capacity,
                                                                    int m_split, int32_t *__restrict__ tile_count) {
  const int nn = clamp_nodes(*n_nodes, capacity);
  const int base = blockIdx.x * kRefineBlock;
  if (base >= nn) return;
  const int i = base + threadIdx.x;
  const bool f = i < nn && splits_now(child, depth, visits, i, m_split);
  int total;
  block_rank(f, &total);
  if (threadIdx.x == 0) tile_count[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the tile counts, the cap, the new node count.
__global__ __launch_bounds__(kRefineBlock) void refine_scan_kernel(const int32_t *__restrict__ tile_count,
                                                                   int32_t *__restrict__ tile_off,
                                                                   int32_t *__restrict__ n_nodes, int capacity,
                                                                   RefineHeader *__restrict__ hdr) {
  __shared__ int wave_sum[kRefineWaves];
  __shared__ int carry_s;
  const int nn = clamp_nodes(*n_nodes, capacity);
  const int tiles = (nn + kRefineBlock - 1) / kRefineBlock;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int t0 = 0; t0 < tiles; t0 += kRefineBlock) {
    const int t = t0 + threadIdx.x;
    const int v = t < tiles ? tile_count[t] : 0;
    int s = v;   // inclusive scan inside the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(s, o, 64);
      if (lane >= o) s += u;
    }
    if (lane == 63) wave_sum[wave] = s;
    __syncthreads();
    int before = carry_s, all = carry_s;
    for (int w = 0; w < kRefineWaves; ++w) {
      before += w < wave ? wave_sum[w] : 0;
      all += wave_sum[w];
    }
    if (t < tiles) tile_off[t] = before + s - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = all;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int room = (capacity - nn) / 4;
    const int splits = min(carry_s, room);
    hdr->old_nodes = nn;
    hdr->splits = splits;
    *n_nodes = nn + 4 * splits;
  }
}

__global__ __launch_bounds__(kRefineBlock) void refine_apply_kernel(
    int32_t *__restrict__ child, int32_t *__restrict__ depth, int32_t *__restrict__ visits,
    const int32_t *__restrict__ tile_off, const RefineHeader *__restrict__ hdr, int m_split,
    ramlt_region_state st, int has_state) {
  const int nn = hdr->old_nodes;
  const int base = blockIdx.x * kRefineBlock;
  if (base >= nn) return;
  const int i = base + threadIdx.x;
  const bool f = i < nn && splits_now(child, depth, visits, i, m_split);
  int total;
  const int r = tile_off[blockIdx.x] + block_rank(f, &total);
  if (i >= nn) return;
  if (visits[i] != 0) visits[i] = 0;
  if (!f || r >= hdr->splits) return;
  const int first = nn + 4 * r;
  const int d = depth[i] + 1;
  child[i] = first;
  double lam = 0.0;
  float lam32 = 0.f;
  int upd = 1;
  if (has_state) {
    lam = st.lambda[i];
    upd = max(1, st.updates[i] / 4);
    if (st.lambda_f32) lam32 = st.lambda_f32[i];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = first + q;
    child[c] = -1;
    depth[c] = d;
    visits[c] = 0;
    if (has_state) {
      st.lambda[c] = lam;
      st.acc[c] = 0.0;
      st.visits[c] = 0;
      st.updates[c] = upd;
      if (st.lambda_f32) st.lambda_f32[c] = lam32;
    }
  }
}

size_t tiles_of(int capacity) { return ((size_t)capacity + kRefineBlock - 1) / kRefineBlock; }

}  // namespace

size_t quadtree_workspace_bytes(int capacity) {
  const size_t t = tiles_of(capacity) * sizeof(int32_t);
  const size_t t_al = (t + 255) / 256 * 256;
  return kHeaderBytes + 2 * t_al;
}

hipError_t launch_quadtree_init(const ramlt_quadtree &t, hipStream_t st) {
  init_kernel<<<(t.n_roots + kInitBlock - 1) / kInitBlock, kInitBlock, 0, st>>>(t.child, t.depth, t.visits,
                                                                                 t.n_nodes, t.n_roots);
  return hipGetLastError();
}

hipError_t launch_quadtree_lookup(const ramlt_quadtree &t, const int32_t *root, const float *x, const float *y,
                                  int32_t *leaf, long long n, int count, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const long long want = (n + kLookupBlock - 1) / kLookupBlock;
  // two resident workgroups per CU, at most 512 (the loop's 32-bit indices rely on it)
  const long long cap = std::min(2LL * (cus > 0 ? cus : 256), 512LL);
  const int grid = (int)(want < cap ? want : cap);
  lookup_kernel<<<grid, kLookupBlock, 0, st>>>(t.child, t.n_nodes, t.visits, root, x, y, leaf, n, t.n_roots,
                                               t.capacity, count);
  return hipGetLastError();
}

hipError_t launch_quadtree_refine(const ramlt_quadtree &t, int m_split, const ramlt_region_state *s, void *ws,
                                  hipStream_t st) {
  const int tiles = (int)tiles_of(t.capacity);
  const size_t t_al = (tiles * sizeof(int32_t) + 255) / 256 * 256;
  char *w = (char *)ws;
  RefineHeader *hdr = (RefineHeader *)w;
  int32_t *tile_count = (int32_t *)(w + kHeaderBytes);
  int32_t *tile_off = (int32_t *)(w + kHeaderBytes + t_al);
  refine_count_kernel<<<tiles, kRefineBlock, 0, st>>>(t.child, t.depth, t.visits, t.n_nodes, t.capacity, m_split,
                                                      tile_count);
  refine_scan_kernel<<<1, kRefineBlock, 0, st>>>(tile_count, tile_off, t.n_nodes, t.capacity, hdr);
  ramlt_region_state none = {};
  refine_apply_kernel<<<tiles, kRefineBlock, 0, st>>>(t.child, t.depth, t.visits, tile_off, hdr, m_split,
                                                      s ? *s : none, s ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ramlt
