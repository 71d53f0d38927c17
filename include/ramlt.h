/*
 * ramlt.h -- per-pixel Monte Carlo chain statistics and the regional reconstruction
 * filter, with its adjoint, on AMD Instinct MI355X (gfx950).
 *
 * The operations follow "Regional Adaptive Metropolis Light Transport" (Otsu et al.):
 *
 *   stats_accumulate  Appendix A: per-pixel estimator mean, sample variance, lag
 *                     autocorrelations rho_k and autocorrelation time
 *                     tau = 1 + 2 sum_k rho_k of each pixel's sample sequence
 *                     (buffer order is the sequence); feature planes get mean and variance.
 *   filter_forward    Sec. 3.1 eq. path_integral: the pixel reconstruction filter h_j
 *                     applied to the per-pixel means, as a normalised Gaussian over the
 *                     (2r+1)^2 window, clipped at the border, whose width
 *                     sigma_k = sqrt(exp(lambda_k)) (Sec. 5.3) is looked up from the
 *                     region of the output pixel on the N x N screen grid
 *                     (Sec. 5.2 state-dependent parameters, Sec. 6.1 grid partition).
 *   loss_seed         MSE against a reference image, L = sum (out - R)^2 / (3P), and its
 *                     gradient U = 2 (out - R) / (3P). (Not in the paper; drives the adjoint.)
 *   filter_backward   The exact adjoint of filter_forward composed with the per-pixel mean:
 *                     dL/dg for every radiance sample and dL/dlambda_k per region, with the
 *                     window weights recomputed from lambda.
 *   region_adapt      Algorithm 1: regional adaptation of lambda_k from a batch of
 *                     (region, acceptance probability) proposals.
 *   quadtree_*        Sec. 6.1-6.3: quadtree partitions (forests for the 2-D and 4-D
 *                     partitions), leaf lookup with visit counts, refinement.
 *   perturb_directions  Sec. 3.3: proposed ray directions with a truncated-normal polar
 *                     angle of scale sigma_k = sqrt(exp(lambda_k)).
 *   rrmse             Sec. 8.2: relative RMS error map and image value.
 *   lens_chain_step   Sec. 3.3 / 6.1 / Alg. 1: one Metropolis step of screen-space chains
 *                     under the regional adaptive lens perturbation (luminance target);
 *                     lens_chain_sort regroups the chains by screen tile between steps.
 *
 * Conventions shared by every entry point
 *   - All pointers inside ramlt_frame are DEVICE pointers into memory the caller owns
 *     (e.g. allocated by PyTorch). The library allocates nothing, never synchronises,
 *     never copies between host and device, keeps no pointer after returning, and only
 *     enqueues work on `stream` (a hipStream_t; NULL = the null stream).
 *   - frames_host is a HOST array of n_frames descriptors. It is read for validation and
 *     launch sizing only. With n_frames == 1, frames_dev may be NULL. With n_frames > 1
 *     frames_dev must be a device-resident copy of the same array (built once by the
 *     caller, e.g. before graph capture); kernels read descriptors from it and process
 *     all frames in one launch per operation (per radius for the filter operations).
 *   - Sample planes are laid out [c][s][y][x] with x contiguous; stride_c, stride_s,
 *     stride_y are element strides (radiance and features each have their own).
 *     Per-pixel planes (mean, var, tau, out, reference, grad_out, grad_radiance,
 *     feat_*) are dense [c][H][W]; lag_corr is dense [3][K_L][H][W].
 *   - Return value: a RAMLT_* status. On failure nothing has been enqueued (validation
 *     runs entirely on the host before any launch) except for RAMLT_EHIP, which reports
 *     a failed HIP call; ramlt_last_error() then holds a message (thread-local).
 *   - NaN or Inf inputs propagate to the outputs; they never abort a call.
 */
#ifndef RAMLT_H
#define RAMLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ramlt_status {
  RAMLT_OK = 0,
  RAMLT_EINVAL = 1,       /* bad argument: null required pointer, size, radius, lag, ... */
  RAMLT_EUNSUPPORTED = 2, /* unknown dtype, non-gfx950 device, plane too large          */
  RAMLT_EWORKSPACE = 3,   /* workspace missing or smaller than ramlt_workspace_size()    */
  RAMLT_EHIP = 4          /* a HIP runtime call or kernel launch failed                   */
};

enum ramlt_feature_dtype { RAMLT_F32 = 0, RAMLT_F16 = 1 };

enum ramlt_op {
  RAMLT_OP_STATS = 0,
  RAMLT_OP_FILTER_FORWARD = 1,
  RAMLT_OP_LOSS_SEED = 2,
  RAMLT_OP_FILTER_BACKWARD = 3
};

/* Launch schedule in ramlt_frame.flags (results do not depend on it beyond fp32 rounding
 * order; 0 selects the defaults). The autotuner (paper_2402_08273_amd/tune.py) picks them.
 *   bits 0-1: output tile of the filter kernels (filter_forward, filter_backward);
 *   bit 2:    RAMLT_SCHED_DIRECT: the filter gathers each (2r+1)^2 window directly instead of
 *             a pass over rows then columns.
 * Frames of one batch with different tiles run in separate launches.
 *
 * Where the loss is formed, also in ramlt_frame.flags:
 *   bit 3:    RAMLT_LOSS_IN_FORWARD: filter_forward forms, besides out, the MSE loss seed
 *             (writes grad_out = U = 2 (out - reference) / (3 W H), accumulates *loss) and the
 *             parameter half of the adjoint (accumulates grad_lambda), from the window sums it
 *             holds for out; filter_backward then forms grad_radiance only, from grad_out
 *             (reference, loss and grad_lambda are left alone). Over the pair the results are
 *             those of filter_forward followed by filter_backward with the seed fused, up to
 *             fp32 rounding order; the per-pixel planes are read and written fewer times.
 * Other bits must be 0. */
enum ramlt_tile { RAMLT_TILE_DEFAULT = 0, RAMLT_TILE_32X8 = 1, RAMLT_TILE_32X16 = 2, RAMLT_TILE_64X8 = 3 };
#define RAMLT_TILE_MASK 3
#define RAMLT_SCHED_DIRECT 4
#define RAMLT_LOSS_IN_FORWARD 8
/* Launch size of stats_accumulate, bits 4-7 (v = (flags >> RAMLT_STATS_WG_SHIFT) & 15):
 * v = 1..14: the frame's 256-pixel tiles are covered by a series of launches of v
 * workgroups per compute unit each, so that every workgroup of a launch is resident from
 * its start; v = 15: one launch covers the whole frame; v = 0: the default (4 per compute
 * unit). A batch takes the value of its first frame. A single frame of fewer than 1024
 * tiles (under 262 144 pixels) ignores it: one launch of a workgroup per (tile, channel).
 * Results do not depend on it. */
#define RAMLT_STATS_WG_SHIFT 4
#define RAMLT_STATS_WG_MASK (15 << RAMLT_STATS_WG_SHIFT)
#define RAMLT_STATS_ONE_LAUNCH 15
#define RAMLT_FLAGS_KNOWN (RAMLT_TILE_MASK | RAMLT_SCHED_DIRECT | RAMLT_LOSS_IN_FORWARD | RAMLT_STATS_WG_MASK)

#define RAMLT_N_RADIANCE 3
#define RAMLT_N_FEATURES 7
#define RAMLT_MAX_RADIUS 15
#define RAMLT_MAX_LAG 32
#define RAMLT_MAX_FRAMES 4096
#define RAMLT_MAX_REGIONS 4096             /* n_regions (grid side N) must not exceed this */
#define RAMLT_MAX_PLANE_ELEMS (1LL << 30) /* (H-1)*stride_y + W and W*H must not exceed this */
#define RAMLT_MAX_SIDE 65536               /* W and H must not exceed this               */

/* One frame of render buffers and its outputs. Fields an operation does not use are
 * ignored by it (they may be NULL/0). "in" = read, "out" = written, "acc" = accumulated (+=). */
typedef struct ramlt_frame {
  int32_t W, H;           /* image size, >= 1                                          */
  int32_t S;              /* samples per pixel, >= 1                                   */
  int32_t max_lag;        /* stats: 0..RAMLT_MAX_LAG; K_L = min(max_lag, S - 1)         */

  /* stats, in: radiance samples g[3][S][H][W] (fp32)                                  */
  const float *radiance;
  int64_t rad_stride_c, rad_stride_s, rad_stride_y;

  /* stats, in: feature samples f[7][S][H][W] (albedo rgb, normal xyz, depth), or NULL */
  const void *features;
  int64_t feat_stride_c, feat_stride_s, feat_stride_y;
  int32_t feat_dtype;     /* RAMLT_F32 or RAMLT_F16                                    */
  int32_t flags;          /* launch schedule, RAMLT_TILE_* | RAMLT_SCHED_*; 0 = defaults */

  /* stats, out: [3][H][W] each; lag_corr [3][K_L][H][W] or NULL                       */
  float *mean, *var, *tau, *lag_corr;
  /* stats, out: [7][H][W] each; required iff features != NULL                          */
  float *feat_mean, *feat_var;

  /* filter parameters: lambda[n_regions * n_regions], row-major (ky, kx), in           */
  const float *lambda;
  int32_t n_regions;      /* grid size N, 1..RAMLT_MAX_REGIONS (the paper's N_top = 20)  */
  int32_t radius;         /* window radius r, 0..RAMLT_MAX_RADIUS; K = 2r + 1           */
  float lambda_min;       /* lower clamp of lambda (the paper uses -30); finite         */
  int32_t _reserved0;

  /* filter_forward: in = mean; out = filtered image [3][H][W]                          */
  float *out;
  /* loss_seed: in = out, reference [3][H][W]; out = grad_out; acc = *loss (fp64)       */
  const float *reference;
  double *loss;           /* may be NULL                                               */
  /* filter_backward: in = grad_out U = dL/dout, mean, out                               */
  float *grad_out;
  /* filter_backward, out: G [3][H][W], dL/dg[c][s][y][x] = G[c][y][x] for every s       */
  float *grad_radiance;
  /* filter_backward, acc: dL/dlambda [n_regions^2] (caller zeroes); may be NULL         */
  float *grad_lambda;
} ramlt_frame;

/* Appendix A per-pixel statistics (mean = the estimator of I_j, Sec. 3.2; variance;
 * rho_k = C_k / M2 with C_k = sum_{s<S-k} (g_s - mean)(g_{s+k} - mean); tau; features:
 * mean and variance). Accumulation is in fp64. var = M2 / (S - 1), 0 for S = 1. A pixel
 * whose samples are all equal gets rho_k = 0 and tau = 1. Requires per frame: radiance,
 * mean, var, tau; features => feat_mean, feat_var. Workspace: see ramlt_workspace_size. */
int stats_accumulate(const ramlt_frame *frames_host, const ramlt_frame *frames_dev,
                     int32_t n_frames, void *workspace, size_t ws_bytes, void *stream);

/* Sec. 3.1 reconstruction filter with per-region width (Sec. 5.2-5.3, 6.1):
 *   k(x,y) = floor((2y+1)N/(2H)) * N + floor((2x+1)N/(2W)),
 *   h_jp = exp(-(dx^2+dy^2) / (2 exp(max(lambda_k(j), lambda_min)))),
 *   out_j = sum_{p in window(j), inside} h_jp mean_p / sum h_jp   (fp32).
 * (A NaN lambda_k gives NaN outputs for its region.)
 * Requires per frame: mean, lambda, out, n_regions >= 1, 0 <= radius <= 15.
 * With RAMLT_LOSS_IN_FORWARD in flags also: reference and grad_out (loss and grad_lambda
 * optional), and a workspace of ramlt_workspace_size(..., RAMLT_OP_FILTER_FORWARD) bytes for
 * the per-tile partial sums of the loss and dL/dlambda, added in a fixed order as
 * filter_backward adds its own (see there). */
int filter_forward(const ramlt_frame *frames_host, const ramlt_frame *frames_dev,
                   int32_t n_frames, void *workspace, size_t ws_bytes, void *stream);

/* grad_out = 2 (out - reference) / (3 W H); *loss += sum (out - reference)^2 / (3 W H)
 * (fp64 accumulation; summed over frames in a batch). Requires: out, reference, grad_out. */
int loss_seed(const ramlt_frame *frames_host, const ramlt_frame *frames_dev,
              int32_t n_frames, void *workspace, size_t ws_bytes, void *stream);

/* Adjoint of filter_forward o per-pixel mean, for U = grad_out:
 *   grad_radiance_p = (1/S) sum_{j : p in window(j)} U_j h_jp / D_j,
 *   grad_lambda_k  += sum_{k(j)=k} sum_c U_jc sum_p h'_jp (mean_pc - out_jc) / D_j,
 *   h'_jp = h_jp (dx^2+dy^2) / (2 sigma^2) if lambda_k >= lambda_min else 0
 *   (and NaN for a NaN lambda_k, which propagates as in filter_forward).
 * With RAMLT_LOSS_IN_FORWARD in flags: grad_radiance only (filter_forward has formed the
 * rest); requires lambda, grad_out, grad_radiance.
 * Otherwise requires: mean, out, lambda, grad_radiance, and either grad_out, or (grad_out NULL)
 * reference: then U = 2 (out - reference) / (3 W H) is formed inside the kernel (the
 * loss seed fused into the adjoint, nothing written to grad_out) and *loss, if not
 * NULL, accumulates the MSE as loss_seed would. grad_lambda may be NULL.
 * Workspace: always needed, ramlt_workspace_size(..., RAMLT_OP_FILTER_BACKWARD) bytes
 * (per-tile partial sums of dL/dlambda and of the loss, then a plan per radius for a
 * batch). The partials are added in a fixed order by a second kernel, one atomic add per
 * (frame, region) and per frame: a single frame whose regions are >= 16 px wide and
 * >= 4 px tall gets run-to-run identical grad_lambda and loss; smaller regions, and frames
 * of a batch that share grad_lambda or loss, are summed in atomic (unordered) order. */
int filter_backward(const ramlt_frame *frames_host, const ramlt_frame *frames_dev,
                    int32_t n_frames, void *workspace, size_t ws_bytes, void *stream);

/* The whole differentiable step of ONE frame in one call: stats_accumulate, then
 * filter_forward with RAMLT_LOSS_IN_FORWARD (out, the MSE seed U in grad_out, *loss and
 * grad_lambda accumulated), then filter_backward (grad_radiance) -- Appendix A and
 * Sec. 3.1 eq. path_integral with Sec. 5.2-5.3, as for those calls -- enqueued in that
 * order on `stream`. Every output is bit for bit what the three calls give with the same
 * descriptor. frame: HOST pointer to one descriptor whose flags include
 * RAMLT_LOSS_IN_FORWARD, with every field the three calls require (radiance, mean, var,
 * tau, features => feat_mean / feat_var, lambda, out, reference, grad_out, grad_radiance;
 * lag_corr, loss and grad_lambda optional; loss and grad_lambda accumulate, the caller
 * zeroes them). Flags bits 4-7 size the statistics launches as for stats_accumulate.
 * workspace: DEVICE, 256-byte aligned, at least ramlt_workspace_size(frame, 1,
 * RAMLT_OP_FILTER_FORWARD) bytes (the per-tile partials). Errors as for the three calls;
 * all validation precedes the first launch. */
int stats_filter_step(const ramlt_frame *frame, void *workspace, size_t ws_bytes, void *stream);

/* filter_backward for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same operation and
 * results, with the workspace taken from a device array the library owns, so the caller
 * passes no workspace. The array holds RAMLT_NOALLOC_WORKSPACE_BYTES on every GPU the
 * library runs on, until the process ends; a call whose ramlt_workspace_size(...,
 * RAMLT_OP_FILTER_BACKWARD) exceeds it returns RAMLT_EWORKSPACE (a single 3840x2160 frame
 * needs about 400 KB). The call allocates nothing. Every call on one GPU uses that GPU's
 * one array: calls that overlap on one GPU (on different streams, or from different host
 * threads without ordering) race and must not be made; calls ordered on one stream are
 * fine. No part of the array needs to start at zero (each call writes every entry it
 * reads). Other arguments and errors as for filter_backward. */
#define RAMLT_NOALLOC_WORKSPACE_BYTES (4u << 20)
int filter_backward_noalloc(const ramlt_frame *frames_host, const ramlt_frame *frames_dev, int32_t n_frames,
                            void *stream);

/* ---------------------------------------------------------------------------------
 * Regional adaptation of the scaling parameters (Algorithm 1 with eqs. est_exp_acc,
 * update_lambda and step_size_n; parameters of Sec. 8.1).
 *
 * A batch of proposals i = 0..n-1 carries the region k_i of the chain's current state
 * (Alg. 1 line 8) and its acceptance probability alpha_i (line 11). Regions are
 * independent (Sec. 5.3, "Criterion for Adaptation"); within a region the proposals are
 * taken in index order, exactly as the sequential algorithm would visit them:
 *   A_k += alpha_i; i_k += 1; once i_k reaches L:
 *     alpha_hat = A_k / L; gamma = min(gamma_max, gamma_scale / sqrt(n_k));
 *     lambda_k = max(lambda_k + gamma * sgn(alpha_hat - alpha_target), lambda_min);
 *     i_k = 0; A_k = 0; n_k += 1.
 * (The listing tests i_k > L but divides by L; the update here fires at i_k == L. The
 * Sec. 5.3 prose states the direction of the update the other way round from eq.
 * update_lambda; the equation is followed. sgn(0) = 0; a NaN alpha gives sgn 0.)
 * alpha is accumulated in fp64 in the proposals' order, so every decision and every state
 * value equals the sequential algorithm's in fp64 (the same IEEE operations in the same
 * order). Proposals whose region is outside [0, n_regions) are skipped. The state carries
 * over between calls: consecutive batches equal one batch of their concatenation. */
typedef struct ramlt_adapt_params {
  int32_t n_regions;      /* m, 1..RAMLT_MAX_ADAPT_REGIONS                               */
  int32_t L;              /* visits per update (the paper's L = 10), 1..RAMLT_MAX_ADAPT_L */
  double gamma_max;       /* eq. step_size_n cap (paper: 1); finite                       */
  double gamma_scale;     /* eq. step_size_n scale (paper: 5); finite                     */
  double alpha_target;    /* alpha* (paper: 0.5); finite                                  */
  double lambda_min;      /* lower limit of lambda (paper: -30); finite                   */
} ramlt_adapt_params;

/* Per-region state, DEVICE arrays of n_regions entries, read and updated in place.
 * Initial values (Alg. 1 lines 2-7): lambda = lambda_init (paper: 1), acc = 0,
 * visits = 0, updates = 1. Invariant kept by every call: 0 <= visits < L. */
typedef struct ramlt_region_state {
  double *lambda;         /* lambda_k = log sigma_k^2                                    */
  double *acc;            /* A_k, accumulated acceptance of the pending visits           */
  int32_t *visits;        /* i_k, visits since the last update                           */
  int32_t *updates;       /* n_k, 1 + number of updates so far                          */
  float *lambda_f32;      /* optional (NULL = none): lambda_k rounded to float, the table
                             filter_forward reads                                        */
} ramlt_region_state;

#define RAMLT_MAX_ADAPT_REGIONS (1 << 24)
#define RAMLT_MAX_ADAPT_L (1 << 20)
#define RAMLT_MAX_PROPOSALS (1LL << 30)

/* region: DEVICE int32[n]; alpha: DEVICE float[n]; n in 0..RAMLT_MAX_PROPOSALS (0 = no
 * work). params, state: HOST structs. workspace: DEVICE, 256-byte aligned, at least
 * ramlt_adapt_workspace_size(n, n_regions) bytes (proposals sorted by region, stably,
 * and region boundaries). The state arrays and the workspace, which the call writes, must
 * not overlap each other or the proposals (RAMLT_EINVAL). Errors as for the other entry
 * points. */
int region_adapt(const ramlt_adapt_params *params, const ramlt_region_state *state, const int32_t *region,
                 const float *alpha, int64_t n_proposals, void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes of region_adapt (0 for n_proposals <= 0 or invalid sizes). */
size_t ramlt_adapt_workspace_size(int64_t n_proposals, int32_t n_regions);

/* ------------------------------------------------------------------------------------
 * Quadtree partitions (Sec. 6.1 "Quadtree Partition", Sec. 6.2 "Refining Quadtree Partition",
 * Sec. 6.3 "4d Partition"; Sec. 7 "Explicit Synchronization for Refinement of Partitions").
 *
 * A forest of n_roots quadtrees, each over the unit square [0,1]^2: one tree for the 2-D
 * screen partition; one tree per screen grid cell for the 4-D partition (the tree then
 * covers the two coordinates of the outgoing direction). The regions are the leaves; a
 * node's index is its region key (for region_adapt and its state arrays).
 *
 * Nodes are numbered in creation order: the roots 0..n_roots-1, then the four children of
 * each split, consecutively (child q covers the quadrant q = right + 2 * top). Node i is
 * stored as child[i] (index of its first child, or -1 for a leaf) and depth[i] (0 for a
 * root; a node at depth d has side 2^-d). Its square follows from the path of quadrants
 * from its root. Leaves deeper than RAMLT_QT_MAX_DEPTH are never made, so every square
 * corner is exact in float32. */
typedef struct ramlt_quadtree {
  int32_t n_roots;        /* trees, 1..capacity                                           */
  int32_t capacity;       /* entries of child / depth / visits, 1..RAMLT_MAX_QT_NODES      */
  int32_t *child;         /* DEVICE [capacity]; entries >= *n_nodes are unused            */
  int32_t *depth;         /* DEVICE [capacity]                                            */
  int32_t *visits;        /* DEVICE [capacity]: lookups counted per leaf since the last
                             refinement (the split criterion; separate from the region
                             state's i_k, which restarts every L visits)                 */
  int32_t *n_nodes;       /* DEVICE [1]: nodes in use                                     */
} ramlt_quadtree;

#define RAMLT_QT_MAX_DEPTH 20
#define RAMLT_MAX_QT_NODES (1 << 26)
#define RAMLT_MAX_QT_POINTS (1LL << 30)

/* Reset the forest to its n_roots roots (each a leaf at depth 0 with no visits); sets
 * *n_nodes = n_roots. The tree struct is HOST memory holding device pointers. */
int quadtree_init(const ramlt_quadtree *tree, void *stream);

/* Region of each point: descend from tree root[i] (root == NULL: tree 0), choosing at a
 * node with lower corner (x0, y0) and side s the child (x >= x0 + s/2) + 2 (y >= y0 + s/2),
 * down to a leaf. leaf[i] = that leaf's index, or -1 when root[i] is outside
 * [0, n_roots), x or y is outside [0, 1] or NaN, or the stored links are inconsistent (a
 * first child outside [n_roots, capacity - 4], or more than RAMLT_QT_MAX_DEPTH levels).
 * count != 0 also adds 1 to visits[leaf] for every point with a region (integer atomics,
 * so the counts do not depend on the order; int32, so more than 2^31 - 1 visits of one
 * leaf between refinements wrap).
 * root: DEVICE int32[n] or NULL; x, y: DEVICE float[n]; leaf: DEVICE int32[n]; n in
 * 0..RAMLT_MAX_QT_POINTS. leaf, and the tree's visits when counting, must not overlap each
 * other, the points or the tree's other arrays. Errors: RAMLT_EINVAL for bad sizes or
 * pointers. */
int quadtree_lookup(const ramlt_quadtree *tree, const int32_t *root, const float *x, const float *y,
                    int32_t *leaf, int64_t n_points, int32_t count, void *stream);

/* One refinement pass: every leaf with more than m_split visits and depth below
 * RAMLT_QT_MAX_DEPTH splits into four children, in increasing node order; children made
 * in this pass are not considered again. When fewer than 4 * (number of such leaves)
 * entries are free, only the first floor((capacity - n_nodes) / 4) of them split. Every
 * visit counter then restarts from 0, and *n_nodes grows by 4 per split.
 * state (optional, NULL = none): the region state (ramlt_region_state, n_regions >=
 * capacity entries) of region_adapt; each child gets the parent's lambda (and lambda_f32)
 * as it is, updates = max(1, floor(parent updates / 4)) (the paper gives n_k / 4; it is
 * rounded down and kept >= 1 so the step size stays finite), and an empty pending window
 * (acc = 0, visits = 0). m_split >= 0. workspace: DEVICE, 256-byte aligned, at least
 * ramlt_quadtree_workspace_size(capacity) bytes. The tree's arrays, the first capacity
 * entries of the state's arrays and the workspace must not overlap (RAMLT_EINVAL). The
 * result is deterministic. */
int quadtree_refine(const ramlt_quadtree *tree, int32_t m_split, const ramlt_region_state *state,
                    void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes of quadtree_refine (0 for an invalid capacity). */
size_t ramlt_quadtree_workspace_size(int32_t capacity);

/* ------------------------------------------------------------------------------------
 * Direction perturbation (Sec. 3.3 "Perturbing Ray Directions"; the scale of region k is
 * sigma_k = sqrt(exp(lambda_k)), Sec. 5.3).
 *
 * For proposal i with region k = region[i], current direction omega_i (unit) and uniforms
 * (u, v) = uv[i] in [0, 1):
 *   theta' = sigma_k Phi^-1(Phi(-a) + u (Phi(a) - Phi(-a))), a = pi / sigma_k: the normal
 *            N(0, sigma_k^2) truncated to [-pi, pi], by its inverse CDF (fp64);
 *   phi'   = 2 pi v;
 *   omega' = sin theta' (cos phi' t + sin phi' b) + cos theta' omega_i (fp32),
 * with (t, b) the orthonormal basis of omega_i of Duff et al., "Building an Orthonormal
 * Basis, Revisited" (JCGT 2017): s = sign(z), a = -1/(s + z), c = x y a,
 * t = (1 + s x^2 a, s c, -s x), b = (c, s + y^2 a, -y). (The paper leaves the azimuth origin
 * open; every choice gives the same distribution.) u = 1/2 leaves omega unchanged; theta'
 * is clamped to [-pi, pi] (reached only at u = 0). A region outside [0, n_regions) gives NaN
 * outputs; NaN inputs propagate. omega is used as given (not renormalised).
 * lambda: DEVICE double[n_regions] (e.g. ramlt_region_state.lambda), 8-byte aligned;
 * region: DEVICE int32[n]; omega, omega_out: DEVICE float[n][3]; uv: DEVICE float[n][2],
 * 8-byte aligned; theta_out: DEVICE float[n] or NULL. n in 0..RAMLT_MAX_PROPOSALS;
 * n_regions in 1..RAMLT_MAX_ADAPT_REGIONS. workspace: DEVICE, 256-byte aligned, at least
 * ramlt_perturb_workspace_size(n_regions) bytes (per-region terms that depend on sigma only,
 * for up to 65536 regions; 0 bytes, and NULL allowed, above that or for n = 0). omega_out
 * may be omega itself; otherwise omega_out, theta_out and the workspace must not overlap
 * each other or an input. Errors: RAMLT_EINVAL for bad sizes/pointers, RAMLT_EWORKSPACE. */
int perturb_directions(const double *lambda, int32_t n_regions, const int32_t *region, const float *omega,
                       const float *uv, float *omega_out, float *theta_out, int64_t n, void *workspace,
                       size_t ws_bytes, void *stream);

/* Workspace bytes of perturb_directions (0 for an invalid n_regions). */
size_t ramlt_perturb_workspace_size(int32_t n_regions);

/* ------------------------------------------------------------------------------------
 * Screen-space chains of the regional adaptive lens perturbation (Sec. 3.3 "Lens
 * Perturbation", "Perturbing Ray Directions"; Sec. 6.1 "2d Partition for the Lens
 * Perturbation"; Alg. 1 lines 8-13), with an image's luminance standing in for the path
 * contribution: one Metropolis step per chain, producing the (region, alpha) stream that
 * region_adapt consumes.
 *
 * The state of chain i is its primary ray direction omega_i of a pinhole camera looking along
 * +z. Its raster position is sx = 1/2 + (1/2)(x / z) / tx, sy = 1/2 + (1/2)(y / z) / ty,
 * tx = tan_half_fov_x, ty = (float)(tx H / W) (from double); it is in the frame iff z > 0
 * and sx, sy in [0, 1), its pixel is (min(floor(sx W), W - 1), min(floor(sy H), H - 1)), and
 * its region the cell of that pixel on the n_regions x n_regions screen grid (the map of
 * filter_forward). Every one of these float operations rounds to nearest on its own.
 *   proposal: omega' as perturb_directions gives it for (u, v) = noise[i][0..1] with
 *             sigma_k = sqrt(exp(lambda[k])) of the current region k;
 *   alpha:    0 if omega' is outside the frame, else 1 if L' >= L, else L' / L (float), with
 *             L, L' the luminance at the two pixels (pi(omega) = L[pixel] is the target
 *             density over directions; the proposal is symmetric);
 *   move:     omega_i = omega' iff noise[i][2] < alpha.
 * region[i] = k, alpha[i] = alpha (Alg. 1 line 8: the region of the state before the move).
 * A chain whose state is outside the frame (or NaN) gets region -1 and alpha NaN and does not
 * move. density: DEVICE float[n] or NULL, read and updated in place: the luminance of each
 * chain's current pixel, carried between steps so that a step reads the image once per chain
 * (at the proposal) instead of twice; an entry below 0 or NaN (e.g. -1 before the first
 * step) is read from the image, and after the step every entry holds the luminance of the
 * chain's pixel (-1 for a chain outside the frame). Results equal those without it as long
 * as the image does not change between steps (reset the entries to -1 when it does).
 * pixel: DEVICE int32[n] or NULL, read and updated in place: each chain's current pixel
 * iy * W + ix under the raster map above (-1 for a chain outside the frame or NaN), carried
 * between steps so that a step skips the raster map of its current state; an entry below -1
 * or >= W * H (e.g. -2 before the first step) is taken from the raster map of omega, and
 * after the step every entry holds the chain's pixel. Results equal those without it as
 * long as the entries are the raster map of omega or below -1 (set them to -2 whenever omega
 * is changed other than by this call; permute them with the chains, as lens_chain_sort's
 * perm allows).
 * luminance: DEVICE float[H][W] (>= 0; NaN gives alpha NaN, never a move); lambda:
 * DEVICE double[n_regions^2], 8-byte aligned (e.g. ramlt_region_state.lambda); omega: DEVICE
 * float[n][3], read and updated in place; noise: DEVICE float[n][3]; region: DEVICE int32[n];
 * alpha: DEVICE float[n]; omega_prop: DEVICE float[n][3] or NULL (the proposals). W, H as for
 * rrmse; tan_half_fov_x finite, > 0; n_regions in 1..RAMLT_MAX_REGIONS; n in
 * 0..RAMLT_MAX_PROPOSALS. workspace: DEVICE, 256-byte aligned, at least
 * ramlt_lens_workspace_size(n_regions) bytes (0, and NULL allowed, above 65536 regions or for
 * n = 0). The buffers the call writes (omega, density, pixel, region, alpha, omega_prop, the
 * workspace) must not overlap each other or an input. Errors: RAMLT_EINVAL,
 * RAMLT_EWORKSPACE. */
int lens_chain_step(const float *luminance, int32_t W, int32_t H, float tan_half_fov_x, const double *lambda,
                    int32_t n_regions, float *omega, float *density, int32_t *pixel, const float *noise,
                    int32_t *region, float *alpha, float *omega_prop, int64_t n, void *workspace, size_t ws_bytes,
                    void *stream);

/* Workspace bytes of lens_chain_step (0 for an invalid n_regions). */
size_t ramlt_lens_workspace_size(int32_t n_regions);

/* Reorder of lens chains by screen tile, for the locality of lens_chain_step's luminance
 * reads. Not an operation of the paper: its chains are independent (Sec. 3.3, Sec. 7), so
 * their order in memory is free, and chains grouped by where they are on the screen read a
 * few KB of the image per workgroup instead of a cache line each.
 * The key of chain i is the T x T pixel tile of its current pixel under lens_chain_step's
 * raster map (tiles numbered row-major, tile = (iy / T) * ceil(W / T) + ix / T), or the tile
 * count for a chain outside the frame or NaN; T = 2^s with s the smallest integer >= 4 that
 * leaves at most 63 tiles (256 at 1920 x 1080, 512 at 3840 x 2160). The chains are written
 * in key order, stably (chains of one tile keep their index order):
 *   omega_out[j] = omega[perm[j]], density_out[j] = density[perm[j]], perm[j] = old index.
 * omega: DEVICE float[n][3] (read); density: DEVICE float[n] or NULL (lens_chain_step's
 * carried luminance, moved with its chain); omega_out: DEVICE float[n][3]; density_out:
 * DEVICE float[n], required iff density is given; perm: DEVICE int32[n] or NULL (the old
 * index of each chain, to reorder any per-chain data the caller keeps). The outputs and the
 * workspace must not overlap the inputs or each other. W, H, tan_half_fov_x as for
 * lens_chain_step; n in
 * 0..RAMLT_MAX_PROPOSALS. workspace: DEVICE, 256-byte aligned, at least
 * ramlt_lens_sort_workspace_size(n) bytes (64 counters per 4096 chains). Errors:
 * RAMLT_EINVAL, RAMLT_EWORKSPACE. */
int lens_chain_sort(int32_t W, int32_t H, float tan_half_fov_x, const float *omega, const float *density, int64_t n,
                    float *omega_out, float *density_out, int32_t *perm, void *workspace, size_t ws_bytes,
                    void *stream);

/* Workspace bytes of lens_chain_sort for n chains (0 for n <= 0). */
size_t ramlt_lens_sort_workspace_size(int64_t n);

/* ------------------------------------------------------------------------------------
 * rRMSE of an image against a reference (Sec. 8.2: the error measure of the paper's
 * equal-time comparisons, shown per pixel and for the whole image; the paper gives no
 * formula). Per pixel j of P = W H:
 *   e_j = (1/3) sum_c (I_cj - R_cj)^2 / (R_cj^2 + eps)   (fp64; eps keeps black reference
 *                                                         pixels finite, e.g. 1e-2)
 *   map[j] = sqrt(e_j) (float), *rrmse_out = sqrt((1/P) sum_j e_j) (double).
 * The image value is summed per workgroup and then in a fixed order: run-to-run identical.
 * image, reference: DEVICE float[3][H][W] (dense planes, e.g. filter_forward's out and the
 * frame's reference); map: DEVICE float[H][W] or NULL; rrmse_out: DEVICE double or NULL
 * (not both NULL); W, H in 1..RAMLT_MAX_SIDE with W H <= RAMLT_MAX_PLANE_ELEMS; eps finite,
 * >= 0. workspace: DEVICE, 256-byte aligned, >= ramlt_rrmse_workspace_size(W, H) bytes.
 * map, rrmse_out and the workspace must not overlap each other or the images. */
int rrmse(const float *image, const float *reference, int32_t W, int32_t H, double eps, float *map,
          double *rrmse_out, void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes of rrmse (0 for invalid sizes). */
size_t ramlt_rrmse_workspace_size(int32_t W, int32_t H);

/* Bytes of device workspace `op` needs for these frames (0 if none). Workspace is
 * caller-owned, 256-byte aligned, and may be reused across calls on one stream. */
size_t ramlt_workspace_size(const ramlt_frame *frames_host, int32_t n_frames, int32_t op);

/* Message for the last non-zero status returned on this thread ("" if none). */
const char *ramlt_last_error(void);

/* ABI version: sizeof(ramlt_frame) in the high 16 bits, revision in the low 16. */
int32_t ramlt_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RAMLT_H */
