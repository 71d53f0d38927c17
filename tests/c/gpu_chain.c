/* One pass of the whole path from C, with no Python or PyTorch in the process: the HIP
 * runtime allocates the buffers and libramlt does every step.
 *
 *   screen grid (N x N regions):  region_adapt -> stats_accumulate -> filter_forward (with
 *                                 the adapted lambda) -> filter_backward (loss seed fused)
 *                                 -> rrmse of the filtered image
 *   quadtree (one tree):          quadtree_init, then `rounds` times: quadtree_lookup
 *                                 (counted) -> region_adapt keyed by leaf ->
 *                                 quadtree_refine (children inherit lambda and n_k / 4);
 *                                 then quadtree_lookup -> perturb_directions with the
 *                                 leaves' lambda
 *   lens chains:                  lens_chain_step on a luminance image with the screen
 *                                 grid's adapted lambda
 *
 * Usage: gpu_chain DIR W H S N r max_lag n_prop capacity n_pts m_split rounds n_chains tan_half_fov_x
 * Inputs are raw little-endian arrays in DIR (radiance.f32 [3][S][H][W], features.f32
 * [7][S][H][W], reference.f32 [3][H][W], region.i32 / alpha.f32 [n_prop], px.f32 / py.f32 /
 * qalpha.f32 [n_pts], omega.f32 [n_pts][3], uv.f32 [n_pts][2], luminance.f32 [H][W],
 * chains.f32 / noise.f32 [n_chains][3]); every output is written to DIR as
 * out_<name>.<type>. Exit status 0 on success, 2 for a HIP error, 3 for a library
 * status, 4 for a file or argument error. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ramlt.h"

static const char *g_dir;

#define HIP_OK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
      exit(2);                                                                         \
    }                                                                                  \
  } while (0)

#define RAMLT_OK_(call)                                                                \
  do {                                                                                 \
    int s_ = (call);                                                                   \
    if (s_ != RAMLT_OK) {                                                              \
      fprintf(stderr, "%s:%d %s -> %d: %s\n", __FILE__, __LINE__, #call, s_, ramlt_last_error()); \
      exit(3);                                                                         \
    }                                                                                  \
  } while (0)

static void *dev_alloc(size_t bytes) {
  void *p = NULL;
  HIP_OK(hipMalloc(&p, bytes ? bytes : 256));
  return p;
}

static void *dev_zeros(size_t bytes) {
  void *p = dev_alloc(bytes);
  HIP_OK(hipMemset(p, 0, bytes ? bytes : 256));
  return p;
}

static void path_of(char *buf, size_t n, const char *name) {
  if ((size_t)snprintf(buf, n, "%s/%s", g_dir, name) >= n) {
    fprintf(stderr, "path too long: %s/%s\n", g_dir, name);
    exit(4);
  }
}

/* Reads exactly `bytes` from DIR/name into new device memory. */
static void *upload(const char *name, size_t bytes) {
  char path[4096];
  path_of(path, sizeof path, name);
  FILE *f = fopen(path, "rb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path);
    exit(4);
  }
  void *host = malloc(bytes ? bytes : 1);
  if (!host) exit(4);
  size_t got = fread(host, 1, bytes, f);
  int extra = fgetc(f);
  fclose(f);
  if (got != bytes || extra != EOF) {
    fprintf(stderr, "%s: expected exactly %zu bytes\n", path, bytes);
    exit(4);
  }
  void *d = dev_alloc(bytes);
  HIP_OK(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
  free(host);
  return d;
}

static void *upload_host(const void *host, size_t bytes) {
  void *d = dev_alloc(bytes);
  HIP_OK(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
  return d;
}

static void download(const char *name, const void *dev, size_t bytes) {
  char path[4096];
  path_of(path, sizeof path, name);
  void *host = malloc(bytes ? bytes : 1);
  if (!host) exit(4);
  HIP_OK(hipMemcpy(host, dev, bytes, hipMemcpyDeviceToHost));
  FILE *f = fopen(path, "wb");
  if (!f || fwrite(host, 1, bytes, f) != bytes || fclose(f) != 0) {
    fprintf(stderr, "cannot write %s\n", path);
    exit(4);
  }
  free(host);
}

/* Region state of Alg. 1 at its initial values (lambda = 1, A = 0, i = 0, n = 1). */
static ramlt_region_state new_state(int32_t m) {
  ramlt_region_state s;
  double *lam = malloc(sizeof(double) * (size_t)m);
  int32_t *ones = malloc(sizeof(int32_t) * (size_t)m);
  float *lam32 = malloc(sizeof(float) * (size_t)m);
  if (!lam || !ones || !lam32) exit(4);
  for (int32_t k = 0; k < m; ++k) {
    lam[k] = 1.0;
    ones[k] = 1;
    lam32[k] = 1.0f;
  }
  s.lambda = upload_host(lam, sizeof(double) * (size_t)m);
  s.acc = dev_zeros(sizeof(double) * (size_t)m);
  s.visits = dev_zeros(sizeof(int32_t) * (size_t)m);
  s.updates = upload_host(ones, sizeof(int32_t) * (size_t)m);
  s.lambda_f32 = upload_host(lam32, sizeof(float) * (size_t)m);
  free(lam);
  free(ones);
  free(lam32);
  return s;
}

static ramlt_adapt_params paper_params(int32_t m) {
  ramlt_adapt_params p;
  memset(&p, 0, sizeof p);
  p.n_regions = m;
  p.L = 10;
  p.gamma_max = 1.0;
  p.gamma_scale = 5.0;
  p.alpha_target = 0.5;
  p.lambda_min = -30.0;
  return p;
}

static void adapt(const ramlt_region_state *st, int32_t m, const int32_t *region, const float *alpha, int64_t n) {
  ramlt_adapt_params p = paper_params(m);
  size_t ws = ramlt_adapt_workspace_size(n, m);
  void *w = dev_alloc(ws);
  RAMLT_OK_(region_adapt(&p, st, region, alpha, n, w, ws, NULL));
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipFree(w));
}

int main(int argc, char **argv) {
  if (argc != 15) {
    fprintf(stderr, "usage: %s DIR W H S N r max_lag n_prop capacity n_pts m_split rounds n_chains tan_half_fov_x\n",
            argv[0]);
    return 4;
  }
  g_dir = argv[1];
  const int32_t W = atoi(argv[2]), H = atoi(argv[3]), S = atoi(argv[4]), N = atoi(argv[5]);
  const int32_t r = atoi(argv[6]), max_lag = atoi(argv[7]);
  const int64_t n_prop = atoll(argv[8]);
  const int32_t capacity = atoi(argv[9]);
  const int64_t n_pts = atoll(argv[10]);
  const int32_t m_split = atoi(argv[11]), rounds = atoi(argv[12]);
  const int64_t n_chains = atoll(argv[13]);
  const float tan_half = (float)atof(argv[14]);
  if (W < 1 || H < 1 || S < 1 || N < 1 || r < 0 || max_lag < 0 || n_prop < 1 || capacity < 1 || n_pts < 1 ||
      m_split < 0 || rounds < 1 || n_chains < 1 || !(tan_half > 0.0f) || (int64_t)W * H * S > (1 << 26)) {
    fprintf(stderr, "bad sizes\n");
    return 4;
  }
  const size_t P = (size_t)W * (size_t)H;
  const int32_t KL = max_lag < S - 1 ? max_lag : S - 1;
  const int32_t m = N * N;

  /* screen grid: adapt lambda from the proposals, then the reconstruction step */
  ramlt_region_state grid = new_state(m);
  int32_t *region = upload("region.i32", sizeof(int32_t) * (size_t)n_prop);
  float *alpha = upload("alpha.f32", sizeof(float) * (size_t)n_prop);
  adapt(&grid, m, region, alpha, n_prop);

  ramlt_frame f;
  memset(&f, 0, sizeof f);
  f.W = W;
  f.H = H;
  f.S = S;
  f.max_lag = max_lag;
  f.radiance = upload("radiance.f32", sizeof(float) * 3 * (size_t)S * P);
  f.rad_stride_c = (int64_t)S * (int64_t)P;
  f.rad_stride_s = (int64_t)P;
  f.rad_stride_y = W;
  f.features = upload("features.f32", sizeof(float) * 7 * (size_t)S * P);
  f.feat_stride_c = (int64_t)S * (int64_t)P;
  f.feat_stride_s = (int64_t)P;
  f.feat_stride_y = W;
  f.feat_dtype = RAMLT_F32;
  f.mean = dev_alloc(sizeof(float) * 3 * P);
  f.var = dev_alloc(sizeof(float) * 3 * P);
  f.tau = dev_alloc(sizeof(float) * 3 * P);
  f.lag_corr = KL > 0 ? dev_alloc(sizeof(float) * 3 * (size_t)KL * P) : NULL;
  f.feat_mean = dev_alloc(sizeof(float) * 7 * P);
  f.feat_var = dev_alloc(sizeof(float) * 7 * P);
  f.lambda = grid.lambda_f32;
  f.n_regions = N;
  f.radius = r;
  f.lambda_min = -30.0f;
  f.out = dev_alloc(sizeof(float) * 3 * P);
  f.reference = upload("reference.f32", sizeof(float) * 3 * P);
  f.loss = dev_zeros(sizeof(double));
  f.grad_out = NULL; /* the loss seed runs inside the adjoint */
  f.grad_radiance = dev_alloc(sizeof(float) * 3 * P);
  f.grad_lambda = dev_zeros(sizeof(float) * (size_t)m);

  size_t ws_bytes = ramlt_workspace_size(&f, 1, RAMLT_OP_STATS);
  const int32_t ops[2] = {RAMLT_OP_FILTER_FORWARD, RAMLT_OP_FILTER_BACKWARD};
  for (int i = 0; i < 2; ++i) {
    size_t b = ramlt_workspace_size(&f, 1, ops[i]);
    if (b > ws_bytes) ws_bytes = b;
  }
  void *ws = dev_alloc(ws_bytes);
  RAMLT_OK_(stats_accumulate(&f, NULL, 1, ws, ws_bytes, NULL));
  RAMLT_OK_(filter_forward(&f, NULL, 1, ws, ws_bytes, NULL));
  RAMLT_OK_(filter_backward(&f, NULL, 1, ws, ws_bytes, NULL));

  size_t rws = ramlt_rrmse_workspace_size(W, H);
  void *rw = dev_alloc(rws);
  float *map = dev_alloc(sizeof(float) * P);
  double *err = dev_alloc(sizeof(double));
  RAMLT_OK_(rrmse(f.out, f.reference, W, H, 1e-2, map, err, rw, rws, NULL));
  HIP_OK(hipDeviceSynchronize());

  download("out_grid_lambda.f64", grid.lambda, sizeof(double) * (size_t)m);
  download("out_grid_lambda.f32", grid.lambda_f32, sizeof(float) * (size_t)m);
  download("out_grid_updates.i32", grid.updates, sizeof(int32_t) * (size_t)m);
  download("out_mean.f32", f.mean, sizeof(float) * 3 * P);
  download("out_var.f32", f.var, sizeof(float) * 3 * P);
  download("out_tau.f32", f.tau, sizeof(float) * 3 * P);
  if (KL > 0) download("out_lag_corr.f32", f.lag_corr, sizeof(float) * 3 * (size_t)KL * P);
  download("out_feat_mean.f32", f.feat_mean, sizeof(float) * 7 * P);
  download("out_feat_var.f32", f.feat_var, sizeof(float) * 7 * P);
  download("out_out.f32", f.out, sizeof(float) * 3 * P);
  download("out_loss.f64", f.loss, sizeof(double));
  download("out_grad_radiance.f32", f.grad_radiance, sizeof(float) * 3 * P);
  download("out_grad_lambda.f32", f.grad_lambda, sizeof(float) * (size_t)m);
  download("out_map.f32", map, sizeof(float) * P);
  download("out_rrmse.f64", err, sizeof(double));

  /* quadtree: grow one tree from counted lookups while its leaves adapt, then perturb */
  ramlt_quadtree t;
  t.n_roots = 1;
  t.capacity = capacity;
  t.child = dev_alloc(sizeof(int32_t) * (size_t)capacity);
  t.depth = dev_alloc(sizeof(int32_t) * (size_t)capacity);
  t.visits = dev_alloc(sizeof(int32_t) * (size_t)capacity);
  t.n_nodes = dev_alloc(sizeof(int32_t));
  ramlt_region_state leaves = new_state(capacity);
  float *px = upload("px.f32", sizeof(float) * (size_t)n_pts);
  float *py = upload("py.f32", sizeof(float) * (size_t)n_pts);
  float *qalpha = upload("qalpha.f32", sizeof(float) * (size_t)n_pts);
  int32_t *leaf0 = dev_alloc(sizeof(int32_t) * (size_t)n_pts);
  int32_t *leaf1 = dev_alloc(sizeof(int32_t) * (size_t)n_pts);
  size_t qws = ramlt_quadtree_workspace_size(capacity);
  void *qw = dev_alloc(qws);
  RAMLT_OK_(quadtree_init(&t, NULL));
  for (int32_t i = 0; i < rounds; ++i) {
    RAMLT_OK_(quadtree_lookup(&t, NULL, px, py, leaf0, n_pts, 1, NULL));
    adapt(&leaves, capacity, leaf0, qalpha, n_pts);
    RAMLT_OK_(quadtree_refine(&t, m_split, &leaves, qw, qws, NULL));
  }
  RAMLT_OK_(quadtree_lookup(&t, NULL, px, py, leaf1, n_pts, 1, NULL));
  HIP_OK(hipDeviceSynchronize());

  float *omega = upload("omega.f32", sizeof(float) * 3 * (size_t)n_pts);
  float *uv = upload("uv.f32", sizeof(float) * 2 * (size_t)n_pts);
  float *omega_out = dev_alloc(sizeof(float) * 3 * (size_t)n_pts);
  float *theta = dev_alloc(sizeof(float) * (size_t)n_pts);
  size_t pws = ramlt_perturb_workspace_size(capacity);
  void *pw = dev_alloc(pws);
  RAMLT_OK_(perturb_directions(leaves.lambda, capacity, leaf1, omega, uv, omega_out, theta, n_pts, pw, pws, NULL));
  HIP_OK(hipDeviceSynchronize());

  int32_t nn = 0;
  HIP_OK(hipMemcpy(&nn, t.n_nodes, sizeof nn, hipMemcpyDeviceToHost));
  if (nn < 1 || nn > capacity) {
    fprintf(stderr, "node count %d outside [1, %d]\n", nn, capacity);
    return 4;
  }
  download("out_n_nodes.i32", t.n_nodes, sizeof(int32_t));
  download("out_child.i32", t.child, sizeof(int32_t) * (size_t)nn);
  download("out_depth.i32", t.depth, sizeof(int32_t) * (size_t)nn);
  download("out_visits.i32", t.visits, sizeof(int32_t) * (size_t)nn);
  download("out_leaf0.i32", leaf0, sizeof(int32_t) * (size_t)n_pts);
  download("out_leaf1.i32", leaf1, sizeof(int32_t) * (size_t)n_pts);
  download("out_leaf_lambda.f64", leaves.lambda, sizeof(double) * (size_t)nn);
  download("out_leaf_updates.i32", leaves.updates, sizeof(int32_t) * (size_t)nn);
  download("out_leaf_acc.f64", leaves.acc, sizeof(double) * (size_t)nn);
  download("out_leaf_ivisits.i32", leaves.visits, sizeof(int32_t) * (size_t)nn);
  download("out_omega.f32", omega_out, sizeof(float) * 3 * (size_t)n_pts);
  download("out_theta.f32", theta, sizeof(float) * (size_t)n_pts);

  /* lens chains on the luminance, with the screen grid's adapted lambda */
  float *lum = upload("luminance.f32", sizeof(float) * P);
  float *chains = upload("chains.f32", sizeof(float) * 3 * (size_t)n_chains);
  float *noise = upload("noise.f32", sizeof(float) * 3 * (size_t)n_chains);
  int32_t *lregion = dev_alloc(sizeof(int32_t) * (size_t)n_chains);
  float *lalpha = dev_alloc(sizeof(float) * (size_t)n_chains);
  float *lprop = dev_alloc(sizeof(float) * 3 * (size_t)n_chains);
  size_t lws = ramlt_lens_workspace_size(N);
  void *lw = dev_alloc(lws);
  RAMLT_OK_(lens_chain_step(lum, W, H, tan_half, grid.lambda, N, chains, NULL, NULL, noise, lregion, lalpha, lprop,
                            n_chains, lw, lws, NULL));
  HIP_OK(hipDeviceSynchronize());
  download("out_lens_region.i32", lregion, sizeof(int32_t) * (size_t)n_chains);
  download("out_lens_alpha.f32", lalpha, sizeof(float) * (size_t)n_chains);
  download("out_lens_prop.f32", lprop, sizeof(float) * 3 * (size_t)n_chains);
  download("out_lens_chains.f32", chains, sizeof(float) * 3 * (size_t)n_chains);
  printf("chain done: %d nodes\n", nn);
  return 0;
}
