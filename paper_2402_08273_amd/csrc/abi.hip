// C ABI of the ramlt library: host-side validation, device check, dispatch.
//
// Every argument check runs on the host before anything is enqueued, so each error
// status can be produced without a GPU. Only after validation does the library touch
// the HIP runtime (device query, launches).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "common.hpp"
#include "launch.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

#define REQUIRE_PTR(i, f, field, align)                                                        \
  do {                                                                                         \
    if ((f).field == nullptr) return fail(RAMLT_EINVAL, "frame %d: " #field " is NULL", (i));  \
    if (!aligned((f).field, (align)))                                                          \
      return fail(RAMLT_EINVAL, "frame %d: " #field " is not %d-byte aligned", (i), (int)(align)); \
  } while (0)

#define OPTIONAL_PTR(i, f, field, align)                                                       \
  do {                                                                                         \
    if ((f).field != nullptr && !aligned((f).field, (align)))                                  \
      return fail(RAMLT_EINVAL, "frame %d: " #field " is not %d-byte aligned", (i), (int)(align)); \
  } while (0)

int check_plane_layout(int i, const char *what, int W, int H, int64_t sc, int64_t ss, int64_t sy) {
  if (sc < 1 || ss < 1 || sy < W)
    return fail(RAMLT_EINVAL, "frame %d: %s strides must satisfy stride_c >= 1, stride_s >= 1, stride_y >= W",
                i, what);
  const long long extent = (long long)(H - 1) * sy + W;
  if (extent > RAMLT_MAX_PLANE_ELEMS)
    return fail(RAMLT_EUNSUPPORTED, "frame %d: %s plane extent %lld exceeds %lld elements", i, what, extent,
                (long long)RAMLT_MAX_PLANE_ELEMS);
  return RAMLT_OK;
}

int check_common(const ramlt_frame *fh, const ramlt_frame *fd, int32_t n) {
  if (fh == nullptr) return fail(RAMLT_EINVAL, "frames_host is NULL");
  if (n < 1 || n > RAMLT_MAX_FRAMES) return fail(RAMLT_EINVAL, "n_frames %d outside 1..%d", n, RAMLT_MAX_FRAMES);
  if (n > 1 && fd == nullptr) return fail(RAMLT_EINVAL, "n_frames > 1 needs the device copy frames_dev");
  if (fd != nullptr && !aligned(fd, 8)) return fail(RAMLT_EINVAL, "frames_dev is not 8-byte aligned");
  for (int i = 0; i < n; ++i) {
    const ramlt_frame &f = fh[i];
    if (f.W < 1 || f.H < 1) return fail(RAMLT_EINVAL, "frame %d: W and H must be >= 1 (got %d x %d)", i, f.W, f.H);
    if (f.W > RAMLT_MAX_SIDE || f.H > RAMLT_MAX_SIDE)
      return fail(RAMLT_EUNSUPPORTED, "frame %d: W and H must be <= %d (got %d x %d)", i, RAMLT_MAX_SIDE, f.W, f.H);
    if ((long long)f.W * f.H > RAMLT_MAX_PLANE_ELEMS)
      return fail(RAMLT_EUNSUPPORTED, "frame %d: W*H exceeds %lld", i, (long long)RAMLT_MAX_PLANE_ELEMS);
    if (f.flags & ~RAMLT_FLAGS_KNOWN) return fail(RAMLT_EINVAL, "frame %d: unknown flags 0x%x", i, (unsigned)f.flags);
  }
  return RAMLT_OK;
}

int check_filter_params(int i, const ramlt_frame &f) {
  if (f.n_regions < 1 || f.n_regions > RAMLT_MAX_REGIONS)
    return fail(RAMLT_EINVAL, "frame %d: n_regions %d outside 1..%d", i, f.n_regions, RAMLT_MAX_REGIONS);
  if (f.radius < 0 || f.radius > RAMLT_MAX_RADIUS)
    return fail(RAMLT_EINVAL, "frame %d: radius %d outside 0..%d", i, f.radius, RAMLT_MAX_RADIUS);
  if (!std::isfinite(f.lambda_min)) return fail(RAMLT_EINVAL, "frame %d: lambda_min is not finite", i);
  REQUIRE_PTR(i, f, lambda, 4);
  return RAMLT_OK;
}

int validate_stats(const ramlt_frame &f, int i) {
  if (f.S < 1) return fail(RAMLT_EINVAL, "frame %d: S must be >= 1 (got %d)", i, f.S);
  if (f.max_lag < 0 || f.max_lag > RAMLT_MAX_LAG)
    return fail(RAMLT_EINVAL, "frame %d: max_lag %d outside 0..%d", i, f.max_lag, RAMLT_MAX_LAG);
  REQUIRE_PTR(i, f, radiance, 4);
  int r = check_plane_layout(i, "radiance", f.W, f.H, f.rad_stride_c, f.rad_stride_s, f.rad_stride_y);
  if (r) return r;
  REQUIRE_PTR(i, f, mean, 4);
  REQUIRE_PTR(i, f, var, 4);
  REQUIRE_PTR(i, f, tau, 4);
  OPTIONAL_PTR(i, f, lag_corr, 4);
  if (f.features != nullptr) {
    if (f.feat_dtype != RAMLT_F32 && f.feat_dtype != RAMLT_F16)
      return fail(RAMLT_EUNSUPPORTED, "frame %d: feat_dtype %d is not RAMLT_F32 or RAMLT_F16", i, f.feat_dtype);
    if (!aligned(f.features, f.feat_dtype == RAMLT_F16 ? 2 : 4))
      return fail(RAMLT_EINVAL, "frame %d: features pointer misaligned for its dtype", i);
    r = check_plane_layout(i, "features", f.W, f.H, f.feat_stride_c, f.feat_stride_s, f.feat_stride_y);
    if (r) return r;
    REQUIRE_PTR(i, f, feat_mean, 4);
    REQUIRE_PTR(i, f, feat_var, 4);
  }
  return RAMLT_OK;
}

int validate_forward(const ramlt_frame &f, int i) {
  int r = check_filter_params(i, f);
  if (r) return r;
  REQUIRE_PTR(i, f, mean, 4);
  REQUIRE_PTR(i, f, out, 4);
  if (f.flags & RAMLT_LOSS_IN_FORWARD) {  // the MSE seed and dL/dlambda in the same pass
    REQUIRE_PTR(i, f, reference, 4);
    REQUIRE_PTR(i, f, grad_out, 4);
    OPTIONAL_PTR(i, f, loss, 8);
    OPTIONAL_PTR(i, f, grad_lambda, 4);
  }
  return RAMLT_OK;
}

int validate_loss(const ramlt_frame &f, int i) {
  REQUIRE_PTR(i, f, out, 4);
  REQUIRE_PTR(i, f, reference, 4);
  REQUIRE_PTR(i, f, grad_out, 4);
  OPTIONAL_PTR(i, f, loss, 8);
  return RAMLT_OK;
}

int validate_backward(const ramlt_frame &f, int i) {
  if (f.S < 1) return fail(RAMLT_EINVAL, "frame %d: S must be >= 1 (got %d)", i, f.S);
  int r = check_filter_params(i, f);
  if (r) return r;
  if (f.flags & RAMLT_LOSS_IN_FORWARD) {  // grad_radiance only, from grad_out
    REQUIRE_PTR(i, f, grad_out, 4);
    REQUIRE_PTR(i, f, grad_radiance, 4);
    return RAMLT_OK;
  }
  if (f.grad_out == nullptr && f.reference == nullptr)
    return fail(RAMLT_EINVAL, "frame %d: filter_backward needs grad_out, or reference for the fused MSE seed", i);
  OPTIONAL_PTR(i, f, grad_out, 4);
  if (f.grad_out == nullptr) {
    REQUIRE_PTR(i, f, reference, 4);
    OPTIONAL_PTR(i, f, loss, 8);
  }
  REQUIRE_PTR(i, f, mean, 4);
  REQUIRE_PTR(i, f, out, 4);
  REQUIRE_PTR(i, f, grad_radiance, 4);
  OPTIONAL_PTR(i, f, grad_lambda, 4);
  return RAMLT_OK;
}

// gfx950 check, once per device.
constexpr int kMaxDevices = 64;
std::once_flag g_dev_once[kMaxDevices];
int g_dev_status[kMaxDevices];
char g_dev_arch[kMaxDevices][64];

int check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(RAMLT_EUNSUPPORTED, "device index %d out of range", dev);
  std::call_once(g_dev_once[dev], [dev] {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      g_dev_status[dev] = RAMLT_EHIP;
      std::snprintf(g_dev_arch[dev], sizeof(g_dev_arch[dev]), "unknown");
      return;
    }
    std::snprintf(g_dev_arch[dev], sizeof(g_dev_arch[dev]), "%s", prop.gcnArchName);
    g_dev_status[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? RAMLT_OK : RAMLT_EUNSUPPORTED;
  });
  if (g_dev_status[dev] == RAMLT_EHIP) return fail(RAMLT_EHIP, "hipGetDeviceProperties failed on device %d", dev);
  if (g_dev_status[dev] != RAMLT_OK)
    return fail(RAMLT_EUNSUPPORTED, "device %d is %s; this library is built for gfx950 only", dev, g_dev_arch[dev]);
  return RAMLT_OK;
}

typedef int (*Validator)(const ramlt_frame &, int);
typedef hipError_t (*Launcher)(const ramlt_frame *, const ramlt_frame *, int, void *, hipStream_t);

int run_op(int op, const char *name, Validator v, Launcher l, const ramlt_frame *fh, const ramlt_frame *fd,
           int32_t n, void *ws, size_t ws_bytes, void *stream) {
  int r = check_common(fh, fd, n);
  if (r) return r;
  for (int i = 0; i < n; ++i) {
    r = v(fh[i], i);
    if (r) return r;
  }
  const size_t need = ramlt::workspace_bytes(fh, n, op);
  if (need > 0) {
    if (ws == nullptr || ws_bytes < need)
      return fail(RAMLT_EWORKSPACE, "%s needs %zu bytes of workspace, got %zu", name, need,
                  ws == nullptr ? (size_t)0 : ws_bytes);
    if (!aligned(ws, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
  }
  r = check_device();
  if (r) return r;
  const hipError_t e = l(fh, fd, n, ws, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "%s: %s", name, hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// A device buffer of an entry point: its address and byte length (0 = absent).
struct Span {
  const void *p;
  size_t bytes;
};

// True if a written buffer overlaps another written buffer or a read one (the kernels of the
// entry point write some buffers at other elements' places while they read the rest).
bool writes_overlap(const Span *wr, int nwr, const Span *rd, int nrd) {
  for (int a = 0; a < nwr; ++a) {
    if (!wr[a].bytes) continue;
    for (int b = 0; b < nrd; ++b)
      if (rd[b].bytes && overlap(wr[a].p, wr[a].bytes, rd[b].p, rd[b].bytes)) return true;
    for (int b = a + 1; b < nwr; ++b)
      if (wr[b].bytes && overlap(wr[a].p, wr[a].bytes, wr[b].p, wr[b].bytes)) return true;
  }
  return false;
}

int validate_adapt(const ramlt_adapt_params *p, const ramlt_region_state *s, const int32_t *region,
                   const float *alpha, int64_t n) {
  if (!p) return fail(RAMLT_EINVAL, "region_adapt: params is NULL");
  if (!s) return fail(RAMLT_EINVAL, "region_adapt: state is NULL");
  if (p->n_regions < 1 || p->n_regions > RAMLT_MAX_ADAPT_REGIONS)
    return fail(RAMLT_EINVAL, "region_adapt: n_regions %d outside 1..%d", p->n_regions, RAMLT_MAX_ADAPT_REGIONS);
  if (p->L < 1 || p->L > RAMLT_MAX_ADAPT_L)
    return fail(RAMLT_EINVAL, "region_adapt: L %d outside 1..%d", p->L, RAMLT_MAX_ADAPT_L);
  if (!std::isfinite(p->gamma_max) || !std::isfinite(p->gamma_scale) || !std::isfinite(p->alpha_target) ||
      !std::isfinite(p->lambda_min))
    return fail(RAMLT_EINVAL, "region_adapt: gamma_max, gamma_scale, alpha_target, lambda_min must be finite");
  if (n < 0 || n > RAMLT_MAX_PROPOSALS)
    return fail(RAMLT_EINVAL, "region_adapt: n_proposals %lld outside 0..%lld", (long long)n,
                (long long)RAMLT_MAX_PROPOSALS);
  if (!s->lambda || !aligned(s->lambda, 8) || !s->acc || !aligned(s->acc, 8))
    return fail(RAMLT_EINVAL, "region_adapt: state.lambda and state.acc must be 8-byte aligned device pointers");
  if (!s->visits || !aligned(s->visits, 4) || !s->updates || !aligned(s->updates, 4))
    return fail(RAMLT_EINVAL, "region_adapt: state.visits and state.updates must be 4-byte aligned device pointers");
  if (s->lambda_f32 && !aligned(s->lambda_f32, 4))
    return fail(RAMLT_EINVAL, "region_adapt: state.lambda_f32 must be 4-byte aligned");
  if (n > 0 && (!region || !aligned(region, 4) || !alpha || !aligned(alpha, 4)))
    return fail(RAMLT_EINVAL, "region_adapt: region and alpha must be 4-byte aligned device pointers");
  return RAMLT_OK;
}

int validate_tree(const char *fn, const ramlt_quadtree *t) {
  if (!t) return fail(RAMLT_EINVAL, "%s: tree is NULL", fn);
  if (t->capacity < 1 || t->capacity > RAMLT_MAX_QT_NODES)
    return fail(RAMLT_EINVAL, "%s: capacity %d outside 1..%d", fn, t->capacity, RAMLT_MAX_QT_NODES);
  if (t->n_roots < 1 || t->n_roots > t->capacity)
    return fail(RAMLT_EINVAL, "%s: n_roots %d outside 1..capacity (%d)", fn, t->n_roots, t->capacity);
  if (!t->child || !aligned(t->child, 4) || !t->depth || !aligned(t->depth, 4) || !t->visits ||
      !aligned(t->visits, 4) || !t->n_nodes || !aligned(t->n_nodes, 4))
    return fail(RAMLT_EINVAL, "%s: child, depth, visits and n_nodes must be 4-byte aligned device pointers", fn);
  return RAMLT_OK;
}

}  // namespace

extern "C" {

int quadtree_init(const ramlt_quadtree *tree, void *stream) {
  int r = validate_tree("quadtree_init", tree);
  if (r) return r;
  r = check_device();
  if (r) return r;
  const hipError_t e = ramlt::launch_quadtree_init(*tree, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "quadtree_init: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

int quadtree_lookup(const ramlt_quadtree *tree, const int32_t *root, const float *x, const float *y,
                    int32_t *leaf, int64_t n_points, int32_t count, void *stream) {
  int r = validate_tree("quadtree_lookup", tree);
  if (r) return r;
  if (n_points < 0 || n_points > RAMLT_MAX_QT_POINTS)
    return fail(RAMLT_EINVAL, "quadtree_lookup: n_points %lld outside 0..%lld", (long long)n_points,
                (long long)RAMLT_MAX_QT_POINTS);
  if (n_points > 0 && (!x || !aligned(x, 4) || !y || !aligned(y, 4) || !leaf || !aligned(leaf, 4)))
    return fail(RAMLT_EINVAL, "quadtree_lookup: x, y and leaf must be 4-byte aligned device pointers");
  if (root && !aligned(root, 4)) return fail(RAMLT_EINVAL, "quadtree_lookup: root is not 4-byte aligned");
  if (n_points > 0) {
    // leaf is written, and the tree's visit counts with count, while the points and the
    // tree's links are read
    const size_t np = (size_t)n_points, c = (size_t)tree->capacity;
    const Span rd[6] = {{x, np * 4},           {y, np * 4},           {root, root ? np * 4 : 0},
                        {tree->child, c * 4},  {tree->depth, c * 4},  {tree->n_nodes, 4}};
    const Span wr[2] = {{leaf, np * 4}, {tree->visits, count ? c * 4 : 0}};
    if (writes_overlap(wr, 2, rd, 6))
      return fail(RAMLT_EINVAL, "quadtree_lookup: leaf (and the visit counts when counting) must not overlap each "
                                "other, the points or the tree's links");
  }
  r = check_device();
  if (r) return r;
  const hipError_t e =
      ramlt::launch_quadtree_lookup(*tree, root, x, y, leaf, n_points, count != 0, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "quadtree_lookup: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

int quadtree_refine(const ramlt_quadtree *tree, int32_t m_split, const ramlt_region_state *state, void *workspace,
                    size_t ws_bytes, void *stream) {
  int r = validate_tree("quadtree_refine", tree);
  if (r) return r;
  if (m_split < 0) return fail(RAMLT_EINVAL, "quadtree_refine: m_split %d is negative", m_split);
  if (state) {
    if (!state->lambda || !aligned(state->lambda, 8) || !state->acc || !aligned(state->acc, 8))
      return fail(RAMLT_EINVAL, "quadtree_refine: state.lambda and state.acc must be 8-byte aligned device pointers");
    if (!state->visits || !aligned(state->visits, 4) || !state->updates || !aligned(state->updates, 4))
      return fail(RAMLT_EINVAL,
                  "quadtree_refine: state.visits and state.updates must be 4-byte aligned device pointers");
    if (state->lambda_f32 && !aligned(state->lambda_f32, 4))
      return fail(RAMLT_EINVAL, "quadtree_refine: state.lambda_f32 must be 4-byte aligned");
  }
  const size_t need = ramlt::quadtree_workspace_bytes(tree->capacity);
  if (workspace == nullptr || ws_bytes < need)
    return fail(RAMLT_EWORKSPACE, "quadtree_refine needs %zu bytes of workspace, got %zu", need,
                workspace == nullptr ? (size_t)0 : ws_bytes);
  if (!aligned(workspace, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
  {
    // children are written past the nodes in use while the parents are read, and the state of
    // every child from its parent's: all of these buffers are written
    const size_t c = (size_t)tree->capacity;
    const Span wr[10] = {{tree->child, c * 4},
                         {tree->depth, c * 4},
                         {tree->visits, c * 4},
                         {tree->n_nodes, 4},
                         {workspace, need},
                         {state ? state->lambda : nullptr, state ? c * 8 : 0},
                         {state ? state->acc : nullptr, state ? c * 8 : 0},
                         {state ? state->visits : nullptr, state ? c * 4 : 0},
                         {state ? state->updates : nullptr, state ? c * 4 : 0},
                         {state ? state->lambda_f32 : nullptr, state && state->lambda_f32 ? c * 4 : 0}};
    if (writes_overlap(wr, 10, nullptr, 0))
      return fail(RAMLT_EINVAL, "quadtree_refine: the tree's arrays, the state's first capacity entries and the "
                                "workspace must not overlap");
  }
  r = check_device();
  if (r) return r;
  const hipError_t e = ramlt::launch_quadtree_refine(*tree, m_split, state, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "quadtree_refine: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

int perturb_directions(const double *lambda, int32_t n_regions, const int32_t *region, const float *omega,
                       const float *uv, float *omega_out, float *theta_out, int64_t n, void *workspace,
                       size_t ws_bytes, void *stream) {
  if (n_regions < 1 || n_regions > RAMLT_MAX_ADAPT_REGIONS)
    return fail(RAMLT_EINVAL, "perturb_directions: n_regions %d outside 1..%d", n_regions,
                RAMLT_MAX_ADAPT_REGIONS);
  if (!lambda || !aligned(lambda, 8))
    return fail(RAMLT_EINVAL, "perturb_directions: lambda must be an 8-byte aligned device pointer");
  if (n < 0 || n > RAMLT_MAX_PROPOSALS)
    return fail(RAMLT_EINVAL, "perturb_directions: n %lld outside 0..%lld", (long long)n,
                (long long)RAMLT_MAX_PROPOSALS);
  if (n > 0) {
    if (!region || !aligned(region, 4) || !omega || !aligned(omega, 4) || !omega_out || !aligned(omega_out, 4))
      return fail(RAMLT_EINVAL, "perturb_directions: region, omega and omega_out must be 4-byte aligned device "
                                "pointers");
    if (!uv || !aligned(uv, 8))
      return fail(RAMLT_EINVAL, "perturb_directions: uv must be an 8-byte aligned device pointer");
    if (theta_out && !aligned(theta_out, 4))
      return fail(RAMLT_EINVAL, "perturb_directions: theta_out is not 4-byte aligned");
    const size_t need = ramlt::perturb_workspace_bytes(n_regions);
    if (need > 0) {
      if (workspace == nullptr || ws_bytes < need)
        return fail(RAMLT_EWORKSPACE, "perturb_directions needs %zu bytes of workspace, got %zu", need,
                    workspace == nullptr ? (size_t)0 : ws_bytes);
      if (!aligned(workspace, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
    }
    // the sigma table is written before the proposals read it, and each proposal's outputs
    // while the others read their inputs: omega_out may be omega itself (a proposal reads its
    // direction before it writes the new one), nothing else may overlap
    const size_t m = (size_t)n_regions, nn = (size_t)n;
    const bool in_place = (const void *)omega_out == (const void *)omega;
    const Span rd[4] = {{lambda, m * 8}, {region, nn * 4}, {omega, in_place ? 0 : nn * 12}, {uv, nn * 8}};
    const Span wr[3] = {{omega_out, nn * 12}, {theta_out, theta_out ? nn * 4 : 0}, {workspace, need}};
    if (writes_overlap(wr, 3, rd, 4))
      return fail(RAMLT_EINVAL, "perturb_directions: omega_out, theta_out and the workspace must not overlap each "
                                "other or the inputs (omega_out may be omega itself)");
  }
  int r = check_device();
  if (r) return r;
  const hipError_t e = ramlt::launch_perturb(lambda, n_regions, region, omega, uv, omega_out, theta_out, n, workspace,
                                             (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "perturb_directions: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

int lens_chain_step(const float *luminance, int32_t W, int32_t H, float tan_half_fov_x, const double *lambda,
                    int32_t n_regions, float *omega, float *density, int32_t *pixel, const float *noise,
                    int32_t *region, float *alpha, float *omega_prop, int64_t n, void *workspace, size_t ws_bytes,
                    void *stream) {
  if (W < 1 || H < 1 || W > RAMLT_MAX_SIDE || H > RAMLT_MAX_SIDE || (long long)W * H > RAMLT_MAX_PLANE_ELEMS)
    return fail(RAMLT_EINVAL, "lens_chain_step: image size %d x %d out of range", W, H);
  if (!std::isfinite(tan_half_fov_x) || !(tan_half_fov_x > 0.0f))
    return fail(RAMLT_EINVAL, "lens_chain_step: tan_half_fov_x must be finite and > 0");
  const float ty = (float)((double)tan_half_fov_x * H / W);
  if (!(ty > 0.0f) || !std::isfinite(ty))
    return fail(RAMLT_EINVAL, "lens_chain_step: tan_half_fov_x * H / W is not a positive float");
  if (n_regions < 1 || n_regions > RAMLT_MAX_REGIONS)
    return fail(RAMLT_EINVAL, "lens_chain_step: n_regions %d outside 1..%d", n_regions, RAMLT_MAX_REGIONS);
  if (!luminance || !aligned(luminance, 4))
    return fail(RAMLT_EINVAL, "lens_chain_step: luminance must be a 4-byte aligned device pointer");
  if (!lambda || !aligned(lambda, 8))
    return fail(RAMLT_EINVAL, "lens_chain_step: lambda must be an 8-byte aligned device pointer");
  if (n < 0 || n > RAMLT_MAX_PROPOSALS)
    return fail(RAMLT_EINVAL, "lens_chain_step: n %lld outside 0..%lld", (long long)n,
                (long long)RAMLT_MAX_PROPOSALS);
  if (n > 0) {
    if (!omega || !aligned(omega, 4) || !noise || !aligned(noise, 4) || !region || !aligned(region, 4) || !alpha ||
        !aligned(alpha, 4))
      return fail(RAMLT_EINVAL, "lens_chain_step: omega, noise, region and alpha must be 4-byte aligned device "
                                "pointers");
    if (omega_prop && !aligned(omega_prop, 4))
      return fail(RAMLT_EINVAL, "lens_chain_step: omega_prop is not 4-byte aligned");
    if (density && !aligned(density, 4))
      return fail(RAMLT_EINVAL, "lens_chain_step: density is not 4-byte aligned");
    if (pixel && !aligned(pixel, 4)) return fail(RAMLT_EINVAL, "lens_chain_step: pixel is not 4-byte aligned");
    const size_t need = ramlt::perturb_workspace_bytes(n_regions * n_regions);
    if (need > 0) {
      if (workspace == nullptr || ws_bytes < need)
        return fail(RAMLT_EWORKSPACE, "lens_chain_step needs %zu bytes of workspace, got %zu", need,
                    workspace == nullptr ? (size_t)0 : ws_bytes);
      if (!aligned(workspace, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
    }
    // the sigma table is written before the chains read it, and each chain's state and
    // outputs while the others read theirs: every written buffer stands alone
    const size_t nn = (size_t)n, m = (size_t)n_regions * (size_t)n_regions, P = (size_t)W * (size_t)H;
    const Span rd[3] = {{luminance, P * 4}, {lambda, m * 8}, {noise, nn * 12}};
    const Span wr[7] = {{omega, nn * 12},      {density, density ? nn * 4 : 0}, {pixel, pixel ? nn * 4 : 0},
                        {region, nn * 4},      {alpha, nn * 4},                 {omega_prop, omega_prop ? nn * 12 : 0},
                        {workspace, need}};
    if (writes_overlap(wr, 7, rd, 3))
      return fail(RAMLT_EINVAL, "lens_chain_step: the chains' state, the outputs and the workspace must not overlap "
                                "each other or the inputs");
  }
  int r = check_device();
  if (r) return r;
  const hipError_t e = ramlt::launch_lens_step(luminance, W, H, tan_half_fov_x, ty, lambda, n_regions, omega, density,
                                               pixel, noise, region, alpha, omega_prop, n, workspace,
                                               (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "lens_chain_step: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

size_t ramlt_lens_workspace_size(int32_t n_regions) {
  if (n_regions < 1 || n_regions > RAMLT_MAX_REGIONS) return 0;
  return ramlt::perturb_workspace_bytes(n_regions * n_regions);
}

int lens_chain_sort(int32_t W, int32_t H, float tan_half_fov_x, const float *omega, const float *density, int64_t n,
                    float *omega_out, float *density_out, int32_t *perm, void *workspace, size_t ws_bytes,
                    void *stream) {
  if (W < 1 || H < 1 || W > RAMLT_MAX_SIDE || H > RAMLT_MAX_SIDE || (long long)W * H > RAMLT_MAX_PLANE_ELEMS)
    return fail(RAMLT_EINVAL, "lens_chain_sort: image size %d x %d out of range", W, H);
  if (!std::isfinite(tan_half_fov_x) || !(tan_half_fov_x > 0.0f))
    return fail(RAMLT_EINVAL, "lens_chain_sort: tan_half_fov_x must be finite and > 0");
  const float ty = (float)((double)tan_half_fov_x * H / W);
  if (!(ty > 0.0f) || !std::isfinite(ty))
    return fail(RAMLT_EINVAL, "lens_chain_sort: tan_half_fov_x * H / W is not a positive float");
  if (n < 0 || n > RAMLT_MAX_PROPOSALS)
    return fail(RAMLT_EINVAL, "lens_chain_sort: n %lld outside 0..%lld", (long long)n,
                (long long)RAMLT_MAX_PROPOSALS);
  if (n > 0) {
    if (!omega || !aligned(omega, 4) || !omega_out || !aligned(omega_out, 4))
      return fail(RAMLT_EINVAL, "lens_chain_sort: omega and omega_out must be 4-byte aligned device pointers");
    if ((density == nullptr) != (density_out == nullptr))
      return fail(RAMLT_EINVAL, "lens_chain_sort: density and density_out go together");
    if (density && (!aligned(density, 4) || !aligned(density_out, 4)))
      return fail(RAMLT_EINVAL, "lens_chain_sort: density and density_out must be 4-byte aligned");
    if (perm && !aligned(perm, 4)) return fail(RAMLT_EINVAL, "lens_chain_sort: perm is not 4-byte aligned");
    const size_t n3 = (size_t)n * 3 * sizeof(float), n1 = (size_t)n * sizeof(float);
    const size_t need = ramlt::lens_sort_workspace_bytes(n);
    if (workspace == nullptr || ws_bytes < need)
      return fail(RAMLT_EWORKSPACE, "lens_chain_sort needs %zu bytes of workspace, got %zu", need,
                  workspace == nullptr ? (size_t)0 : ws_bytes);
    if (!aligned(workspace, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
    // the outputs are written at other chains' places while the inputs are read, and the
    // workspace's counters while both are in use
    const Span in[2] = {{omega, n3}, {density, density ? n1 : 0}};
    const Span out[4] = {{omega_out, n3}, {density_out, density_out ? n1 : 0}, {perm, perm ? n1 : 0},
                         {workspace, need}};
    if (writes_overlap(out, 4, in, 2))
      return fail(RAMLT_EINVAL, "lens_chain_sort: outputs and workspace must not overlap the inputs or each other");
  }
  int r = check_device();
  if (r) return r;
  const hipError_t e = ramlt::launch_lens_sort(W, H, tan_half_fov_x, ty, omega, density, n, omega_out, density_out,
                                               perm, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "lens_chain_sort: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

size_t ramlt_lens_sort_workspace_size(int64_t n) {
  if (n <= 0 || n > RAMLT_MAX_PROPOSALS) return 0;
  return ramlt::lens_sort_workspace_bytes(n);
}

int rrmse(const float *image, const float *reference, int32_t W, int32_t H, double eps, float *map,
          double *rrmse_out, void *workspace, size_t ws_bytes, void *stream) {
  if (W < 1 || H < 1 || W > RAMLT_MAX_SIDE || H > RAMLT_MAX_SIDE || (long long)W * H > RAMLT_MAX_PLANE_ELEMS)
    return fail(RAMLT_EINVAL, "rrmse: image size %d x %d out of range", W, H);
  if (!std::isfinite(eps) || eps < 0) return fail(RAMLT_EINVAL, "rrmse: eps must be finite and >= 0");
  if (!image || !aligned(image, 4) || !reference || !aligned(reference, 4))
    return fail(RAMLT_EINVAL, "rrmse: image and reference must be 4-byte aligned device pointers");
  if (!map && !rrmse_out) return fail(RAMLT_EINVAL, "rrmse: map and rrmse_out are both NULL");
  if (map && !aligned(map, 4)) return fail(RAMLT_EINVAL, "rrmse: map is not 4-byte aligned");
  if (rrmse_out && !aligned(rrmse_out, 8)) return fail(RAMLT_EINVAL, "rrmse: rrmse_out is not 8-byte aligned");
  const size_t need = ramlt::rrmse_workspace_bytes((long long)W * H);
  if (workspace == nullptr || ws_bytes < need)
    return fail(RAMLT_EWORKSPACE, "rrmse needs %zu bytes of workspace, got %zu", need,
                workspace == nullptr ? (size_t)0 : ws_bytes);
  if (!aligned(workspace, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
  {
    const size_t P = (size_t)W * (size_t)H;
    const Span rd[2] = {{image, P * 12}, {reference, P * 12}};
    const Span wr[3] = {{map, map ? P * 4 : 0}, {rrmse_out, rrmse_out ? (size_t)8 : 0}, {workspace, need}};
    if (writes_overlap(wr, 3, rd, 2))
      return fail(RAMLT_EINVAL, "rrmse: map, rrmse_out and the workspace must not overlap each other or the images");
  }
  int r = check_device();
  if (r) return r;
  const hipError_t e =
      ramlt::launch_rrmse(image, reference, (long long)W * H, eps, map, rrmse_out, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "rrmse: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

size_t ramlt_rrmse_workspace_size(int32_t W, int32_t H) {
  if (W < 1 || H < 1 || W > RAMLT_MAX_SIDE || H > RAMLT_MAX_SIDE || (long long)W * H > RAMLT_MAX_PLANE_ELEMS)
    return 0;
  return ramlt::rrmse_workspace_bytes((long long)W * H);
}

size_t ramlt_perturb_workspace_size(int32_t n_regions) {
  if (n_regions < 1 || n_regions > RAMLT_MAX_ADAPT_REGIONS) return 0;
  return ramlt::perturb_workspace_bytes(n_regions);
}

size_t ramlt_quadtree_workspace_size(int32_t capacity) {
  if (capacity < 1 || capacity > RAMLT_MAX_QT_NODES) return 0;
  return ramlt::quadtree_workspace_bytes(capacity);
}

int region_adapt(const ramlt_adapt_params *params, const ramlt_region_state *state, const int32_t *region,
                 const float *alpha, int64_t n_proposals, void *workspace, size_t ws_bytes, void *stream) {
  int r = validate_adapt(params, state, region, alpha, n_proposals);
  if (r) return r;
  const size_t need = ramlt::adapt_workspace_bytes(n_proposals, params->n_regions);
  if (need > 0) {
    if (workspace == nullptr || ws_bytes < need)
      return fail(RAMLT_EWORKSPACE, "region_adapt needs %zu bytes of workspace, got %zu", need,
                  workspace == nullptr ? (size_t)0 : ws_bytes);
    if (!aligned(workspace, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
  }
  {
    // the sorted stream is written to the workspace while the proposals are read, and the state
    // is updated in place
    const size_t m = (size_t)params->n_regions, np = (size_t)(n_proposals > 0 ? n_proposals : 0);
    const Span rd[2] = {{region, np * 4}, {alpha, np * 4}};
    const Span wr[6] = {{state->lambda, m * 8},  {state->acc, m * 8},
                        {state->visits, m * 4},  {state->updates, m * 4},
                        {state->lambda_f32, state->lambda_f32 ? m * 4 : 0}, {workspace, need}};
    if (writes_overlap(wr, 6, rd, 2))
      return fail(RAMLT_EINVAL, "region_adapt: the state arrays and the workspace must not overlap each other or "
                                "the proposals");
  }
  r = check_device();
  if (r) return r;
  const hipError_t e = ramlt::launch_region_adapt(*params, *state, region, alpha, n_proposals, workspace,
                                                  (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "region_adapt: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

size_t ramlt_adapt_workspace_size(int64_t n_proposals, int32_t n_regions) {
  if (n_proposals <= 0 || n_proposals > RAMLT_MAX_PROPOSALS || n_regions < 1 ||
      n_regions > RAMLT_MAX_ADAPT_REGIONS)
    return 0;
  return ramlt::adapt_workspace_bytes(n_proposals, n_regions);
}

int stats_accumulate(const ramlt_frame *frames_host, const ramlt_frame *frames_dev, int32_t n_frames,
                     void *workspace, size_t ws_bytes, void *stream) {
  return run_op(RAMLT_OP_STATS, "stats_accumulate", validate_stats, ramlt::launch_stats, frames_host, frames_dev,
                n_frames, workspace, ws_bytes, stream);
}

int filter_forward(const ramlt_frame *frames_host, const ramlt_frame *frames_dev, int32_t n_frames,
                   void *workspace, size_t ws_bytes, void *stream) {
  return run_op(RAMLT_OP_FILTER_FORWARD, "filter_forward", validate_forward, ramlt::launch_filter_forward,
                frames_host, frames_dev, n_frames, workspace, ws_bytes, stream);
}

int loss_seed(const ramlt_frame *frames_host, const ramlt_frame *frames_dev, int32_t n_frames, void *workspace,
              size_t ws_bytes, void *stream) {
  return run_op(RAMLT_OP_LOSS_SEED, "loss_seed", validate_loss, ramlt::launch_loss_seed, frames_host, frames_dev,
                n_frames, workspace, ws_bytes, stream);
}

int filter_backward(const ramlt_frame *frames_host, const ramlt_frame *frames_dev, int32_t n_frames,
                    void *workspace, size_t ws_bytes, void *stream) {
  return run_op(RAMLT_OP_FILTER_BACKWARD, "filter_backward", validate_backward, ramlt::launch_filter_backward,
                frames_host, frames_dev, n_frames, workspace, ws_bytes, stream);
}

int stats_filter_step(const ramlt_frame *frame, void *workspace, size_t ws_bytes, void *stream) {
  int r = check_common(frame, nullptr, 1);
  if (r) return r;
  if (!(frame->flags & RAMLT_LOSS_IN_FORWARD))
    return fail(RAMLT_EINVAL, "stats_filter_step: the frame's flags must include RAMLT_LOSS_IN_FORWARD");
  if ((r = validate_stats(*frame, 0)) || (r = validate_forward(*frame, 0)) || (r = validate_backward(*frame, 0)))
    return r;
  const size_t need = ramlt::workspace_bytes(frame, 1, RAMLT_OP_FILTER_FORWARD);
  if (workspace == nullptr || ws_bytes < need)
    return fail(RAMLT_EWORKSPACE, "stats_filter_step needs %zu bytes of workspace, got %zu", need,
                workspace == nullptr ? (size_t)0 : ws_bytes);
  if (!aligned(workspace, 256)) return fail(RAMLT_EWORKSPACE, "workspace must be 256-byte aligned");
  r = check_device();
  if (r) return r;
  const hipError_t e = ramlt::launch_step(*frame, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "stats_filter_step: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

int filter_backward_noalloc(const ramlt_frame *frames_host, const ramlt_frame *frames_dev, int32_t n_frames,
                            void *stream) {
  int r = check_common(frames_host, frames_dev, n_frames);
  if (r) return r;
  for (int i = 0; i < n_frames; ++i) {
    r = validate_backward(frames_host[i], i);
    if (r) return r;
  }
  const size_t need = ramlt::workspace_bytes(frames_host, n_frames, RAMLT_OP_FILTER_BACKWARD);
  if (need > ramlt::kNoallocWorkspaceBytes)
    return fail(RAMLT_EWORKSPACE, "filter_backward_noalloc needs %zu bytes of workspace; the library's own holds %zu",
                need, (size_t)ramlt::kNoallocWorkspaceBytes);
  r = check_device();
  if (r) return r;
  void *ws = nullptr;
  hipError_t e = ramlt::noalloc_workspace(&ws);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "filter_backward_noalloc: workspace address: %s", hipGetErrorString(e));
  e = ramlt::launch_filter_backward(frames_host, frames_dev, n_frames, ws, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAMLT_EHIP, "filter_backward_noalloc: %s", hipGetErrorString(e));
  g_last_error.clear();
  return RAMLT_OK;
}

size_t ramlt_workspace_size(const ramlt_frame *frames_host, int32_t n_frames, int32_t op) {
  if (frames_host == nullptr || n_frames < 1 || n_frames > RAMLT_MAX_FRAMES) return 0;
  return ramlt::workspace_bytes(frames_host, n_frames, op);
}

const char *ramlt_last_error(void) { return g_last_error.c_str(); }

int32_t ramlt_abi_version(void) { return (int32_t)((sizeof(ramlt_frame) << 16) | 3); }

}  // extern "C"
