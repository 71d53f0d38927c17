"""ctypes binding of ``include/ramlt.h`` (argument marshalling only).

The entry points keep the C names: :func:`stats_accumulate`, :func:`filter_forward`,
:func:`loss_seed`, :func:`filter_backward`, :func:`workspace_size`, :func:`last_error`.
Each takes a sequence of :class:`RamltFrame` descriptors holding device pointers, an
optional device copy of that table, an optional workspace pointer and a stream handle,
and raises :class:`RamltError` on a non-zero status.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# RAMLT_LIBRARY names another build of the same library (the host tests load the
# AddressSanitizer build this way); the default is the in-tree libramlt.so
LIB_PATH = os.environ.get("RAMLT_LIBRARY") or os.path.join(_HERE, "libramlt.so")

RAMLT_OK = 0
RAMLT_EINVAL = 1
RAMLT_EUNSUPPORTED = 2
RAMLT_EWORKSPACE = 3
RAMLT_EHIP = 4

RAMLT_F32 = 0
RAMLT_F16 = 1

# ramlt_frame.flags: launch schedule (include/ramlt.h)
RAMLT_TILE_DEFAULT = 0
RAMLT_TILE_32X8 = 1
RAMLT_TILE_32X16 = 2
RAMLT_TILE_64X8 = 3
RAMLT_TILE_MASK = 3
RAMLT_SCHED_DIRECT = 4
RAMLT_LOSS_IN_FORWARD = 8  # the MSE seed and dL/dlambda in filter_forward; filter_backward: G only
# stats_accumulate launch size: v workgroups per compute unit per launch (1..14), one launch
# (15), or the default (0), in bits 4-7
RAMLT_STATS_WG_SHIFT = 4
RAMLT_STATS_WG_MASK = 15 << RAMLT_STATS_WG_SHIFT
RAMLT_STATS_ONE_LAUNCH = 15
TILE_SHAPES = {RAMLT_TILE_32X8: (32, 8), RAMLT_TILE_32X16: (32, 16), RAMLT_TILE_64X8: (64, 8)}

OP_STATS = 0
OP_FILTER_FORWARD = 1
OP_LOSS_SEED = 2
OP_FILTER_BACKWARD = 3

MAX_RADIUS = 15
MAX_LAG = 32
MAX_FRAMES = 4096
MAX_REGIONS = 4096

EXPORTED = (
    "stats_accumulate",
    "filter_forward",
    "loss_seed",
    "filter_backward",
    "filter_backward_noalloc",
    "stats_filter_step",
    "ramlt_workspace_size",
    "ramlt_last_error",
    "ramlt_abi_version",
    "region_adapt",
    "ramlt_adapt_workspace_size",
    "quadtree_init",
    "quadtree_lookup",
    "quadtree_refine",
    "ramlt_quadtree_workspace_size",
    "perturb_directions",
    "ramlt_perturb_workspace_size",
    "lens_chain_step",
    "ramlt_lens_workspace_size",
    "lens_chain_sort",
    "ramlt_lens_sort_workspace_size",
    "rrmse",
    "ramlt_rrmse_workspace_size",
)

MAX_ADAPT_REGIONS = 1 << 24
MAX_ADAPT_L = 1 << 20
MAX_PROPOSALS = 1 << 30
QT_MAX_DEPTH = 20
MAX_QT_NODES = 1 << 26
MAX_QT_POINTS = 1 << 30


class RamltFrame(ctypes.Structure):
    """Mirror of ``ramlt_frame``; every pointer field is a device address (int)."""

    _fields_ = [
        ("W", ctypes.c_int32),
        ("H", ctypes.c_int32),
        ("S", ctypes.c_int32),
        ("max_lag", ctypes.c_int32),
        ("radiance", ctypes.c_void_p),
        ("rad_stride_c", ctypes.c_int64),
        ("rad_stride_s", ctypes.c_int64),
        ("rad_stride_y", ctypes.c_int64),
        ("features", ctypes.c_void_p),
        ("feat_stride_c", ctypes.c_int64),
        ("feat_stride_s", ctypes.c_int64),
        ("feat_stride_y", ctypes.c_int64),
        ("feat_dtype", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("mean", ctypes.c_void_p),
        ("var", ctypes.c_void_p),
        ("tau", ctypes.c_void_p),
        ("lag_corr", ctypes.c_void_p),
        ("feat_mean", ctypes.c_void_p),
        ("feat_var", ctypes.c_void_p),
        ("lambda_", ctypes.c_void_p),
        ("n_regions", ctypes.c_int32),
        ("radius", ctypes.c_int32),
        ("lambda_min", ctypes.c_float),
        ("_reserved0", ctypes.c_int32),
        ("out", ctypes.c_void_p),
        ("reference", ctypes.c_void_p),
        ("loss", ctypes.c_void_p),
        ("grad_out", ctypes.c_void_p),
        ("grad_radiance", ctypes.c_void_p),
        ("grad_lambda", ctypes.c_void_p),
    ]


class RamltAdaptParams(ctypes.Structure):
    """Mirror of ``ramlt_adapt_params`` (host struct)."""

    _fields_ = [
        ("n_regions", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("gamma_max", ctypes.c_double),
        ("gamma_scale", ctypes.c_double),
        ("alpha_target", ctypes.c_double),
        ("lambda_min", ctypes.c_double),
    ]


class RamltRegionState(ctypes.Structure):
    """Mirror of ``ramlt_region_state`` (host struct of device pointers)."""

    _fields_ = [
        ("lambda_", ctypes.c_void_p),
        ("acc", ctypes.c_void_p),
        ("visits", ctypes.c_void_p),
        ("updates", ctypes.c_void_p),
        ("lambda_f32", ctypes.c_void_p),
    ]


class RamltQuadtree(ctypes.Structure):
    """Mirror of ``ramlt_quadtree`` (host struct of device pointers)."""

    _fields_ = [
        ("n_roots", ctypes.c_int32),
        ("capacity", ctypes.c_int32),
        ("child", ctypes.c_void_p),
        ("depth", ctypes.c_void_p),
        ("visits", ctypes.c_void_p),
        ("n_nodes", ctypes.c_void_p),
    ]


class RamltError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"ramlt status {status}: {message}")
        self.status = status


_lib = None


def load():
    """Load ``libramlt.so`` (built in-tree). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2402_08273_amd.build` "
            "(there is no fallback implementation)"
        )
    lib = ctypes.CDLL(LIB_PATH)
    sig = [ctypes.POINTER(RamltFrame), ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
           ctypes.c_size_t, ctypes.c_void_p]
    for name in ("stats_accumulate", "filter_forward", "loss_seed", "filter_backward"):
        fn = getattr(lib, name)
        fn.argtypes = sig
        fn.restype = ctypes.c_int
    lib.filter_backward_noalloc.argtypes = [ctypes.POINTER(RamltFrame), ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_void_p]
    lib.filter_backward_noalloc.restype = ctypes.c_int
    lib.stats_filter_step.argtypes = [ctypes.POINTER(RamltFrame), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.stats_filter_step.restype = ctypes.c_int
    lib.ramlt_workspace_size.argtypes = [ctypes.POINTER(RamltFrame), ctypes.c_int32, ctypes.c_int32]
    lib.ramlt_workspace_size.restype = ctypes.c_size_t
    lib.ramlt_last_error.argtypes = []
    lib.ramlt_last_error.restype = ctypes.c_char_p
    lib.ramlt_abi_version.argtypes = []
    lib.ramlt_abi_version.restype = ctypes.c_int32
    lib.region_adapt.argtypes = [ctypes.POINTER(RamltAdaptParams), ctypes.POINTER(RamltRegionState),
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                                 ctypes.c_void_p]
    lib.region_adapt.restype = ctypes.c_int
    lib.ramlt_adapt_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.ramlt_adapt_workspace_size.restype = ctypes.c_size_t
    qt = ctypes.POINTER(RamltQuadtree)
    lib.quadtree_init.argtypes = [qt, ctypes.c_void_p]
    lib.quadtree_init.restype = ctypes.c_int
    lib.quadtree_lookup.argtypes = [qt, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]
    lib.quadtree_lookup.restype = ctypes.c_int
    lib.quadtree_refine.argtypes = [qt, ctypes.c_int32, ctypes.POINTER(RamltRegionState), ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p]
    lib.quadtree_refine.restype = ctypes.c_int
    lib.perturb_directions.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.rrmse.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.rrmse.restype = ctypes.c_int
    lib.ramlt_rrmse_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.ramlt_rrmse_workspace_size.restype = ctypes.c_size_t
    lib.lens_chain_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.lens_chain_step.restype = ctypes.c_int
    lib.ramlt_lens_workspace_size.argtypes = [ctypes.c_int32]
    lib.ramlt_lens_workspace_size.restype = ctypes.c_size_t
    lib.lens_chain_sort.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.lens_chain_sort.restype = ctypes.c_int
    lib.ramlt_lens_sort_workspace_size.argtypes = [ctypes.c_int64]
    lib.ramlt_lens_sort_workspace_size.restype = ctypes.c_size_t
    lib.ramlt_perturb_workspace_size.argtypes = [ctypes.c_int32]
    lib.ramlt_perturb_workspace_size.restype = ctypes.c_size_t
    lib.perturb_directions.restype = ctypes.c_int
    lib.ramlt_quadtree_workspace_size.argtypes = [ctypes.c_int32]
    lib.ramlt_quadtree_workspace_size.restype = ctypes.c_size_t
    if (lib.ramlt_abi_version() >> 16) != ctypes.sizeof(RamltFrame):
        raise RuntimeError("ramlt_frame layout mismatch between libramlt.so and the binding")
    _lib = lib
    return lib


def _table(frames):
    if isinstance(frames, RamltFrame):
        frames = [frames]
    n = len(frames)
    arr = (RamltFrame * n)(*frames)
    return arr, n


def _call(name, frames, frames_dev=None, workspace=None, ws_bytes=0, stream=None):
    lib = load()
    arr, n = _table(frames)
    st = getattr(lib, name)(arr, frames_dev, n, workspace, ws_bytes, stream)
    if st != RAMLT_OK:
        raise RamltError(st, lib.ramlt_last_error().decode())
    return st


def stats_accumulate(frames, frames_dev=None, workspace=None, ws_bytes=0, stream=None):
    return _call("stats_accumulate", frames, frames_dev, workspace, ws_bytes, stream)


def filter_forward(frames, frames_dev=None, workspace=None, ws_bytes=0, stream=None):
    return _call("filter_forward", frames, frames_dev, workspace, ws_bytes, stream)


def loss_seed(frames, frames_dev=None, workspace=None, ws_bytes=0, stream=None):
    return _call("loss_seed", frames, frames_dev, workspace, ws_bytes, stream)


def filter_backward(frames, frames_dev=None, workspace=None, ws_bytes=0, stream=None):
    return _call("filter_backward", frames, frames_dev, workspace, ws_bytes, stream)


def filter_backward_noalloc(frames, frames_dev=None, stream=None):
    """filter_backward with the library's own device workspace (no workspace argument)."""
    lib = load()
    arr, n = _table(frames)
    st = lib.filter_backward_noalloc(arr, frames_dev, n, stream)
    if st != RAMLT_OK:
        raise RamltError(st, lib.ramlt_last_error().decode())
    return st


def stats_filter_step_status(frame, workspace=None, ws_bytes=0, stream=None):
    """Raw status of stats_filter_step on one descriptor (no exception)."""
    return load().stats_filter_step(ctypes.byref(frame), workspace, ws_bytes, stream)


def stats_filter_step(frame, workspace=None, ws_bytes=0, stream=None):
    """stats_accumulate + filter_forward (loss in the forward pass) + filter_backward of one
    frame in one call."""
    st = stats_filter_step_status(frame, workspace, ws_bytes, stream)
    if st != RAMLT_OK:
        raise RamltError(st, load().ramlt_last_error().decode())
    return st


def workspace_size(frames, op):
    lib = load()
    arr, n = _table(frames)
    return int(lib.ramlt_workspace_size(arr, n, op))


def last_error():
    return load().ramlt_last_error().decode()


def status_of(name, frames, frames_dev=None, workspace=None, ws_bytes=0, stream=None):
    """Raw status code of an entry point (no exception); used by host-validation tests."""
    lib = load()
    arr, n = _table(frames)
    return getattr(lib, name)(arr, frames_dev, n, workspace, ws_bytes, stream)


def region_adapt(params, state, region, alpha, n, workspace=None, ws_bytes=0, stream=None):
    """Call ``region_adapt``; raises RamltError on a non-zero status."""
    lib = load()
    st = lib.region_adapt(ctypes.byref(params) if params is not None else None,
                          ctypes.byref(state) if state is not None else None, region, alpha, n, workspace,
                          ws_bytes, stream)
    if st != RAMLT_OK:
        raise RamltError(st, last_error())
    return st


def adapt_status(params, state, region, alpha, n, workspace=None, ws_bytes=0, stream=None):
    """Status of a ``region_adapt`` call (no exception), for validation tests."""
    lib = load()
    return lib.region_adapt(ctypes.byref(params) if params is not None else None,
                            ctypes.byref(state) if state is not None else None, region, alpha, n, workspace,
                            ws_bytes, stream)


def adapt_workspace_size(n, m):
    return int(load().ramlt_adapt_workspace_size(n, m))


def _ref(x):
    return ctypes.byref(x) if x is not None else None


def _check(st):
    if st != RAMLT_OK:
        raise RamltError(st, last_error())
    return st


def quadtree_init_status(tree, stream=None):
    return load().quadtree_init(_ref(tree), stream)


def quadtree_lookup_status(tree, root, x, y, leaf, n, count, stream=None):
    return load().quadtree_lookup(_ref(tree), root, x, y, leaf, n, int(count), stream)


def quadtree_refine_status(tree, m_split, state, workspace=None, ws_bytes=0, stream=None):
    return load().quadtree_refine(_ref(tree), m_split, _ref(state), workspace, ws_bytes, stream)


def quadtree_init(tree, stream=None):
    return _check(quadtree_init_status(tree, stream))


def quadtree_lookup(tree, root, x, y, leaf, n, count, stream=None):
    return _check(quadtree_lookup_status(tree, root, x, y, leaf, n, count, stream))


def quadtree_refine(tree, m_split, state, workspace=None, ws_bytes=0, stream=None):
    return _check(quadtree_refine_status(tree, m_split, state, workspace, ws_bytes, stream))


def quadtree_workspace_size(capacity):
    return int(load().ramlt_quadtree_workspace_size(capacity))


def perturb_directions_status(lam, n_regions, region, omega, uv, omega_out, theta_out, n, workspace=None,
                              ws_bytes=0, stream=None):
    return load().perturb_directions(lam, n_regions, region, omega, uv, omega_out, theta_out, n, workspace,
                                     ws_bytes, stream)


def perturb_directions(lam, n_regions, region, omega, uv, omega_out, theta_out, n, workspace=None, ws_bytes=0,
                       stream=None):
    return _check(perturb_directions_status(lam, n_regions, region, omega, uv, omega_out, theta_out, n, workspace,
                                            ws_bytes, stream))


def perturb_workspace_size(n_regions):
    return int(load().ramlt_perturb_workspace_size(n_regions))


def lens_chain_step_status(luminance, W, H, tan_half_fov_x, lam, n_regions, omega, noise, region, alpha,
                           omega_prop, n, workspace=None, ws_bytes=0, stream=None, density=None, pixel=None):
    return load().lens_chain_step(luminance, W, H, tan_half_fov_x, lam, n_regions, omega, density, pixel, noise,
                                  region, alpha, omega_prop, n, workspace, ws_bytes, stream)


def lens_chain_step(luminance, W, H, tan_half_fov_x, lam, n_regions, omega, noise, region, alpha, omega_prop, n,
                    workspace=None, ws_bytes=0, stream=None, density=None, pixel=None):
    return _check(lens_chain_step_status(luminance, W, H, tan_half_fov_x, lam, n_regions, omega, noise, region,
                                         alpha, omega_prop, n, workspace, ws_bytes, stream, density, pixel))


def lens_workspace_size(n_regions):
    return int(load().ramlt_lens_workspace_size(n_regions))


def lens_chain_sort_status(W, H, tan_half_fov_x, omega, density, n, omega_out, density_out, perm, workspace=None,
                           ws_bytes=0, stream=None):
    return load().lens_chain_sort(W, H, tan_half_fov_x, omega, density, n, omega_out, density_out, perm, workspace,
                                  ws_bytes, stream)


def lens_chain_sort(W, H, tan_half_fov_x, omega, density, n, omega_out, density_out, perm, workspace=None,
                    ws_bytes=0, stream=None):
    return _check(lens_chain_sort_status(W, H, tan_half_fov_x, omega, density, n, omega_out, density_out, perm,
                                         workspace, ws_bytes, stream))


def lens_sort_workspace_size(n):
    return int(load().ramlt_lens_sort_workspace_size(n))


def rrmse_status(image, reference, W, H, eps, map_, out, workspace=None, ws_bytes=0, stream=None):
    return load().rrmse(image, reference, W, H, eps, map_, out, workspace, ws_bytes, stream)


def rrmse(image, reference, W, H, eps, map_, out, workspace=None, ws_bytes=0, stream=None):
    return _check(rrmse_status(image, reference, W, H, eps, map_, out, workspace, ws_bytes, stream))


def rrmse_workspace_size(W, H):
    return int(load().ramlt_rrmse_workspace_size(W, H))
