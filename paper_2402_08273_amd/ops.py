"""PyTorch-facing wrappers around the C ABI: device memory and streams come from torch,
every computation runs in the HIP kernels of ``libramlt.so``.

All tensors must be CUDA (HIP) tensors on the current device. Sample planes are
``[C, S, H, W]`` views with unit x stride (any other strides); per-pixel planes are dense
``[C, H, W]`` float32.
"""

from typing import NamedTuple, Optional

import torch

from . import _abi
from ._abi import RamltFrame

LAMBDA_MIN_DEFAULT = -30.0
N_REGIONS_DEFAULT = 20


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _check_samples(t, name, channels, dtypes):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 4 or t.shape[0] != channels:
        raise ValueError(f"{name} must be [{channels}, S, H, W], got {tuple(t.shape)}")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} dtype {t.dtype} not in {dtypes}")
    if t.stride(3) != 1:
        raise ValueError(f"{name} must have unit x stride")


def _check_plane(t, name, channels=3, hw=None):
    """A dense float32 device plane [channels, H, W] (and [.., H, W] == hw when given)."""
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous()
            or t.dim() != 3 or t.shape[0] != channels):
        raise ValueError(f"{name} must be a contiguous float32 device tensor [{channels}, H, W]")
    if hw is not None and tuple(t.shape[1:]) != tuple(hw):
        raise ValueError(f"{name} must be [{channels}, {hw[0]}, {hw[1]}], got {tuple(t.shape)}")


def _check_vector(t, name, n, dtype):
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous()
            or t.numel() != n):
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor with {n} entries")


def _check_stats_out(out, K_L, H, W, features):
    """Every output plane a caller passes in must hold what the kernel writes into it."""
    for name in ("mean", "var", "tau"):
        _check_plane(getattr(out, name), f"out.{name}", 3, (H, W))
    if out.lag_corr is not None:
        t = out.lag_corr
        if (not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous()
                or tuple(t.shape) != (3, K_L, H, W)):
            raise ValueError(f"out.lag_corr must be a contiguous float32 device tensor [3, {K_L}, {H}, {W}]")
    if features is not None:
        for name in ("feat_mean", "feat_var"):
            t = getattr(out, name)
            if t is None:
                raise ValueError(f"out.{name} is required with features")
            _check_plane(t, f"out.{name}", 7, (H, W))


def workspace_for(frames, op, device):
    """(tensor, 256-byte-aligned pointer, bytes) of the workspace ``op`` needs on
    ``frames`` (``(None, None, 0)`` when it needs none)."""
    need = _abi.workspace_size(frames, op)
    if need == 0:
        return None, None, 0
    t = torch.empty(need + 256, device=device, dtype=torch.uint8)
    return t, (t.data_ptr() + 255) // 256 * 256, need


class Stats(NamedTuple):
    mean: torch.Tensor
    var: torch.Tensor
    tau: torch.Tensor
    lag_corr: Optional[torch.Tensor]
    feat_mean: Optional[torch.Tensor]
    feat_var: Optional[torch.Tensor]


def stats_frame(radiance, features=None, max_lag=8, out: Optional[Stats] = None, with_lag_corr=True):
    """Descriptor + output tensors for :func:`stats` (allocates outputs unless given)."""
    _check_samples(radiance, "radiance", 3, (torch.float32,))
    _, S, H, W = radiance.shape
    dev = radiance.device
    K_L = max(0, min(int(max_lag), S - 1))
    if out is not None:
        _check_stats_out(out, K_L, H, W, features)
    if out is None:
        mk = lambda c: torch.empty((c, H, W), device=dev, dtype=torch.float32)  # noqa: E731
        out = Stats(
            mk(3), mk(3), mk(3),
            torch.empty((3, K_L, H, W), device=dev, dtype=torch.float32) if with_lag_corr else None,
            mk(7) if features is not None else None,
            mk(7) if features is not None else None,
        )
    f = RamltFrame()
    f.W, f.H, f.S, f.max_lag = W, H, S, int(max_lag)
    f.radiance = radiance.data_ptr()
    f.rad_stride_c, f.rad_stride_s, f.rad_stride_y = radiance.stride(0), radiance.stride(1), radiance.stride(2)
    if features is not None:
        _check_samples(features, "features", 7, (torch.float32, torch.float16))
        if features.shape[1:] != radiance.shape[1:]:
            raise ValueError("features and radiance must have the same S, H, W")
        f.features = features.data_ptr()
        f.feat_stride_c, f.feat_stride_s, f.feat_stride_y = features.stride(0), features.stride(1), features.stride(2)
        f.feat_dtype = _abi.RAMLT_F16 if features.dtype == torch.float16 else _abi.RAMLT_F32
        f.feat_mean, f.feat_var = _ptr(out.feat_mean), _ptr(out.feat_var)
    f.mean, f.var, f.tau = _ptr(out.mean), _ptr(out.var), _ptr(out.tau)
    f.lag_corr = _ptr(out.lag_corr)
    return f, out


def stats(radiance, features=None, max_lag=8, with_lag_corr=True, out: Optional[Stats] = None) -> Stats:
    """Per-pixel Appendix A statistics of radiance (and feature) sample planes."""
    f, out = stats_frame(radiance, features, max_lag, out, with_lag_corr)
    _abi.stats_accumulate([f], stream=_stream())
    return out


def filter_frame(mean, lam, radius, n_regions=None, lambda_min=LAMBDA_MIN_DEFAULT, schedule=0):
    _check_plane(mean, "mean")
    if n_regions is None:
        n_regions = int(round(lam.numel() ** 0.5))
    if lam.dtype != torch.float32 or not lam.is_cuda or lam.numel() != n_regions * n_regions or not lam.is_contiguous():
        raise ValueError("lam must be a contiguous float32 device tensor with n_regions**2 entries")
    f = RamltFrame()
    f.W, f.H = mean.shape[2], mean.shape[1]
    f.mean = mean.data_ptr()
    f.lambda_ = lam.data_ptr()
    f.n_regions = int(n_regions)
    f.radius = int(radius)
    f.lambda_min = float(lambda_min)
    f.flags = int(schedule)  # RAMLT_TILE_* | RAMLT_SCHED_*: launch schedule only
    return f


def filter_forward(mean, lam, radius, n_regions=None, lambda_min=LAMBDA_MIN_DEFAULT, out=None, schedule=0):
    """Regional reconstruction filter of per-pixel means -> [3, H, W]. ``schedule``:
    ramlt_frame.flags (tile shape, direct gather), e.g. from :mod:`.tune`."""
    f = filter_frame(mean, lam, radius, n_regions, lambda_min, schedule)
    if out is None:
        out = torch.empty_like(mean)
    _check_plane(out, "out", 3, mean.shape[1:])
    f.out = out.data_ptr()
    _abi.filter_forward([f], stream=_stream())
    return out


def loss_seed(out, reference, grad_out=None, loss=None):
    """MSE loss (accumulated into a float64 [1] tensor) and its gradient w.r.t. ``out``."""
    _check_plane(out, "out")
    _check_plane(reference, "reference", 3, out.shape[1:])
    if grad_out is None:
        grad_out = torch.empty_like(out)
    _check_plane(grad_out, "grad_out", 3, out.shape[1:])
    if loss is None:
        loss = torch.zeros(1, device=out.device, dtype=torch.float64)
    _check_vector(loss, "loss", 1, torch.float64)
    f = RamltFrame()
    f.W, f.H = out.shape[2], out.shape[1]
    f.out, f.reference, f.grad_out, f.loss = out.data_ptr(), reference.data_ptr(), grad_out.data_ptr(), loss.data_ptr()
    _abi.loss_seed([f], stream=_stream())
    return loss, grad_out


def filter_backward(grad_out, mean, out, lam, radius, S, n_regions=None, lambda_min=LAMBDA_MIN_DEFAULT,
                    want_grad_lambda=True, grad_radiance=None, grad_lambda=None, reference=None, loss=None,
                    schedule=0):
    """Adjoint of the filter: (G [3,H,W] = dL/dg for every sample, dL/dlambda [N*N]).

    With ``grad_out=None`` and a ``reference`` image, the MSE loss seed is fused into the
    adjoint (U is never written); ``loss`` (fp64 [1]), if given, accumulates the MSE.
    ``schedule``: as for :func:`filter_forward`."""
    f = filter_frame(mean, lam, radius, n_regions, lambda_min, schedule)
    hw = mean.shape[1:]
    _check_plane(out, "out", 3, hw)
    if grad_out is None:
        if reference is None:
            raise ValueError("filter_backward needs grad_out or a reference image")
        _check_plane(reference, "reference", 3, hw)
        f.reference = reference.data_ptr()
        if loss is not None:
            _check_vector(loss, "loss", 1, torch.float64)
        f.loss = _ptr(loss)
    else:
        _check_plane(grad_out, "grad_out", 3, hw)
        f.grad_out = grad_out.data_ptr()
    f.S = int(S)
    if grad_radiance is None:
        grad_radiance = torch.empty_like(mean)
    _check_plane(grad_radiance, "grad_radiance", 3, hw)
    if want_grad_lambda and grad_lambda is None:
        grad_lambda = torch.zeros_like(lam)
    if want_grad_lambda:
        _check_vector(grad_lambda, "grad_lambda", f.n_regions * f.n_regions, torch.float32)
    f.out = out.data_ptr()
    f.grad_radiance = grad_radiance.data_ptr()
    f.grad_lambda = _ptr(grad_lambda) if want_grad_lambda else None
    ws, ws_ptr, ws_bytes = workspace_for([f], _abi.OP_FILTER_BACKWARD, mean.device)
    _abi.filter_backward([f], workspace=ws_ptr, ws_bytes=ws_bytes, stream=_stream())
    del ws  # freed blocks are reused in stream order, after this launch
    return grad_radiance, grad_lambda


def filter_forward_loss(mean, lam, radius, reference, n_regions=None, lambda_min=LAMBDA_MIN_DEFAULT, out=None,
                        grad_out=None, loss=None, grad_lambda=None, want_grad_lambda=True, schedule=0):
    """The filter with the MSE loss seed and dL/dlambda formed in the same pass
    (RAMLT_LOSS_IN_FORWARD): returns (out, U = dL/dout, loss, grad_lambda); ``loss`` (fp64
    [1]) and ``grad_lambda`` are accumulated into (zeros when not given). The radiance
    gradient then comes from :func:`filter_backward_radiance` on U."""
    f = filter_frame(mean, lam, radius, n_regions, lambda_min, schedule | _abi.RAMLT_LOSS_IN_FORWARD)
    hw = mean.shape[1:]
    _check_plane(reference, "reference", 3, hw)
    out = torch.empty_like(mean) if out is None else out
    grad_out = torch.empty_like(mean) if grad_out is None else grad_out
    loss = torch.zeros(1, device=mean.device, dtype=torch.float64) if loss is None else loss
    _check_plane(out, "out", 3, hw)
    _check_plane(grad_out, "grad_out", 3, hw)
    _check_vector(loss, "loss", 1, torch.float64)
    if want_grad_lambda:
        grad_lambda = torch.zeros_like(lam) if grad_lambda is None else grad_lambda
        _check_vector(grad_lambda, "grad_lambda", f.n_regions * f.n_regions, torch.float32)
    f.out, f.reference, f.grad_out, f.loss = out.data_ptr(), reference.data_ptr(), grad_out.data_ptr(), loss.data_ptr()
    f.grad_lambda = _ptr(grad_lambda) if want_grad_lambda else None
    ws, ws_ptr, ws_bytes = workspace_for([f], _abi.OP_FILTER_FORWARD, mean.device)
    _abi.filter_forward([f], workspace=ws_ptr, ws_bytes=ws_bytes, stream=_stream())
    del ws  # freed blocks are reused in stream order, after this launch
    return out, grad_out, loss, (grad_lambda if want_grad_lambda else None)


def filter_backward_radiance(grad_out, lam, radius, S, n_regions=None, lambda_min=LAMBDA_MIN_DEFAULT,
                             grad_radiance=None, schedule=0):
    """The radiance half of the adjoint: G [3, H, W] = dL/dg for every sample, from U
    (RAMLT_LOSS_IN_FORWARD: dL/dlambda and the loss come from :func:`filter_forward_loss`)."""
    _check_plane(grad_out, "grad_out")
    f = filter_frame(grad_out, lam, radius, n_regions, lambda_min, schedule | _abi.RAMLT_LOSS_IN_FORWARD)
    f.mean = 0
    f.grad_out = grad_out.data_ptr()
    f.S = int(S)
    if grad_radiance is None:
        grad_radiance = torch.empty_like(grad_out)
    _check_plane(grad_radiance, "grad_radiance", 3, grad_out.shape[1:])
    f.grad_radiance = grad_radiance.data_ptr()
    ws, ws_ptr, ws_bytes = workspace_for([f], _abi.OP_FILTER_BACKWARD, grad_out.device)
    _abi.filter_backward([f], workspace=ws_ptr, ws_bytes=ws_bytes, stream=_stream())
    del ws
    return grad_radiance


class StepResult(NamedTuple):
    stats: Stats
    out: torch.Tensor
    grad_out: torch.Tensor
    grad_radiance: torch.Tensor
    loss: torch.Tensor
    grad_lambda: Optional[torch.Tensor]


def step_frame(radiance, features, lam, radius, reference, max_lag=8, n_regions=None,
               lambda_min=LAMBDA_MIN_DEFAULT, schedule=0, with_lag_corr=False, want_grad_lambda=True):
    """Descriptor (flags with RAMLT_LOSS_IN_FORWARD) and zeroed / fresh output tensors of one
    frame's whole step, for :func:`stats_filter_step` or for the three calls in sequence."""
    f, st = stats_frame(radiance, features, max_lag, None, with_lag_corr)
    fl = filter_frame(st.mean, lam, radius, n_regions, lambda_min, int(schedule) | _abi.RAMLT_LOSS_IN_FORWARD)
    hw = st.mean.shape[1:]
    _check_plane(reference, "reference", 3, hw)
    out, grad_out, grad_radiance = (torch.empty_like(st.mean) for _ in range(3))
    loss = torch.zeros(1, device=st.mean.device, dtype=torch.float64)
    grad_lambda = torch.zeros_like(lam) if want_grad_lambda else None
    f.lambda_, f.n_regions, f.radius, f.lambda_min = fl.lambda_, fl.n_regions, fl.radius, fl.lambda_min
    f.flags = fl.flags
    f.out, f.reference, f.grad_out = out.data_ptr(), reference.data_ptr(), grad_out.data_ptr()
    f.grad_radiance, f.loss, f.grad_lambda = grad_radiance.data_ptr(), loss.data_ptr(), _ptr(grad_lambda)
    return f, StepResult(st, out, grad_out, grad_radiance, loss, grad_lambda)


def stats_filter_step(radiance, features, lam, radius, reference, max_lag=8, n_regions=None,
                      lambda_min=LAMBDA_MIN_DEFAULT, schedule=0, with_lag_corr=False, want_grad_lambda=True):
    """The whole differentiable step of one frame in one library call: statistics, the
    filter with the MSE seed, the loss and dL/dlambda, and the radiance adjoint G. Same
    results as :func:`stats`, :func:`filter_forward_loss` and
    :func:`filter_backward_radiance`."""
    f, res = step_frame(radiance, features, lam, radius, reference, max_lag, n_regions, lambda_min, schedule,
                        with_lag_corr, want_grad_lambda)
    ws, ws_ptr, ws_bytes = workspace_for([f], _abi.OP_FILTER_FORWARD, radiance.device)
    _abi.stats_filter_step(f, workspace=ws_ptr, ws_bytes=ws_bytes, stream=_stream())
    del ws
    return res


class RegionalFilter(torch.autograd.Function):
    """out = filter(mean over samples of radiance; lambda). Differentiable in radiance and
    lambda; the statistics outputs and features carry no gradient.

    ``RegionalFilter.apply(radiance, features, lam, radius, n_regions, lambda_min, max_lag)``
    """

    @staticmethod
    def forward(ctx, radiance, features, lam, radius, n_regions=None, lambda_min=LAMBDA_MIN_DEFAULT, max_lag=8):
        # the lag correlations are not needed by the filter or its adjoint: not written
        st = stats(radiance, features, max_lag, with_lag_corr=False)
        out = filter_forward(st.mean, lam, radius, n_regions, lambda_min)
        ctx.save_for_backward(st.mean, out, lam)
        ctx.cfg = (int(radius), n_regions, float(lambda_min), radiance.shape)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        mean, out, lam = ctx.saved_tensors
        radius, n_regions, lambda_min, shape = ctx.cfg
        G, gl = filter_backward(grad_out.contiguous(), mean, out, lam, radius, shape[1], n_regions, lambda_min,
                                want_grad_lambda=ctx.needs_input_grad[2])
        g_rad = G.unsqueeze(1).expand(shape) if ctx.needs_input_grad[0] else None
        return g_rad, None, gl, None, None, None, None


class MSELoss(torch.autograd.Function):
    """L = mean((out - reference)^2) in float64, with the gradient formed by the loss_seed
    kernel during the forward pass."""

    @staticmethod
    def forward(ctx, out, reference):
        loss, grad = loss_seed(out.contiguous(), reference.contiguous())
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g.to(grad.dtype), None


# ---------------------------------------------------------------------------- adaptation
class RegionAdapter:
    """Per-region adaptive scaling parameters (Algorithm 1) on the device.

    Holds the state (lambda_k and its float copy for the filter, A_k, i_k, n_k) for
    ``n_regions`` regions and feeds batches of proposals (region int32 [n], acceptance
    probability float32 [n], device tensors) through ``region_adapt``. Defaults are the
    paper's parameters (Sec. 8.1): L = 10, gamma_max = 1, gamma_scale = 5, alpha* = 0.5,
    lambda_init = 1, lambda_min = -30.
    """

    def __init__(self, n_regions, L=10, gamma_max=1.0, gamma_scale=5.0, alpha_target=0.5,
                 lambda_init=1.0, lambda_min=LAMBDA_MIN_DEFAULT, device="cuda"):
        dev = torch.device(device)
        m = int(n_regions)
        self.lam = torch.full((m,), float(lambda_init), device=dev, dtype=torch.float64)
        self.acc = torch.zeros(m, device=dev, dtype=torch.float64)
        self.visits = torch.zeros(m, device=dev, dtype=torch.int32)
        self.updates = torch.ones(m, device=dev, dtype=torch.int32)
        self.lam_f32 = self.lam.float()  # the filter's lambda table
        self.params = _abi.RamltAdaptParams(m, int(L), float(gamma_max), float(gamma_scale), float(alpha_target),
                                            float(lambda_min))
        self.state = _abi.RamltRegionState(self.lam.data_ptr(), self.acc.data_ptr(), self.visits.data_ptr(),
                                           self.updates.data_ptr(), self.lam_f32.data_ptr())
        self.device = dev
        self._ws = None
        self._ws_bytes = 0

    def workspace(self, n):
        need = _abi.adapt_workspace_size(n, self.params.n_regions)
        if need > self._ws_bytes:
            self._ws = torch.empty(need + 256, device=self.device, dtype=torch.uint8)
            self._ws_bytes = need
        if need == 0:
            return None, 0
        return (self._ws.data_ptr() + 255) // 256 * 256, need

    def step(self, region, alpha):
        """Adapt on one batch of proposals, in index order within each region."""
        if region.dtype != torch.int32 or alpha.dtype != torch.float32 or not region.is_cuda or not alpha.is_cuda:
            raise ValueError("region must be an int32 and alpha a float32 device tensor")
        if region.dim() != 1 or region.shape != alpha.shape or not region.is_contiguous() or not alpha.is_contiguous():
            raise ValueError("region and alpha must be contiguous 1-D tensors of equal length")
        n = region.numel()
        ws, ws_bytes = self.workspace(n)
        _abi.region_adapt(self.params, self.state, region.data_ptr() if n else None,
                          alpha.data_ptr() if n else None, n, ws, ws_bytes, _stream())
        return self


class Quadtree:
    """A forest of quadtrees on the device (Sec. 6.1-6.3): ``n_roots`` trees over [0,1]^2,
    storage for ``capacity`` nodes. Leaves are regions; a node index is a region key for
    :class:`RegionAdapter` (give it ``n_regions >= capacity``).

    ``lookup(x, y, root=None, count=True)`` returns the leaf of every point (int32, -1 for
    none) and counts visits per leaf; ``refine(m_split, adapter=None)`` splits the leaves
    visited more than ``m_split`` times since the last refinement, passing lambda and
    n_k / 4 on to the children in ``adapter``'s state."""

    def __init__(self, n_roots, capacity, device="cuda"):
        dev = torch.device(device)
        cap = int(capacity)
        self.child = torch.empty(cap, device=dev, dtype=torch.int32)
        self.depth = torch.empty(cap, device=dev, dtype=torch.int32)
        self.visits = torch.empty(cap, device=dev, dtype=torch.int32)
        self.n_nodes_dev = torch.empty(1, device=dev, dtype=torch.int32)
        self.tree = _abi.RamltQuadtree(int(n_roots), cap, self.child.data_ptr(), self.depth.data_ptr(),
                                       self.visits.data_ptr(), self.n_nodes_dev.data_ptr())
        self.device = dev
        need = _abi.quadtree_workspace_size(cap)
        self._ws = torch.empty(need + 256, device=dev, dtype=torch.uint8)
        self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        self._ws_bytes = need
        _abi.quadtree_init(self.tree, _stream())

    @property
    def n_nodes(self):
        return int(self.n_nodes_dev.item())

    def reset(self):
        _abi.quadtree_init(self.tree, _stream())
        return self

    def lookup(self, x, y, root=None, count=True, out=None):
        for t in (x, y):
            if t.dtype != torch.float32 or not t.is_cuda or t.dim() != 1 or not t.is_contiguous():
                raise ValueError("x and y must be contiguous 1-D float32 device tensors")
        if x.shape != y.shape:
            raise ValueError("x and y differ in length")
        if root is not None and (root.dtype != torch.int32 or not root.is_cuda or root.shape != x.shape
                                 or not root.is_contiguous()):
            raise ValueError("root must be a contiguous int32 device tensor like x")
        n = x.numel()
        leaf = out if out is not None else torch.empty(n, device=self.device, dtype=torch.int32)
        if leaf.dtype != torch.int32 or leaf.shape != x.shape or not leaf.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor like x")
        _abi.quadtree_lookup(self.tree, root.data_ptr() if (root is not None and n) else None,
                             x.data_ptr() if n else None, y.data_ptr() if n else None,
                             leaf.data_ptr() if n else None, n, 1 if count else 0, _stream())
        return leaf

    def refine(self, m_split, adapter=None):
        if adapter is not None and adapter.params.n_regions < self.tree.capacity:
            raise ValueError("the adapter needs n_regions >= the tree capacity")
        _abi.quadtree_refine(self.tree, int(m_split), adapter.state if adapter is not None else None,
                             self._ws_ptr, self._ws_bytes, _stream())
        return self


def perturb_directions(lam, region, omega, uv, theta=False):
    """Proposed directions (Sec. 3.3, truncated-normal polar angle with sigma_k =
    sqrt(exp(lambda_k)) of each proposal's region): lam float64 [m] (e.g.
    ``RegionAdapter.lam``), region int32 [n], omega float32 [n, 3] (unit), uv float32
    [n, 2] uniforms. Returns omega' [n, 3] (and theta' [n] with ``theta=True``)."""
    n = region.numel()
    if lam.dtype != torch.float64 or lam.dim() != 1 or not lam.is_contiguous() or not lam.is_cuda:
        raise ValueError("lam must be a contiguous 1-D float64 device tensor")
    if region.dtype != torch.int32 or region.dim() != 1 or not region.is_contiguous():
        raise ValueError("region must be a contiguous 1-D int32 tensor")
    if omega.dtype != torch.float32 or tuple(omega.shape) != (n, 3) or not omega.is_contiguous():
        raise ValueError("omega must be a contiguous float32 [n, 3] tensor")
    if uv.dtype != torch.float32 or tuple(uv.shape) != (n, 2) or not uv.is_contiguous():
        raise ValueError("uv must be a contiguous float32 [n, 2] tensor")
    for name, t in (("region", region), ("omega", omega), ("uv", uv)):
        if t.device != lam.device:
            raise ValueError(f"{name} must be on lam's device ({lam.device})")
    out = torch.empty_like(omega)
    th = torch.empty(n, device=omega.device, dtype=torch.float32) if theta else None
    p = (lambda t: t.data_ptr() if (t is not None and n) else None)
    need = _abi.perturb_workspace_size(lam.numel())
    ws = torch.empty(need + 256, device=omega.device, dtype=torch.uint8) if need else None
    wp = (ws.data_ptr() + 255) // 256 * 256 if need else None
    _abi.perturb_directions(lam.data_ptr(), lam.numel(), p(region), p(omega), p(uv), p(out), p(th), n, wp, need,
                            _stream())
    return (out, th) if theta else out


def lens_chain_step(luminance, tan_half_fov_x, lam, n_regions, omega, noise, want_proposals=False, density=None,
                    pixel=None):
    """One Metropolis step of screen-space chains under the regional adaptive lens
    perturbation (Sec. 3.3, Sec. 6.1, Alg. 1 lines 8-13) with the luminance image as target:
    luminance float32 [H, W]; lam float64 [n_regions^2] (e.g. ``RegionAdapter.lam``); omega
    float32 [n, 3] primary directions, updated in place; noise float32 [n, 3] = (u, v,
    acceptance uniform); density (optional) float32 [n], the luminance of each chain's pixel
    carried between steps (start it at -1; updated in place); pixel (optional) int32 [n], the
    pixel of each chain carried between steps (start it at -2; updated in place). Returns
    (region int32 [n],
    alpha float32 [n]) for :class:`RegionAdapter` (and the proposals [n, 3] with
    ``want_proposals=True``)."""
    if luminance.dtype != torch.float32 or luminance.dim() != 2 or not luminance.is_contiguous() \
            or not luminance.is_cuda:
        raise ValueError("luminance must be a contiguous float32 [H, W] device tensor")
    n = omega.shape[0] if omega.dim() == 2 else -1
    if omega.dtype != torch.float32 or tuple(omega.shape) != (n, 3) or not omega.is_contiguous():
        raise ValueError("omega must be a contiguous float32 [n, 3] tensor")
    if noise.dtype != torch.float32 or tuple(noise.shape) != (n, 3) or not noise.is_contiguous():
        raise ValueError("noise must be a contiguous float32 [n, 3] tensor")
    if lam.dtype != torch.float64 or lam.numel() != n_regions * n_regions or not lam.is_contiguous() \
            or not lam.is_cuda:
        raise ValueError("lam must be a contiguous float64 device tensor of n_regions**2 entries")
    if density is not None and (density.dtype != torch.float32 or tuple(density.shape) != (n,)
                                or not density.is_contiguous()):
        raise ValueError("density must be a contiguous float32 [n] tensor")
    if pixel is not None and (pixel.dtype != torch.int32 or tuple(pixel.shape) != (n,) or not pixel.is_contiguous()):
        raise ValueError("pixel must be a contiguous int32 [n] tensor")
    for name, t in (("omega", omega), ("noise", noise), ("lam", lam), ("density", density), ("pixel", pixel)):
        if t is not None and t.device != luminance.device:
            raise ValueError(f"{name} must be on the luminance's device ({luminance.device})")
    H, W = luminance.shape
    region = torch.empty(n, device=omega.device, dtype=torch.int32)
    alpha = torch.empty(n, device=omega.device, dtype=torch.float32)
    prop = torch.empty_like(omega) if want_proposals else None
    p = (lambda t: t.data_ptr() if (t is not None and n) else None)
    need = _abi.lens_workspace_size(n_regions)
    ws = torch.empty(need + 256, device=omega.device, dtype=torch.uint8) if need else None
    wp = (ws.data_ptr() + 255) // 256 * 256 if need else None
    _abi.lens_chain_step(luminance.data_ptr(), W, H, float(tan_half_fov_x), lam.data_ptr(), n_regions, p(omega),
                         p(noise), p(region), p(alpha), p(prop), n, wp, need, _stream(), density=p(density),
                         pixel=p(pixel))
    return (region, alpha, prop) if want_proposals else (region, alpha)


def lens_chain_sort(omega, W, H, tan_half_fov_x, density=None, want_perm=True):
    """Regroup lens chains by the screen tile of their current pixel (stable; the tile side is
    the smallest power of two >= 16 leaving at most 63 tiles), so that the next steps'
    luminance reads stay in cache. omega float32 [n, 3]; density (optional) float32 [n], the
    carried luminance, moved with its chain. Returns (omega_sorted, density_sorted or None,
    perm int32 [n] or None) with omega_sorted[j] = omega[perm[j]]."""
    n = omega.shape[0] if omega.dim() == 2 else -1
    if omega.dtype != torch.float32 or tuple(omega.shape) != (n, 3) or not omega.is_contiguous() \
            or not omega.is_cuda:
        raise ValueError("omega must be a contiguous float32 [n, 3] device tensor")
    if density is not None and (density.dtype != torch.float32 or tuple(density.shape) != (n,)
                                or not density.is_contiguous() or density.device != omega.device):
        raise ValueError("density must be a contiguous float32 [n] tensor on omega's device")
    om2 = torch.empty_like(omega)
    d2 = torch.empty_like(density) if density is not None else None
    perm = torch.empty(n, device=omega.device, dtype=torch.int32) if want_perm else None
    p = (lambda t: t.data_ptr() if (t is not None and n) else None)
    need = _abi.lens_sort_workspace_size(n)
    ws = torch.empty(need + 256, device=omega.device, dtype=torch.uint8) if need else None
    wp = (ws.data_ptr() + 255) // 256 * 256 if need else None
    _abi.lens_chain_sort(int(W), int(H), float(tan_half_fov_x), p(omega), p(density), n, p(om2), p(d2), p(perm), wp,
                         need, _stream())
    return om2, d2, perm


def rrmse(image, reference, eps=1e-2, want_map=True):
    """rRMSE of ``image`` against ``reference`` (float32 [3, H, W] device tensors, Sec. 8.2):
    returns (map float32 [H, W] or None, rRMSE as a float64 device tensor of shape [])."""
    for t in (image, reference):
        if t.dtype != torch.float32 or t.dim() != 3 or t.shape[0] != 3 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("image and reference must be contiguous float32 [3, H, W] device tensors")
    if image.shape != reference.shape:
        raise ValueError("image and reference differ in shape")
    _, H, W = image.shape
    m = torch.empty((H, W), device=image.device, dtype=torch.float32) if want_map else None
    out = torch.empty((), device=image.device, dtype=torch.float64)
    need = _abi.rrmse_workspace_size(W, H)
    ws = torch.empty(need + 256, device=image.device, dtype=torch.uint8)
    _abi.rrmse(image.data_ptr(), reference.data_ptr(), W, H, float(eps), m.data_ptr() if m is not None else None,
               out.data_ptr(), (ws.data_ptr() + 255) // 256 * 256, need, _stream())
    return m, out


class QuadtreeAdapter:
    """Regional adaptation over a quadtree partition (Sec. 6.1-6.3 with Algorithm 1): every
    batch of proposals is looked up in the forest (leaf = region, visits counted), adapted
    region by region, and after every ``m_refine`` proposals the forest refines, handing
    lambda and n_k / 4 to the children. Defaults: the paper's M_split = 5000,
    M_refine = 10^7 (Sec. 8.1) and the adaptation defaults of :class:`RegionAdapter`."""

    def __init__(self, n_roots, capacity, m_split=5000, m_refine=10_000_000, device="cuda", **adapt_kw):
        self.tree = Quadtree(n_roots, capacity, device)
        self.adapter = RegionAdapter(capacity, device=device, **adapt_kw)
        self.m_split = int(m_split)
        self.m_refine = int(m_refine)
        self.pending = 0   # proposals since the last refinement

    @property
    def lam(self):
        return self.adapter.lam

    def step(self, x, y, alpha, root=None):
        """One batch: (x, y) in the trees' unit squares (float32), alpha float32, root int32
        or None; returns the proposals' regions (int32, -1 for none)."""
        leaf = self.tree.lookup(x, y, root)
        self.adapter.step(leaf, alpha)
        self.pending += x.numel()
        if self.pending >= self.m_refine:
            self.tree.refine(self.m_split, self.adapter)
            self.pending = 0
        return leaf
