"""Regional reconstruction filter over per-pixel means, its adjoint, and the MSE loss seed,
in float64.

TEST INFRASTRUCTURE (see the package docstring): only tests/, smoke() and bench.py's
cpu_baseline leg may use it.

Sources in the paper and the readings taken where it is silent:

* Pixel intensity I_j is the integral of h_j f (Sec. 3.1, eq. path_integral); MCMC
  rendering "splats" path contributions to the screen through the reconstruction
  filter h_j. The paper gives h_j no functional form. Reading: an isotropic Gaussian,
  truncated to the square window |dx|, |dy| <= r (the paper's own kernels are
  truncated normals, Sec. 3.3 "Perturbing Ray Directions"), evaluated at integer pixel
  offsets, clipped at the image border, normalised by the sum of in-image weights.
* Its width comes from the region parameter lambda_k = log sigma_k^2,
  sigma_k = sqrt(exp(lambda_k)) (Sec. 5.3), looked up state-dependently,
  sigma(x) = sum_k 1_{P_k}(x) sigma_k (Sec. 5.2), on the uniform N x N grid over the
  raster position in [0,1]^2 (Sec. 5.4 "2d Partition for the Lens Perturbation",
  Sec. 6.1 "Grid Partition"). The region is that of the OUTPUT pixel j, at its centre:
  k_x = floor((2x + 1) N / (2W)), k_y = floor((2y + 1) N / (2H)), k = k_y N + k_x.
* lambda is clamped below at the paper's minimum scaling parameter, -30 (Sec. 8.1
  "Parameters"); N defaults to the paper's top-level grid size 20 (same paragraph).

    h_jp   = exp(-(dx^2 + dy^2) / (2 sigma_{k(j)}^2)),  sigma^2 = exp(max(lambda, lambda_min))
    D_j    = sum_{p in W(j)} h_jp
    out_jc = sum_{p in W(j)} h_jp mean_pc / D_j

Adjoint, for a loss L with U = dL/dout:

    G_pc       = (1/S) sum_{j : p in W(j)} U_jc h_jp / D_j      (= dL/dg_{p,s,c} for every s)
    dL/dlam_k  = sum_{j : k(j) = k} sum_c U_jc sum_{p in W(j)} h'_jp (mean_pc - out_jc) / D_j
    h'_jp      = h_jp (dx^2 + dy^2) / (2 sigma^2)  if lambda_k >= lambda_min, else 0

MSE loss against a reference R (no counterpart in the paper; it exists to drive the
adjoint): L = sum (out - R)^2 / (3P), U = 2 (out - R) / (3P).
"""

import numpy as np

LAMBDA_MIN_DEFAULT = -30.0
N_REGIONS_DEFAULT = 20


def region_index(W, H, n_regions, origin=(0, 0), shape=None):
    """Region k(x, y) of every pixel centre of a W x H image, int64 [H, W]; or, with
    ``origin = (x0, y0)`` and ``shape = (h, w)``, of the pixels x0 <= x < x0 + w,
    y0 <= y < y0 + h only (a crop keeps the regions of the full image)."""
    h, w = (H, W) if shape is None else shape
    x = origin[0] + np.arange(w, dtype=np.int64)
    y = origin[1] + np.arange(h, dtype=np.int64)
    kx = ((2 * x + 1) * n_regions) // (2 * W)
    ky = ((2 * y + 1) * n_regions) // (2 * H)
    return ky[:, None] * n_regions + kx[None, :]


def region_sigma_sq(lam, lambda_min=LAMBDA_MIN_DEFAULT):
    """sigma_k^2 = exp(max(lambda_k, lambda_min)) for every region, float64."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.exp(np.maximum(lam, lambda_min))


def _shift(img, dx, dy):
    """out[..., y, x] = img[..., y+dy, x+dx] where inside, plus the inside mask [H, W]."""
    H, W = img.shape[-2], img.shape[-1]
    out = np.zeros_like(img)
    mask = np.zeros((H, W), dtype=bool)
    y0, y1 = max(0, -dy), min(H, H - dy)
    x0, x1 = max(0, -dx), min(W, W - dx)
    if y0 < y1 and x0 < x1:
        out[..., y0:y1, x0:x1] = img[..., y0 + dy : y1 + dy, x0 + dx : x1 + dx]
        mask[y0:y1, x0:x1] = True
    return out, mask


def _crop_geometry(arr, origin, image_size):
    """(W, H, origin) of the image that the [.., h, w] array ``arr`` is a crop of.

    Crops: the array holds pixels origin[0] <= x < origin[0] + w, origin[1] <= y < ...
    of a W x H image. Regions and the border clipping are those of the full image, and
    pixels outside the array count as outside; so a result is the full image's result
    where every pixel it reads lies in the array (see each function)."""
    h, w = arr.shape[-2:]
    if image_size is None:
        if tuple(origin) != (0, 0):
            raise ValueError("a crop needs image_size")
        return w, h, (0, 0)
    W, H = image_size
    x0, y0 = origin
    if x0 < 0 or y0 < 0 or x0 + w > W or y0 + h > H:
        raise ValueError("crop outside the image")
    return W, H, (x0, y0)


def _pixel_sigma_sq(W, H, lam, n_regions, lambda_min, origin=(0, 0), shape=None):
    k = region_index(W, H, n_regions, origin, shape)
    return region_sigma_sq(lam, lambda_min)[k], k


def filter_forward(mean, lam, n_regions=N_REGIONS_DEFAULT, radius=3,
                   lambda_min=LAMBDA_MIN_DEFAULT, origin=(0, 0), image_size=None):
    """Filtered image from per-pixel means.

    mean: [C, H, W]; lam: [n_regions**2]. Returns (out [C,H,W], D [H,W]) in float64.
    On a crop (``origin``, ``image_size = (W, H)``), out_j and D_j are exact for every j
    whose window, clipped to the image, lies in the crop: j at least ``radius`` pixels
    from each crop edge that is not an image edge.
    """
    mean = np.asarray(mean, dtype=np.float64)
    W, H, origin = _crop_geometry(mean, origin, image_size)
    s2, _ = _pixel_sigma_sq(W, H, lam, n_regions, lambda_min, origin, mean.shape[-2:])
    num = np.zeros_like(mean)
    den = np.zeros(mean.shape[-2:])
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            h = np.exp(-(dx * dx + dy * dy) / (2.0 * s2))
            mu_p, inside = _shift(mean, dx, dy)
            h = np.where(inside, h, 0.0)
            num += h[None] * mu_p
            den += h
    return num / den[None], den


def mse_loss_seed(out, reference, count=None):
    """L = sum (out - R)^2 / (3P) and U = dL/dout = 2 (out - R) / (3P); 3P = out.size,
    or ``count`` (the full image's 3P when out and R are crops: L is then the crop's share)."""
    out = np.asarray(out, dtype=np.float64)
    ref = np.asarray(reference, dtype=np.float64)
    n = out.size if count is None else int(count)
    diff = out - ref
    return float((diff * diff).sum() / n), 2.0 * diff / n


def filter_backward(grad_out, mean, out, lam, n_regions=N_REGIONS_DEFAULT, radius=3,
                    lambda_min=LAMBDA_MIN_DEFAULT, S=1, origin=(0, 0), image_size=None):
    """Adjoint of :func:`filter_forward` composed with the per-pixel mean of S samples.

    grad_out U, mean, out: [C, H, W]. Returns (G [C,H,W], grad_lambda [n_regions**2]),
    where G_pc is dL/dg_{p,s,c} for every sample s of pixel p.
    On a crop (``origin``, ``image_size``), with U and out valid on the whole crop: G_p is
    exact for p at least 2 ``radius`` pixels from each crop edge that is not an image
    edge, and grad_lambda[k] for a region k whose pixels all lie ``radius`` pixels inside
    such edges (other entries hold partial sums).
    """
    U = np.asarray(grad_out, dtype=np.float64)
    mean = np.asarray(mean, dtype=np.float64)
    out = np.asarray(out, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    W, H, origin = _crop_geometry(mean, origin, image_size)
    s2, k = _pixel_sigma_sq(W, H, lam, n_regions, lambda_min, origin, mean.shape[-2:])
    live = (lam >= lambda_min)[k]  # [H, W]: gradient passes through the clamp
    # D_j, recomputed from the same weights as the forward pass.
    den = np.zeros(mean.shape[-2:])
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            _, inside = _shift(mean, dx, dy)
            den += np.where(inside, np.exp(-(dx * dx + dy * dy) / (2.0 * s2)), 0.0)
    a = U / den[None]  # U_j / D_j
    G = np.zeros_like(U)
    per_pixel = np.zeros(mean.shape[-2:])
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            d2 = float(dx * dx + dy * dy)
            h = np.exp(-d2 / (2.0 * s2))  # h_jp with j the array position, p = j + (dx, dy)
            mu_p, inside = _shift(mean, dx, dy)
            h = np.where(inside, h, 0.0)
            # scatter U_j h_jp / D_j from j onto p = j + (dx, dy)
            contrib = a * h[None]
            back, inside_j = _shift(contrib, -dx, -dy)
            G += back
            # derivative of the weights with respect to lambda_{k(j)}
            hprime = np.where(live, h * d2 / (2.0 * s2), 0.0)
            per_pixel += (U * hprime[None] * (mu_p - out)).sum(axis=0) / den
    grad_lambda = np.bincount(k.ravel(), weights=per_pixel.ravel(),
                              minlength=n_regions * n_regions)
    return G / float(S), grad_lambda
