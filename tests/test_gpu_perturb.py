"""GPU parity of perturb_directions (Sec. 3.3 direction perturbation, sigma_k from lambda_k of
Sec. 5.3) against the FP64 oracle.

Tolerances, from the arithmetic: theta' is computed in fp64 (erf and erfc within a few ulp,
erfinv from polynomials within 2e-10 relative, pinned in test_erfinv_poly_host.py) and stored
as float32: 2^-24 rounding + 2e-10 < 2^-23, so |theta_gpu - theta| <= 2^-23 |theta|. The direction is formed
in float32: theta' and phi' rounded (<= 2^-24 relative, phi' <= 2 pi), sin/cos within an ulp,
the basis vectors within a few roundings of unit-size terms; each component of omega' is a
sum of three such products: |error| <= 4e-6."""

import math

import numpy as np
import pytest
import torch

from oracle import direction_sampler as ods
from paper_2402_08273_amd import ops
from synth.directions import make_lambda_table, make_perturb_inputs

pytestmark = pytest.mark.gpu

DIR_TOL = 4e-6


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(name, lam, region, omega, uv):
    out, th = ops.perturb_directions(_dev(lam), _dev(region), _dev(omega), _dev(uv), theta=True)
    out, th = out.cpu().numpy(), th.cpu().numpy()
    want, wth = ods.perturb_directions(lam, region, omega, uv)
    nan = np.isnan(wth)
    assert np.array_equal(np.isnan(th), nan), name
    assert np.array_equal(np.isnan(out), np.isnan(want)), name
    ok = ~nan
    err = np.abs(th[ok] - wth[ok])
    assert np.all(err <= 2.0 ** -23 * np.abs(wth[ok]) + 1e-45), (name, float(err.max()))
    okd = ~np.isnan(want)
    derr = np.abs(out[okd] - want[okd])
    assert derr.size == 0 or derr.max() <= DIR_TOL, (name, float(derr.max()))
    return out, th, want, wth


@pytest.mark.parametrize("m,n", [(1, 1000), (400, 200_000), (65_536, 300_000), (70_000, 300_000)])
def test_perturb_parity(m, n):
    print(f"perturb parity m={m} n={n}", flush=True)
    lam = make_lambda_table(m, seed=m)
    region, omega, uv = make_perturb_inputs(n, m, seed=m + 1)
    out, th, _, wth = _compare(f"m={m}", lam, region, omega, uv)
    ok = ~np.isnan(wth)
    # unit length and the polar angle, independent of the frame convention
    o = out[ok].astype(np.float64)
    w = omega[ok].astype(np.float64)
    assert np.allclose(np.sum(o * o, axis=1), np.sum(w * w, axis=1), atol=2 * DIR_TOL)
    assert np.allclose(np.sum(o * w, axis=1), np.cos(wth[ok]), atol=2 * DIR_TOL)


def test_perturb_edge_cases():
    lam = np.array([-30.0, 0.0, 1.0, 6.0, 40.0, 700.0, -745.0, np.inf, -np.inf, np.nan])
    w = [[0, 0, 1], [0, 0, -1], [0, 0, -0.0], [1, 0, 0], [0, -1, 0], [0.6, 0.8, 0], [0, 0.6, -0.8],
         [np.nan, 0, 1], [0, 0, 1], [0.36, 0.48, 0.8]]
    uvs = [[0.0, 0.0], [0.5, 0.3], [1 - 2 ** -24, 0.999], [0.25, 0.5], [2 ** -24, 0.75], [0.5, 0.0],
           [0.75, 0.1], [0.3, 0.2], [np.nan, 0.2], [0.9, np.nan]]
    region, omega, uv = [], [], []
    for k in range(-1, lam.size + 1):
        for a, b in zip(w, uvs):
            region.append(k)
            omega.append(a)
            uv.append(b)
    region = np.array(region, dtype=np.int32)
    omega = np.array(omega, dtype=np.float32)
    uv = np.array(uv, dtype=np.float32)
    out, th, want, wth = _compare("edges", lam, region, omega, uv)
    valid = (region >= 0) & (region < lam.size)
    assert np.all(np.isnan(out[~valid])) and np.all(np.isnan(th[~valid]))
    # u = 0: theta' = -pi exactly for every sigma; u = 1/2: omega unchanged
    u0 = valid & (uv[:, 0] == 0.0) & (region < 7)   # finite sigma
    assert np.all(th[u0] == np.float32(-math.pi))
    half = valid & (uv[:, 0] == 0.5) & ~np.isnan(omega).any(axis=1) & (region < 7)
    assert np.array_equal(out[half], omega[half])
    # empty batch
    e = torch.empty(0, device="cuda")
    r = ops.perturb_directions(_dev(lam), e.int(), e.view(0, 3).float().contiguous(),
                               e.view(0, 2).float().contiguous())
    assert r.shape == (0, 3)


def test_perturb_statistics_on_gpu():
    # the GPU's theta' for one region over a seeded stream follows the truncated normal:
    # KS distance against the exact CDF and the closed-form second moment
    lam = np.array([math.log(0.8 ** 2)])
    n = 1 << 20
    region = np.zeros(n, dtype=np.int32)
    _, omega, uv = make_perturb_inputs(n, 1, seed=9)
    _, th = ops.perturb_directions(_dev(lam), _dev(region), _dev(omega), _dev(uv), theta=True)
    th = np.sort(th.cpu().numpy().astype(np.float64))
    F = ods.truncated_normal_cdf(th, 0.8)
    i = np.arange(1, n + 1)
    D = max(np.max(i / n - F), np.max(F - (i - 1) / n))
    assert D < 1.95 / math.sqrt(n)
    a = math.pi / 0.8
    from scipy import special
    Z = special.ndtr(a) - special.ndtr(-a)
    var = 0.64 * (1 - 2 * a * math.exp(-0.5 * a * a) / math.sqrt(2 * math.pi) / Z)
    assert abs(np.mean(th * th) - var) < 5 * var * math.sqrt(2.0 / n) + 1e-6


@pytest.mark.slow
@pytest.mark.parametrize("m", [400, 20 * 20 * 50 * 50])
def test_perturb_full_size(m):
    n = 1 << 24
    print(f"perturb full size m={m} n={n}", flush=True)
    lam = make_lambda_table(m, seed=5)
    region, omega, uv = make_perturb_inputs(n, m, seed=6)
    _compare(f"full m={m}", lam, region, omega, uv)
