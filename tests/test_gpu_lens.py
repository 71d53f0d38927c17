"""GPU parity of lens_chain_step (screen-space chains under the regional adaptive lens
perturbation: Sec. 3.3, Sec. 6.1, Alg. 1 lines 8-13) against the oracle, and the closed
adaptation loop (lens_chain_step -> region_adapt) reaching the target acceptance.

Tolerances (tests/lens_check.py). The region of the current state is decided in float32 on
both sides with the same IEEE operations: exact. The proposal omega' is the direction
perturbation's (float32 trigonometry and frame against the fp64 oracle): within 4e-6 per
component. alpha equals the oracle's decision on the GPU's proposal exactly, and is one of
the values that a proposal within 4e-6 of the oracle's can give (the single one away from
pixel and frame edges; at most 1 % of the chains are near an edge); the move is taken iff the
uniform is below alpha."""

import math

import numpy as np
import pytest
import torch

from oracle import lens_chain as olc
from paper_2402_08273_amd import ops
from paper_2402_08273_amd.ops import RegionAdapter
from synth.directions import make_lambda_table
from synth.lens import make_lens_chains, make_lens_noise, make_luminance

import lens_check as lc

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(name, L, tx, lam, N, omega, noise, sample=None):
    """One step on the GPU against the oracle's step on the same inputs (or on a sample of
    the chains), through lens_check.check_step."""
    om = _dev(omega)
    region, alpha, prop = ops.lens_chain_step(_dev(L), tx, _dev(lam), N, om, _dev(noise), want_proposals=True)
    torch.cuda.synchronize()
    g = [t.cpu().numpy() for t in (om, region, alpha, prop)]
    idx = np.arange(omega.shape[0]) if sample is None else sample
    o = olc.step(L, tx, lam, N, omega[idx], noise[idx])
    g = [a[idx] for a in g]
    lc.check_step(L, tx, omega[idx], noise[idx], o, g, name=name)
    return g[2], o[1] >= 0


@pytest.mark.parametrize("W,H,tx,N,n", [(320, 200, 0.6, 20, 200_000), (77, 45, 1.2, 3, 50_000),
                                        (640, 360, 0.4, 300, 100_000), (1, 1, 0.5, 1, 1000)])
def test_lens_step_parity(W, H, tx, N, n):
    print(f"lens parity W={W} H={H} tx={tx} N={N} n={n}", flush=True)
    L = make_luminance(W, H, seed=W + H)
    lam = make_lambda_table(N * N, seed=N)
    if N * N >= 3:
        lam[:3] = [-30.0, 6.0, 0.0]     # tiny sigma, nearly uniform proposals, sigma = 1
    else:
        lam[:] = 0.0
    omega = make_lens_chains(n, W, H, tx, seed=n)
    noise = make_lens_noise(n, seed=W, batch=1)
    alpha, valid = _compare(f"W={W} N={N}", L, tx, lam, N, omega, noise)
    assert valid.mean() > 0.99 and (alpha[valid] == 0).any() and (alpha[valid] == 1).any()


def test_lens_step_full_size_sampled():
    # the bench's configuration: 1920 x 1080 luminance, 20 x 20 regions, 16 M chains; the
    # oracle recomputes a sample of 100 000 chains from the same inputs
    W, H, tx, N, n = 1920, 1080, 0.6, 20, 1 << 24
    print("lens full size", flush=True)
    L = make_luminance(W, H, seed=5)
    lam = make_lambda_table(N * N, seed=7)
    omega = make_lens_chains(n, W, H, tx, seed=8)
    noise = make_lens_noise(n, seed=9)
    sample = np.sort(np.random.default_rng(3).choice(n, 100_000, replace=False))
    _compare("full", L, tx, lam, N, omega, noise, sample=sample)


def test_lens_adaptation_loop_reaches_the_target_acceptance():
    # Closed loop on the GPU: every round the chains step with the current lambda and the
    # regions adapt from the (region, alpha) stream (Alg. 1, L = 10, alpha* = 1/2). Regions
    # of different contrast settle on different scales, each with acceptance near 1/2.
    W, H, tx, N, n, rounds = 256, 160, 0.5, 4, 1 << 16, 80
    print("lens adaptation loop", flush=True)
    L = _dev(make_luminance(W, H, seed=2))
    ad = RegionAdapter(N * N, L=10)
    om = _dev(make_lens_chains(n, W, H, tx, seed=3))
    sums = torch.zeros(N * N, dtype=torch.float64, device="cuda")
    counts = torch.zeros(N * N, dtype=torch.float64, device="cuda")
    for r in range(rounds):
        region, alpha = ops.lens_chain_step(L, tx, ad.lam, N, om, _dev(make_lens_noise(n, seed=4, batch=r)))
        ad.step(region, alpha)
        if r >= rounds - 20:
            ok = region >= 0
            sums.index_add_(0, region[ok].long(), alpha[ok].double())
            counts.index_add_(0, region[ok].long(), torch.ones_like(alpha[ok], dtype=torch.float64))
    torch.cuda.synchronize()
    acc = (sums / counts.clamp(min=1)).cpu().numpy()
    cnt = counts.cpu().numpy()
    lam = ad.lam.cpu().numpy()
    busy = cnt > 20 * 2000
    assert busy.sum() >= 8, cnt
    # the update follows sgn(alpha_hat - alpha*) of windows of L = 10 (eq. update_lambda), so
    # a region settles where its window means are above the target half of the time: its mean
    # acceptance is near, not at, 1/2 (within 0.07 in the oracle's run of this loop)
    assert np.all(np.abs(acc[busy] - 0.5) < 0.1), (acc[busy], lam)
    assert abs(float(np.mean(acc[busy])) - 0.5) < 0.03, (acc[busy], lam)
    assert lam.max() - lam.min() > 1.0, lam                  # the scales differ by region
    assert np.all(lam > -30) and np.all(np.isfinite(lam))
    assert math.isfinite(float(acc[busy].mean()))


def test_lens_step_edge_cases():
    print("lens edge cases", flush=True)
    # no chains
    L = _dev(make_luminance(64, 40, seed=1))
    lam = _dev(np.zeros(4))
    region, alpha = ops.lens_chain_step(L, 0.5, lam, 2, _dev(np.zeros((0, 3), np.float32)),
                                        _dev(np.zeros((0, 3), np.float32)))
    assert region.numel() == 0 and alpha.numel() == 0
    # a black image: every proposal inside the frame is accepted, every one outside rejected;
    # NaN luminance: alpha NaN and no move, on both sides
    for name, img in (("black", np.zeros((40, 64), np.float32)),
                      ("nan", np.where(np.arange(64 * 40).reshape(40, 64) % 7 == 0, np.nan, 1.0).astype(np.float32))):
        om = make_lens_chains(20_000, 64, 40, 0.5, seed=2)
        nz = make_lens_noise(20_000, seed=3)
        lam_h = np.array([-2.0, 0.0, -1.0, -3.0])
        g_alpha, ok = _compare(name, img, 0.5, lam_h, 2, om, nz)
        if name == "black":
            assert set(np.unique(g_alpha[ok]).tolist()) == {0.0, 1.0}
        else:
            assert np.isnan(g_alpha[ok]).any()
    # a one-row image with a wide field of view
    W, H, tx = 3000, 1, 2.0
    img = make_luminance(W, H, seed=4)
    lam_h = make_lambda_table(9, seed=5)
    _compare("one row", img, tx, lam_h, 3, make_lens_chains(50_000, W, H, tx, seed=6), make_lens_noise(50_000, seed=7))


def test_lens_carried_density_gives_the_same_steps():
    # carrying each chain's luminance between steps (read once, at the proposal) changes
    # nothing in the results: five steps with and without it agree bit for bit, and the
    # carried value is the luminance at the chain's pixel
    W, H, tx, N, n = 320, 200, 0.6, 20, 100_000
    print("lens carried density", flush=True)
    img = make_luminance(W, H, seed=8)
    L = _dev(img)
    lam = _dev(make_lambda_table(N * N, seed=9))
    om_a = _dev(make_lens_chains(n, W, H, tx, seed=10))
    om_b = om_a.clone()
    dens = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    for r in range(5):
        nz = _dev(make_lens_noise(n, seed=11, batch=r))
        ra, aa = ops.lens_chain_step(L, tx, lam, N, om_a, nz)
        rb, ab = ops.lens_chain_step(L, tx, lam, N, om_b, nz, density=dens)
        torch.cuda.synchronize()
        assert torch.equal(ra, rb), r
        assert np.array_equal(aa.cpu().numpy(), ab.cpu().numpy(), equal_nan=True), r
        assert np.array_equal(om_a.cpu().numpy(), om_b.cpu().numpy(), equal_nan=True), r
    # the pixel of each final state by the header's raster map (float32, one rounding per
    # operation), a property of the GPU's own states rather than an oracle comparison
    w = om_b.cpu().numpy()
    f32 = np.float32
    ty = f32(float(f32(tx)) * H / W)
    with np.errstate(divide="ignore", invalid="ignore"):
        sx = f32(0.5) + f32(0.5) * ((w[:, 0] / w[:, 2]) / f32(tx))
        sy = f32(0.5) + f32(0.5) * ((w[:, 1] / w[:, 2]) / ty)
        inside = (w[:, 2] > 0) & (sx >= 0) & (sx < 1) & (sy >= 0) & (sy < 1)
    ix = np.minimum((np.where(inside, sx, 0) * f32(W)).astype(np.int64), W - 1)
    iy = np.minimum((np.where(inside, sy, 0) * f32(H)).astype(np.int64), H - 1)
    d = dens.cpu().numpy()
    assert np.array_equal(d[inside], img[iy[inside], ix[inside]]) and np.all(d[~inside] == -1.0)


@pytest.mark.parametrize("W,H,N", [(320, 200, 20), (1920, 1080, 20), (77, 45, 3), (1, 1, 1)])
def test_lens_carried_pixel_gives_the_same_steps(W, H, N):
    # carrying each chain's pixel between steps (no raster map of the current state) changes
    # nothing in the results: five steps with the pixel (and with pixel and luminance) agree
    # bit for bit with five steps without either, chains outside the frame and NaN states
    # included; entries below -1 or past the image are taken from the raster map
    tx, n = 0.6, 100_003
    print(f"lens carried pixel W={W} H={H} N={N}", flush=True)
    L = _dev(make_luminance(W, H, seed=12))
    lam = _dev(make_lambda_table(N * N, seed=13))
    om0 = make_lens_chains(n, W, H, tx, seed=14)
    om0[:50] = [0.0, 0.0, -1.0]          # behind the camera
    om0[50:60] = [np.nan, 0.0, 1.0]
    om0[60:70] = [5.0, 0.0, 1.0]         # outside the field of view
    om_a, om_b, om_c = _dev(om0), _dev(om0), _dev(om0)
    pix_b = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    pix_b[1::7] = W * H + 5              # past the image: recomputed as well
    pix_c = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    dens_c = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    for r in range(5):
        nz = _dev(make_lens_noise(n, seed=15, batch=r))
        ra, aa, pa = ops.lens_chain_step(L, tx, lam, N, om_a, nz, want_proposals=True)
        rb, ab, pb = ops.lens_chain_step(L, tx, lam, N, om_b, nz, want_proposals=True, pixel=pix_b)
        rc, ac = ops.lens_chain_step(L, tx, lam, N, om_c, nz, density=dens_c, pixel=pix_c)
        torch.cuda.synchronize()
        for rr, aa2 in ((rb, ab), (rc, ac)):
            assert torch.equal(ra, rr), r
            assert np.array_equal(aa.cpu().numpy(), aa2.cpu().numpy(), equal_nan=True), r
        assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy(), equal_nan=True), r
        for o in (om_b, om_c):
            assert np.array_equal(om_a.cpu().numpy(), o.cpu().numpy(), equal_nan=True), r
    # the carried pixel is the oracle's raster map of each final state
    inside, ix, iy = olc.raster(om_a.cpu().numpy(), W, H, tx)
    want = np.where(inside, iy * W + ix, -1)
    assert np.array_equal(pix_b.cpu().numpy(), want) and np.array_equal(pix_c.cpu().numpy(), want)
    assert (want[:70] == -1).all() and (ra[:70] == -1).all()


@pytest.mark.parametrize("W,H,n", [(1920, 1080, 300_037), (3840, 2160, 70_001), (100, 40, 4097), (1, 1, 5000),
                                   (640, 360, 1), (640, 360, 0), (1000, 1000, 4096)])
def test_lens_chain_sort_matches_the_stable_tile_order(W, H, n):
    # the reorder groups chains by the screen tile of their pixel (oracle.lens_chain.tile_order:
    # float32 raster map, stable sort): order, directions and carried luminance bit for bit
    print(f"lens sort W={W} H={H} n={n}", flush=True)
    tx = 0.6
    omega = make_lens_chains(max(n, 1), W, H, tx, seed=n + 1)[:n]
    rng = np.random.default_rng(n)
    dens = rng.random(n).astype(np.float32)
    dens[rng.random(n) < 0.1] = -1.0
    om2, d2, perm = ops.lens_chain_sort(_dev(omega), W, H, tx, density=_dev(dens))
    torch.cuda.synchronize()
    keys, want = olc.tile_order(omega, W, H, tx)
    assert np.array_equal(perm.cpu().numpy(), want)
    assert np.array_equal(om2.cpu().numpy(), omega[want], equal_nan=True)
    assert np.array_equal(d2.cpu().numpy(), dens[want])
    if n > 1:  # a key per tile, non-decreasing
        assert np.all(np.diff(keys[want]) >= 0)


def test_lens_step_after_the_sort_is_the_permuted_step():
    # chains are independent: the step of the reordered chains (with their noise reordered
    # the same way) is the reordered step, bit for bit; the carried luminance moves along
    W, H, tx, N, n = 640, 360, 0.6, 20, 200_000
    L = _dev(make_luminance(W, H, seed=4))
    lam = _dev(make_lambda_table(N * N, seed=6))
    omega = _dev(make_lens_chains(n, W, H, tx, seed=7))
    noise = _dev(make_lens_noise(n, seed=8))
    dens = torch.full((n,), -1.0, device="cuda")
    ops.lens_chain_step(L, tx, lam, N, omega, noise, density=dens)  # the carried values are set
    om_s, dens_s, perm = ops.lens_chain_sort(omega, W, H, tx, density=dens)
    p = perm.long()
    noise_s = noise[p].contiguous()
    r1, a1 = ops.lens_chain_step(L, tx, lam, N, omega, noise, density=dens)
    r2, a2 = ops.lens_chain_step(L, tx, lam, N, om_s, noise_s, density=dens_s)
    torch.cuda.synchronize()
    assert torch.equal(r2, r1[p]) and torch.equal(a2.isnan(), a1[p].isnan())
    assert torch.equal(torch.nan_to_num(a2, 7.0), torch.nan_to_num(a1[p], 7.0))
    assert torch.equal(om_s.isnan(), omega[p].isnan())
    assert torch.equal(torch.nan_to_num(om_s, 7.0), torch.nan_to_num(omega[p], 7.0))
    assert torch.equal(dens_s, dens[p])
