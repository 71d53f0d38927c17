"""Pins of the lens-perturbation chain oracle (oracle/lens_chain.py; Sec. 3.3 lens
perturbation, Sec. 6.1 screen partition, Alg. 1 lines 8-13): the raster map against pixel
centres and the frame's edges; the Metropolis step's stationary distribution against the
closed form (luminance times each pixel's solid angle, by the exact rectangle formula) with a
chi-square test; the degenerate cases (tiny sigma, states outside the frame, black
pixels); and, closing the loop with the adaptation, the direction of the lambda update."""

import math

import numpy as np

from oracle import lens_chain as lc
from oracle.regional_filter import region_index

F32 = np.float32


def test_raster_round_trip_and_frame_edges():
    W, H, tx = 7, 5, 0.6
    d = lc.pixel_centre_directions(W, H, tx)
    inside, ix, iy = lc.raster(d, W, H, tx)
    assert inside.all()
    assert np.array_equal(iy * W + ix, np.arange(W * H))
    # behind the camera, on the axis plane, outside the field of view, NaN
    w = np.array([[0, 0, -1], [0.1, 0, 0], [0.7, 0, 1], [0, 0.5, 1], [np.nan, 0, 1], [0, 0, 1]], dtype=F32)
    inside, ix, iy = lc.raster(w, W, H, tx)
    assert inside.tolist() == [False, False, False, False, False, True]
    assert (ix[-1], iy[-1]) == (W // 2, H // 2)
    # the solid angles of the pixels add up to the frame's: 4 asin(sin a sin b), a, b the half angles
    a, b = math.atan(float(F32(tx))), math.atan(float(lc.tan_half_y(tx, W, H)))
    assert abs(lc.pixel_solid_angles(W, H, tx).sum() - 4 * math.asin(math.sin(a) * math.sin(b))) < 1e-12


def test_stationary_distribution_is_luminance_times_solid_angle():
    # Independent chains with a fixed sigma: after burn-in the pixel of each chain is drawn
    # from pi(omega) = L(pixel) over directions, i.e. P(pixel j) = L_j Omega_j / sum L Omega.
    W, H, tx, N = 6, 4, 0.8, 2
    rng = np.random.default_rng(11)
    L = rng.uniform(0.2, 3.0, size=(H, W)).astype(F32)
    L[1, 2] = 0.0                          # a black pixel: never entered
    lam = np.full(N * N, math.log(0.3 ** 2))
    n, steps = 20000, 150
    start = rng.choice(np.flatnonzero(L.ravel() > 0), size=n)
    omega = lc.pixel_centre_directions(W, H, tx)[start]
    for _ in range(steps):
        noise = rng.random((n, 3)).astype(F32)
        omega, region, alpha, _ = lc.step(L, tx, lam, N, omega, noise)
    inside, ix, iy = lc.raster(omega, W, H, tx)
    assert inside.all()
    counts = np.bincount(iy * W + ix, minlength=W * H)
    p = (L.astype(np.float64) * lc.pixel_solid_angles(W, H, tx)).ravel()
    p /= p.sum()
    assert counts[1 * W + 2] == 0
    live = p > 0
    chi2 = float((((counts - n * p) ** 2)[live] / (n * p[live])).sum())
    assert chi2 < 49.7, chi2                # 23 degrees of freedom, 0.1 % critical value
    # a Metropolis ratio taken the wrong way round, or luminance alone, is far off
    q = (1.0 / np.where(L > 0, L, np.inf)).ravel() * lc.pixel_solid_angles(W, H, tx).ravel()
    q /= q.sum()
    assert float((((counts - n * q) ** 2)[live] / (n * q[live])).sum()) > 1000
    r = L.astype(np.float64).ravel() / L.sum()
    assert float((((counts - n * r) ** 2)[live] / (n * r[live])).sum()) > 100


def test_degenerate_cases():
    W, H, tx, N = 8, 6, 0.5, 3
    rng = np.random.default_rng(3)
    L = rng.uniform(0.5, 2.0, size=(H, W)).astype(F32)
    L[0, 0] = 0.0
    d = lc.pixel_centre_directions(W, H, tx)
    noise = rng.random((d.shape[0], 3)).astype(F32)
    # sigma = e^-15: the proposal stays in the pixel and is always accepted
    nxt, region, alpha, prop = lc.step(L, tx, np.full(N * N, -30.0), N, d, noise)
    assert np.all(alpha == 1) and np.allclose(nxt, d, atol=1e-6)
    assert np.array_equal(region, region_index(W, H, N).ravel())
    # states outside the frame: no region, alpha NaN, no move
    bad = np.array([[0, 0, -1], [np.nan, 0, 1], [0.9, 0, 0.1]], dtype=F32)
    nxt, region, alpha, prop = lc.step(L, tx, np.zeros(N * N), N, bad, rng.random((3, 3)).astype(F32))
    assert region.tolist() == [-1, -1, -1] and np.all(np.isnan(alpha)) and np.all(np.isnan(prop))
    assert np.array_equal(nxt, bad, equal_nan=True)
    # a black current pixel accepts any proposal inside the frame; outside the frame, alpha = 0
    one = d[:1]
    nxt, region, alpha, prop = lc.step(L, tx, np.zeros(N * N), N, np.repeat(one, 200, 0),
                                       rng.random((200, 3)).astype(F32))
    ins, _, _ = lc.raster(prop, W, H, tx)
    assert np.all(alpha[ins] == 1) and np.all(alpha[~ins] == 0) and (~ins).any()


def test_closed_loop_pins_the_direction_of_the_update():
    # Reading A2: eq. update_lambda raises lambda when the estimated acceptance is above the
    # target, while the prose states the opposite. Closing the loop with the lens chains shows
    # which one adapts: with the equation every region settles near alpha* = 1/2; with the
    # prose's direction (the same update fed 1 - alpha, which flips sgn(alpha_hat - 1/2)) the
    # scales run away (here upwards, from an initial sigma of 1.6 rad that already accepts
    # less than half) and the acceptance with them.
    from oracle import region_adapt as ora

    W, H, tx, N, n, rounds = 64, 40, 0.5, 2, 8192, 60
    rng = np.random.default_rng(21)
    L = rng.uniform(0.2, 3.0, size=(H, W)).astype(F32)

    def run(flip):
        st = ora.initial_state(N * N)
        omega = lc.pixel_centre_directions(W, H, tx)[rng.integers(0, W * H, n)]
        acc = np.zeros(N * N)
        cnt = np.zeros(N * N)
        for r in range(rounds):
            omega, region, alpha, _ = lc.step(L, tx, st["lambda"], N, omega, rng.random((n, 3)).astype(F32))
            ora.adapt(st, region, (F32(1) - alpha) if flip else alpha, L=10)
            if r >= rounds - 20:
                ok = region >= 0
                np.add.at(acc, region[ok], alpha[ok])
                np.add.at(cnt, region[ok], 1)
        return acc / np.maximum(cnt, 1), st["lambda"]

    acc, lam = run(False)
    assert np.all(np.abs(acc - 0.5) < 0.1), (acc, lam)
    with np.errstate(over="ignore", invalid="ignore"):
        acc_f, lam_f = run(True)
    assert np.all(np.abs(acc_f - 0.5) > 0.4) and np.all(np.abs(lam_f) > 20), (acc_f, lam_f)


def test_tile_order_of_the_chain_reorder():
    # tile side: the smallest power of two >= 16 leaving at most 63 tiles
    assert lc.sort_tile_side(1920, 1080) == 256  # 8 x 5 = 40 tiles (128: 15 x 9 = 135)
    assert lc.sort_tile_side(3840, 2160) == 512
    assert lc.sort_tile_side(16, 16) == 16 and lc.sort_tile_side(1, 1) == 16
    assert lc.sort_tile_side(65536, 65536) == 16384  # 4 x 4 (8192: 8 x 8 = 64 tiles)
    assert lc.sort_tile_side(16 * 63, 16) == 16 and lc.sort_tile_side(16 * 64, 16) == 32
    # chains through known pixel centres, in a shuffled order, with some outside the frame:
    # the keys are the tiles of those pixels, written out by hand, and the order is the one a
    # stable insertion sort by key gives
    W, H, tx = 100, 40, 0.6
    T = lc.sort_tile_side(W, H)
    assert T == 16  # 7 x 3 tiles
    d = lc.pixel_centre_directions(W, H, tx)
    rng = np.random.default_rng(3)
    pick = rng.integers(0, W * H, 500)
    om = d[pick].copy()
    out = rng.random(500) < 0.05
    om[out] = [0.0, 0.0, -1.0]
    om[7] = [np.nan, 0.0, 1.0]
    out[7] = True
    keys, perm = lc.tile_order(om, W, H, tx)
    px, py = pick % W, pick // W
    want = np.where(out, 7 * 3, (py // 16) * 7 + px // 16)
    assert np.array_equal(keys, want)
    order = []  # stable insertion sort
    for i in range(len(want)):
        j = len(order)
        while j > 0 and want[order[j - 1]] > want[i]:
            j -= 1
        order.insert(j, i)
    assert np.array_equal(perm, order)
