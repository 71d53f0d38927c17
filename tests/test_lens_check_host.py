"""The lens-step checker (tests/lens_check.py) on the CPU: it accepts a correct step whose
proposals differ from the oracle's within the direction bound, and it catches a wrong alpha
at a pixel edge, at the frame edge and for a proposal clearly outside the frame (Sec. 3.3
"Lens Perturbation": a proposal outside the frame is rejected, alpha = 0)."""

import numpy as np
import pytest

from oracle import lens_chain as olc
from synth.directions import make_lambda_table
from synth.lens import make_lens_chains, make_lens_noise, make_luminance
import lens_check as lc

F32 = np.float32
W, H, TX, N = 96, 60, 0.6, 4


def _step(omega, noise, lam, L=None):
    L = make_luminance(W, H, seed=11) if L is None else L
    return L, olc.step(L, TX, lam, N, omega, noise)


def _nudged(L, omega, noise, o, seed=0, size=1.5e-6):
    """A correct step whose proposals differ from the oracle's by up to ``size`` per
    component: alpha and the move re-decided on the nudged proposals."""
    o_next, o_region, o_alpha, o_prop = o
    rng = np.random.default_rng(seed)
    valid = o_region >= 0
    prop = o_prop.copy()
    prop[valid] = (o_prop[valid] + rng.uniform(-size, size, o_prop[valid].shape)).astype(F32)
    alpha = o_alpha.copy()
    alpha[valid] = olc.acceptance(L, TX, omega[valid], prop[valid])
    nxt = omega.copy()
    mv = valid & (noise[:, 2] < alpha)
    nxt[mv] = prop[mv]
    return [nxt, o_region.copy(), alpha, prop]


def _edge_chains(n, sx_edge, sy, lam_region_value=-30.0):
    """Chains just inside the frame at raster x = sx_edge (every row position sy), with a
    region scale so small that their proposals stay within ~1e-6 of them."""
    tx = float(F32(TX))
    ty = float(olc.tan_half_y(TX, W, H))
    d = np.stack([np.full(n, (2.0 * sx_edge - 1.0) * tx), (2.0 * sy - 1.0) * ty, np.ones(n)], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    lam = np.full(N * N, lam_region_value)
    return d.astype(F32), lam


def test_checker_accepts_correct_steps_near_edges():
    lam = make_lambda_table(N * N, seed=3)
    omega = make_lens_chains(60_000, W, H, TX, seed=4)
    noise = make_lens_noise(60_000, seed=5)
    L, o = _step(omega, noise, lam)
    g = _nudged(L, omega, noise, o)
    n_edge = lc.check_step(L, TX, omega, noise, o, g, name="nudged")
    assert n_edge > 0  # some proposals lie within the bound of a pixel edge
    # the oracle's own step passes as well
    lc.check_step(L, TX, omega, noise, o, [a.copy() for a in o], name="self")


def test_checker_catches_a_wrong_alpha_at_a_pixel_edge():
    lam = make_lambda_table(N * N, seed=3)
    omega = make_lens_chains(60_000, W, H, TX, seed=4)
    noise = make_lens_noise(60_000, seed=5)
    L, o = _step(omega, noise, lam)
    valid = o[1] >= 0
    single, multi = lc.candidate_alphas(L, TX, omega[valid], o[3][valid])
    vidx = np.flatnonzero(valid)
    _, px, py = olc.raster(omega, W, H, TX)
    planted = 0
    for i, cands in multi.items():
        if 0.0 in cands:
            continue  # a pixel edge inside the frame
        j = vidx[i]
        # a wrong luminance index: the pixel two columns over from the oracle's proposal
        _, qx, qy = olc.raster(o[3][j:j + 1], W, H, TX)
        q = (int(qy[0]), int(min(qx[0] + 2, W - 1)) if qx[0] + 2 < W else int(qx[0] - 2))
        wrong = float(olc.ratio(L[q], L[py[j], px[j]]))
        if lc._alpha_in(wrong, cands):
            continue
        g = [a.copy() for a in o]
        g[2][j] = wrong
        g[0][j] = g[3][j] if noise[j, 2] < wrong else omega[j]
        with pytest.raises(AssertionError, match="alpha"):
            lc.check_step(L, TX, omega, noise, o, g, name="pixel edge")
        # the candidate check alone catches it too (it does not look at the checked proposal)
        s2, m2 = lc.candidate_alphas(L, TX, omega[valid], o[3][valid])
        assert not lc._alpha_in(wrong, m2[i])
        planted += 1
        if planted == 3:
            break
    assert planted == 3


def test_checker_catches_a_wrong_alpha_at_the_frame_edge():
    n = H
    sy = (np.arange(n) + 0.5) / n
    omega, lam = _edge_chains(n, 1.0 - 3e-7, sy)
    noise = make_lens_noise(n, seed=6)
    L = make_luminance(W, H, seed=12)
    L, o = _step(omega, noise, lam, L)
    inside, px, py = olc.raster(omega, W, H, TX)
    assert inside.all() and np.all(px == W - 1)
    valid = o[1] >= 0
    single, multi = lc.candidate_alphas(L, TX, omega[valid], o[3][valid])
    edge = [i for i, c in multi.items() if 0.0 in c]
    assert len(edge) > n // 2  # the box reaches both the last column and outside
    planted = 0
    for i in edge:
        j = np.flatnonzero(valid)[i]
        # plausible bugs: the column index wrapped to the start of the row, or the proposal's
        # pixel one column or one row off
        y, x = py[j], px[j]
        wrongs = [float(olc.ratio(L[q], L[y, x])) for q in ((y, 0), (y, x - 1), ((y + 1) % H, x), (y - 1, x))]
        wrongs = [v for v in wrongs if not lc._alpha_in(v, multi[i])]
        if not wrongs:
            continue
        wrong = wrongs[0]
        g = _nudged(L, omega, noise, o, seed=1, size=1e-7)
        g[2][j] = wrong
        g[0][j] = g[3][j] if noise[j, 2] < wrong else omega[j]
        with pytest.raises(AssertionError, match="alpha"):
            lc.check_step(L, TX, omega, noise, o, g, name="frame edge", edge_budget=1.0)
        planted += 1
    assert planted >= 5
    # and the correct step passes with every one of those chains at the edge
    lc.check_step(L, TX, omega, noise, o, _nudged(L, omega, noise, o, seed=2, size=1e-7), edge_budget=1.0)


def test_checker_catches_a_ratio_for_a_proposal_outside_the_frame():
    lam = make_lambda_table(N * N, seed=3)
    lam[:] = 5.0  # wide proposals: many leave the frame
    omega = make_lens_chains(20_000, W, H, TX, seed=7)
    noise = make_lens_noise(20_000, seed=8)
    L, o = _step(omega, noise, lam)
    valid = o[1] >= 0
    out_in, qx, qy = olc.raster(o[3], W, H, TX)
    _, px, py = olc.raster(omega, W, H, TX)
    far = np.flatnonzero(valid & ~out_in & (o[3][:, 2] > 0.1))
    assert far.size > 100
    # a plausible bug: the proposal's pixel clamped into the image instead of rejected
    tx = F32(TX)
    ty = olc.tan_half_y(TX, W, H)
    caught = 0
    for j in far[:20]:
        p = o[3][j]
        sx = F32(0.5) + F32(0.5) * ((p[0] / p[2]) / tx)
        sy = F32(0.5) + F32(0.5) * ((p[1] / p[2]) / ty)
        cx = int(np.clip(np.floor(sx * W), 0, W - 1))
        cy = int(np.clip(np.floor(sy * H), 0, H - 1))
        wrong = float(olc.ratio(L[cy, cx], L[py[j], px[j]]))
        if wrong == 0.0:
            continue
        g = [a.copy() for a in o]
        g[2][j] = wrong
        g[0][j] = g[3][j] if noise[j, 2] < wrong else omega[j]
        with pytest.raises(AssertionError, match="alpha"):
            lc.check_step(L, TX, omega, noise, o, g, name="outside")
        caught += 1
    assert caught >= 10


@pytest.mark.parametrize("kind", ["black", "nan"])
def test_checker_on_black_and_nan_images(kind):
    # a black image accepts every proposal inside the frame (alpha 1) and rejects the rest;
    # NaN luminance gives NaN alpha and no move: the checker takes NaN as a value of its own
    img = np.zeros((H, W), F32) if kind == "black" else \
        np.where(np.arange(W * H).reshape(H, W) % 7 == 0, np.nan, 1.0).astype(F32)
    lam = make_lambda_table(N * N, seed=9)
    omega = make_lens_chains(20_000, W, H, TX, seed=10)
    noise = make_lens_noise(20_000, seed=11)
    _, o = _step(omega, noise, lam, img)
    lc.check_step(img, TX, omega, noise, o, _nudged(img, omega, noise, o, seed=3), name=kind)
    g = [a.copy() for a in o]
    j = int(np.flatnonzero((o[1] >= 0) & ~np.isnan(o[2]))[0])
    g[2][j] = 0.5
    with pytest.raises(AssertionError, match="alpha"):
        lc.check_step(img, TX, omega, noise, o, g, name=kind)
