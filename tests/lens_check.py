"""Checks of one step of lens-perturbation chains (Sec. 3.3 "Lens Perturbation", Sec. 6.1,
Alg. 1 lines 8-13) computed elsewhere against the oracle's step on the same inputs.

Several results can be correct for one chain: the proposal omega' is compared within a
bound (DIR_TOL per component: float32 trigonometry and frame against the fp64 sampler), and a
proposal that close to a pixel edge, or to the frame edge, may land in either pixel, or
outside. Everything that follows from omega' (its pixel, alpha, the move) is therefore
checked in two ways:

* exactly, against the oracle's decision taken on the checked proposal itself
  (``oracle.lens_chain.acceptance``: float32, one rounding per operation on both sides);
* against the set of values that every float32 direction within DIR_TOL of the ORACLE's
  proposal can give: min(1, L[q] / L[p]) for each pixel q the box of such directions can
  reach, and 0 where it can reach outside the frame. Where the set holds one value the
  alpha must be that value; the chains with more than one (near an edge) are counted.

The second check uses nothing the checked side produced to choose the candidates.
"""

import numpy as np

from oracle import lens_chain as olc

DIR_TOL = 4e-6
F32 = np.float32
# float32 rounding of the raster map (a division, a quotient by tx, a sum, a product by W),
# as an absolute bound on sx or sy in [0, 1]: far above the few ulps those operations make
RASTER_SLACK = 2.0 ** -20


def _tangent_range(a, z, tol):
    """Interval of a' / z' over |a' - a| <= tol, |z' - z| <= tol, for z - tol > 0 (the
    quotient is monotone in each argument there, so the extremes are at the corners)."""
    c = np.stack([(a - tol) / (z - tol), (a - tol) / (z + tol), (a + tol) / (z - tol), (a + tol) / (z + tol)])
    return c.min(axis=0), c.max(axis=0)


def candidate_boxes(o_prop, W, H, tan_half_x, tol=DIR_TOL):
    """For each oracle proposal [n, 3]: (ix_lo, ix_hi, iy_lo, iy_hi, may_be_inside,
    may_be_outside) over every direction within ``tol`` of it per component. A pixel range
    is empty where the proposal cannot be inside the frame."""
    o = np.asarray(o_prop, dtype=np.float64)
    n = o.shape[0]
    tx = float(F32(tan_half_x))
    ty = float(olc.tan_half_y(tan_half_x, W, H))
    x, y, z = o[:, 0], o[:, 1], o[:, 2]
    front = z - tol > 0
    zz = np.where(front, z, 1.0)
    qx_lo, qx_hi = _tangent_range(x, zz, tol)
    qy_lo, qy_hi = _tangent_range(y, zz, tol)
    sx_lo = 0.5 + 0.5 * qx_lo / tx - RASTER_SLACK
    sx_hi = 0.5 + 0.5 * qx_hi / tx + RASTER_SLACK
    sy_lo = 0.5 + 0.5 * qy_lo / ty - RASTER_SLACK
    sy_hi = 0.5 + 0.5 * qy_hi / ty + RASTER_SLACK
    inside = front & (sx_hi >= 0) & (sx_lo < 1) & (sy_hi >= 0) & (sy_lo < 1)
    outside = ~front | (sx_lo < 0) | (sx_hi >= 1) | (sy_lo < 0) | (sy_hi >= 1)
    # at or behind the image plane's horizon: outside unless the tangent can still be in
    # the frame (impossible for a unit direction with z this small; reported as undecided)
    undecided = ~front & (z + tol > 0) & (np.abs(x) - tol <= tx * (z + tol)) & (np.abs(y) - tol <= ty * (z + tol))
    if undecided.any():
        raise AssertionError(f"{int(undecided.sum())} proposals at the horizon: the box check cannot decide them")
    ix_lo = np.clip(np.floor(sx_lo * W), 0, W - 1).astype(np.int64)
    ix_hi = np.clip(np.floor(sx_hi * W), 0, W - 1).astype(np.int64)
    iy_lo = np.clip(np.floor(sy_lo * H), 0, H - 1).astype(np.int64)
    iy_hi = np.clip(np.floor(sy_hi * H), 0, H - 1).astype(np.int64)
    assert ix_lo.shape == (n,)
    return ix_lo, ix_hi, iy_lo, iy_hi, inside, outside


def candidate_alphas(L, tan_half_x, omega, o_prop, tol=DIR_TOL):
    """(single [n] float32, multi {i: tuple}) for chains whose state is inside the frame:
    single[i] is the one alpha every proposal within ``tol`` of the oracle's gives (NaN where
    there is more than one, listed in ``multi`` as the sorted tuple of all of them)."""
    L = np.asarray(L, dtype=F32)
    H, W = L.shape
    inside_p, px, py = olc.raster(omega, W, H, tan_half_x)
    assert inside_p.all(), "candidates are for chains inside the frame"
    ix_lo, ix_hi, iy_lo, iy_hi, may_in, may_out = candidate_boxes(o_prop, W, H, tan_half_x, tol)
    cur = L[py, px]
    one_px = may_in & ~may_out & (ix_lo == ix_hi) & (iy_lo == iy_hi)
    single = np.full(omega.shape[0], np.nan, dtype=F32)
    single[one_px] = olc.ratio(L[iy_lo[one_px], ix_lo[one_px]], cur[one_px])
    single[~may_in & may_out] = 0.0
    multi = {}
    for i in np.flatnonzero(~one_px & may_in):
        vals = {0.0} if may_out[i] else set()
        block = L[iy_lo[i]:iy_hi[i] + 1, ix_lo[i]:ix_hi[i] + 1].ravel()
        vals.update(float(v) for v in olc.ratio(block, np.full(block.shape, cur[i], F32)))
        nan = any(np.isnan(v) for v in vals)
        vals = sorted(v for v in vals if not np.isnan(v)) + ([float("nan")] if nan else [])
        if len(vals) == 1:
            single[i] = vals[0]  # several pixels, one value: decided all the same
        else:
            multi[int(i)] = tuple(vals)
    return single, multi


def _alpha_in(a, cands):
    a = float(a)
    return any((np.isnan(a) and np.isnan(c)) or a == c for c in cands)


def check_step(L, tan_half_x, omega, noise, oracle, checked, tol=DIR_TOL, edge_budget=0.05, name=""):
    """Compare one step. ``oracle`` = (next, region, alpha, prop) of ``oracle.lens_chain.step``
    on (omega, noise); ``checked`` = the same four arrays from the side under test. Raises
    AssertionError on any mismatch; returns the number of chains near an edge (more than one
    possible alpha).

    The share of such chains is a property of the inputs and the bound, not of the checked
    side: a proposal within tol per component moves its tangent x / z by up to ~2 tol in the
    frame, so at 1920 px across tan = 0.6 (pixels 6.25e-4 wide in the tangent) about 2.4 % of
    the proposals lie that close to a vertical pixel edge. ``edge_budget`` only guards against
    a candidate check that has become vacuous."""
    o_next, o_region, o_alpha, o_prop = oracle
    g_next, g_region, g_alpha, g_prop = checked
    omega = np.asarray(omega, dtype=F32)
    u_acc = np.asarray(noise, dtype=F32)[:, 2]
    # region of the current state: exact; no region -> alpha NaN, proposal NaN, no move
    assert np.array_equal(g_region, o_region), (name, "region")
    valid = o_region >= 0
    assert np.all(np.isnan(g_alpha[~valid])) and np.all(np.isnan(g_prop[~valid])), (name, "invalid chains")
    assert np.array_equal(g_next[~valid], omega[~valid], equal_nan=True), (name, "invalid chains moved")
    # the proposals, within the direction bound
    err = np.abs(g_prop[valid].astype(np.float64) - o_prop[valid])
    assert err.size == 0 or float(err.max()) <= tol, (name, "proposal", float(err.max()))
    # alpha: the oracle's decision on the checked proposal, exactly
    a_own = olc.acceptance(L, tan_half_x, omega[valid], g_prop[valid])
    assert np.array_equal(g_alpha[valid], a_own, equal_nan=True), (name, "alpha of the proposal")
    # alpha: one of the values a proposal within the bound of the oracle's can give
    single, multi = candidate_alphas(L, tan_half_x, omega[valid], o_prop[valid], tol)
    ga = g_alpha[valid]
    oa = o_alpha[valid]
    one = np.ones(ga.shape, dtype=bool)
    one[list(multi)] = False
    assert np.array_equal(oa[one], single[one], equal_nan=True), (name, "oracle alpha outside its candidates")
    bad = np.flatnonzero(one & ~((ga == single) | (np.isnan(ga) & np.isnan(single))))
    assert bad.size == 0, (name, "alpha differs where only one value is possible", int(np.flatnonzero(valid)[bad[0]]),
                           float(ga[bad[0]]), float(single[bad[0]]))
    for i, c in multi.items():
        assert _alpha_in(oa[i], c), (name, "oracle alpha outside its own candidates", i)
        assert _alpha_in(ga[i], c), (name, "alpha outside the candidates", int(np.flatnonzero(valid)[i]), ga[i], c)
    n_edge = len(multi)
    # the move: taken iff the uniform is below the checked alpha, to the checked proposal
    mv = valid & (u_acc < g_alpha)
    stay = valid & ~mv
    assert np.array_equal(g_next[mv], g_prop[mv]), (name, "move")
    assert np.array_equal(g_next[stay], omega[stay], equal_nan=True), (name, "stay")
    assert n_edge <= max(20, edge_budget * valid.sum()), (name, "near-edge chains", n_edge)
    return n_edge
