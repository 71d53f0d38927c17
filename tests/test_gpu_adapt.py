"""GPU parity of region_adapt (regional adaptation, Algorithm 1) against the sequential
FP64 oracle: integer state and every update decision exactly, A_k exactly (the same fp64
additions in the same order), lambda_k within the rounding bound of summing its updates
in a different association (lambda_tol), on streams spanning one to three radix passes
(both paths: the single-pass one of grids under 512 regions and the multi-pass one),
several batches in a row, and the edge cases (L = 1, one region, out-of-range keys,
acceptance exactly at the target, NaN acceptance, empty batches)."""

import numpy as np
import pytest
import torch

from oracle import region_adapt as ora
from paper_2402_08273_amd.ops import RegionAdapter
from synth.proposals import make_proposals

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def lambda_tol(updates):
    """|lambda_gpu - lambda_oracle| bound for a region that applied `updates` window updates
    in the batch: both sum the same deltas (|delta| <= gamma_max = 1) in fp64, the oracle
    one after another, the GPU in up to 64 blocks then block by block, so each side's
    rounding error is at most (updates + 1) ulp of a partial sum of magnitude
    <= |lambda_0| + updates <= 31 + updates."""
    u = np.asarray(updates, dtype=np.float64)
    return 2.0 * (u + 1.0) * (31.0 + u) * 2.0 ** -52 + 1e-15


def _compare(name, ad, st, regions=None, updates_before=None, extra=0):
    """State of the GPU adapter against the oracle's; ``extra`` roundings (one per batch
    folded into lambda) are added to the lambda bound."""
    torch.cuda.synchronize()
    sel = slice(None) if regions is None else regions
    vis = ad.visits.cpu().numpy()[sel]
    upd = ad.updates.cpu().numpy()[sel]
    acc = ad.acc.cpu().numpy()[sel]
    lam = ad.lam.cpu().numpy()[sel]
    lam32 = ad.lam_f32.cpu().numpy()[sel]
    assert np.array_equal(vis, st["visits"][sel]), name
    assert np.array_equal(upd, st["updates"][sel]), name
    assert np.array_equal(acc, st["acc"][sel]), (name, np.abs(acc - st["acc"][sel]).max())
    before = 1 if updates_before is None else updates_before[sel]
    err = np.abs(lam - st["lambda"][sel])
    tol = lambda_tol(st["updates"][sel] - before + extra)
    assert np.all(err <= tol), (name, float(err.max()), float(tol.min()))
    assert np.array_equal(lam32, lam.astype(np.float32)), name


# m < 512 takes the single-pass path (8-bit keys up to m = 255, 9-bit from 256 to 511);
# m = 512 is the first grid of the multi-pass path
@pytest.mark.parametrize("m,n,L,batches", [(1, 50, 1, 2), (5, 997, 2, 3), (400, 200_000, 10, 3),
                                           (3000, 150_000, 37, 2), (70_000, 300_000, 10, 2),
                                           (20, 80_000, 64, 2), (20, 80_000, 65, 2), (7, 300_000, 1000, 2),
                                           (255, 100_000, 3, 2), (256, 100_000, 10, 2), (511, 100_000, 1, 2),
                                           (512, 100_000, 10, 2)])
def test_region_adapt_parity(m, n, L, batches):
    print(f"region_adapt parity m={m} n={n} L={L} batches={batches}", flush=True)
    ad = RegionAdapter(m, L=L)
    st = ora.initial_state(m)
    for b in range(batches):
        region, alpha = make_proposals(n, m, seed=m + L, batch=b)
        ad.step(_dev(region), _dev(alpha))
        ora.adapt(st, region, alpha, L=L)
        # the two run on their own: every update decision depends on alpha and n_k only, so
        # lambda differs by rounding alone, the updates since the start plus one per batch
        _compare(f"m={m} batch {b}", ad, st, extra=b + 1)


@pytest.mark.parametrize("m,n,L", [(1 << 24, 400_000, 10), (2, 2_500_000, 1 << 20)])
def test_region_adapt_maximum_sizes(m, n, L):
    # the most regions (24-bit keys: three radix passes) and the longest windows (2^20
    # visits summed in order in fp64 before an update)
    print(f"region_adapt maximum sizes m={m} n={n} L={L}", flush=True)
    region, alpha = make_proposals(n, m, seed=17)
    ad = RegionAdapter(m, L=L)
    ad.step(_dev(region), _dev(alpha))
    st = ora.adapt(ora.initial_state(m), region, alpha, L=L)
    assert int(st["updates"].max()) >= 2
    _compare(f"maximum m={m} L={L}", ad, st)


def test_region_adapt_edge_cases():
    m, L = 4, 3
    ad = RegionAdapter(m, L=L)
    st = ora.initial_state(m)
    cases = [
        (np.array([], np.int32), np.array([], np.float32)),                     # empty batch
        (np.array([-5, 4, 99, -1], np.int32), np.array([0.9] * 4, np.float32)),  # all out of range
        (np.array([0, 0, 0, 1, 1, 1], np.int32), np.array([0.5] * 6, np.float32)),  # mean == target: sgn 0
        (np.array([2, 2, 2], np.int32), np.array([np.nan, 0.9, 0.9], np.float32)),  # NaN: sgn 0
        (np.array([3] * 31, np.int32), np.full(31, 0.0625, np.float32)),         # many updates, one region
    ]
    for i, (region, alpha) in enumerate(cases):
        ad.step(_dev(region), _dev(alpha))
        ora.adapt(st, region, alpha, L=L)
        torch.cuda.synchronize()
        vis, upd = ad.visits.cpu().numpy(), ad.updates.cpu().numpy()
        acc, lam = ad.acc.cpu().numpy(), ad.lam.cpu().numpy()
        assert np.array_equal(vis, st["visits"]) and np.array_equal(upd, st["updates"]), i
        # NaN propagates into a pending A_k on both sides; compare with NaN == NaN
        assert np.array_equal(acc, st["acc"], equal_nan=True), i
        assert np.all(np.abs(lam - st["lambda"]) <= lambda_tol(st["updates"])), i


def test_region_adapt_batches_compose_on_gpu():
    m, n = 400, 120_000
    region, alpha = make_proposals(n, m, seed=11)
    one = RegionAdapter(m)
    one.step(_dev(region), _dev(alpha))
    two = RegionAdapter(m)
    two.step(_dev(region[:50_001]), _dev(alpha[:50_001]))
    two.step(_dev(region[50_001:]), _dev(alpha[50_001:]))
    torch.cuda.synchronize()
    for a, b in [(one.acc, two.acc), (one.visits, two.visits), (one.updates, two.updates)]:
        assert torch.equal(a, b)
    tol = torch.from_numpy(lambda_tol(one.updates.cpu().numpy())).cuda()
    assert torch.all((one.lam - two.lam).abs() <= tol)


@pytest.mark.slow
@pytest.mark.parametrize("m", [400, 20 * 20 * 50 * 50])
def test_region_adapt_full_size_sampled_regions(m):
    # 16 M proposals, the bench's launch configuration; regions are independent, so the
    # oracle replays the sub-streams of sampled regions (each in its own order)
    n = 1 << 24
    print(f"region_adapt full size m={m} n={n}", flush=True)
    region, alpha = make_proposals(n, m, seed=3)
    ad = RegionAdapter(m)
    ad.step(_dev(region), _dev(alpha))
    counts = np.bincount(region[(region >= 0) & (region < m)], minlength=m)
    picks = np.unique(np.concatenate([[0, 1, m - 1], np.argsort(counts)[-3:],
                                      np.random.default_rng(0).integers(0, m, 8)]))
    st = ora.initial_state(m)
    for k in picks:
        sel = region == k
        ora.adapt(st, region[sel], alpha[sel])
    _compare(f"full size m={m}", ad, st, regions=picks)
