"""GPU parity of the quadtree partition (quadtree_init / quadtree_lookup / quadtree_refine)
against the pointer-based oracle: leaf of every point, visit counters, the node arrays after
every refinement and the node count exactly; with region adaptation in the loop, the region
state as in the region_adapt tests (integers and A_k exactly, lambda within the rounding
bound of the updates applied along the node's lineage). Edge cases: one tree and many,
points on square edges and corners, x or y = 1, NaN, invalid roots, empty batches,
lookups that do not count, capacity and depth limits, inconsistent links."""

import numpy as np
import pytest
import torch

from oracle import quadtree as oqt
from oracle import region_adapt as ora
from paper_2402_08273_amd import _abi
from paper_2402_08273_amd.ops import Quadtree, RegionAdapter
from synth.points import make_points
from synth.proposals import make_proposals
from synth.workloads import QUADTREE_2D, QUADTREE_4D

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def lambda_tol(updates):
    """Rounding bound of a lambda that summed `updates` window deltas (|delta| <= 1) in fp64
    in a different association than the oracle (see the region_adapt parity tests)."""
    u = np.asarray(updates, dtype=np.float64)
    return 2.0 * (u + 1.0) * (31.0 + u) * 2.0 ** -52 + 1e-15


def _arrays(t):
    torch.cuda.synchronize()
    n = t.n_nodes
    return n, t.child[:n].cpu().numpy(), t.depth[:n].cpu().numpy(), t.visits[:n].cpu().numpy()


def _check_tree(name, t, f):
    n, child, depth, visits = _arrays(t)
    assert n == len(f.nodes), (name, n, len(f.nodes))
    assert np.array_equal(child, np.asarray(f.child_array())), name
    assert np.array_equal(depth, np.asarray(f.depth_array())), name
    assert np.array_equal(visits, np.asarray(f.visits_array())), name


def _lookup_both(name, t, f, root, x, y, count=True):
    leaf = t.lookup(_dev(x), _dev(y), None if root is None else _dev(root), count=count)
    want = f.lookup_many(root, x, y, count=count)
    got = leaf.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (name, bad[:5], got[bad[:5]], want[bad[:5]])
    return got


@pytest.mark.parametrize("n_roots,capacity,n,m_split,rounds", [
    (1, 4096, 20_000, 100, 6),
    (3, 20_000, 50_000, 300, 6),
    (20, 20_000, 60_000, 60, 5),
    (400, 30_000, 120_000, 40, 4),
    (2, 40_000, 200_000, 5, 7),
    (100, 20_000, 80_000, 30, 4),
    (600, 30_000, 150_000, 30, 4),
])
def test_quadtree_growth_parity(n_roots, capacity, n, m_split, rounds):
    print(f"quadtree growth R={n_roots} cap={capacity} n={n} M_split={m_split}", flush=True)
    t = Quadtree(n_roots, capacity)
    f = oqt.Forest(n_roots, capacity)
    _check_tree("init", t, f)
    for r in range(rounds):
        root, x, y = make_points(n, n_roots, seed=11 + n_roots, batch=r)
        _lookup_both(f"refinement {r}", t, f, None if n_roots == 1 else root, x, y)
        _check_tree(f"visits {r}", t, f)
        t.refine(m_split)
        f.refine(m_split)
        _check_tree(f"refine {r}", t, f)
    assert len(f.nodes) > 4 * n_roots


def test_quadtree_with_region_adaptation():
    # the loop of the quadtree partition: lookups give the proposals' regions, the
    # regions adapt, and every refinement passes lambda and n_k / 4 to the children
    R, cap, n, m_split, L = 2, 8192, 60_000, 200, 10
    print(f"quadtree + region_adapt R={R} cap={cap} n={n}", flush=True)
    t = Quadtree(R, cap)
    ad = RegionAdapter(cap, L=L)
    f = oqt.Forest(R, cap)
    st = ora.initial_state(cap)
    applied = np.zeros(cap, dtype=np.int64)   # window updates applied along each lineage
    for r in range(6):
        root, x, y = make_points(n, R, seed=21, batch=r)
        _, alpha = make_proposals(n, 7, seed=22, batch=r)
        leaf = _lookup_both(f"refinement {r}", t, f, root, x, y)
        ad.step(_dev(leaf), _dev(alpha))
        before = st["updates"].copy()
        ora.adapt(st, leaf, alpha, L=L)
        applied += st["updates"] - before
        old = len(f.nodes)
        t.refine(m_split, ad)
        f.refine(m_split, st)
        _check_tree(f"refine {r}", t, f)
        for p, c in enumerate(f.child_array()[:old]):
            if c >= old:
                applied[c:c + 4] = applied[p]
        torch.cuda.synchronize()
        nn = len(f.nodes)
        for name, got in (("visits", ad.visits), ("updates", ad.updates), ("acc", ad.acc)):
            assert np.array_equal(got.cpu().numpy()[:nn], st[name][:nn]), (r, name)
        lam = ad.lam.cpu().numpy()[:nn]
        err = np.abs(lam - st["lambda"][:nn])
        tol = lambda_tol(applied[:nn] + r + 1)   # + one rounding per call along the lineage
        assert np.all(err <= tol), (r, float(err.max()))
        assert np.array_equal(ad.lam_f32.cpu().numpy()[:nn], lam.astype(np.float32)), r
    # the children took max(1, floor(n / 4)) updates and lambda from their parents
    assert int(st["updates"][R:len(f.nodes)].min()) >= 1
    assert len(f.nodes) > 50


def test_quadtree_capacity_limit():
    # 9 nodes of storage: the root's split (5 nodes) fits, then only one more split
    t = Quadtree(1, 9)
    f = oqt.Forest(1, 9)
    x = np.array([0.1, 0.6, 0.1, 0.6] * 10, dtype=np.float32)
    y = np.array([0.1, 0.1, 0.6, 0.6] * 10, dtype=np.float32)
    for r in range(3):
        _lookup_both(f"refinement {r}", t, f, None, x, y)
        t.refine(5)
        f.refine(5)
        _check_tree(f"refine {r}", t, f)
    assert t.n_nodes == 9 and f.child_array() == [1, 5, -1, -1, -1, -1, -1, -1, -1]


def test_quadtree_depth_limit():
    t = Quadtree(1, 200)
    f = oqt.Forest(1, 200)
    x = np.full(7, 0.3, dtype=np.float32)
    y = np.full(7, 0.7, dtype=np.float32)
    for r in range(oqt.MAX_DEPTH + 3):
        _lookup_both(f"refinement {r}", t, f, None, x, y)
        t.refine(0)
        f.refine(0)
    _check_tree("deep", t, f)
    assert t.n_nodes == 1 + 4 * oqt.MAX_DEPTH
    assert int(t.depth[:t.n_nodes].max()) == oqt.MAX_DEPTH


def test_quadtree_edge_points():
    t = Quadtree(3, 4096)
    f = oqt.Forest(3, 4096)
    for r in range(4):
        root, x, y = make_points(30_000, 3, seed=5, batch=r)
        _lookup_both(f"grow {r}", t, f, root, x, y)
        t.refine(50)
        f.refine(50)
    g = np.array([0.0, 0.25, 0.5, 0.75, 1.0, 0.125, 0.375, 1.0 - 2.0 ** -24, 2.0 ** -20], dtype=np.float32)
    xx, yy = np.meshgrid(g, g)
    x = np.concatenate([xx.ravel(), [np.nan, 0.5, -0.0, -1e-30, 1.0000001, np.inf, 0.3, 0.3]]).astype(np.float32)
    y = np.concatenate([yy.ravel(), [0.5, np.nan, 0.0, 0.5, 0.5, 0.5, 0.3, 0.3]]).astype(np.float32)
    root = np.resize(np.array([0, 1, 2], dtype=np.int32), x.size)
    root[-2:] = [-1, 3]
    got = _lookup_both("edges", t, f, root, x, y)
    assert got[-2] == -1 and got[-1] == -1 and got[-8] == -1 and got[-7] == -1   # invalid roots, NaN
    # count=False leaves the counters alone; an empty batch is a no-op
    before = t.visits.clone()
    _lookup_both("no count", t, f, root, x, y, count=False)
    empty = torch.empty(0, device="cuda", dtype=torch.float32)
    assert t.lookup(empty, empty).numel() == 0
    torch.cuda.synchronize()
    assert torch.equal(before, t.visits)
    _check_tree("after edges", t, f)
    # init restores the roots
    t.reset()
    n, child, depth, visits = _arrays(t)
    assert n == 3 and child.tolist() == [-1] * 3 and depth.tolist() == [0] * 3 and visits.tolist() == [0] * 3


def test_quadtree_inconsistent_links_give_no_region():
    # links that leave the stored nodes or cycle are answered with -1, within bounds
    t = Quadtree(1, 64)
    x = np.array([0.0, 0.7, 0.2, 0.7], dtype=np.float32)   # (0, 0) stays in quadrant 0 at every level
    y = np.array([0.0, 0.2, 0.7, 0.7], dtype=np.float32)
    t.lookup(_dev(x), _dev(y))
    t.refine(0)                                   # nodes 0..4
    t.child[1] = 1                                # node 1 claims itself as its first child
    t.child[2] = 3                                # node 2's children would run past n_nodes
    t.child[3] = 0                                # a root as a child
    got = t.lookup(_dev(x), _dev(y)).cpu().numpy()
    assert got.tolist() == [-1, -1, -1, 4]


@pytest.mark.slow
@pytest.mark.parametrize("wl", [QUADTREE_2D, QUADTREE_4D], ids=["2d", "4d"])
def test_quadtree_full_size(wl):
    # the bench's workload: the forest grown over its refinement rounds, then the timed
    # lookup batch, all compared in full
    R = wl["n_roots"]
    print(f"quadtree full size R={R} rounds={wl['rounds']}", flush=True)
    t = Quadtree(R, wl["capacity"])
    f = oqt.Forest(R, wl["capacity"])
    root, x, y = make_points(wl["grow_points"], R, seed=wl["seed"], batch=0)
    r_dev = None if R == 1 else _dev(root)
    x_dev, y_dev = _dev(x), _dev(y)
    for r in range(wl["rounds"]):
        leaf = t.lookup(x_dev, y_dev, r_dev)
        want = f.lookup_many(None if R == 1 else root, x, y)
        assert np.array_equal(leaf.cpu().numpy(), want), r
        t.refine(wl["m_split"])
        f.refine(wl["m_split"])
        _check_tree(f"refinement {r}", t, f)
    print(f"  nodes {len(f.nodes)} depth {max(f.depth_array())}", flush=True)
    root, x, y = make_points(wl["lookup_points"], R, seed=wl["seed"], batch=1)
    leaf = t.lookup(_dev(x), _dev(y), None if R == 1 else _dev(root))
    want = f.lookup_many(None if R == 1 else root, x, y)
    assert np.array_equal(leaf.cpu().numpy(), want)
    _check_tree("timed batch", t, f)


def test_quadtree_forest_larger_than_the_lds_table():
    # more nodes than the lookup keeps in LDS: descents continue in global memory and the
    # visits of the later nodes are counted with global atomics
    t = Quadtree(3, 120_000)
    f = oqt.Forest(3, 120_000)
    r = 0
    while len(f.nodes) <= 20_000:
        root, x, y = make_points(300_000, 3, seed=61, batch=r)
        _lookup_both(f"grow {r}", t, f, root, x, y)
        t.refine(8)
        f.refine(8)
        _check_tree(f"refine {r}", t, f)
        r += 1
        assert r < 12
    for b in range(2):
        root, x, y = make_points(400_000, 3, seed=62, batch=b)
        _lookup_both(f"large forest {b}", t, f, root, x, y)
        _check_tree(f"large forest visits {b}", t, f)


def test_quadtree_adapter_follows_the_oracle_loop():
    # the convenience loop: lookup -> adapt -> refine every m_refine proposals
    from paper_2402_08273_amd.ops import QuadtreeAdapter

    R, cap, n = 2, 8192, 30_000
    qa = QuadtreeAdapter(R, cap, m_split=150, m_refine=60_000)
    f = oqt.Forest(R, cap)
    st = ora.initial_state(cap)
    pending = 0
    for r in range(6):
        root, x, y = make_points(n, R, seed=71, batch=r)
        _, alpha = make_proposals(n, 5, seed=72, batch=r)
        leaf = qa.step(_dev(x), _dev(y), _dev(alpha), _dev(root)).cpu().numpy()
        want = f.lookup_many(root, x, y)
        assert np.array_equal(leaf, want), r
        ora.adapt(st, want, alpha)
        pending += n
        if pending >= 60_000:
            f.refine(150, st)
            pending = 0
        _check_tree(f"refinement {r}", qa.tree, f)
        nn = len(f.nodes)
        torch.cuda.synchronize()
        assert np.array_equal(qa.adapter.updates.cpu().numpy()[:nn], st["updates"][:nn]), r
        assert np.array_equal(qa.adapter.acc.cpu().numpy()[:nn], st["acc"][:nn]), r
        # rounding bound of the re-associated update sums, with every window of the run
        # counted for every lineage (the per-lineage bound is pinned in the test above)
        tol = lambda_tol((r + 1) * n // 10 + r + 1)
        assert np.allclose(qa.lam.cpu().numpy()[:nn], st["lambda"][:nn], rtol=0, atol=tol), r
