"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bar: bit-exact neighbour indices and FP32 squared distances, and the GPU tree
identical to the oracle tree node by node (split dimensions, split values,
ranges, tight boxes, packed order).
"""
import math

import numpy as np
import pytest

import oracle
import pins
from gpu_util import assert_same, compare_trees, dev, gpu_knn, log
from paper_1607_08220_amd import inputs
from treecheck import check_knn_lists, check_tree

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_08220_amd as knn
    knn.load_library()
    return knn


def _full_check(knn, X, Q, k, leaf, self_ids=None, r2=np.inf, what="", subtree_points=0,
                split_block_nodes=0):
    log(f"[case] {what} n={len(X)} d={X.shape[1]} m={len(Q)} k={k} leaf={leaf} "
        f"self={self_ids is not None} r2={r2} W={subtree_points} sbn={split_block_nodes}")
    T = oracle.build(X, leaf)
    _, _, tree = gpu_knn(X, Q[:1], 1, leaf=leaf, subtree_points=subtree_points,
                         split_block_nodes=split_block_nodes)
    g = tree.export()
    check_tree(X, g, leaf)
    compare_trees(g, T)
    gi, gd, _ = gpu_knn(X, Q, k, self_ids=self_ids, r2=r2, tree=tree)
    oi, od = T.query(Q, k, self_ids=self_ids, r2=r2)
    assert_same(gi, gd, oi, od, what)
    check_knn_lists(gi, gd)
    gi1, gd1, _ = gpu_knn(X, Q, k, self_ids=self_ids, r2=r2, order=1, tree=tree)
    assert_same(gi1, gd1, oi, od, what + " (input order)")
    # small batches default to one wavefront per query: the lane-per-query
    # forms answer the same batch too
    for trav in (1, 2):
        for order in (0, 1):
            gi2, gd2, _ = gpu_knn(X, Q, k, self_ids=self_ids, r2=r2, tree=tree, traversal=trav,
                                  order=order)
            assert_same(gi2, gd2, oi, od, what + f" (traversal {trav}, order {order})")
    for team in (8, 16, 32):  # a team of lanes per query (where k and the depth fit)
        gi3, gd3, _ = gpu_knn(X, Q, k, self_ids=self_ids, r2=r2, tree=tree, traversal=4,
                              team_lanes=team)
        assert_same(gi3, gd3, oi, od, what + f" (team of {team})")
    tree.free()


def test_tiny_uniform_workload(knn):
    """65,536 uniform 3-D points, 4,096 fresh queries, k = 5, leaf 32."""
    w = inputs.workload("tiny_uniform")
    _full_check(knn, w.points, w.queries, w.k, w.leaf, what="tiny_uniform")
    bi, bd = oracle.bf32(w.points, w.queries, w.k)
    gi, gd, t = gpu_knn(w.points, w.queries, w.k, leaf=w.leaf)
    assert_same(gi, gd, bi, bd, "tiny_uniform vs brute force")
    t.free()


def test_golden_examples(knn):
    import json
    for name in ("alg1_radius_update.json", "alg1_cell_bound.json"):
        g = json.load(open(f"{pins.GOLD}/{name}"))
        X = np.array(g["points"], np.float32)
        q = np.array([g["query"]], np.float32)
        log(f"[case] golden {name}")
        gi, gd, t = gpu_knn(X, q, g["k"], leaf=g["leaf"])
        assert gi[0].tolist() == g["expected_idx"] and gd[0].tolist() == g["expected_d2"]
        t.free()


def test_fp32_summation_order(knn):
    """Hand-derived value: left-to-right unfused FP32 sum (catches FMA contraction)."""
    import json
    g = json.load(open(f"{pins.GOLD}/fp32_sum_order.json"))
    x = np.array([pins._hexf(h) for h in g["x_hex"]], np.float32)[None, :]
    q = np.array([g["q"]], np.float32)
    log("[case] fp32 summation order")
    gi, gd, t = gpu_knn(x, q, 1, leaf=1)
    assert pins._bits(gd[0, 0]) == pins._bits(pins._hexf(g["expected_d2_hex"]))
    t.free()


def test_grid_shells(knn):
    r3 = pins._gold("sum_of_three_squares.json")["r3"]
    X = pins.grid_points()
    c = int(np.flatnonzero((X == 4).all(1))[0])
    k = sum(r3[1:6])  # shells D = 1..5: 56 neighbours
    for leaf in (1, 4, 32):
        log(f"[case] grid shells leaf={leaf}")
        gi, gd, t = gpu_knn(X, X[c:c + 1], k, leaf=leaf, self_ids=np.array([c]))
        bi, bd = oracle.bf32(X, X[c:c + 1], k, self_ids=np.array([c]))
        assert_same(gi, gd, bi, bd, f"grid leaf={leaf}")
        for D in range(1, 6):
            assert int((gd[0] == D).sum()) == r3[D]
        t.free()


def test_small_adversarial_sets(knn):
    """The oracle's small random and adversarial sets: every d from 1 to 16,
    k from 1 to more than n, self exclusion and a radius."""
    rng = np.random.default_rng(3)
    for name, X, leaf in pins._cases(21):
        n, d = X.shape
        Q = np.concatenate([X[rng.integers(0, n, 30)],
                            rng.random((20, d)).astype(np.float32) * 3 - 1]).astype(np.float32)
        sid = np.concatenate([rng.integers(0, n, 30), -np.ones(20)]).astype(np.int32)
        T = oracle.build(X, leaf)
        log(f"[case] {name}")
        _, _, tree = gpu_knn(X, Q[:1], 1, leaf=leaf)
        g = tree.export()
        check_tree(X, g, leaf)
        compare_trees(g, T)
        for k in (1, 5, 17, min(64, n + 3)):
            for r2 in (np.inf, 0.01):
                for s in (None, sid):
                    gi, gd, _ = gpu_knn(X, Q, k, self_ids=s, r2=r2, tree=tree)
                    bi, bd = oracle.bf32(X, Q, k, self_ids=s, r2=r2)
                    assert_same(gi, gd, bi, bd, f"{name} k={k} r2={r2} self={s is not None}")
        tree.free()


@pytest.mark.parametrize("d,leaf,k", [(3, 32, 8), (4, 16, 16), (2, 8, 33), (6, 32, 5),
                                      (10, 32, 5), (16, 64, 64), (1, 5, 7)])
def test_ragged_sizes_span_level_passes(knn, d, leaf, k):
    """Sizes that need several level passes plus ragged tails, clustered data."""
    rng = np.random.default_rng(100 + d)
    n = 100_003 if d <= 4 else 40_009
    if d == 3:
        X = inputs.clustered(n, seed=77, n_clusters=50)
    else:
        X = inputs.corr_gauss(n, d, seed=78)
    ids = rng.choice(n, 3_001, replace=False).astype(np.int32)
    # some cases choose every split with one wavefront per node
    sbn = -1 if d in (4, 10, 1) else 0
    _full_check(knn, X, X[ids], k, leaf, self_ids=ids, what=f"ragged d={d}", split_block_nodes=sbn)


def test_small_subtree_width(knn):
    """A small per-wavefront subtree forces many level passes and all code paths."""
    X = inputs.clustered(50_000, seed=79, n_clusters=20)
    rng = np.random.default_rng(5)
    ids = rng.choice(len(X), 2_000, replace=False).astype(np.int32)
    _full_check(knn, X, X[ids], 8, 4, self_ids=ids, what="W=64", subtree_points=64)


def test_heavy_duplicates_and_identical_big_nodes(knn):
    """Identical points above the level-pass size become one oversized bucket;
    a constant sample over a non-constant node takes the extent rule."""
    rng = np.random.default_rng(9)
    X = np.concatenate([np.full((20_000, 3), 0.5, np.float32),
                        rng.random((300, 3)).astype(np.float32),
                        np.repeat(rng.random((4, 3)).astype(np.float32), 5_000, 0)])
    X = X[rng.permutation(len(X))]
    Q = np.concatenate([X[:500], rng.random((100, 3)).astype(np.float32)])
    _full_check(knn, X, Q, 9, 32, what="duplicates")
    Y = np.concatenate([np.zeros((5000, 2), np.float32), np.ones((3, 2), np.float32)])
    Y = Y[rng.permutation(len(Y))]
    for sbn in (0, -1):  # the split (and its left counts) by a workgroup, then a wavefront
        _full_check(knn, Y, Y[:50], 4, 2, what="constant sample", subtree_points=64,
                    split_block_nodes=sbn)


def test_subtree_nodes_above_the_lds_tile(knn):
    """Subtree nodes larger than the finish's LDS tile are split straight from
    HBM: two such levels at 16 dimensions (tile 256 of 1024 points), buckets
    larger than the tile (leaf 600), and children still above the tile after
    an HBM split because of duplicates."""
    rng = np.random.default_rng(21)
    X = rng.standard_normal((12_000, 16)).astype(np.float32)
    ids = rng.choice(len(X), 600, replace=False).astype(np.int32)
    _full_check(knn, X, X[ids], 6, 8, self_ids=ids, what="d=16 two HBM levels")
    X = (np.floor(rng.random((30_000, 3)) * 40) / 40).astype(np.float32)
    ids = rng.choice(len(X), 800, replace=False).astype(np.int32)
    _full_check(knn, X, X[ids], 7, 600, self_ids=ids, what="leaf 600, grid duplicates")
    x = np.concatenate([np.full(700, 0.25), np.full(200, 0.75), rng.random(100)])
    X = np.stack([x, np.zeros(1000)], 1).astype(np.float32)
    X = np.tile(X, (20, 1))
    X[:, 1] = np.repeat(np.arange(20), 1000).astype(np.float32) * 10.0
    X = X[rng.permutation(len(X))]
    _full_check(knn, X, X[::13], 5, 16, self_ids=np.arange(0, len(X), 13),
                what="duplicate children above the tile", subtree_points=1024)


@pytest.mark.parametrize("n", [8191, 8192, 8193, 12289, 65537])
def test_presampled_children_around_the_threshold(knn, n):
    """Children of at least 4,096 points get their sample written by the
    partition that creates them; roots of 8,191 .. 65,537 points put the
    children of the first levels on both sides of that size (and children of
    exactly 4,096 points), under the workgroup and the wavefront samplers."""
    X = inputs.clustered(n, seed=n, n_clusters=7)
    rng = np.random.default_rng(n)
    ids = rng.choice(n, 300, replace=False).astype(np.int32)
    for sbn in (0, -1):
        _full_check(knn, X, X[ids], 6, 32, self_ids=ids, what=f"presampled n={n}",
                    split_block_nodes=sbn)


def test_split_outside_sample_window(knn):
    """The level histogram resolves only the sample ranks around the middle;
    these inputs put the point closest to half outside that window (the
    systematic sample positions hit only the large, or only the small,
    values of the split dimension), so the full-histogram path decides."""
    rng = np.random.default_rng(5)
    # 4,096 points: sample positions 4j + 2; 20,480 (five partition blocks of
    # 4,096, counted one by one): 10 (2j + 1); all even either way
    for n, big_even in ((4096, True), (4096, False), (20480, True)):
        x = np.empty(n, np.float32)
        hi = (1.0 + rng.random(n // 2) * 0.01).astype(np.float32)
        lo = (rng.random(n // 2) * 0.001).astype(np.float32)
        x[0::2], x[1::2] = (hi, lo) if big_even else (lo, hi)
        X = np.stack([x, (rng.random(n) * 1e-4).astype(np.float32)], 1)
        for sbn in (0, -1):  # split chosen by a workgroup, then by a wavefront
            _full_check(knn, X, X[::7], 5, 32, self_ids=np.arange(0, n, 7),
                        what=f"window n={n} big_even={big_even}", split_block_nodes=sbn)


def test_determinism_and_order_independence(knn):
    w = inputs.workload("cosmo_clustered", scale=1 / 256)
    log(f"[case] determinism n={len(w.points)}")
    a_i, a_d, t1 = gpu_knn(w.points, w.queries, w.k, self_ids=w.self_ids)
    b_i, b_d, t2 = gpu_knn(w.points, w.queries, w.k, self_ids=w.self_ids)
    e1, e2 = t1.export(), t2.export()
    for key in ("dim", "split", "left", "parent", "start", "count", "lo", "hi", "perm"):
        assert np.array_equal(e1[key], e2[key]), key
    assert_same(a_i, a_d, b_i, b_d, "repeat")
    p = np.random.default_rng(1).permutation(len(w.queries))
    half = len(p) // 2
    for trav in (0, 1, 2, 3):  # every traversal form: order and batch do not matter
        for order in ((0, 1) if trav in (1, 2) else (0,)):
            what = f"traversal {trav} order {order}"
            c_i, c_d, _ = gpu_knn(w.points, w.queries[p], w.k, self_ids=w.self_ids[p], tree=t1,
                                  traversal=trav, order=order)
            assert_same(c_i, c_d, a_i[p], a_d[p], "permuted queries, " + what)
            d_i, d_d, _ = gpu_knn(w.points, w.queries[:half], w.k, self_ids=w.self_ids[:half],
                                  tree=t1, traversal=trav, order=order)
            assert_same(d_i, d_d, a_i[:half], a_d[:half], "batch split, " + what)
    # the leaf-batch knob only reschedules the traversal: identical results
    import torch
    Q, S = dev(w.queries), dev(w.self_ids)
    for lb in (1, 17, 64):
        idx, d2 = knn.knn_query_ex(t1, Q, w.k, self_ids=S, leaf_batch=lb, traversal=1)
        torch.cuda.synchronize()
        assert_same(idx.cpu().numpy(), d2.cpu().numpy(), a_i, a_d, f"leaf_batch={lb}")
    with pytest.raises(knn.KnnError):
        knn.knn_query_ex(t1, Q, w.k, leaf_batch=65)
    t1.free()
    t2.free()


def test_radius_at_or_below_zero(knn):
    """r2_max <= 0 admits no point (D < r2_max is never true for D >= 0); a
    radius equal to a distance excludes that point (strict)."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0], [3, 0, 0]], np.float32)
    log("[case] radius <= 0 and strict radius")
    for r2 in (0.0, -1.0, -np.inf):
        gi, gd, t = gpu_knn(X, X[:2], 3, r2=r2)
        assert (gi == -1).all() and np.isinf(gd).all(), r2
        bi, bd = oracle.bf32(X, X[:2], 3, r2=r2)
        assert_same(gi, gd, bi, bd, f"r2={r2}")
        t.free()
    gi, gd, t = gpu_knn(X, X[:1], 4, r2=4.0)  # D = 0, 1 qualify; D = 4 is not < 4
    assert gi.tolist() == [[0, 1, -1, -1]] and gd[0, :2].tolist() == [0.0, 1.0]
    bi, bd = oracle.bf32(X, X[:1], 4, r2=4.0)
    assert_same(gi, gd, bi, bd, "strict radius")
    t.free()


def test_empty_and_degenerate_calls(knn):
    import torch
    X = np.random.default_rng(2).random((10, 3)).astype(np.float32)
    log("[case] empty/degenerate calls")
    gi, gd, t = gpu_knn(X, X[:0], 3)
    assert gi.shape == (0, 3)
    gi, gd, _ = gpu_knn(X, X[:2], 64, tree=t)  # k > n pads
    assert (gi[:, 10:] == -1).all() and np.isinf(gd[:, 10:]).all()
    gi, gd, t1 = gpu_knn(X[:1], X[:1], 2)       # n = 1
    assert gi.tolist() == [[0, -1]] and gd[0, 0] == 0.0
    P = torch.from_numpy(X).cuda()
    with pytest.raises(knn.KnnError):
        knn.knn_query(t, torch.from_numpy(X).cuda(), 0)
    with pytest.raises(knn.KnnError):
        knn.knn_query(t, torch.from_numpy(X).cuda(), 65)
    with pytest.raises(knn.KnnError):
        knn.knn_build_ex(P, leaf_size=1, max_depth=1)  # depth above max_depth
    # a NaN or infinite coordinate stops the build before any split is computed
    for bad in (np.nan, np.inf, -np.inf):
        Xb = np.tile(X, (300, 1))
        Xb[1234, 1] = bad
        with pytest.raises(knn.KnnError) as e:
            knn.knn_build(torch.from_numpy(Xb).cuda(), 8)
        assert e.value.code == knn.KNN_ENOTFINITE
        with pytest.raises(knn.KnnError) as e:
            knn.knn_build_batch(torch.from_numpy(Xb).cuda(), [0, 1000, len(Xb)])
        assert e.value.code == knn.KNN_ENOTFINITE
    t.free()
    t1.free()


@pytest.mark.parametrize("d", [3, 4, 10, 16])
def test_fp64_cross_check(knn, d):
    """GPU vs FP64 brute force.  The GPU result must be the exact FP32 answer
    (== BF32 bit for bit); then every rank where it differs from the FP64
    brute force is either allowed by the 1e-6 relative rule or is a legal
    FP32 reorder (the two FP64 distances closer than the FP32 forward-error
    bound allows FP32 to resolve); both kinds are counted and logged, and any
    other difference fails.  Uniform data and a near-tie set (lattice points
    moved by ~3e-7, queries at cell centres) where FP32 and FP64 disagree
    often; the seeds are not chosen."""
    import fp64rule
    rng = np.random.default_rng(1000 + d)
    n = 20_000
    near = (rng.integers(0, 8, size=(n, d)) + rng.standard_normal((n, d)) * 3e-7).astype(np.float32)
    sets = [("uniform", rng.random((n, d)).astype(np.float32), rng.random((256, d)).astype(np.float32)),
            ("near-ties", near, (rng.integers(0, 8, size=(256, d)) + 0.5).astype(np.float32))]
    for name, X, Q in sets:
        log(f"[case] fp64 cross-check {name} d={d}")
        gi, gd, t = gpu_knn(X, Q, 8)
        bi, bd = oracle.bf32(X, Q, 8)
        assert_same(gi, gd, bi, bd, f"{name} d={d} vs BF32")
        i64, d64 = oracle.bf64(X, Q, 8)
        c = fp64rule.classify(X, Q, gi, i64, d64)
        log(f"  differing ranks {c['differing_ranks']}: {c['rule']} within 1e-6, "
            f"{c['fp32']} legal FP32 reorders beyond it, {len(c['bad'])} mismatches")
        assert not c["bad"], c["bad"][:5]
        if name == "near-ties":
            assert c["differing_ranks"] > 0, "the near-tie set should exercise the rule"
        t.free()


@pytest.mark.parametrize("d", [1, 3, 6, 10, 16])
def test_both_traversals_match_oracle(knn, d):
    """The stack-free walk, the explicit-stack form and the one-wavefront-per-
    query form give the oracle's result on the same tree, in both query
    orders."""
    import torch
    n = 60_011
    X = inputs.clustered(n, seed=90, n_clusters=40) if d == 3 else inputs.corr_gauss(n, d, seed=91)
    ids = np.random.default_rng(d).choice(n, 2_000, replace=False).astype(np.int32)
    log(f"[case] traversals d={d}")
    t = knn.knn_build(dev(X), 32)
    bi, bd = oracle.bf32(X, X[ids], 9, self_ids=ids)
    for trav, team in ((1, 0), (2, 0), (3, 0), (4, 16), (4, 32)):
        for order in (0, 1):
            gi, gd = knn.knn_query_ex(t, dev(X[ids]), 9, self_ids=dev(ids), traversal=trav,
                                      order=order, team_lanes=team)
            torch.cuda.synchronize()
            assert_same(gi.cpu().numpy(), gd.cpu().numpy(), bi, bd,
                        f"traversal {trav} (team {team}) order {order}")
    t.free()


@pytest.mark.parametrize("d", [2, 10])
def test_wavefront_per_query_edge_cases(knn, d):
    """One wavefront per query: k up to 64 (every lane a heap entry), a radius
    at, below and above zero, a single query, and a bucket of 3,000 identical
    points (larger than a wavefront's 64 lanes)."""
    import torch
    rng = np.random.default_rng(40 + d)
    n = 20_000
    X = inputs.corr_gauss(n, d, seed=92 + d)
    X[:3_000] = X[0]  # 3,000 identical points: an oversized bucket of > 64 rows
    X = X[rng.permutation(n)]
    ids = rng.choice(n, 300, replace=False).astype(np.int32)
    log(f"[case] wavefront per query d={d}")
    t = knn.knn_build(dev(X), 16)
    for k in (1, 7, 16, 32, 64):
        bi, bd = oracle.bf32(X, X[ids], k, self_ids=ids)
        gi, gd = knn.knn_query_ex(t, dev(X[ids]), k, self_ids=dev(ids), traversal=3)
        torch.cuda.synchronize()
        assert_same(gi.cpu().numpy(), gd.cpu().numpy(), bi, bd, f"wave k={k}")
        for team in (8, 16, 32):  # teams with k at and above their size (the latter fall back)
            gi, gd = knn.knn_query_ex(t, dev(X[ids]), k, self_ids=dev(ids), traversal=4,
                                      team_lanes=team)
            torch.cuda.synchronize()
            assert_same(gi.cpu().numpy(), gd.cpu().numpy(), bi, bd, f"team {team} k={k}")
    for r2 in (0.0, -1.0, 0.5):
        bi, bd = oracle.bf32(X, X[ids[:1]], 5, self_ids=ids[:1], r2=r2)
        for trav in (3, 4):
            gi, gd = knn.knn_query_ex(t, dev(X[ids[:1]]), 5, self_ids=dev(ids[:1]), r2_max=r2,
                                      traversal=trav, team_lanes=8)
            torch.cuda.synchronize()
            assert_same(gi.cpu().numpy(), gd.cpu().numpy(), bi, bd, f"form {trav} r2={r2}")
    with pytest.raises(knn.KnnError):
        knn.knn_query_ex(t, dev(X[ids]), 5, traversal=4, team_lanes=12)
    t.free()
