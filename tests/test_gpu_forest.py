"""Batched build + query (many independent trees in one forest): every tree of
the forest equals the oracle tree over its own rows node by node, and every
query's neighbours equal brute force over its own tree's points and the
per-call GPU result."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, compare_trees, dev, log
from paper_1607_08220_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_08220_amd as knn
    knn.load_library()
    return knn


def compare_forest_tree(g: dict, t: int, off: int, o: oracle.Tree) -> None:
    """Tree t of the forest export g (root node t, rows from off) against the
    oracle tree over the same rows."""
    assert g["parent"][t] == -1
    compare_trees(g, o, root=t, off=off)


@pytest.mark.parametrize("d,lo,hi,ntrees", [(6, 3.0, 14.0, 37), (3, 5.0, 17.0, 9), (2, 0.0, 6.0, 50)])
def test_forest_matches_oracle_and_single_trees(knn, d, lo, hi, ntrees):
    import torch
    f = inputs.forest(ntrees, d=d, lo_exp=lo, hi_exp=hi, q_per_tree=64, seed=77 + d)
    log(f"[case] forest d={d} trees={ntrees} rows={len(f.points)} sizes "
        f"{np.diff(f.offsets).min()}..{np.diff(f.offsets).max()}")
    P = dev(f.points)
    forest = knn.knn_build_batch(P, f.offsets, leaf_size=f.leaf)
    info = forest.info()
    assert info["trees"] == ntrees and info["n"] == len(f.points)
    g = forest.export()
    Q, T, S = dev(f.queries), dev(f.tree_ids), dev(f.self_ids)
    fi, fd = knn.knn_query_batch(forest, Q, T, f.k, self_ids=S)
    torch.cuda.synchronize()
    fi, fd = fi.cpu().numpy(), fd.cpu().numpy()
    # every traversal form in both orders: the lane-per-query forms start at
    # the home leaf of each query's own tree (grouped across trees) or at its
    # root; the wavefront form takes input order
    for trav, team in ((1, 0), (2, 0), (3, 0), (4, 8), (4, 32)):
        for order in (0, 1):
            ti, td = knn.knn_query_batch(forest, Q, T, f.k, self_ids=S, order=order,
                                         traversal=trav, team_lanes=team)
            torch.cuda.synchronize()
            assert_same(ti.cpu().numpy(), td.cpu().numpy(), fi, fd,
                        f"traversal {trav} (team {team}) order {order} vs default")
    assert knn.knn_tree_errors(forest) == 0
    for t in range(ntrees):
        a, b = int(f.offsets[t]), int(f.offsets[t + 1])
        X = f.points[a:b]
        compare_forest_tree(g, t, a, oracle.build(X, f.leaf))
        sel = np.flatnonzero(f.tree_ids == t)
        bi, bd = oracle.bf32(X, f.queries[sel], f.k, self_ids=f.self_ids[sel] - a)
        bi = np.where(bi >= 0, bi + a, bi)
        assert_same(fi[sel], fd[sel], bi, bd, f"tree {t} vs brute force")
        if t % 8 == 0:  # the per-call path gives the same answer
            single = knn.knn_build(dev(X), f.leaf)
            si, sd = knn.knn_query_ex(single, dev(f.queries[sel]), f.k,
                                      self_ids=dev((f.self_ids[sel] - a).astype(np.int32)))
            torch.cuda.synchronize()
            si = si.cpu().numpy()
            assert_same(fi[sel], fd[sel], np.where(si >= 0, si + a, si), sd.cpu().numpy(),
                        f"tree {t} vs per-call")
            single.free()
    with pytest.raises(knn.KnnError):
        knn.knn_query(forest, Q, 3)  # a forest needs tree ids
    forest.free()


def test_forest_argument_errors(knn):
    X = dev(np.zeros((10, 3), np.float32))
    for bad in ([0, 5, 5, 10], [1, 10], [0, 4, 11]):
        with pytest.raises((knn.KnnError, ValueError)):
            knn.knn_build_batch(X, bad)


def test_autotune_picks_a_listed_config(knn):
    from paper_1607_08220_amd import autotune
    f = inputs.forest(6, d=4, lo_exp=6.0, hi_exp=12.0, q_per_tree=128, seed=3)
    log("[case] autotune")
    r = autotune.tune(dev(f.points), dev(f.queries), f.k, self_ids=dev(f.self_ids),
                      offsets=f.offsets, tree_ids=dev(f.tree_ids), leaf_sizes=(16, 32),
                      leaf_batches=(48, 64), orders=(0, 1), reps=1)
    assert (r["leaf_size"], r["leaf_batch"], r["order"]) in {
        (a["leaf_size"], a["leaf_batch"], a["order"]) for a in r["table"]}
    # 2 leaf sizes x 2 leaf batches x 2 orders x 5 traversal forms (two team sizes)
    assert len(r["table"]) == 40 and r["ms"] == min(a["ms"] for a in r["table"])
    assert {(a["traversal"], a["team_lanes"]) for a in r["table"]} == {
        (1, 0), (2, 0), (3, 0), (4, 16), (4, 32)}


@pytest.mark.parametrize("trav", [1, 2, 3, 4])
def test_forest_query_graph_replay(knn, trav):
    """The batched query captured once in a graph and replayed, with eager
    work and synchronization between replays, gives the eager result every
    time -- for the lane-per-query forms (their grouping kernels, counting
    sort and workspace included) and the wavefront form."""
    import torch
    f = inputs.forest(20, d=6, lo_exp=8.0, hi_exp=15.0, q_per_tree=256, seed=21)
    log(f"[case] graph replay rows={len(f.points)} traversal={trav}")
    forest = knn.knn_build_batch(dev(f.points), f.offsets, leaf_size=32)
    Q, T, S = dev(f.queries), dev(f.tree_ids), dev(f.self_ids)
    ei, ed = knn.knn_query_batch(forest, Q, T, f.k, self_ids=S)
    torch.cuda.synchronize()
    ei, ed = ei.cpu().numpy(), ed.cpu().numpy()
    bi, bd = [], []
    for t in range(20):  # brute force over each query's own tree
        a, b = int(f.offsets[t]), int(f.offsets[t + 1])
        sel = np.flatnonzero(f.tree_ids == t)
        ii, dd = oracle.bf32(f.points[a:b], f.queries[sel], f.k, self_ids=f.self_ids[sel] - a)
        bi.append((sel, np.where(ii >= 0, ii + a, ii), dd))
    for sel, ii, dd in bi:
        assert_same(ei[sel], ed[sel], ii, dd, "eager vs brute force")
    oi = torch.empty((len(f.queries), f.k), dtype=torch.int32, device="cuda")
    od = torch.empty((len(f.queries), f.k), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm up on the capture stream
        knn.knn_query_batch(forest, Q, T, f.k, self_ids=S, out=(oi, od), traversal=trav)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        knn.knn_query_batch(forest, Q, T, f.k, self_ids=S, out=(oi, od), traversal=trav)
    for rep in range(4):
        oi.fill_(-7)
        od.fill_(-7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_same(oi.cpu().numpy(), od.cpu().numpy(), ei, ed, f"replay {rep}")
    del g
    forest.free()


def test_out_of_range_tree_ids(knn):
    """Tree ids outside [0, trees) read no node: those queries get padding
    rows, the others their own tree's answer, in every traversal form and
    order, and knn_tree_errors reports the count (then clears it)."""
    import torch
    f = inputs.forest(5, d=3, lo_exp=6.0, hi_exp=11.0, q_per_tree=40, seed=5)
    log(f"[case] out-of-range tree ids rows={len(f.points)}")
    forest = knn.knn_build_batch(dev(f.points), f.offsets, leaf_size=16)
    ids = f.tree_ids.copy()
    bad = np.arange(0, len(ids), 7)
    ids[bad] = np.resize(np.array([-1, 5, 1000, -(2 ** 31), 2 ** 31 - 1], np.int32), len(bad))
    good = np.setdiff1d(np.arange(len(ids)), bad)
    ref = {}
    for t in range(5):
        a, b = int(f.offsets[t]), int(f.offsets[t + 1])
        sel = good[f.tree_ids[good] == t]
        ii, dd = oracle.bf32(f.points[a:b], f.queries[sel], f.k, self_ids=f.self_ids[sel] - a)
        ref[t] = (sel, np.where(ii >= 0, ii + a, ii), dd)
    Q, T, S = dev(f.queries), dev(ids), dev(f.self_ids)
    for trav in (1, 2, 3, 4):
        for order in (0, 1):
            gi, gd = knn.knn_query_batch(forest, Q, T, f.k, self_ids=S, order=order,
                                         traversal=trav, team_lanes=16)
            torch.cuda.synchronize()
            gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
            assert (gi[bad] == -1).all() and np.isinf(gd[bad]).all(), (trav, order)
            for t, (sel, ii, dd) in ref.items():
                assert_same(gi[sel], gd[sel], ii, dd, f"tree {t} traversal {trav} order {order}")
            with pytest.raises(knn.KnnError) as e:
                knn.knn_tree_errors(forest)
            assert e.value.code == knn.KNN_EINVAL and f"{len(bad)} queries" in str(e.value)
            assert knn.knn_tree_errors(forest) == 0  # cleared
    forest.free()
