"""Batched build + query (many independent trees in one forest): every tree of
the forest equals the oracle tree over its own rows node by node, and every
query's neighbours equal brute force over its own tree's points and the
per-call GPU result."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, dev, log
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
    n_t = len(o.perm)
    assert np.array_equal(g["perm"][off:off + n_t] - off, o.perm), f"tree {t}: packed order"
    assert g["parent"][t] == -1
    stack = [(t, 0)]
    while stack:
        a, b = stack.pop()
        assert g["start"][a] - off == o.start[b] and g["count"][a] == o.count[b], (t, a, b)
        assert np.array_equal(g["lo"][a], o.lo[b]) and np.array_equal(g["hi"][a], o.hi[b]), (t, a)
        if o.dim[b] < 0:
            assert g["dim"][a] < 0, f"tree {t}: node {a} splits, oracle node {b} is a leaf"
            continue
        assert g["dim"][a] == o.dim[b] and g["split"][a] == o.split[b], (t, a, b)
        stack.append((int(g["left"][a]), int(o.left[b])))
        stack.append((int(g["left"][a]) + 1, int(o.right[b])))


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
    fi2, fd2 = knn.knn_query_batch(forest, Q, T, f.k, self_ids=S, order=1)
    torch.cuda.synchronize()
    fi, fd, fi2, fd2 = fi.cpu().numpy(), fd.cpu().numpy(), fi2.cpu().numpy(), fd2.cpu().numpy()
    assert_same(fi, fd, fi2, fd2, "grouped vs input order")
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
    # 2 leaf sizes x 2 leaf batches x 2 orders x 3 traversal forms
    assert len(r["table"]) == 24 and r["ms"] == min(a["ms"] for a in r["table"])
    assert {a["traversal"] for a in r["table"]} == {1, 2, 3}


def test_forest_query_graph_replay(knn):
    """The batched query captured once in a graph and replayed, with eager
    work and synchronization between replays, gives the eager result every
    time."""
    import torch
    f = inputs.forest(20, d=6, lo_exp=8.0, hi_exp=15.0, q_per_tree=256, seed=21)
    log(f"[case] graph replay rows={len(f.points)}")
    forest = knn.knn_build_batch(dev(f.points), f.offsets, leaf_size=32)
    Q, T, S = dev(f.queries), dev(f.tree_ids), dev(f.self_ids)
    ei, ed = knn.knn_query_batch(forest, Q, T, f.k, self_ids=S)
    torch.cuda.synchronize()
    ei, ed = ei.cpu().numpy(), ed.cpu().numpy()
    oi = torch.empty((len(f.queries), f.k), dtype=torch.int32, device="cuda")
    od = torch.empty((len(f.queries), f.k), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm up on the capture stream
        knn.knn_query_batch(forest, Q, T, f.k, self_ids=S, out=(oi, od))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        knn.knn_query_batch(forest, Q, T, f.k, self_ids=S, out=(oi, od))
    for rep in range(4):
        oi.fill_(-7)
        od.fill_(-7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_same(oi.cpu().numpy(), od.cpu().numpy(), ei, ed, f"replay {rep}")
    del g
    forest.free()
