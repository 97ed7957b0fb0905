"""Build plans: a build whose runs only enqueue kernels, captured in a graph
together with queries on its tree and replayed over new point values.

Every run's tree equals the eager build's tree array by array (and so the
oracle's, which the eager build is held to elsewhere); a run is also compared
node by node with the oracle tree directly.  Graph replays over fresh point
values give the eager build + query result each time; failed runs leave a
tree that answers with index -1 and report their error from finish."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import assert_same, check_links, compare_trees, dev, log
from paper_1607_08220_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("dim", "split", "left", "parent", "start", "count", "lo", "hi", "perm", "packed")


@pytest.fixture(scope="module")
def knn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_08220_amd as knn
    knn.load_library()
    return knn


def same_export(a: dict, b: dict, what: str) -> None:
    for key in KEYS:
        x, y = np.asarray(a[key]), np.asarray(b[key])
        assert x.shape == y.shape, f"{what}: {key} shape {x.shape} vs {y.shape}"
        if x.dtype.kind == "f":
            x, y = x.view(np.uint32), y.view(np.uint32)
        assert np.array_equal(x, y), f"{what}: {key} differs"


def test_plan_tree_equals_eager_and_oracle(knn):
    import torch
    X = inputs.clustered(200_000, seed=41)
    log(f"[case] plan single tree n={len(X)}")
    P = dev(X)
    plan = knn.BuildPlan(len(X), 3, leaf_size=32)
    for rep in range(2):  # a second run over the same plan starts from clean state
        plan.run(P)
        tree = plan.finish()
        g = tree.export()
        check_links(g, len(X))
        eager = knn.knn_build_ex(P, leaf_size=32)
        same_export(g, eager.export(), f"run {rep} vs eager")
        eager.free()
    seen = compare_trees(g, oracle.build(X, 32))
    log(f"[case] plan tree: {seen} nodes identical to the oracle tree")
    info = tree.info()
    # the depth a plan's tree reports is its bound: the balanced depth of
    # 200,000 points in buckets of 32 (13 halvings) + 8
    assert info["nodes"] == len(g["dim"]) and info["depth"] == 13 + 8
    # the plan owns its tree: the C-ABI free refuses it
    assert knn.load_library().knn_tree_free(tree.handle) == knn.KNN_EINVAL
    plan.destroy()


@pytest.mark.parametrize("d,lo,hi,ntrees", [(6, 3.0, 14.0, 37), (3, 5.0, 16.0, 9)])
def test_plan_forest_equals_eager(knn, d, lo, hi, ntrees):
    import torch
    f = inputs.forest(ntrees, d=d, lo_exp=lo, hi_exp=hi, q_per_tree=64, seed=5 + d)
    log(f"[case] plan forest d={d} trees={ntrees} rows={len(f.points)}")
    P = dev(f.points)
    plan = knn.BuildPlan(len(f.points), d, offsets=f.offsets, leaf_size=f.leaf)
    plan.run(P)
    tree = plan.finish()
    eager = knn.knn_build_batch(P, f.offsets, leaf_size=f.leaf)
    same_export(tree.export(), eager.export(), "plan forest vs eager forest")
    Q, T, S = dev(f.queries), dev(f.tree_ids), dev(f.self_ids)
    pi, pd = knn.knn_query_batch(tree, Q, T, f.k, self_ids=S)
    ei, ed = knn.knn_query_batch(eager, Q, T, f.k, self_ids=S)
    torch.cuda.synchronize()
    assert_same(pi.cpu().numpy(), pd.cpu().numpy(), ei.cpu().numpy(), ed.cpu().numpy(),
                "forest queries: plan tree vs eager tree")
    eager.free()
    plan.destroy()


@pytest.mark.parametrize("trav", [0, 2, 3])
def test_plan_build_and_query_graph_replay(knn, trav):
    """Build + query captured once; each replay over new point values (copied
    into the captured input buffer) equals the eager build + query on those
    values, with eager work and synchronisation between replays."""
    import torch
    n, m, k = 150_000, 20_000, 8
    log(f"[case] plan graph replay n={n} m={m} k={k} traversal={trav}")
    sets = [inputs.clustered(n, seed=300 + s) for s in range(3)]
    P = dev(sets[0])
    Q = dev(inputs.uniform(m, 3, seed=77) * np.float32(0.9))
    plan = knn.BuildPlan(n, 3, leaf_size=32)
    plan.run(P)
    plan.finish()
    oi = torch.empty((m, k), dtype=torch.int32, device="cuda")
    od = torch.empty((m, k), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm up on the capture stream
        plan.run(P)
        knn.knn_query_ex(plan.tree, Q, k, out=(oi, od), traversal=trav)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(P)
        knn.knn_query_ex(plan.tree, Q, k, out=(oi, od), traversal=trav)
    for rep in range(4):
        X = sets[rep % len(sets)]
        P.copy_(torch.from_numpy(X))
        oi.fill_(-7)
        od.fill_(-7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        plan.finish()
        eager = knn.knn_build_ex(dev(X), leaf_size=32)
        ei, ed = knn.knn_query_ex(eager, Q, k, traversal=trav)
        torch.cuda.synchronize()
        ri, rd = oi.cpu().numpy(), od.cpu().numpy()
        assert_same(ri, rd, ei.cpu().numpy(), ed.cpu().numpy(), f"replay {rep} vs eager")
        same_export(plan.tree.export(), eager.export(), f"replay {rep} tree vs eager")
        eager.free()
        if rep == 0:
            pick = np.arange(0, m, 97)
            bi, bd = oracle.bf32(X, inputs.uniform(m, 3, seed=77)[pick] * np.float32(0.9), k)
            assert_same(ri[pick], rd[pick], bi, bd, "replay vs brute force")
    del g
    torch.cuda.synchronize()
    plan.destroy()


def test_plan_errors_leave_a_safe_tree(knn):
    """A non-finite coordinate, or a tree deeper than the plan allows, is
    reported by finish; the tree then answers with index -1 everywhere, and
    the next good run restores it."""
    import torch
    n, m, k = 50_000, 512, 4
    X = inputs.clustered(n, seed=9)
    P = dev(X)
    Q = dev(X[:m])
    log(f"[case] plan errors n={n}")
    plan = knn.BuildPlan(n, 3, leaf_size=32)
    bad = X.copy()
    bad[1234, 1] = np.nan
    plan.run(dev(bad))
    with pytest.raises(knn.KnnError) as e:
        plan.finish()
    assert e.value.code == knn.KNN_ENOTFINITE
    ii, _ = knn.knn_query_ex(plan.tree, Q, k)
    torch.cuda.synchronize()
    assert (ii.cpu().numpy() == -1).all()
    plan.run(P)
    plan.finish()
    gi, gd = knn.knn_query_ex(plan.tree, Q, k)
    torch.cuda.synchronize()
    bi, bd = oracle.bf32(X, X[:m], k)
    assert_same(gi.cpu().numpy(), gd.cpu().numpy(), bi, bd, "after a failed run")
    plan.destroy()
    shallow = knn.BuildPlan(n, 3, leaf_size=32, max_depth=6)
    shallow.run(P)
    with pytest.raises(knn.KnnError) as e:
        shallow.finish()
    assert e.value.code == knn.KNN_EDEPTH
    ii, _ = knn.knn_query_ex(shallow.tree, Q, k)
    torch.cuda.synchronize()
    assert (ii.cpu().numpy() == -1).all()
    shallow.destroy()


def test_plan_argument_errors(knn):
    import torch
    with pytest.raises(knn.KnnError):
        knn.BuildPlan(0, 3)
    with pytest.raises(ValueError):
        knn.BuildPlan(100, 3, offsets=[0, 50, 99])
    plan = knn.BuildPlan(1000, 3)
    with pytest.raises(ValueError):
        plan.run(torch.zeros((999, 3), device="cuda"))
    with pytest.raises(ValueError):
        plan.run(torch.zeros((1000, 2), device="cuda"))
    with pytest.raises(knn.KnnError):
        plan.finish()  # nothing ran yet
    plan.destroy()
    assert knn.load_library().knn_build_plan_destroy(None) == knn.KNN_OK
