"""Full-size parity, in the launch configuration the bench times.

Clustered 3-D workload (2^26 points, 2^22 queries drawn from the data with
self excluded, k = 8, leaf 32): the oracle tree is built over all points; the
GPU tree passes the invariant checks and equals the oracle tree node by node,
and ALL 2^22 GPU results equal the oracle's Algorithm 1 results bit for bit.
256 sampled queries are also recomputed by brute force over all points
(the oracle's kd-tree pinned against the definition at this size).

Plasma-like 4-D workload (2^28 points, 2^24 queries, k = 16): the GPU tree
equals the oracle tree node by node and 2^20 of the queries (a random
subset) equal the oracle's results bit for bit; 64 sampled queries equal brute
force.

The oracle builds with one thread per host core (the same tree as one
thread) so that both cases finish in a few minutes."""
import os
import time

import numpy as np
import pytest

import oracle
from gpu_util import assert_same, compare_trees, log
from paper_1607_08220_amd import inputs
from treecheck import check_knn_lists, check_tree

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def knn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_08220_amd as knn
    knn.load_library()
    return knn


def _gpu_build_query(knn, w):
    import torch
    P = torch.from_numpy(w.points).cuda()
    Q = torch.from_numpy(w.queries).cuda()
    S = torch.from_numpy(w.self_ids).cuda()
    tree = knn.knn_build(P, w.leaf)
    idx, d2 = knn.knn_query_ex(tree, Q, w.k, self_ids=S)
    torch.cuda.synchronize()
    del P, Q, S
    return tree, idx, d2


@pytest.mark.parametrize("name,n_check,n_bf,tree_check", [
    ("cosmo_clustered", None, 256, True),
    ("plasma_4d", 1 << 20, 64, False),
])
def test_full_size(knn, name, n_check, n_bf, tree_check):
    t0 = time.time()
    w = inputs.workload(name)
    n, m = len(w.points), len(w.queries)
    log(f"[case] full size {name}: n={n} m={m} k={w.k} leaf={w.leaf} "
        f"(generated in {time.time() - t0:.0f} s)")
    tree, idx, d2 = _gpu_build_query(knn, w)
    info = tree.info()
    assert info["n"] == n and info["leaves"] * 2 - 1 == info["nodes"]
    t0 = time.time()
    g = tree.export()
    tree.free()
    T = oracle.build(w.points, w.leaf, nthreads=THREADS)
    log(f"[case] {name}: oracle tree {len(T.dim)} nodes in {time.time() - t0:.0f} s")
    if tree_check:
        check_tree(w.points, g, w.leaf)
    seen = compare_trees(g, T)
    log(f"[case] {name}: {seen} nodes identical to the oracle tree")
    del g
    rows = (np.arange(m) if n_check is None
            else np.sort(np.random.default_rng(9).choice(m, n_check, replace=False)))
    gi = idx.cpu().numpy()[rows]
    gd = d2.cpu().numpy()[rows]
    t0 = time.time()
    oi, od = T.query(w.queries[rows], w.k, self_ids=w.self_ids[rows], nthreads=THREADS)
    log(f"[case] {name}: oracle answered {len(rows)} queries in {time.time() - t0:.1f} s")
    assert_same(gi, gd, oi, od, f"{name}: GPU vs oracle kd-tree")
    check_knn_lists(gi, gd)
    assert (gi != w.self_ids[rows][:, None]).all()
    pick = np.random.default_rng(10).choice(len(rows), n_bf, replace=False)
    bi, bd = oracle.bf32(w.points, w.queries[rows[pick]], w.k, self_ids=w.self_ids[rows[pick]],
                         nthreads=THREADS)
    assert_same(gi[pick], gd[pick], bi, bd, f"{name}: sampled vs brute force")
    T.close()
