"""Helpers for the GPU parity tests (compare the HIP path with the oracle)."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_knn(points, queries, k, leaf=32, self_ids=None, r2=np.inf, order=0, tree=None,
            subtree_points=0, split_block_nodes=0, traversal=0, team_lanes=0):
    """Build (unless a tree is given) and query through the C-ABI; host arrays out."""
    import torch
    import paper_1607_08220_amd as knn
    P = dev(np.asarray(points, np.float32))
    if tree is None:
        tree = knn.knn_build_ex(P, leaf_size=leaf, subtree_points=subtree_points,
                                split_block_nodes=split_block_nodes)
        check_links(tree.export(), len(points))
    Q = dev(np.asarray(queries, np.float32))
    S = dev(np.asarray(self_ids, np.int32)) if self_ids is not None else None
    idx, d2 = knn.knn_query_ex(tree, Q, k, self_ids=S, r2_max=r2, order=order,
                               traversal=traversal, team_lanes=team_lanes)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), d2.cpu().numpy(), tree


def check_links(g: dict, n: int) -> None:
    """Child ids above the parent id and in range, parents pointing back,
    buckets inside [0, n): checked on the host before a query walks the tree."""
    N = len(g["dim"])
    inner = np.flatnonzero(g["dim"] >= 0)
    L = g["left"][inner].astype(np.int64)
    assert (L > inner).all() and (L + 1 < N).all(), "child id out of order or range"
    assert (g["parent"][L] == inner).all() and (g["parent"][L + 1] == inner).all(), "bad parent"
    assert g["parent"][0] == -1
    leaves = np.flatnonzero(g["dim"] < 0)
    st, ct = g["start"][leaves].astype(np.int64), g["count"][leaves].astype(np.int64)
    assert (st >= 0).all() and (ct >= 1).all() and (st + ct <= n).all(), "bucket out of range"
    assert int(ct.sum()) == n, "buckets do not cover the points"


def compare_trees(g: dict, o: oracle.Tree, root: int = 0, off: int = 0) -> int:
    """Walk the GPU tree (from node `root`, rows from `off`: a forest's tree)
    and the oracle tree from their roots in lockstep, a level at a time, and
    require identical split dimensions, split values, ranges and boxes, and
    an identical packed order.  Returns the number of nodes compared."""
    n_t = len(o.perm)
    assert np.array_equal(g["perm"][off:off + n_t].astype(np.int64) - off, o.perm), \
        "packed order differs"
    a = np.array([root], np.int64)
    b = np.array([0], np.int64)
    seen = 0
    while a.size:
        seen += a.size

        def first_bad(ok, what):
            if not ok.all():
                j = int(np.flatnonzero(~ok)[0])
                raise AssertionError(f"{what}: GPU node {a[j]} vs oracle node {b[j]}")
        first_bad((g["start"][a].astype(np.int64) - off == o.start[b])
                  & (g["count"][a] == o.count[b]), "range")
        first_bad((g["lo"][a] == o.lo[b]).all(1) & (g["hi"][a] == o.hi[b]).all(1), "box")
        leaf = o.dim[b] < 0
        first_bad(~leaf | (g["dim"][a] < 0), "GPU splits where the oracle has a leaf")
        ai, bi = a[~leaf], b[~leaf]
        a, b = ai, bi
        first_bad(g["dim"][ai] == o.dim[bi], "split dimension")
        first_bad(g["split"][ai] == o.split[bi], "split value")
        gl = g["left"][ai].astype(np.int64)
        a = np.concatenate([gl, gl + 1])
        b = np.concatenate([o.left[bi], o.right[bi]])
    assert seen == len(o.dim), (seen, len(o.dim))
    if root == 0 and off == 0 and n_t == len(g["perm"]):  # a single tree: nothing else
        assert seen == len(g["dim"]), (seen, len(g["dim"]))
    return seen


def assert_same(a_idx, a_d, b_idx, b_d, what=""):
    bad = np.argwhere((a_idx != b_idx) | (a_d.view(np.uint32) != b_d.view(np.uint32)))
    if len(bad):
        r = int(bad[0][0])
        raise AssertionError(f"{what}: {len(bad)} entries differ; first query {r}: "
                             f"{a_idx[r].tolist()} {a_d[r].tolist()} vs "
                             f"{b_idx[r].tolist()} {b_d[r].tolist()}")
