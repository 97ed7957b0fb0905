"""Invariant checks for an exported kd-tree (oracle or GPU), numpy only.

A tree is a mapping with node arrays ``dim`` (-1 = leaf), ``split``, ``left``,
``right``, ``start``, ``count``, ``lo``/``hi`` [nodes, d], and ``perm`` [n]
(packed position -> original index); ``packed`` [n, d] and ``parent`` are
checked when present.  Node 0 is the root.

Invariants (Section III-A of the paper: the tree partitions the input, each
split sends x[dim] < split left, buckets hold at most `leaf` points, buckets
are contiguous after packing):
  * perm is a permutation of 0..n-1 and packed == points[perm]
  * every node is reached exactly once from the root
  * children split their parent's range: left first, then right, both nonempty
  * all points of a left child have x[dim] < split, of a right child >= split
  * a leaf holds <= leaf points unless all its points are identical
  * every node's box is tight (min / max of its points), so every point lies
    inside its leaf's box
"""
from __future__ import annotations

import numpy as np


def _levels(t):
    """Breadth-first node lists from the root; asserts each node is seen once."""
    N = len(t["dim"])
    seen = np.zeros(N, bool)
    levels = []
    cur = np.array([0], np.int64)
    while cur.size:
        assert not seen[cur].any(), "node reached twice"
        seen[cur] = True
        levels.append(cur)
        inner = cur[t["dim"][cur] >= 0]
        cur = np.concatenate([t["left"][inner], t["right"][inner]]).astype(np.int64)
    assert seen.all(), f"{int((~seen).sum())} nodes not reachable from the root"
    return levels


def _seg_reduce(col, starts, counts, fn):
    """fn.reduceat over disjoint segments given by starts/counts (counts > 0)."""
    order = np.argsort(starts, kind="stable")
    s, c = starts[order], counts[order]
    idx = np.empty(2 * len(s), np.int64)
    idx[0::2] = s
    idx[1::2] = s + c
    flat = fn.reduceat(col, idx[:-1] if idx[-1] == len(col) else idx)[0::2]
    out = np.empty_like(flat)
    out[order] = flat
    return out


def check_tree(points: np.ndarray, t: dict, leaf: int, check_parent: bool = True) -> dict:
    X = np.asarray(points, np.float32)
    n, d = X.shape
    perm = np.asarray(t["perm"], np.int64)
    assert perm.shape == (n,)
    assert np.array_equal(np.sort(perm), np.arange(n)), "perm is not a permutation"
    P = X[perm]
    if "packed" in t and t["packed"] is not None:
        assert np.array_equal(np.asarray(t["packed"], np.float32), P), "packed != points[perm]"
    dim, split = np.asarray(t["dim"]), np.asarray(t["split"], np.float32)
    left, right = np.asarray(t["left"], np.int64), np.asarray(t["right"], np.int64)
    start, count = np.asarray(t["start"], np.int64), np.asarray(t["count"], np.int64)
    lo, hi = np.asarray(t["lo"], np.float32), np.asarray(t["hi"], np.float32)
    assert start[0] == 0 and count[0] == n, "root must cover the input"
    levels = _levels(t)
    depth = len(levels) - 1
    for lv in levels:
        # box tightness, per dimension, over the level's disjoint ranges
        for j in range(d):
            mn = _seg_reduce(P[:, j], start[lv], count[lv], np.minimum)
            mx = _seg_reduce(P[:, j], start[lv], count[lv], np.maximum)
            assert np.array_equal(mn, lo[lv, j]), f"box lo not tight (dim {j})"
            assert np.array_equal(mx, hi[lv, j]), f"box hi not tight (dim {j})"
        inner = lv[dim[lv] >= 0]
        leaves = lv[dim[lv] < 0]
        if inner.size:
            L, R = left[inner], right[inner]
            assert (count[L] >= 1).all() and (count[R] >= 1).all(), "empty child"
            assert np.array_equal(start[L], start[inner]), "left child must start the range"
            assert np.array_equal(start[R], start[inner] + count[L]), "right child follows left"
            assert np.array_equal(count[L] + count[R], count[inner]), "children lose points"
            if check_parent and "parent" in t:
                par = np.asarray(t["parent"], np.int64)
                assert np.array_equal(par[L], inner) and np.array_equal(par[R], inner)
            # split sides: max over left < split <= min over right, per split dim
            for j in np.unique(dim[inner]):
                sel = inner[dim[inner] == j]
                lmax = _seg_reduce(P[:, j], start[left[sel]], count[left[sel]], np.maximum)
                rmin = _seg_reduce(P[:, j], start[right[sel]], count[right[sel]], np.minimum)
                assert (lmax < split[sel]).all(), "a left point is not < split"
                assert (rmin >= split[sel]).all(), "a right point is not >= split"
        big = leaves[count[leaves] > leaf]
        for v in big:  # oversized buckets only when all points coincide
            seg = P[start[v]:start[v] + count[v]]
            assert (seg == seg[0]).all(), "oversized leaf with distinct points"
    if check_parent and "parent" in t:
        assert int(np.asarray(t["parent"])[0]) == -1
    n_leaves = int((dim < 0).sum())
    return {"depth": depth, "nodes": len(dim), "leaves": n_leaves}


def check_knn_lists(idx: np.ndarray, d2: np.ndarray) -> None:
    """Each list ascends by (D, idx); padding (-1, +inf) only at the end."""
    idx = np.asarray(idx)
    d2 = np.asarray(d2)
    pad = idx < 0
    assert np.all(np.isinf(d2[pad])), "padding must carry +inf"
    # once padding starts it continues
    assert not np.any(pad[:, :-1] & ~pad[:, 1:]), "padding must be trailing"
    a, b = d2[:, :-1], d2[:, 1:]
    ia, ib = idx[:, :-1], idx[:, 1:]
    ok = (a < b) | ((a == b) & ((ia < ib) | (ib < 0)))
    assert np.all(ok | pad[:, 1:]), "neighbour list not ascending by (D, idx)"
