"""Pick the schedule knobs of a workload by measuring them on the device.

The knobs change speed only, never results: the bucket size (Section III-A1
reports 32 as the best for its data; other data and hardware may differ),
the traversal's leaf batch (how many of a wavefront's 64 lanes must hold a
bucket before it scans), the query order (grouped by home leaf, or as given)
and the traversal form (stack-free walk from the home leaf, Algorithm 1's
explicit stack with a lane per query, or with a wavefront per query).  ``tune`` builds the trees for each bucket size, times the
queries for every leaf batch, order and traversal form, and returns the
fastest combination.  Every
timed call goes through the C-ABI (``knn_build_batch``/``knn_query_batch``
for forests, ``knn_build_ex``/``knn_query_ex`` otherwise).
"""
from __future__ import annotations

import itertools
import time

import numpy as np

import paper_1607_08220_amd as knn


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - a)
    return best


def tune(points, queries, k: int, self_ids=None, offsets=None, tree_ids=None,
         leaf_sizes=(16, 32, 64), leaf_batches=(32, 48, 64), orders=(0, 1),
         traversals=(1, 2, 3, (4, 16), (4, 32)), reps: int = 3,
         build_weight: float = 1.0) -> dict:
    """Return {"leaf_size", "leaf_batch", "order", "traversal", "team_lanes", "ms",
    "table"}: the knobs minimising build_weight * build time + query time on
    this sample.  A traversal entry is a form (1, 2, 3) or (4, lanes) for a
    team of lanes per query.  The best form depends on the batch size (one
    wavefront or a team per query pays off for small batches), so tune on
    batches of the size the knobs will serve, or leave forms 3 and 4 out of
    ``traversals`` when the sample is smaller.
    ``points``/``queries`` are CUDA float32 tensors; for a forest pass the host
    ``offsets`` and the CUDA int32 ``tree_ids`` of the queries."""
    table = []
    for leaf in leaf_sizes:
        if offsets is not None:
            build = lambda: knn.knn_build_batch(points, offsets, leaf_size=leaf)  # noqa: E731
        else:
            build = lambda: knn.knn_build_ex(points, leaf_size=leaf)  # noqa: E731
        t_build = _time(lambda: build().free(), reps)
        tree = build()
        for lb, order, form in itertools.product(leaf_batches, orders, traversals):
            trav, team = form if isinstance(form, tuple) else (form, 0)
            if offsets is not None:
                q = lambda: knn.knn_query_batch(tree, queries, tree_ids, k,  # noqa: E731
                                                self_ids=self_ids, order=order, leaf_batch=lb,
                                                traversal=trav, team_lanes=team)
            else:
                q = lambda: knn.knn_query_ex(tree, queries, k, self_ids=self_ids,  # noqa: E731
                                             order=order, leaf_batch=lb, traversal=trav,
                                             team_lanes=team)
            t_query = _time(q, reps)
            table.append({"leaf_size": leaf, "leaf_batch": lb, "order": order, "traversal": trav,
                          "team_lanes": team, "build_ms": t_build * 1e3,
                          "query_ms": t_query * 1e3,
                          "ms": (build_weight * t_build + t_query) * 1e3})
        tree.free()
    best = min(table, key=lambda r: r["ms"])
    return {**{key: best[key] for key in ("leaf_size", "leaf_batch", "order", "traversal",
                                          "team_lanes", "ms")},
            "table": table}
