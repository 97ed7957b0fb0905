"""The FP64 cross-check of an FP32 k-NN result (numpy only).

The exact FP32 result (indices and FP32 squared distances, ties by index) is
compared with a brute force in FP64 arithmetic.  Where the two lists differ at
a rank, the two neighbours' FP64 distances a and b decide:

  * |a - b| < 1e-6 max(a, b), or a == b: allowed by the 1e-6 relative rule;
  * otherwise |a - b| <= (d + 2) u (a + b) (1 + (d + 2) u), u = 2^-24: the two
    FP32 distances may legally order the points either way, since each FP32
    distance lies within (d + 2) u D of its exact value (the forward-error
    bound of d subtractions, d squares and d - 1 additions, each rounded
    once).  Such a case is counted apart, not called a bug, provided the FP32
    result is the exact FP32 answer (the caller checks FP32 == brute force);
  * anything else is a real mismatch.

The same test is applied to the sorted FP64 distances of the returned set
against the FP64 brute force's distances rank by rank.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def dist64(X: np.ndarray, q: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """FP64 squared distances of points X[ids] from q, summed left to right."""
    Xd = X[ids].astype(np.float64)
    qd = q.astype(np.float64)
    acc = np.zeros(len(ids))
    for j in range(X.shape[1]):
        t = qd[j] - Xd[:, j]
        acc = acc + t * t
    return acc


def _classify_pair(a: float, b: float, d: int) -> str:
    if a == b or abs(a - b) < 1e-6 * max(a, b):
        return "rule"
    g = (d + 2) * U32
    if abs(a - b) <= g * (a + b) * (1 + g):
        return "fp32"
    return "bad"


def classify(X, Q, idx32, idx64, d64) -> dict:
    """Compare an FP32 result (idx32) with the FP64 brute force (idx64, d64).
    Returns counts of ranks allowed by the 1e-6 rule, of legal FP32 reorders
    beyond it, and the list of real mismatches (row, rank, a, b)."""
    X = np.asarray(X, np.float32)
    Q = np.asarray(Q, np.float32)
    d = X.shape[1]
    out = {"rows": len(Q), "differing_ranks": 0, "rule": 0, "fp32": 0, "bad": []}
    rows = np.flatnonzero((idx32 != idx64).any(1))
    for r in rows:
        valid = idx32[r] >= 0
        if not np.array_equal(valid, idx64[r] >= 0):
            out["bad"].append((int(r), -1, "padding differs", None))
            continue
        mine = dist64(X, Q[r], idx32[r][valid])
        # rank by rank, where the indices differ
        for j in np.flatnonzero(idx32[r][valid] != idx64[r][valid]):
            out["differing_ranks"] += 1
            v = _classify_pair(float(mine[j]), float(d64[r, j]), d)
            if v == "bad":
                out["bad"].append((int(r), int(j), float(mine[j]), float(d64[r, j])))
            else:
                out[v] += 1
        # the multiset of FP64 distances of the returned set, rank by rank
        for j, (a, b) in enumerate(zip(np.sort(mine), d64[r][valid])):
            if _classify_pair(float(a), float(b), d) == "bad":
                out["bad"].append((int(r), int(j), float(a), float(b)))
    return out
