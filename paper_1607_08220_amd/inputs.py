"""Seeded synthetic workloads (numpy only; no k-NN arithmetic lives here).

The paper measures on cosmology (Gadget N-body), plasma (VPIC) and Daya Bay
datasets that are not available; these generators stand in for them with the
same shapes: 3-D clustered positions, 4-D space+energy records, and correlated
Gaussian feature vectors.  Every generator draws from
``numpy.random.Generator(PCG64(seed))`` in FP64 and rounds to FP32 (RNE).
The same module feeds the GPU path and the CPU oracle.

Workloads:
  uniform        n points uniform in [0,1)^d
  clustered      80 % of points in Gaussian clusters (sigma 1e-3, Pareto(1.5)
                 sizes, centres uniform) + 20 % uniform background; shuffled
  plasma         x from density 1 + 0.5 sin(2 pi 4 x) on [0,1), y ~ U[0,1),
                 z ~ U[0,0.25), energy LogNormal(0,1) min-max scaled to [0,1)
  corr_gauss     x = Q diag(i^-1/2) z, Q Haar-orthogonal, z ~ N(0, I_d)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n: int, d: int = 3, seed: int = 1001) -> np.ndarray:
    return _rng(seed).random((n, d)).astype(np.float32)


def clustered(n: int, seed: int = 1002, n_clusters: int = 10_000, sigma: float = 1e-3,
              frac_clustered: float = 0.8, alpha: float = 1.5) -> np.ndarray:
    """3-D cosmology-like points: Pareto-sized isotropic Gaussian clusters plus a
    uniform background, in random order."""
    rng = _rng(seed)
    n_bg = int(round((1.0 - frac_clustered) * n))
    n_cl = n - n_bg
    n_clusters = max(1, min(n_clusters, n_cl)) if n_cl > 0 else 0
    out = np.empty((n, 3), np.float32)
    out[:n_bg] = rng.random((n_bg, 3))
    if n_cl > 0:
        w = (1.0 - rng.random(n_clusters)) ** (-1.0 / alpha)  # Pareto, x_m = 1
        raw = n_cl * w / w.sum()
        sizes = np.floor(raw).astype(np.int64)
        rem = n_cl - int(sizes.sum())
        if rem > 0:  # remainder by largest fractional part
            order = np.argsort(-(raw - sizes), kind="stable")
            sizes[order[:rem]] += 1
        centers = rng.random((n_clusters, 3))
        pos = n_bg
        chunk = 1 << 22
        owner = np.repeat(np.arange(n_clusters, dtype=np.int64), sizes)
        for a in range(0, n_cl, chunk):
            b = min(n_cl, a + chunk)
            pts = centers[owner[a:b]] + sigma * rng.standard_normal((b - a, 3))
            out[pos + a:pos + b] = pts
        del owner
    perm = rng.permutation(n)
    return out[perm]


def plasma(n: int, seed: int = 1003) -> np.ndarray:
    """4-D plasma-like records (x, y, z, energy)."""
    rng = _rng(seed)
    out = np.empty((n, 4), np.float32)
    # x by rejection from 1 + 0.5 sin(2 pi 4 x) (max 1.5) on [0, 1)
    filled = 0
    while filled < n:
        want = int((n - filled) * 1.6) + 1024
        x = rng.random(want)
        u = rng.random(want) * 1.5
        keep = x[u < 1.0 + 0.5 * np.sin(2.0 * np.pi * 4.0 * x)]
        take = min(n - filled, keep.shape[0])
        out[filled:filled + take, 0] = keep[:take]
        filled += take
    out[:, 1] = rng.random(n)
    out[:, 2] = 0.25 * rng.random(n)
    E = rng.lognormal(0.0, 1.0, n)
    e = (E - E.min()) / (E.max() - E.min()) * (1.0 - 2.0 ** -24)
    out[:, 3] = e
    return out


def corr_gauss(n: int, d: int, seed: int) -> np.ndarray:
    """Correlated Gaussian with eigenvalues decaying as 1/i (random rotation)."""
    rng = _rng(seed)
    A = rng.standard_normal((d, d))
    Qm, R = np.linalg.qr(A)
    Qm = Qm * np.sign(np.diag(R))[None, :]  # Haar sign fix
    scale = np.arange(1, d + 1, dtype=np.float64) ** -0.5
    z = rng.standard_normal((n, d))
    return ((z * scale[None, :]) @ Qm.T).astype(np.float32)


def sample_queries(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct data indices (queries drawn from the data, self excluded)."""
    rng = _rng(seed)
    if m >= n:
        return rng.permutation(n).astype(np.int32)[:m]
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)[
        rng.permutation(m)]


@dataclass
class ForestWorkload:
    name: str
    points: np.ndarray      # all trees' points, concatenated [N, d]
    offsets: np.ndarray     # [trees + 1] int64 row offsets
    queries: np.ndarray     # [m, d]
    tree_ids: np.ndarray    # [m] int32: the tree each query searches
    self_ids: np.ndarray    # [m] int32: the query's own row (excluded)
    k: int
    leaf: int


def forest(n_trees: int, d: int = 6, lo_exp: float = 10.0, hi_exp: float = 20.0,
           q_per_tree: int = 1024, seed: int = 1004, k: int = 5, leaf: int = 32) -> ForestWorkload:
    """Many independent trees of log-uniform sizes round(2^(lo + (hi - lo) u)),
    each a correlated Gaussian with its own rotation (eigenvalues 1/i), each
    queried by up to q_per_tree of its own points with the point excluded.
    Tree t draws from its own stream (seed, t), so a prefix of the trees does
    not depend on how many follow."""
    sizes = np.rint(2.0 ** (lo_exp + (hi_exp - lo_exp) * _rng(seed).random(n_trees))).astype(np.int64)
    sizes = np.maximum(sizes, 1)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts, qs, tids, sids = [], [], [], []
    for t in range(n_trees):
        rng = np.random.Generator(np.random.PCG64([seed, t]))
        A = rng.standard_normal((d, d))
        Qm, R = np.linalg.qr(A)
        Qm = Qm * np.sign(np.diag(R))[None, :]
        scale = np.arange(1, d + 1, dtype=np.float64) ** -0.5
        X = ((rng.standard_normal((int(sizes[t]), d)) * scale[None, :]) @ Qm.T).astype(np.float32)
        m = min(q_per_tree, int(sizes[t]))
        own = rng.choice(int(sizes[t]), size=m, replace=False).astype(np.int64)
        pts.append(X)
        qs.append(X[own])
        tids.append(np.full(m, t, np.int32))
        sids.append((own + offsets[t]).astype(np.int32))
    return ForestWorkload(f"forest{n_trees}", np.concatenate(pts), offsets, np.concatenate(qs),
                          np.concatenate(tids), np.concatenate(sids), k, leaf)


@dataclass
class Workload:
    name: str
    points: np.ndarray
    queries: np.ndarray
    self_ids: np.ndarray | None
    k: int
    leaf: int


def workload(name: str, scale: float = 1.0) -> Workload:
    """The named workloads; ``scale`` < 1 shrinks n and m (same distribution).

    tiny_uniform   n = 65,536 uniform 3-D, 4,096 fresh uniform queries, k = 5
    cosmo_clustered n = 2^26 clustered 3-D, 2^22 data queries (self excluded), k = 8
    plasma_4d      n = 2^28 4-D, 2^24 data queries (self excluded), k = 16
    """
    if name == "tiny_uniform":
        n, m = max(1, int(65_536 * scale)), max(1, int(4_096 * scale))
        return Workload(name, uniform(n, 3, 1001), uniform(m, 3, 2001), None, 5, 32)
    if name == "cosmo_clustered":
        n, m = max(2, int((1 << 26) * scale)), max(1, int((1 << 22) * scale))
        X = clustered(n, 1002)
        ids = sample_queries(n, m, 2002)
        return Workload(name, X, X[ids], ids, 8, 32)
    if name == "plasma_4d":
        n, m = max(2, int((1 << 28) * scale)), max(1, int((1 << 24) * scale))
        X = plasma(n, 1003)
        ids = sample_queries(n, m, 2003)
        return Workload(name, X, X[ids], ids, 16, 32)
    raise KeyError(name)
