"""CPU oracle for exact kd-tree k-NN (test infrastructure only).

Plain C in ``oracle.c`` (built with gcc ``-O2 -ffp-contract=off``), wrapped here
with ctypes over numpy arrays.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may use this package; the GPU library never
does, and the two share no code.

Functions and the passages they follow (arXiv 1607.08220):
  bf32 / bf64   the k-NN problem of Section I, by brute force
  build         the local kd-tree of Section III-A (sampled median, variance
                split dimension, stable index shuffle, buckets, packing)
  query         Algorithm 1 of Section III-B/C with the readings listed at the
                top of oracle.c (R1-R10)
  merge         Section III-B step 5: the k nearest of two candidate lists
  vote          the majority vote of the k neighbours' labels (Section V-C)
  regress       the mean of the neighbours' values (Section I)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC", "-pthread"]


def compile_oracle(out_path: str = _LIB, mutant: int = 0) -> str:
    """Compile oracle.c with gcc; ``mutant`` > 0 plants a numbered mistake
    (used only by the tests that show the pins catch such mistakes)."""
    cmd = ["gcc", *CFLAGS, f"-DORC_MUTANT={int(mutant)}", _SRC, "-o", out_path, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def _bind(lib):
    lib.orc_bf32.argtypes = [_p, _i64, ctypes.c_int, _p, _i64, ctypes.c_int, _p,
                             ctypes.c_float, _p, _p, ctypes.c_int]
    lib.orc_bf32.restype = ctypes.c_int
    lib.orc_bf64.argtypes = [_p, _i64, ctypes.c_int, _p, _i64, ctypes.c_int, _p,
                             ctypes.c_double, _p, _p, ctypes.c_int]
    lib.orc_bf64.restype = ctypes.c_int
    lib.orc_dist32.argtypes = [_p, _p, ctypes.c_int]
    lib.orc_dist32.restype = ctypes.c_float
    lib.orc_build.argtypes = [_p, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int)]
    lib.orc_build.restype = _p
    lib.orc_build_mt.argtypes = [_p, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int)]
    lib.orc_build_mt.restype = _p
    lib.orc_tree_free.argtypes = [_p]
    lib.orc_tree_free.restype = None
    lib.orc_tree_nodes.argtypes = [_p]
    lib.orc_tree_nodes.restype = _i64
    lib.orc_tree_depth.argtypes = [_p]
    lib.orc_tree_depth.restype = ctypes.c_int
    lib.orc_tree_export.argtypes = [_p] * 12
    lib.orc_tree_export.restype = None
    lib.orc_query.argtypes = [_p, _p, _i64, ctypes.c_int, _p, ctypes.c_float, _p, _p,
                              ctypes.c_int, _p]
    lib.orc_query.restype = ctypes.c_int
    return lib


_lib_cache: dict[str, ctypes.CDLL] = {}


def load(path: str = _LIB) -> ctypes.CDLL:
    """Load (compiling first if absent) the oracle shared library."""
    if path not in _lib_cache:
        if path == _LIB and not os.path.exists(path):
            compile_oracle(path)
        _lib_cache[path] = _bind(ctypes.CDLL(path))
    return _lib_cache[path]


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _self(self_ids, m):
    if self_ids is None:
        return None
    s = np.ascontiguousarray(self_ids, dtype=np.int32)
    assert s.shape == (m,)
    return s


def bf32(points, queries, k, self_ids=None, r2=np.inf, nthreads=0, lib=None):
    """Brute-force FP32 k-NN: (idx int32 [m,k], D float32 [m,k])."""
    lib = lib or load()
    X, Q = _f32(points), _f32(queries)
    n, d = X.shape
    m = Q.shape[0]
    s = _self(self_ids, m)
    oi = np.empty((m, k), np.int32)
    od = np.empty((m, k), np.float32)
    rc = lib.orc_bf32(_ptr(X), n, d, _ptr(Q), m, k, _ptr(s), float(r2), _ptr(oi), _ptr(od),
                      nthreads)
    if rc:
        raise ValueError(f"orc_bf32 failed: {rc}")
    return oi, od


def bf64(points, queries, k, self_ids=None, r2=np.inf, nthreads=0, lib=None):
    """Brute-force k-NN in FP64 arithmetic on the FP32 inputs."""
    lib = lib or load()
    X, Q = _f32(points), _f32(queries)
    n, d = X.shape
    m = Q.shape[0]
    s = _self(self_ids, m)
    oi = np.empty((m, k), np.int32)
    od = np.empty((m, k), np.float64)
    rc = lib.orc_bf64(_ptr(X), n, d, _ptr(Q), m, k, _ptr(s), float(r2), _ptr(oi), _ptr(od),
                      nthreads)
    if rc:
        raise ValueError(f"orc_bf64 failed: {rc}")
    return oi, od


def dist32(q, x, lib=None) -> np.float32:
    lib = lib or load()
    q, x = _f32(q), _f32(x)
    return np.float32(lib.orc_dist32(_ptr(q), _ptr(x), q.shape[0]))


@dataclass
class Tree:
    """Host copy of an oracle kd-tree.  Node arrays are indexed by node id;
    ``start``/``count`` give each node's range in the packed order."""
    n: int
    d: int
    leaf: int
    depth: int
    dim: np.ndarray      # int32, -1 for leaves
    split: np.ndarray    # float32
    left: np.ndarray     # int64, -1 for leaves
    right: np.ndarray
    start: np.ndarray    # int64
    count: np.ndarray
    level: np.ndarray    # int32
    lo: np.ndarray       # float32 [nodes, d]
    hi: np.ndarray
    perm: np.ndarray     # int32 [n]: packed position -> original index
    packed: np.ndarray   # float32 [n, d]
    _handle: int = 0
    _lib: object = None

    def query(self, queries, k, self_ids=None, r2=np.inf, nthreads=0, stats=False):
        """Algorithm 1 on this tree; returns (idx, D) or (idx, D, stats[m,3])."""
        Q = _f32(queries)
        m = Q.shape[0]
        s = _self(self_ids, m)
        oi = np.empty((m, k), np.int32)
        od = np.empty((m, k), np.float32)
        st = np.empty((m, 3), np.int64) if stats else None
        rc = self._lib.orc_query(self._handle, _ptr(Q), m, k, _ptr(s), float(r2), _ptr(oi),
                                 _ptr(od), nthreads, _ptr(st))
        if rc:
            raise ValueError(f"orc_query failed: {rc}")
        return (oi, od, st) if stats else (oi, od)

    def close(self):
        if self._handle:
            self._lib.orc_tree_free(self._handle)
            self._handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build(points, leaf=32, max_depth=64, lib=None, nthreads=1) -> Tree:
    """Build the oracle kd-tree (Section III-A).  ``nthreads`` > 1 builds the
    subtrees below the top levels on their own threads; the tree (node ids
    included) is the same as with one thread."""
    lib = lib or load()
    X = _f32(points)
    n, d = X.shape
    st = ctypes.c_int(0)
    if nthreads == 1:
        h = lib.orc_build(_ptr(X), n, d, leaf, max_depth, ctypes.byref(st))
    else:
        if nthreads <= 0:
            nthreads = os.cpu_count() or 1
        h = lib.orc_build_mt(_ptr(X), n, d, leaf, max_depth, nthreads, ctypes.byref(st))
    if not h:
        raise ValueError(f"orc_build failed: {st.value}")
    N = lib.orc_tree_nodes(h)
    arrs = dict(dim=np.empty(N, np.int32), split=np.empty(N, np.float32),
                left=np.empty(N, np.int64), right=np.empty(N, np.int64),
                start=np.empty(N, np.int64), count=np.empty(N, np.int64),
                level=np.empty(N, np.int32), lo=np.empty((N, d), np.float32),
                hi=np.empty((N, d), np.float32), perm=np.empty(n, np.int32),
                packed=np.empty((n, d), np.float32))
    lib.orc_tree_export(h, *[_ptr(arrs[k]) for k in ("dim", "split", "left", "right", "start",
                                                      "count", "level", "lo", "hi", "perm",
                                                      "packed")])
    return Tree(n=n, d=d, leaf=leaf, depth=int(lib.orc_tree_depth(h)), _handle=h, _lib=lib,
                **arrs)


def merge(ia, da, ib, db, k):
    """k smallest (D, idx) keys of two per-query lists (padding idx < 0
    ignored, an entry present in both counted once), padded (-1, +inf)."""
    m = ia.shape[0]
    oi = np.full((m, k), -1, np.int32)
    od = np.full((m, k), np.inf, np.float32)
    for q in range(m):
        keys = {(float(d), int(i)) for i, d in zip(ia[q], da[q]) if i >= 0}
        keys |= {(float(d), int(i)) for i, d in zip(ib[q], db[q]) if i >= 0}
        for j, (d, i) in enumerate(sorted(keys)[:k]):
            oi[q, j], od[q, j] = i, d
    return oi, od


def vote(idx, labels):
    """Majority label of each row of neighbour indices (ascending distance,
    -1 padding): most votes; among equally many, the label whose first
    neighbour comes first; -1 for an empty row.  Returns (label, votes)."""
    m = idx.shape[0]
    out = np.full(m, -1, np.int32)
    votes = np.zeros(m, np.int32)
    for q in range(m):
        row = [int(labels[i]) for i in idx[q] if i >= 0]
        counts = {}
        for c in row:
            counts[c] = counts.get(c, 0) + 1
        best = None
        for c in row:  # the first occurrence order is the distance order
            if best is None or counts[c] > counts[best]:
                best = c
        if best is not None:
            out[q], votes[q] = best, counts[best]
    return out, votes


def regress(idx, values):
    """Mean of the neighbours' values: float32 sum in neighbour order, left to
    right, divided by the count (NaN for an empty row)."""
    m = idx.shape[0]
    out = np.full(m, np.nan, np.float32)
    for q in range(m):
        vals = [np.float32(values[i]) for i in idx[q] if i >= 0]
        if vals:
            acc = vals[0]
            for v in vals[1:]:
                acc = np.float32(acc + v)
            out[q] = np.float32(acc / np.float32(len(vals)))
    return out
