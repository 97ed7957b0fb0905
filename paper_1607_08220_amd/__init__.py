"""Exact kd-tree k-NN on MI355X (gfx950): Python binding of libknn.so.

Argument marshalling only: every step runs in the HIP kernels of libknn.so
(built by ``python -m paper_1607_08220_amd.build``).  PyTorch supplies device
memory and the current stream.  If the library is missing the import of any
function below raises; there is no CPU fallback.

    import torch, paper_1607_08220_amd as knn
    tree = knn.knn_build(points_cuda_f32, leaf_size=32)
    idx, d2 = knn.knn_query(tree, queries_cuda_f32, k=8)
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknn.so")

KNN_OK, KNN_EINVAL, KNN_ENOMEM, KNN_EDEVICE, KNN_EDEPTH, KNN_ENOTFINITE = 0, -1, -2, -3, -4, -5
KNN_MAX_DIM, KNN_MAX_K, KNN_PHASES, KNN_QUERY_STATS, KNN_SERVER_STATS = 16, 64, 12, 9, 10
PHASES = ("build_ingest", "build_levels", "build_finish", "build_compact", "build_total",
          "query_locate", "query_group", "query_traverse", "query_total",
          "build_partition_ms", "build_partition_launches", "build_partition_mpts")


class KnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"knn error {code}: {msg}")
        self.code = code


class _BuildParams(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("subtree_points", ctypes.c_int32), ("split_block_nodes", ctypes.c_int32)]


class _QueryParams(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("leaf_batch", ctypes.c_int32),
                ("stats", ctypes.c_void_p), ("traversal", ctypes.c_int32),
                ("team_lanes", ctypes.c_int32)]


class _ServerParams(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("slot_max_queries", ctypes.c_int32), ("slot_workgroups_per_cu", ctypes.c_int32),
                ("slot_idle_us", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("subtree_points", ctypes.c_int32),
                ("nodes", ctypes.c_int64), ("leaves", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("trees", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class _Host(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("dim", "split", "left", "parent", "start", "count", "lo", "hi", "perm",
                 "packed")]


_lib = None
EXPORTED = ("knn_build", "knn_build_ex", "knn_build_batch", "knn_query", "knn_query_ex",
            "knn_query_noalloc", "knn_query_batch", "knn_query_radius", "knn_merge", "knn_classify", "knn_regress",
            "knn_server_create", "knn_server_create_ex",
            "knn_server_submit", "knn_server_wait", "knn_server_stats", "knn_server_destroy",
            "knn_build_plan_create", "knn_build_plan_run", "knn_build_plan_finish",
            "knn_build_plan_tree", "knn_build_plan_destroy",
            "knn_tree_free", "knn_tree_errors", "knn_tree_info", "knn_tree_export",
            "knn_last_error", "knn_strerror", "knn_release_memory", "knn_set_profiling",
            "knn_get_profile")


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libknn.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_1607_08220_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.knn_build.argtypes = [vp, i64, i32, i32, vp, ctypes.POINTER(vp)]
    lib.knn_build_ex.argtypes = [vp, i64, i32, ctypes.POINTER(_BuildParams), vp,
                                 ctypes.POINTER(vp)]
    lib.knn_build_batch.argtypes = [vp, vp, i32, i32, ctypes.POINTER(_BuildParams), vp,
                                    ctypes.POINTER(vp)]
    lib.knn_build_plan_create.argtypes = [i64, i32, vp, i32, ctypes.POINTER(_BuildParams), vp,
                                          ctypes.POINTER(vp)]
    lib.knn_build_plan_run.argtypes = [vp, vp, vp]
    lib.knn_build_plan_finish.argtypes = [vp, vp, ctypes.POINTER(vp)]
    lib.knn_build_plan_tree.argtypes = [vp]
    lib.knn_build_plan_destroy.argtypes = [vp]
    lib.knn_query.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    lib.knn_query_batch.argtypes = [vp, vp, vp, i64, i32, vp, ctypes.c_float,
                                    ctypes.POINTER(_QueryParams), vp, vp, vp]
    lib.knn_query_ex.argtypes = [vp, vp, i64, i32, vp, ctypes.c_float,
                                 ctypes.POINTER(_QueryParams), vp, vp, vp]
    lib.knn_query_noalloc.argtypes = [vp, vp, i64, i32, vp, ctypes.c_float,
                                      ctypes.POINTER(_QueryParams), vp, vp, vp]
    lib.knn_query_radius.argtypes = [vp, vp, i64, i32, vp, vp, ctypes.POINTER(_QueryParams), vp,
                                     vp, vp]
    lib.knn_merge.argtypes = [vp, vp, i32, vp, vp, i32, i64, i32, vp, vp, vp]
    lib.knn_server_create.argtypes = [ctypes.POINTER(vp), i32, i64, i32, ctypes.POINTER(vp)]
    lib.knn_server_create_ex.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(_ServerParams),
                                         ctypes.POINTER(vp)]
    lib.knn_server_submit.argtypes = [vp, i32, vp, i64, i32, vp, vp, vp,
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.knn_server_wait.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
    lib.knn_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.knn_server_destroy.argtypes = [vp]
    lib.knn_classify.argtypes = [vp, i64, i32, vp, vp, vp, vp]
    lib.knn_regress.argtypes = [vp, i64, i32, vp, vp, vp]
    lib.knn_tree_free.argtypes = [vp]
    lib.knn_tree_errors.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.knn_tree_info.argtypes = [vp, ctypes.POINTER(_Info)]
    lib.knn_tree_export.argtypes = [vp, ctypes.POINTER(_Host)]
    lib.knn_last_error.argtypes = []
    lib.knn_last_error.restype = ctypes.c_char_p
    lib.knn_strerror.argtypes = [ctypes.c_int]
    lib.knn_strerror.restype = ctypes.c_char_p
    lib.knn_release_memory.argtypes = []
    lib.knn_set_profiling.argtypes = [i32]
    lib.knn_get_profile.argtypes = [ctypes.POINTER(ctypes.c_float)]
    for name in EXPORTED:
        if name not in ("knn_last_error", "knn_strerror", "knn_build_plan_tree"):
            getattr(lib, name).restype = ctypes.c_int
    lib.knn_build_plan_tree.restype = vp
    _lib = lib
    return lib


def _check(rc: int):
    if rc != KNN_OK:
        lib = load_library()
        raise KnnError(rc, f"{lib.knn_strerror(rc).decode()}: {lib.knn_last_error().decode()}")


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev_f32(t, name, cols=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 [rows, dim] tensor")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name} has {t.shape[1]} columns, expected {cols}")
    return t


class Tree:
    """A kd-tree resident in device memory (owns it until free())."""

    def __init__(self, handle: int, dim: int, device, owned: bool = True):
        self._h = ctypes.c_void_p(handle)
        self.dim = dim
        self.device = device
        self._owned = owned  # False: a build plan's tree, freed with the plan

    @property
    def handle(self):
        if not self._h.value:
            raise ValueError("tree already freed")
        return self._h

    def info(self) -> dict:
        return knn_tree_info(self)

    def query(self, queries, k, self_ids=None, r2_max=math.inf, order=0, out=None):
        return knn_query_ex(self, queries, k, self_ids=self_ids, r2_max=r2_max, order=order,
                            out=out)

    def export(self) -> dict:
        return knn_tree_export(self)

    def free(self):
        if self._h.value:
            if self._owned:
                _check(load_library().knn_tree_free(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def knn_build_ex(points, leaf_size: int = 0, max_depth: int = 0, subtree_points: int = 0,
                 split_block_nodes: int = 0) -> Tree:
    """Build the kd-tree over ``points`` (CUDA float32 [n, dim])."""
    lib = load_library()
    _dev_f32(points, "points")
    p = _BuildParams(leaf_size, max_depth, subtree_points, split_block_nodes)
    out = ctypes.c_void_p()
    _check(lib.knn_build_ex(ctypes.c_void_p(points.data_ptr()), points.shape[0], points.shape[1],
                            ctypes.byref(p), _stream(points), ctypes.byref(out)))
    return Tree(out.value, points.shape[1], points.device)


def knn_build(points, leaf_size: int = 32) -> Tree:
    lib = load_library()
    _dev_f32(points, "points")
    out = ctypes.c_void_p()
    _check(lib.knn_build(ctypes.c_void_p(points.data_ptr()), points.shape[0], points.shape[1],
                         leaf_size, _stream(points), ctypes.byref(out)))
    return Tree(out.value, points.shape[1], points.device)


def knn_build_batch(points, offsets, leaf_size: int = 0, max_depth: int = 0,
                    subtree_points: int = 0, split_block_nodes: int = 0) -> Tree:
    """Build one tree per row range: tree t over rows offsets[t]..offsets[t+1]-1
    of ``points`` (CUDA float32 [N, dim]); ``offsets`` is a host sequence of
    trees + 1 increasing integers starting at 0."""
    lib = load_library()
    _dev_f32(points, "points")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or len(off) < 2 or off[-1] != points.shape[0]:
        raise ValueError("offsets must be trees + 1 values ending at the number of rows")
    p = _BuildParams(leaf_size, max_depth, subtree_points, split_block_nodes)
    out = ctypes.c_void_p()
    _check(lib.knn_build_batch(ctypes.c_void_p(points.data_ptr()),
                               off.ctypes.data_as(ctypes.c_void_p), len(off) - 1,
                               points.shape[1], ctypes.byref(p), _stream(points),
                               ctypes.byref(out)))
    return Tree(out.value, points.shape[1], points.device)


class BuildPlan:
    """A build plan (knn_build_plan_*): the kd-tree build for a fixed point
    count, dimension and forest layout (``offsets``, host sequence, or None
    for one tree), with all device memory taken at creation.  ``run(points)``
    only enqueues kernels on the current stream (no allocation, copy or wait),
    so it can be captured in a ``torch.cuda.CUDAGraph`` and replayed over new
    point values; ``finish()`` waits and raises the latest run's error.
    ``tree`` is the plan's tree (the same handle for the plan's life)."""

    def __init__(self, n: int, dim: int, offsets=None, leaf_size: int = 0, max_depth: int = 0,
                 subtree_points: int = 0, split_block_nodes: int = 0, device=None):
        import torch
        lib = load_library()
        self.device = torch.device(device if device is not None else "cuda")
        self.n, self.dim = int(n), int(dim)
        off_ptr, trees = None, 1
        if offsets is not None:
            off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
            if off.ndim != 1 or len(off) < 2 or off[-1] != n:
                raise ValueError("offsets must be trees + 1 values ending at n")
            self._off = off
            off_ptr, trees = off.ctypes.data_as(ctypes.c_void_p), len(off) - 1
        p = _BuildParams(leaf_size, max_depth, subtree_points, split_block_nodes)
        out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            _check(lib.knn_build_plan_create(self.n, self.dim, off_ptr, trees, ctypes.byref(p), st,
                                             ctypes.byref(out)))
        self._h = out
        self.tree = Tree(lib.knn_build_plan_tree(self._h), self.dim, self.device, owned=False)

    @property
    def handle(self):
        if not self._h.value:
            raise ValueError("plan already destroyed")
        return self._h

    def run(self, points):
        _dev_f32(points, "points", self.dim)
        if points.shape[0] != self.n:
            raise ValueError(f"points has {points.shape[0]} rows, the plan {self.n}")
        _check(load_library().knn_build_plan_run(self.handle, ctypes.c_void_p(points.data_ptr()),
                                                 _stream(points)))

    def finish(self) -> Tree:
        import torch
        out = ctypes.c_void_p()
        st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _check(load_library().knn_build_plan_finish(self.handle, st, ctypes.byref(out)))
        return self.tree

    def destroy(self):
        if self._h.value:
            self.tree._h = ctypes.c_void_p(0)
            _check(load_library().knn_build_plan_destroy(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def knn_build_plan_create(n: int, dim: int, offsets=None, leaf_size: int = 0,
                          max_depth: int = 0, subtree_points: int = 0,
                          split_block_nodes: int = 0) -> BuildPlan:
    return BuildPlan(n, dim, offsets=offsets, leaf_size=leaf_size, max_depth=max_depth,
                     subtree_points=subtree_points, split_block_nodes=split_block_nodes)


def knn_build_plan_run(plan: BuildPlan, points) -> None:
    plan.run(points)


def knn_build_plan_finish(plan: BuildPlan) -> Tree:
    return plan.finish()


def knn_build_plan_tree(plan: BuildPlan) -> Tree:
    return plan.tree


def knn_build_plan_destroy(plan: BuildPlan) -> None:
    plan.destroy()


def _outputs(queries, k, out):
    import torch
    m = queries.shape[0]
    if out is None:
        return (torch.empty((m, k), dtype=torch.int32, device=queries.device),
                torch.empty((m, k), dtype=torch.float32, device=queries.device))
    idx, d2 = out
    if idx.shape != (m, k) or d2.shape != (m, k) or idx.dtype != torch.int32 \
            or d2.dtype != torch.float32 or not idx.is_contiguous() or not d2.is_contiguous():
        raise ValueError("out must be (int32 [m,k], float32 [m,k]) contiguous tensors")
    return idx, d2


def knn_query(tree: Tree, queries, k: int, out=None):
    """k nearest neighbours: (int32 [m,k] indices, float32 [m,k] squared distances)."""
    lib = load_library()
    _dev_f32(queries, "queries", tree.dim)
    idx, d2 = _outputs(queries, k, out)
    _check(lib.knn_query(tree.handle, ctypes.c_void_p(queries.data_ptr()), queries.shape[0], k,
                         ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                         _stream(queries)))
    return idx, d2


def knn_query_ex(tree: Tree, queries, k: int, self_ids=None, r2_max: float = math.inf,
                 order: int = 0, out=None, stats=None, leaf_batch: int = 0, traversal: int = 0,
                 team_lanes: int = 0):
    """knn_query with self exclusion (int32 [m], -1 = none), radius and order.
    ``stats``: optional CUDA int64 [KNN_QUERY_STATS] tensor the traversal adds
    its counters to (see knn_query_params in knn.h)."""
    import torch
    lib = load_library()
    _dev_f32(queries, "queries", tree.dim)
    idx, d2 = _outputs(queries, k, out)
    sp = None
    if self_ids is not None:
        if not (isinstance(self_ids, torch.Tensor) and self_ids.is_cuda
                and self_ids.dtype == torch.int32 and self_ids.is_contiguous()
                and self_ids.shape == (queries.shape[0],)):
            raise TypeError("self_ids must be a contiguous CUDA int32 [m] tensor")
        sp = ctypes.c_void_p(self_ids.data_ptr())
    st = None
    if stats is not None:
        if not (isinstance(stats, torch.Tensor) and stats.is_cuda and stats.dtype == torch.int64
                and stats.numel() >= KNN_QUERY_STATS and stats.is_contiguous()):
            raise TypeError(f"stats must be a contiguous CUDA int64 tensor of "
                            f"{KNN_QUERY_STATS} counters")
        st = stats.data_ptr()
    p = _QueryParams(order, leaf_batch, st, traversal, team_lanes)
    _check(lib.knn_query_ex(tree.handle, ctypes.c_void_p(queries.data_ptr()), queries.shape[0],
                            k, sp, ctypes.c_float(r2_max), ctypes.byref(p),
                            ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                            _stream(queries)))
    return idx, d2


def knn_query_noalloc(tree: Tree, queries, k: int, self_ids=None, r2_max: float = math.inf,
                      order: int = 0, out=None, leaf_batch: int = 0, traversal: int = 0,
                      team_lanes: int = 0):
    """knn_query_ex on the library's static device workspace (the call
    allocates no device memory; calls that overlap on one device race).
    ``out`` (the result tensors) must be given: allocating them here would
    defeat the purpose."""
    lib = load_library()
    _dev_f32(queries, "queries", tree.dim)
    if out is None:
        raise ValueError("knn_query_noalloc writes into caller tensors: pass out=(idx, d2)")
    idx, d2 = _outputs(queries, k, out)
    m = queries.shape[0]
    sp = _dev_i32_vec(self_ids, "self_ids", m) if self_ids is not None else None
    p = _QueryParams(order, leaf_batch, None, traversal, team_lanes)
    _check(lib.knn_query_noalloc(tree.handle, ctypes.c_void_p(queries.data_ptr()), m, k, sp,
                                 ctypes.c_float(r2_max), ctypes.byref(p),
                                 ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                                 _stream(queries)))
    return idx, d2


def _dev_i32_vec(t, name, m):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32
            and t.is_contiguous() and t.shape == (m,)):
        raise TypeError(f"{name} must be a contiguous CUDA int32 [{m}] tensor")
    return ctypes.c_void_p(t.data_ptr())


def knn_query_batch(forest: Tree, queries, tree_ids, k: int, self_ids=None,
                    r2_max: float = math.inf, order: int = 0, out=None, leaf_batch: int = 0,
                    traversal: int = 0, team_lanes: int = 0):
    """k nearest neighbours of each query within its own tree of a forest
    (``tree_ids``: CUDA int32 [m])."""
    lib = load_library()
    _dev_f32(queries, "queries", forest.dim)
    m = queries.shape[0]
    idx, d2 = _outputs(queries, k, out)
    tp = _dev_i32_vec(tree_ids, "tree_ids", m)
    sp = _dev_i32_vec(self_ids, "self_ids", m) if self_ids is not None else None
    p = _QueryParams(order, leaf_batch, None, traversal, team_lanes)
    _check(lib.knn_query_batch(forest.handle, ctypes.c_void_p(queries.data_ptr()), tp, m, k, sp,
                               ctypes.c_float(r2_max), ctypes.byref(p),
                               ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                               _stream(queries)))
    return idx, d2


def knn_query_radius(tree: Tree, queries, k: int, r2, self_ids=None, order: int = 0, out=None,
                     leaf_batch: int = 0, traversal: int = 0, team_lanes: int = 0):
    """k nearest neighbours with one squared radius per query (CUDA float32 [m])."""
    import torch
    lib = load_library()
    _dev_f32(queries, "queries", tree.dim)
    m = queries.shape[0]
    if not (isinstance(r2, torch.Tensor) and r2.is_cuda and r2.dtype == torch.float32
            and r2.is_contiguous() and r2.shape == (m,)):
        raise TypeError("r2 must be a contiguous CUDA float32 [m] tensor")
    idx, d2 = _outputs(queries, k, out)
    sp = _dev_i32_vec(self_ids, "self_ids", m) if self_ids is not None else None
    p = _QueryParams(order, leaf_batch, None, traversal, team_lanes)
    _check(lib.knn_query_radius(tree.handle, ctypes.c_void_p(queries.data_ptr()), m, k, sp,
                                ctypes.c_void_p(r2.data_ptr()), ctypes.byref(p),
                                ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                                _stream(queries)))
    return idx, d2


def knn_merge(a, b, k: int, out=None):
    """Merge two (idx int32 [m,ka], dist2 float32 [m,ka]) lists into the k nearest."""
    import torch
    lib = load_library()
    (ia, da), (ib, db) = a, b
    m = ia.shape[0]
    for t, dt in ((ia, torch.int32), (da, torch.float32), (ib, torch.int32), (db, torch.float32)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.dim() == 2
                and t.is_contiguous() and t.shape[0] == m):
            raise TypeError("lists must be contiguous CUDA (int32, float32) [m, k] tensors")
    if ia.shape != da.shape or ib.shape != db.shape:
        raise ValueError("index and distance lists differ in shape")
    if out is None:
        out = (torch.empty((m, k), dtype=torch.int32, device=ia.device),
               torch.empty((m, k), dtype=torch.float32, device=ia.device))
    oi, od = out
    _check(lib.knn_merge(ctypes.c_void_p(ia.data_ptr()), ctypes.c_void_p(da.data_ptr()),
                         ia.shape[1], ctypes.c_void_p(ib.data_ptr()),
                         ctypes.c_void_p(db.data_ptr()), ib.shape[1], m, k,
                         ctypes.c_void_p(oi.data_ptr()), ctypes.c_void_p(od.data_ptr()),
                         _stream(ia)))
    return oi, od


class Server:
    """Serving loop over resident trees (knn_server_* in knn.h).  Keep the
    trees, and every submitted request's tensors, alive until waited for."""

    def __init__(self, trees, hbm_budget_bytes: int = 0, streams: int = 0,
                 slot_max_queries: int = 0, slot_workgroups_per_cu: int = 0,
                 slot_idle_us: int = 0):
        """``slot_max_queries``: 0 (default), every request forms batches;
        n > 0, requests of at most n queries go to the trees' slot kernels
        (persistent launches that take requests over while they run)."""
        lib = load_library()
        self._trees = list(trees)
        arr = (ctypes.c_void_p * len(self._trees))(*[t.handle.value for t in self._trees])
        h = ctypes.c_void_p()
        p = _ServerParams(hbm_budget_bytes, streams, slot_max_queries, slot_workgroups_per_cu,
                          slot_idle_us)
        _check(lib.knn_server_create_ex(arr, len(self._trees), ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, tree: int, queries, k: int, self_ids=None, out=None) -> int:
        """Queue a request; returns its ticket.  Results land in ``out`` (or in
        tensors allocated here) once :meth:`wait` returns."""
        lib = load_library()
        dim = self._trees[tree].dim if 0 <= tree < len(self._trees) else None  # else the library rejects it
        _dev_f32(queries, "queries", dim)
        m = queries.shape[0]
        idx, d2 = _outputs(queries, k, out)
        sp = _dev_i32_vec(self_ids, "self_ids", m) if self_ids is not None else None
        ticket = ctypes.c_int64()
        _check(lib.knn_server_submit(self._h, tree, ctypes.c_void_p(queries.data_ptr()), m, k, sp,
                                     ctypes.c_void_p(idx.data_ptr()),
                                     ctypes.c_void_p(d2.data_ptr()), ctypes.byref(ticket)))
        self._keep[ticket.value] = (queries, self_ids, idx, d2)
        return ticket.value

    def wait(self, ticket: int):
        """Block until the request is done: (idx, dist2, latency_ms)."""
        lat = ctypes.c_double()
        _check(load_library().knn_server_wait(self._h, ticket, ctypes.byref(lat)))
        _, _, idx, d2 = self._keep.pop(ticket)
        return idx, d2, lat.value

    def stats(self) -> dict:
        buf = (ctypes.c_int64 * KNN_SERVER_STATS)()
        _check(load_library().knn_server_stats(self._h, buf))
        return dict(zip(("requests", "batches", "queries", "peak_bytes", "max_requests_per_batch",
                         "peak_batches_in_flight", "max_k_per_batch", "joined_while_running",
                         "slot_requests", "slot_launches"), list(buf)))

    def close(self):
        if self._h and self._h.value:
            _check(load_library().knn_server_destroy(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def knn_server_create(trees, hbm_budget_bytes: int = 0, streams: int = 0) -> Server:
    return Server(trees, hbm_budget_bytes, streams)


def knn_server_create_ex(trees, hbm_budget_bytes: int = 0, streams: int = 0,
                         slot_max_queries: int = 0, slot_workgroups_per_cu: int = 0,
                         slot_idle_us: int = 0) -> Server:
    return Server(trees, hbm_budget_bytes, streams, slot_max_queries, slot_workgroups_per_cu,
                  slot_idle_us)


def knn_server_submit(server: Server, tree: int, queries, k: int, self_ids=None, out=None) -> int:
    return server.submit(tree, queries, k, self_ids=self_ids, out=out)


def knn_server_wait(server: Server, ticket: int):
    return server.wait(ticket)


def knn_server_stats(server: Server) -> dict:
    return server.stats()


def knn_server_destroy(server: Server):
    server.close()


def _idx_list(idx):
    import torch
    if not (isinstance(idx, torch.Tensor) and idx.is_cuda and idx.dtype == torch.int32
            and idx.dim() == 2 and idx.is_contiguous()):
        raise TypeError("idx must be a contiguous CUDA int32 [m, k] tensor")
    return idx.shape[0], idx.shape[1]


def knn_classify(idx, labels, votes: bool = False):
    """Majority label of each query's neighbours: int32 [m] (and the vote counts)."""
    import torch
    m, k = _idx_list(idx)
    if not (isinstance(labels, torch.Tensor) and labels.is_cuda and labels.dtype == torch.int32
            and labels.is_contiguous()):
        raise TypeError("labels must be a contiguous CUDA int32 tensor")
    out = torch.empty(m, dtype=torch.int32, device=idx.device)
    vo = torch.empty(m, dtype=torch.int32, device=idx.device) if votes else None
    _check(load_library().knn_classify(ctypes.c_void_p(idx.data_ptr()), m, k,
                                       ctypes.c_void_p(labels.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(vo.data_ptr()) if votes else None,
                                       _stream(idx)))
    return (out, vo) if votes else out


def knn_regress(idx, values):
    """Mean of each query's neighbours' values: float32 [m]."""
    import torch
    m, k = _idx_list(idx)
    if not (isinstance(values, torch.Tensor) and values.is_cuda and values.dtype == torch.float32
            and values.is_contiguous()):
        raise TypeError("values must be a contiguous CUDA float32 tensor")
    out = torch.empty(m, dtype=torch.float32, device=idx.device)
    _check(load_library().knn_regress(ctypes.c_void_p(idx.data_ptr()), m, k,
                                      ctypes.c_void_p(values.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _stream(idx)))
    return out


def knn_tree_info(tree: Tree) -> dict:
    info = _Info()
    _check(load_library().knn_tree_info(tree.handle, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in _Info._fields_}


def knn_tree_export(tree: Tree) -> dict:
    """Host copy of the tree as numpy arrays (see knn_tree_host in knn.h)."""
    info = knn_tree_info(tree)
    N, n, d = info["nodes"], info["n"], info["dim"]
    arrs = dict(dim=np.empty(N, np.int32), split=np.empty(N, np.float32),
                left=np.empty(N, np.int32), parent=np.empty(N, np.int32),
                start=np.empty(N, np.int32), count=np.empty(N, np.int32),
                lo=np.empty((N, d), np.float32), hi=np.empty((N, d), np.float32),
                perm=np.empty(n, np.int32), packed=np.empty((n, d), np.float32))
    h = _Host(**{k: v.ctypes.data for k, v in arrs.items()})
    _check(load_library().knn_tree_export(tree.handle, ctypes.byref(h)))
    arrs["right"] = np.where(arrs["left"] >= 0, arrs["left"] + 1, -1)
    arrs["depth"] = info["depth"]
    return arrs


def knn_tree_free(tree: Tree):
    tree.free()


def knn_tree_errors(tree: Tree, stream=None) -> int:
    """Count of queries that named an out-of-range tree id since the last
    call (waits for the stream, clears the count); raises KnnError
    (KNN_EINVAL) when it is nonzero."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(tree.device)
    c = ctypes.c_int64()
    _check(load_library().knn_tree_errors(tree.handle, ctypes.c_void_p(s.cuda_stream),
                                          ctypes.byref(c)))
    return c.value


def knn_release_memory():
    """Wait for the device and return the build pool's unused memory to it."""
    _check(load_library().knn_release_memory())


def knn_strerror(code: int) -> str:
    return load_library().knn_strerror(code).decode()


def knn_last_error() -> str:
    return load_library().knn_last_error().decode()


def knn_set_profiling(enable):
    """False/0: off; True/1: phase events; 2: also an event around every
    launch of the build's partition kernel (which idles the device a few
    microseconds per event)."""
    level = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
    _check(load_library().knn_set_profiling(level))


def knn_get_profile() -> dict:
    buf = (ctypes.c_float * KNN_PHASES)()
    _check(load_library().knn_get_profile(buf))
    return {name: float(buf[i]) for i, name in enumerate(PHASES)}
