"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

Each pin takes an oracle library handle and returns None on success or a short
failure message, so the same pin can be run on the real oracle (must pass) and
on an oracle built with a planted mistake (must fail).
"""
from __future__ import annotations

import json
import os
import struct
from fractions import Fraction

import numpy as np

import fp64rule
import oracle
from treecheck import check_tree

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _hexf(h):
    return struct.unpack(">f", bytes.fromhex(h[2:]))[0]


def _bits(x):
    return struct.unpack(">I", struct.pack(">f", float(x)))[0]


# --- golden worked examples -------------------------------------------------

def pin_golden_alg1(lib):
    """Hand-worked counterexamples to the printed radius update and far-child
    bound of Algorithm 1; the corrected algorithm must give the true k-NN."""
    for name in ("alg1_radius_update.json", "alg1_cell_bound.json"):
        g = _gold(name)
        X = np.array(g["points"], np.float32)
        q = np.array([g["query"]], np.float32)
        T = oracle.build(X, g["leaf"], lib=lib)
        i, dd = T.query(q, g["k"])
        if i[0].tolist() != g["expected_idx"] or dd[0].tolist() != g["expected_d2"]:
            return f"{name}: tree gives {i[0].tolist()} {dd[0].tolist()}"
        i, dd = oracle.bf32(X, q, g["k"], lib=lib)
        if i[0].tolist() != g["expected_idx"]:
            return f"{name}: brute force gives {i[0].tolist()}"
    return None


def pin_fp32_sum_order(lib):
    """Hand-derived FP32 value that distinguishes the left-to-right unfused sum
    from a fused or reordered one."""
    g = _gold("fp32_sum_order.json")
    q = np.array(g["q"], np.float32)
    x = np.array([_hexf(h) for h in g["x_hex"]], np.float32)
    got = oracle.dist32(q, x, lib=lib)
    want = _hexf(g["expected_d2_hex"])
    if _bits(got) != _bits(want):
        return f"dist32 = {float(got)!r}, expected {want!r}"
    i, dd = oracle.bf32(x[None, :], q[None, :], 1, lib=lib)
    if _bits(dd[0, 0]) != _bits(want):
        return "brute force distance differs from the hand-derived value"
    return None


# --- closed forms -------------------------------------------------------------

def grid_points(side=9, seed=7):
    g = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    return g[rng.permutation(len(g))].astype(np.float32)


def pin_grid_shells(lib, leafs=(1, 4, 32)):
    """Integer grid: neighbours of the centre fall on shells of r_3(D) points
    (OEIS A005875), D exact, ties ascending by index; the k = 5 answer is the
    five lowest-index unit neighbours."""
    r3 = _gold("sum_of_three_squares.json")["r3"]
    X = grid_points()
    c = int(np.flatnonzero((X == 4).all(1))[0])
    q = X[c:c + 1]
    k = sum(r3[1:7])  # shells D = 1..6
    for solver in ["bf"] + [f"kd{l}" for l in leafs]:
        if solver == "bf":
            i, dd = oracle.bf32(X, q, k, self_ids=np.array([c]), lib=lib)
        else:
            T = oracle.build(X, int(solver[2:]), lib=lib)
            i, dd = T.query(q, k, self_ids=np.array([c]))
        i, dd = i[0], dd[0]
        for D in range(1, 7):
            sel = dd == D
            if sel.sum() != r3[D]:
                return f"{solver}: {int(sel.sum())} neighbours at D={D}, expected {r3[D]}"
            ids = i[sel]
            if not (np.diff(ids) > 0).all():
                return f"{solver}: ties at D={D} not ascending by index"
            exact = ((X[ids] - q) ** 2).sum(1)
            if not (exact == D).all():
                return f"{solver}: shell D={D} holds a point at another distance"
        unit = np.sort(np.flatnonzero(((X - q) ** 2).sum(1) == 1))[:5]
        i5 = oracle.bf32(X, q, 5, self_ids=np.array([c]), lib=lib)[0][0] if solver == "bf" \
            else T.query(q, 5, self_ids=np.array([c]))[0][0]
        if i5.tolist() != unit.tolist():
            return f"{solver}: k=5 gives {i5.tolist()}, expected {unit.tolist()}"
    return None


def pin_bf64_exact_on_integers(lib, seed=11):
    """Small integer coordinates: every FP32 step is exact, so FP32 and FP64
    brute force agree exactly (indices and distances)."""
    rng = np.random.default_rng(seed)
    for d in (1, 2, 3, 5, 8):
        X = rng.integers(-60, 61, size=(700, d)).astype(np.float32)
        Q = rng.integers(-60, 61, size=(40, d)).astype(np.float32)
        i32, d32 = oracle.bf32(X, Q, 9, lib=lib)
        i64, d64 = oracle.bf64(X, Q, 9, lib=lib)
        if not (np.array_equal(i32, i64) and np.array_equal(d32.astype(np.float64), d64)):
            return f"d={d}: FP32 and FP64 brute force differ on integer data"
    return None


def pin_dist32_error_bound(lib, seed=12):
    """|D32 - D| <= (d+2) u D (1 + (d+2) u), u = 2^-24, against exact rationals."""
    rng = np.random.default_rng(seed)
    u = Fraction(1, 1 << 24)
    for d in (1, 2, 3, 4, 7, 10, 16):
        for _ in range(200):
            q = rng.standard_normal(d).astype(np.float32)
            x = (q + rng.standard_normal(d) * 10.0 ** rng.integers(-6, 2)).astype(np.float32)
            got = Fraction(float(oracle.dist32(q, x, lib=lib)))
            ex = sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(q, x))
            g = (d + 2) * u
            if abs(got - ex) > g * ex * (1 + g):
                return f"d={d}: D32 outside the forward-error bound"
    return None


def pin_bf64_exact_rationals(lib, seed=14):
    """FP64 brute force against exact rational arithmetic on non-integer data
    of mixed scales: every returned distance lies within d * 2^-52 of the
    exact squared distance (relative), and the neighbours are the exact k
    nearest, ordered by exact distance then index.  An FP32 accumulation
    misses the distance bound by about eight orders of magnitude."""
    rng = np.random.default_rng(seed)
    for d in (1, 2, 3, 5, 10, 16):
        n, m, k = 120, 6, 9
        scale = 10.0 ** rng.integers(-3, 3, size=(1, d))
        X = (rng.standard_normal((n, d)) * scale).astype(np.float32)
        Q = (rng.standard_normal((m, d)) * scale).astype(np.float32)
        oi, od = oracle.bf64(X, Q, k, lib=lib)
        for r in range(m):
            q = [Fraction(float(v)) for v in Q[r]]
            exact = [sum((qj - Fraction(float(xj))) ** 2 for qj, xj in zip(q, X[i]))
                     for i in range(n)]
            want = sorted(range(n), key=lambda i: (exact[i], i))[:k]
            if oi[r].tolist() != want:
                return f"d={d} query {r}: FP64 brute force {oi[r].tolist()}, exact {want}"
            bound = Fraction(d, 1 << 52)
            for j, i in enumerate(want):
                if abs(Fraction(float(od[r, j])) - exact[i]) > bound * exact[i]:
                    return f"d={d} query {r} rank {j}: FP64 distance outside d * 2^-52"
    return None


def pin_fp64_near_tie(lib):
    """Hand-derived near-tie that FP32 and FP64 order differently
    (tests/golden/fp64_near_tie.json): FP32 ties two points and orders them
    by index, FP64 separates them by 2^-26; the gap is inside the 1e-6 rule."""
    g = _gold("fp64_near_tie.json")
    X = np.array([[_hexf(h) for h in row] for row in g["points_hex"]], np.float32)
    q = np.array([g["q"]], np.float32)
    i32, d32 = oracle.bf32(X, q, g["k"], lib=lib)
    if i32[0].tolist() != g["fp32_idx"] or d32[0].tolist() != g["fp32_d2"]:
        return f"FP32 brute force gives {i32[0].tolist()} {d32[0].tolist()}"
    i64, d64 = oracle.bf64(X, q, g["k"], lib=lib)
    if i64[0].tolist() != g["fp64_idx"] or d64[0].tolist() != g["fp64_d2"]:
        return f"FP64 brute force gives {i64[0].tolist()} {d64[0].tolist()}"
    T = oracle.build(X, 1, lib=lib)
    ti, td = T.query(q, g["k"])
    if ti[0].tolist() != g["fp32_idx"]:
        return f"KD32 gives {ti[0].tolist()}"
    c = fp64rule.classify(X, q, ti, i64, d64)
    if c["bad"] or c["rule"] != 2:
        return f"cross-check classification {c}"
    return None


def pin_fp64_cross_check(lib, seed=13):
    """KD32 equals BF32, and against FP64 brute force every differing rank is
    allowed by the 1e-6 relative rule or is a legal FP32 reorder (inside the
    FP32 forward-error bound); both kinds are counted, any other is a bug."""
    rng = np.random.default_rng(seed)
    for d in (2, 3, 4, 10, 16):
        # uniform data, and integer lattice points moved by ~3e-7 with queries
        # at cell centres: many neighbours whose distances FP32 cannot separate
        near = (rng.integers(0, 6, size=(3000, d)) +
                rng.standard_normal((3000, d)) * 3e-7).astype(np.float32)
        sets = [("uniform", rng.random((3000, d)).astype(np.float32),
                 rng.random((64, d)).astype(np.float32)),
                ("near-ties", near, (rng.integers(0, 6, size=(64, d)) + 0.5).astype(np.float32))]
        for name, X, Q in sets:
            i32, d32 = oracle.bf32(X, Q, 8, lib=lib)
            T = oracle.build(X, 8, lib=lib)
            ti, td = T.query(Q, 8)
            if not (np.array_equal(ti, i32) and np.array_equal(td, d32)):
                return f"{name} d={d}: KD32 != BF32"
            i64, d64 = oracle.bf64(X, Q, 8, lib=lib)
            c = fp64rule.classify(X, Q, ti, i64, d64)
            if c["bad"]:
                return f"{name} d={d}: mismatch beyond the FP32 error bound {c['bad'][:3]}"
            if name == "near-ties" and c["differing_ranks"] == 0:
                return f"d={d}: the near-tie set produced no FP32/FP64 difference"
            # the check itself: a list with a far point in place of a neighbour fails
            wrong = ti.copy()
            wrong[0, 0] = int(np.argmax(fp64rule.dist64(X, Q[0], np.arange(len(X)))))
            if not fp64rule.classify(X, Q, wrong, i64, d64)["bad"]:
                return f"{name} d={d}: the cross-check accepted a wrong neighbour"
    return None


# --- brute force on small inputs (pins the tree and Algorithm 1) ---------------

def _cases(seed):
    rng = np.random.default_rng(seed)
    for d in (1, 2, 3, 4, 6, 10, 16):
        for leaf in (1, 3, 8, 32):
            n = int(rng.integers(1, 600))
            X = rng.random((n, d)).astype(np.float32)
            yield f"uniform d={d} leaf={leaf} n={n}", X, leaf
    X = np.repeat(rng.random((5, 3)).astype(np.float32), 40, axis=0)  # duplicates
    yield "duplicates", X[rng.permutation(len(X))], 4
    yield "identical", np.full((300, 2), 0.25, np.float32), 8
    t = rng.random(400).astype(np.float32)
    yield "collinear", np.stack([t, 2 * t, -t], 1).astype(np.float32), 2
    yield "grid", grid_points(7, seed), 5
    yield "int-1d", rng.integers(0, 30, size=(500, 1)).astype(np.float32), 1
    X = np.concatenate([np.zeros((1500, 2)), rng.random((3, 2))]).astype(np.float32)
    yield "heavy-dup", X[rng.permutation(len(X))], 8


def pin_kd_equals_bf(lib, seed=21):
    """KD32 == BF32 bit for bit on small random and adversarial sets, with
    k from 1 to more than n, self exclusion and a radius bound."""
    rng = np.random.default_rng(seed + 1)
    for name, X, leaf in _cases(seed):
        n, d = X.shape
        Q = np.concatenate([X[rng.integers(0, n, 30)],
                            rng.random((20, d)).astype(np.float32) * 3 - 1]).astype(np.float32)
        self_ids = np.concatenate([rng.integers(0, n, 30), -np.ones(20)]).astype(np.int32)
        T = oracle.build(X, leaf, lib=lib)
        for k in (1, 2, 5, 17, n + 3):
            for r2 in (np.inf, 0.01):
                for sid in (None, self_ids):
                    a = T.query(Q, k, self_ids=sid, r2=r2)
                    b = oracle.bf32(X, Q, k, self_ids=sid, r2=r2, lib=lib)
                    if not (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])):
                        return f"{name} k={k} r2={r2} self={sid is not None}: KD32 != BF32"
    return None


def pin_1d_window(lib, seed=31):
    """d = 1: the k-NN set is what a two-pointer walk outward from q over the
    sorted data returns (all ties at the k-th distance kept, then (D, idx))."""
    rng = np.random.default_rng(seed)
    for trial in range(6):
        n = int(rng.integers(50, 3000))
        X = (rng.integers(0, n // 3 + 2, n) * 0.37).astype(np.float32)[:, None]
        Q = (rng.random(60) * (n // 3 + 8) * 0.37 - 1).astype(np.float32)[:, None]
        leaf = int(rng.choice([1, 2, 5, 32]))
        T = oracle.build(X, leaf, lib=lib)
        order = np.argsort(X[:, 0], kind="stable")
        vals = X[order, 0]
        for k in (1, 4, 13):
            got_i, got_d = T.query(Q, k)
            for r in range(len(Q)):
                q = Q[r, 0]
                D = lambda p: np.float32(np.float32(q - vals[p]) * np.float32(q - vals[p]))
                R = int(np.searchsorted(vals, q))
                L = R - 1
                taken = []
                while L >= 0 or R < n:
                    dl = D(L) if L >= 0 else np.float32(np.inf)
                    dr = D(R) if R < n else np.float32(np.inf)
                    if len(taken) >= k and min(dl, dr) > taken[k - 1][0]:
                        break
                    if dl <= dr:
                        taken.append((dl, int(order[L])))
                        L -= 1
                    else:
                        taken.append((dr, int(order[R])))
                        R += 1
                    taken.sort()
                want = taken[:k]
                if [w[1] for w in want] != got_i[r].tolist():
                    return f"trial {trial} k={k}: tree {got_i[r].tolist()} vs walk {want}"
    return None


# --- tree construction ----------------------------------------------------------

def pin_tree_invariants(lib, seed=41):
    for name, X, leaf in _cases(seed):
        T = oracle.build(X, leaf, lib=lib)
        t = {k: getattr(T, k) for k in ("dim", "split", "left", "right", "start", "count",
                                         "lo", "hi", "perm", "packed")}
        try:
            check_tree(X, t, leaf)
        except AssertionError as e:
            return f"{name}: {e}"
    return None


def recount_split(X, idx_sorted, leaf):
    """The split the sampled-median rule must choose for a node whose points
    (in their pre-split order, i.e. ascending original index) are idx_sorted;
    computed by direct counting, without histogram or pairwise sums.
    Returns (dims_allowed, split) or None for a leaf."""
    c = len(idx_sorted)
    if c <= leaf:
        return None
    s = min(1024, c)
    pos = ((2 * np.arange(s, dtype=np.int64) + 1) * c) // (2 * s)
    S = X[idx_sorted[pos]].astype(np.float64)
    var = S.var(axis=0)
    if var.max() == 0.0:
        pts = X[idx_sorted].astype(np.float64)
        ext = pts.max(0) - pts.min(0)
        if ext.max() == 0.0:
            return None
        j = int(np.argmax(ext))
        return [j], float(X[idx_sorted, j].max())
    near = np.flatnonzero(var >= var.max() * (1 - 1e-9))
    j = int(near[0]) if len(near) == 1 else None
    out = {}
    for jj in near:
        col = X[idx_sorted, jj]
        cand = np.unique(X[idx_sorted[pos], jj])
        C = (col[None, :] < cand[:, None]).sum(1)
        ok = (C > 0) & (C < c)
        gap = np.abs(2 * C - c).astype(np.int64)
        gap[~ok] = np.iinfo(np.int64).max
        out[int(jj)] = float(cand[int(np.argmin(gap))])
    if j is not None:
        return [j], out[j]
    return list(out), out


def pin_split_rule(lib, seed=51):
    """Every split matches the sampled-median rule recounted directly: sample
    positions in ascending-index order, max-variance dimension (near-ties
    allowed either way), the sample value whose count below is closest to half
    (ties to the smaller value)."""
    rng = np.random.default_rng(seed)
    sets = [(rng.random((5000, 3)).astype(np.float32), 16),
            (np.repeat(rng.random((50, 2)).astype(np.float32), 60, 0), 8),
            (rng.integers(0, 4, size=(3000, 4)).astype(np.float32), 3),
            (np.concatenate([np.zeros((4000, 2)), rng.random((30, 2))]).astype(np.float32), 4)]
    for X, leaf in sets:
        X = X[rng.permutation(len(X))]
        T = oracle.build(X, leaf, lib=lib)
        for v in range(len(T.dim)):
            ids = np.sort(T.perm[T.start[v]:T.start[v] + T.count[v]])
            want = recount_split(X, ids, leaf)
            if want is None:
                if T.dim[v] >= 0:
                    return f"node {v} split although it must be a leaf"
                continue
            dims, split = want
            if T.dim[v] not in dims:
                return f"node {v}: dim {T.dim[v]} not the max-variance dim {dims}"
            sv = split if not isinstance(split, dict) else split[int(T.dim[v])]
            if np.float32(sv) != T.split[v]:
                return f"node {v}: split {T.split[v]} != recounted {sv}"
    return None


ALL_PINS = [pin_golden_alg1, pin_fp32_sum_order, pin_grid_shells, pin_bf64_exact_on_integers,
            pin_dist32_error_bound, pin_bf64_exact_rationals, pin_fp64_near_tie,
            pin_fp64_cross_check, pin_kd_equals_bf, pin_1d_window,
            pin_tree_invariants, pin_split_rule]
