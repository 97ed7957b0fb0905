"""CPU tests of the oracle against its pins, and proof that the pins catch
plausible mistakes planted in the oracle (compiled variants, CPU only)."""
import os

import numpy as np
import pytest

import oracle
import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_oracle_pin(orc, pin):
    msg = pin(orc)
    assert msg is None, msg


# mutant id -> (what it plants, the pins that must notice)
MUTANTS = {
    1: ("Algorithm 1 radius update taken literally (r' <- d[x])",
        [pins.pin_golden_alg1, pins.pin_kd_equals_bf]),
    2: ("Algorithm 1 far bound taken literally (adds on top of the parent bound)",
        [pins.pin_golden_alg1, pins.pin_kd_equals_bf, pins.pin_1d_window]),
    3: ("strict bound test: equal-distance subtrees pruned",
        [pins.pin_kd_equals_bf, pins.pin_grid_shells]),
    4: ("tie-break reversed (larger index first)",
        [pins.pin_grid_shells]),
    5: ("partition sends x == split to the left",
        [pins.pin_tree_invariants]),
    7: ("distance accumulated with a fused multiply-add",
        [pins.pin_fp32_sum_order]),
    8: ("sample positions shifted",
        [pins.pin_split_rule]),
    9: ("FP64 brute force accumulates in FP32",
        [pins.pin_bf64_exact_rationals, pins.pin_fp64_near_tie]),
}


@pytest.mark.parametrize("mid", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, mid):
    what, catchers = MUTANTS[mid]
    lib = oracle.load(oracle.compile_oracle(str(tmp_path / f"m{mid}.so"), mid))
    failures = [p.__name__ for p in catchers if p(lib) is not None]
    assert failures, f"no pin noticed mutant {mid}: {what}"


def test_oracle_tiny_uniform_kd_equals_bf(orc):
    """The 65,536-point uniform workload: KD32 == BF32 on all 4,096 queries."""
    from paper_1607_08220_amd import inputs
    w = inputs.workload("tiny_uniform")
    T = oracle.build(w.points, w.leaf, lib=orc)
    a = T.query(w.queries, w.k)
    b = oracle.bf32(w.points, w.queries, w.k, lib=orc)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_oracle_depth_matches_log(orc):
    """Depth of the sampled-median tree is close to ceil(log2(n / bucket)); the
    paper reports depth 21 for 50 M points with bucket 32 (Section V-B2), which
    is ceil(log2(5e7 / 32))."""
    from paper_1607_08220_amd import inputs
    assert int(np.ceil(np.log2(5e7 / 32))) == 21
    X = inputs.clustered(1 << 18, seed=5)
    T = oracle.build(X, 32, lib=orc)
    base = int(np.ceil(np.log2(len(X) / 32)))
    assert base <= T.depth <= base + 3, T.depth


def test_vote_regress_merge_hand_examples():
    """Hand-worked cases of the application functions (Section V-C majority
    vote, Section I regression, Section III-B step 5 merge)."""
    labels = np.array([2, 0, 1, 0, 2, 1], np.int32)
    idx = np.array([[4, 1, 3, 0],    # labels 2, 0, 0, 2 -> tie 2:2, the nearer (2) wins
                    [1, 2, 5, -1],   # labels 0, 1, 1     -> 1 with 2 votes
                    [-1, -1, -1, -1],
                    [5, 0, 4, 1]], np.int32)  # 1, 2, 2, 0 -> 2 with 2 votes
    c, v = oracle.vote(idx, labels)
    assert c.tolist() == [2, 1, -1, 2] and v.tolist() == [2, 2, 0, 2]
    vals = np.array([1.0, 2.0 ** -24, 2.0 ** -24, 3.0, 0.5, 1e8], np.float32)
    r = oracle.regress(np.array([[0, 1, 2, -1], [5, 0, -1, -1], [-1, -1, -1, -1]], np.int32), vals)
    # 1 + 2^-24 rounds back to 1 twice (left to right), then / 3
    assert r[0] == np.float32(np.float32(1.0) / np.float32(3.0))
    assert r[1] == np.float32(np.float32(1e8 + 1.0) / np.float32(2.0)) and np.isnan(r[2])
    ia = np.array([[3, 5, -1]], np.int32); da = np.array([[1.0, 2.0, np.inf]], np.float32)
    ib = np.array([[5, 7]], np.int32); db = np.array([[2.0, 2.0]], np.float32)
    oi, od = oracle.merge(ia, da, ib, db, 4)
    assert oi.tolist() == [[3, 5, 7, -1]] and od[0, :3].tolist() == [1.0, 2.0, 2.0]


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc, host code only) runs every entry point on small random, integer and
    constant inputs without a report, and its answers still check out."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-pthread",
           os.path.join(here, "oracle_sanitize_main.c"),
           os.path.join(os.path.dirname(here), "oracle", "oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok: 0 failing cases" in r.stdout and "runtime error" not in r.stderr, r.stderr
