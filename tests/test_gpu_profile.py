"""Profiling levels of knn_set_profiling, which the bench reads: level 1
records the phase boundaries only; level 2 also times every launch of the
build's partition kernel (one per level pass). Turning profiling on or off
changes no result."""
import numpy as np
import pytest

from gpu_util import assert_same, dev, log
from paper_1607_08220_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_08220_amd as knn
    knn.load_library()
    return knn


def test_profiling_levels(knn):
    import torch
    X = inputs.clustered(300_000, seed=5)
    P, Q = dev(X), dev(X[:4096])
    log(f"[case] profiling levels n={len(X)}")
    out = {}
    try:
        for level in (0, 1, 2):
            knn.knn_set_profiling(level)
            tree = knn.knn_build(P, 32)
            pb = knn.knn_get_profile()
            idx, d2 = knn.knn_query_ex(tree, Q, 8)
            pq = knn.knn_get_profile()
            torch.cuda.synchronize()
            out[level] = (idx.cpu().numpy(), d2.cpu().numpy())
            tree.free()
            if level >= 1:
                assert pb["build_total"] > 0 and pb["build_levels"] > 0
                assert pq["query_total"] > 0 and pq["query_traverse"] > 0
            if level == 2:
                # 300,000 points with subtrees of 1,024: a partition launch per level pass
                assert pb["build_partition_launches"] >= 8
                assert pb["build_partition_ms"] > 0
                assert pb["build_partition_mpts"] > 0
            if level == 1:
                assert pb["build_partition_launches"] == 0
    finally:
        knn.knn_set_profiling(0)
    for level in (1, 2):
        assert_same(out[level][0], out[level][1], out[0][0], out[0][1],
                    f"profiling level {level} vs off")
