"""k-NN classification and regression on the GPU equal the oracle's vote and
mean on the same neighbour lists (and on lists padded with -1)."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, log
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


@pytest.mark.parametrize("k", [1, 5, 16, 64])
def test_classify_and_regress_match_oracle(knn, k):
    import torch
    rng = np.random.default_rng(k)
    X = inputs.clustered(50_000, seed=31, n_clusters=20)
    labels = (np.floor(X[:, 0] * 3) + 3 * (X[:, 2] > 0.5)).astype(np.int32)  # 6 spatial classes
    values = (X[:, 1] * 10.0).astype(np.float32)
    ids = rng.choice(len(X), 2000, replace=False).astype(np.int32)
    log(f"[case] classify k={k}")
    t = knn.knn_build(dev(X), 32)
    r2 = 1e-4 if k == 64 else np.inf  # some rows padded with -1
    idx, _ = knn.knn_query_ex(t, dev(X[ids]), k, self_ids=dev(ids), r2_max=r2)
    c, v = knn.knn_classify(idx, dev(labels), votes=True)
    mean = knn.knn_regress(idx, dev(values))
    torch.cuda.synchronize()
    hi = idx.cpu().numpy()
    oc, ov = oracle.vote(hi, labels)
    om = oracle.regress(hi, values)
    assert np.array_equal(c.cpu().numpy(), oc) and np.array_equal(v.cpu().numpy(), ov)
    gm = mean.cpu().numpy()
    assert np.array_equal(np.isnan(gm), np.isnan(om))
    assert np.array_equal(gm[~np.isnan(gm)].view(np.uint32), om[~np.isnan(om)].view(np.uint32))
    t.free()
