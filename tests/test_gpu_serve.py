"""Serving loop: requests of uneven size, k and tree, submitted while others
run, each give exactly the result of the same request alone."""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("budget,streams", [(0, 0), (1 << 20, 2), (64 << 20, 1)])
def test_mixed_requests_equal_alone(knn, budget, streams):
    import torch
    rng = np.random.default_rng(11)
    X3 = inputs.clustered(200_003, seed=5, n_clusters=100)
    X10 = inputs.corr_gauss(50_021, 10, seed=6)
    data = [X3, X10]
    trees = [knn.knn_build(dev(X3), 32), knn.knn_build(dev(X10), 32)]
    log(f"[case] serving budget={budget} streams={streams}")
    server = knn.Server(trees, hbm_budget_bytes=budget, streams=streams)
    reqs = []
    for r in range(60):
        t = int(rng.integers(2))
        b = int(2 ** (rng.random() * 13))
        k = int(rng.choice([1, 5, 16, 32]))
        ids = rng.choice(len(data[t]), size=b, replace=False).astype(np.int32)
        use_self = bool(rng.integers(2))
        Q, S = dev(data[t][ids]), (dev(ids) if use_self else None)
        ticket = server.submit(t, Q, k, self_ids=S)
        reqs.append((ticket, t, Q, S, k, ids, use_self))
    lat = []
    for ticket, t, Q, S, k, ids, use_self in reqs:
        gi, gd, ms = server.wait(ticket)
        lat.append(ms)
        ai, ad = knn.knn_query_ex(trees[t], Q, k, self_ids=S)
        torch.cuda.synchronize()
        assert_same(gi.cpu().numpy(), gd.cpu().numpy(), ai.cpu().numpy(), ad.cpu().numpy(),
                    f"request {ticket} tree {t} m={len(ids)} k={k}")
        if ticket % 10 == 0:  # and against brute force
            bi, bd = oracle.bf32(data[t], data[t][ids], k, self_ids=ids if use_self else None)
            assert_same(gi.cpu().numpy(), gd.cpu().numpy(), bi, bd, f"request {ticket} vs oracle")
    st = server.stats()
    log(f"  stats {st}, latency p50 {np.percentile(lat, 50):.3f} ms")
    assert st["requests"] == 60 and st["queries"] == sum(len(r[5]) for r in reqs)
    assert min(lat) >= 0.0
    # continuous batching, not a queue of single requests: requests submitted
    # together share batches, and a batch mixes requests of different k
    assert st["batches"] < 60 and st["max_requests_per_batch"] > 1, st
    assert st["max_k_per_batch"] > 1, st
    if streams == 0:  # four streams and a large budget: batches overlap on the device
        assert st["peak_batches_in_flight"] >= 2 and st["joined_while_running"] >= 1, st
    server.close()
    for t in trees:
        t.free()


def test_request_joins_while_others_run(knn):
    """A small request submitted after a long batch has been launched is
    admitted at once on another stream, runs beside it and completes first;
    both results equal the requests run alone."""
    import time
    import torch
    rng = np.random.default_rng(12)
    X10 = inputs.corr_gauss(1 << 20, 10, seed=7)
    X3 = inputs.clustered(200_003, seed=8, n_clusters=100)
    trees = [knn.knn_build(dev(X10), 32), knn.knn_build(dev(X3), 32)]
    server = knn.Server(trees)
    ida = rng.choice(len(X10), 1 << 16, replace=False).astype(np.int32)
    idb = rng.choice(len(X3), 37, replace=False).astype(np.int32)
    QA, SA, QB, SB = dev(X10[ida]), dev(ida), dev(X3[idb]), dev(idb)
    log("[case] a request joins while a long batch runs")
    sa = time.perf_counter()
    ta = server.submit(0, QA, 32, self_ids=SA)
    while server.stats()["batches"] < 1:  # the long batch is on the device
        time.sleep(1e-4)
    sb = time.perf_counter()
    tb = server.submit(1, QB, 5, self_ids=SB)
    bi, bd, lb = server.wait(tb)
    ai, ad, la = server.wait(ta)
    st = server.stats()
    log(f"  long request {la:.1f} ms, short request {lb:.2f} ms submitted "
        f"{(sb - sa) * 1e3:.2f} ms later; stats {st}")
    assert st["batches"] == 2 and st["peak_batches_in_flight"] == 2, st
    assert st["joined_while_running"] == 1, st
    assert (sb - sa) * 1e3 + lb < la, "the short request did not finish while the long one ran"
    for (gi, gd), tr, Q, S, k in (((ai, ad), trees[0], QA, SA, 32), ((bi, bd), trees[1], QB, SB, 5)):
        ei, ed = knn.knn_query_ex(tr, Q, k, self_ids=S)
        torch.cuda.synchronize()
        assert_same(gi.cpu().numpy(), gd.cpu().numpy(), ei.cpu().numpy(), ed.cpu().numpy(),
                    "served vs alone")
    server.close()
    for t in trees:
        t.free()


def test_server_argument_errors(knn):
    X = dev(np.random.default_rng(1).random((100, 3)).astype(np.float32))
    t = knn.knn_build(X, 32)
    server = knn.Server([t])
    with pytest.raises(knn.KnnError):
        server.submit(1, X, 3)            # no such tree
    with pytest.raises(knn.KnnError):
        server.submit(0, X, 65)           # k too large
    ticket = server.submit(0, X, 3)
    gi, gd, _ = server.wait(ticket)
    assert gi.shape == (100, 3)
    server.close()
    t.free()
