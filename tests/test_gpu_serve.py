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


@pytest.mark.parametrize("budget,streams,slots", [(0, 0, 0), (1 << 20, 2, 0), (64 << 20, 1, 0),
                                                  (0, 0, 4096), (1 << 20, 2, 4096)])
def test_mixed_requests_equal_alone(knn, budget, streams, slots):
    """60 requests of 1..8192 queries, k from {1, 5, 16, 32}, on a 3-D and a
    10-D tree, submitted at once: with batches only (slots 0) and with the
    slot kernels answering the requests of at most 4096 queries."""
    import torch
    rng = np.random.default_rng(11)
    X3 = inputs.clustered(200_003, seed=5, n_clusters=100)
    X10 = inputs.corr_gauss(50_021, 10, seed=6)
    data = [X3, X10]
    trees = [knn.knn_build(dev(X3), 32), knn.knn_build(dev(X10), 32)]
    log(f"[case] serving budget={budget} streams={streams} slots={slots}")
    server = knn.Server(trees, hbm_budget_bytes=budget, streams=streams, slot_max_queries=slots)
    staged = []  # every request's inputs on the device first, then one quick submission loop
    for r in range(60):
        t = int(rng.integers(2))
        b = int(2 ** (rng.random() * 13))
        k = int(rng.choice([1, 5, 16, 32]))
        ids = rng.choice(len(data[t]), size=b, replace=False).astype(np.int32)
        use_self = bool(rng.integers(2))
        Q, S = dev(data[t][ids]), (dev(ids) if use_self else None)
        staged.append((t, Q, S, k, ids, use_self))
    torch.cuda.synchronize()
    reqs = [(server.submit(t, Q, k, self_ids=S), t, Q, S, k, ids, use_self)
            for t, Q, S, k, ids, use_self in staged]
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
    small = sum(len(r[5]) <= 4096 for r in reqs)
    if slots == 0:
        # continuous batching, not a queue of single requests: requests
        # submitted together share batches, and a batch mixes requests of
        # different k
        assert st["slot_requests"] == 0 and st["slot_launches"] == 0, st
        assert st["batches"] < 60 and st["max_requests_per_batch"] > 1, st
        assert st["max_k_per_batch"] > 1, st
        if streams == 0:  # four streams and a large budget: batches overlap on the device
            assert st["peak_batches_in_flight"] >= 2 and st["joined_while_running"] >= 1, st
    else:
        # the small requests went to the slot kernels, the others formed
        # batches (whether a request found its slot kernel already running
        # depends on when the worker took it: test_request_joins_while_others_run
        # shows the join itself)
        assert st["slot_requests"] == small and st["slot_launches"] >= 1, st
        assert st["batches"] >= 1 and st["max_requests_per_batch"] >= 1, st
    server.close()
    for t in trees:
        t.free()


@pytest.mark.parametrize("slots", [0, 4096])
def test_request_joins_while_others_run(knn, slots):
    """A small request submitted after a long one is on the device is
    admitted at once -- on another stream beside the long batch (slots 0),
    or into the running slot kernel, whose workers take the request with the
    fewest queries left first -- and completes first; both results
    equal the requests run alone."""
    import time
    import torch
    rng = np.random.default_rng(12)
    X10 = inputs.corr_gauss(1 << 20, 10, seed=7)
    trees = [knn.knn_build(dev(X10), 32)]
    if slots == 0:
        X3 = inputs.clustered(200_003, seed=8, n_clusters=100)
        trees.append(knn.knn_build(dev(X3), 32))
        other, Xo = 1, X3
    else:  # the same tree and slot kernel
        other, Xo = 0, X10
    server = knn.Server(trees, slot_max_queries=slots)
    ida = rng.choice(len(X10), (1 << 16) if slots == 0 else 4096, replace=False).astype(np.int32)
    idb = rng.choice(len(Xo), 37, replace=False).astype(np.int32)
    QA, SA, QB, SB = dev(X10[ida]), dev(ida), dev(Xo[idb]), dev(idb)
    log(f"[case] a request joins while a long one runs, slots={slots}")
    sa = time.perf_counter()
    ta = server.submit(0, QA, 32, self_ids=SA)
    key = "batches" if slots == 0 else "slot_launches"
    while server.stats()[key] < 1:  # the long request is on the device
        time.sleep(1e-4)
    if slots > 0:
        time.sleep(2e-3)  # well into the long request
    sb = time.perf_counter()
    tb = server.submit(other, QB, 5, self_ids=SB)
    bi, bd, lb = server.wait(tb)
    ai, ad, la = server.wait(ta)
    st = server.stats()
    log(f"  long request {la:.1f} ms, short request {lb:.2f} ms submitted "
        f"{(sb - sa) * 1e3:.2f} ms later; stats {st}")
    if slots == 0:
        assert st["batches"] == 2 and st["peak_batches_in_flight"] == 2, st
    else:
        assert st["slot_requests"] == 2 and st["batches"] == 0 and st["slot_launches"] == 1, st
    assert st["joined_while_running"] == 1, st
    assert (sb - sa) * 1e3 + lb < la, "the short request did not finish while the long one ran"
    for (gi, gd), tr, Q, S, k in (((ai, ad), trees[0], QA, SA, 32),
                                  ((bi, bd), trees[other], QB, SB, 5)):
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


def test_slot_kernel_relaunch(knn):
    """The slot kernel ends once idle and is launched again for the next
    request; requests posted from several threads at once, each answered
    exactly as alone."""
    import threading
    import time
    import torch
    rng = np.random.default_rng(13)
    X = inputs.clustered(100_003, seed=9, n_clusters=50)
    tree = knn.knn_build(dev(X), 32)
    server = knn.Server([tree], slot_max_queries=4096)
    log("[case] slot kernel relaunch")
    ids = [rng.choice(len(X), int(rng.integers(1, 300)), replace=False).astype(np.int32)
           for _ in range(48)]
    Qs = [(dev(X[i]), dev(i)) for i in ids]
    t0 = server.submit(0, Qs[0][0], 7, self_ids=Qs[0][1])
    r0 = server.wait(t0)
    time.sleep(0.05)  # far past the idle time: the launch has ended
    tickets = [None] * len(ids)

    def submit(lo):
        for j in range(1 + lo, len(ids), 4):
            tickets[j] = server.submit(0, Qs[j][0], 1 + j % 17, self_ids=Qs[j][1])
    th = [threading.Thread(target=submit, args=(lo,)) for lo in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    res = [server.wait(t) for t in tickets[1:]]
    st = server.stats()
    log(f"  stats {st}")
    assert st["slot_launches"] >= 2 and st["slot_requests"] == len(ids), st
    for j, (gi, gd, _) in [(0, r0)] + list(enumerate(res, 1)):
        ei, ed = knn.knn_query_ex(tree, Qs[j][0], gi.shape[1], self_ids=Qs[j][1])
        torch.cuda.synchronize()
        assert_same(gi.cpu().numpy(), gd.cpu().numpy(), ei.cpu().numpy(), ed.cpu().numpy(),
                    f"request {j}")
    server.close()
    tree.free()
