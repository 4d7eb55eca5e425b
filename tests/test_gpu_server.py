"""GPU serving: continuous batching must not change any result.

Each request's result (pairs, certificate counts, per-edge counts) served in a
mix of concurrent requests on several graphs equals the same query run alone,
and both equal the oracle.
"""
import threading
import time

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2507_17215_amd import folty, synth

pytestmark = pytest.mark.gpu
INF = folty.DELTA_INF


def say(*a):
    print("[case]", *a, flush=True)


def _graphs():
    gs = [synth.tiny(seed=21), synth.c1_family(20_000, seed=22), synth.bruteforce_size(seed=23)]
    return gs, [folty.Graph(g.n, g.src, g.dst, g.t).build() for g in gs]


def _queries(rng, k, ng):
    out = []
    for _ in range(k):
        out.append((int(rng.integers(0, ng)),
                    dict(delta=int(rng.choice([600, 86400, 400_000, 10**6, INF])),
                         theta=(int(rng.integers(0, 5)), 4), variant=int(rng.choice([0, 3])),
                         universe=int(rng.integers(0, 3)))))
    return out


def test_served_results_equal_alone_results():
    gs, Gs = _graphs()
    rng = np.random.default_rng(7)
    qs = _queries(rng, 60, len(gs))
    alone = [Gs[gi].query(**q) for gi, q in qs]
    oracles = [Oracle(g.n, g.src, g.dst, g.t) for g in gs]
    srv = folty.Server(workers=4, max_batch=8)
    tickets = [None] * len(qs)

    def submitter(idx):
        r = np.random.default_rng(100 + idx[0])
        for i in idx:
            time.sleep(float(r.exponential(0.002)))
            gi, q = qs[i]
            tickets[i] = srv.submit(Gs[gi], **q)

    threads = [threading.Thread(target=submitter, args=(list(range(t, len(qs), 3)),)) for t in range(3)]
    say("server: submitting", len(qs))
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    # a burst on one graph while the others are still queued: requests that wait
    # together share a pass, and passes of several workers run at once
    burst = [(1, dict(delta=int(d), theta=(1, 4), variant=int(v)))
             for d, v in zip(rng.choice([600, 86400, 10**6], size=24), rng.choice([0, 3], size=24))]
    burst_alone = [Gs[gi].query(**q) for gi, q in burst]
    burst_tickets = [srv.submit(Gs[gi], **q) for gi, q in burst]
    served = [srv.wait(t) for t in tickets]
    burst_served = [srv.wait(t) for t in burst_tickets]
    info = srv.info()
    say("server info", info)
    assert info["completed"] == len(qs) + len(burst) and info["rejected"] == 0
    assert info["batches"] > 0 and info["batched_requests"] > info["batches"]
    assert info["peak_concurrent_passes"] > 1
    assert max(s.stats["batch_size"] for s in burst_served) > 1
    for a, s in zip(burst_alone, burst_served):
        assert s.pairs() == a.pairs() and s.n_certificates == a.n_certificates
        assert np.array_equal(s.counts(), a.counts())
    for (gi, q), a, s in zip(qs, alone, served):
        assert s.pairs() == a.pairs()
        assert s.n_certificates == a.n_certificates
        assert np.array_equal(s.counts(), a.counts())
        assert s.stats["latency_ms"] >= s.stats["queue_ms"] >= 0
    for (gi, q), s in list(zip(qs, served))[:12]:
        w = oracles[gi].query(q["delta"], q["theta"][0], q["theta"][1], q["variant"], q["universe"])
        assert np.array_equal(s.counts(), w["counts"]) and s.n_certificates == w["n_certificates"]
    srv.close()


def test_budget_forces_waits_and_rejects_oversized():
    gs, Gs = _graphs()
    rng = np.random.default_rng(8)
    qs = _queries(rng, 20, len(gs))
    # room for roughly one request at a time on the largest graph
    probe = folty.Server(workers=1, hbm_budget_bytes=1 << 40)
    tk = probe.submit(Gs[1], delta=600)
    probe.wait(tk)
    probe.close()
    srv = folty.Server(workers=4, max_batch=1, hbm_budget_bytes=12_000_000)
    say("budget server")
    tickets = []
    for gi, q in qs:
        try:
            tickets.append((gi, q, srv.submit(Gs[gi], **q)))
        except folty.FoltyError as e:
            assert e.code == folty.ENOMEM
            tickets.append((gi, q, None))
    for gi, q, t in tickets:
        if t is None:
            continue
        s = srv.wait(t)
        a = Gs[gi].query(**q)
        assert s.pairs() == a.pairs() and np.array_equal(s.counts(), a.counts())
    info = srv.info()
    say("budget info", info)
    assert info["peak_in_use_bytes"] <= info["budget_bytes"]
    srv.close()
    tiny = folty.Server(workers=1, hbm_budget_bytes=1000)
    with pytest.raises(folty.FoltyError) as ei:
        tiny.submit(Gs[1], delta=600)
    assert ei.value.code == folty.ENOMEM
    assert tiny.info()["rejected"] == 1
    tiny.close()


def test_budget_bounds_device_memory():
    """Under a budget that holds about two requests, the device memory the server
    takes (requests in flight, workspaces kept between passes, cached blocks)
    stays within it: free device memory while serving never falls more than the
    budget (plus a small allowance for runtime objects) below what it was."""
    import torch
    gs = [synth.c1_family(2_000_000, seed=31), synth.c1_family(1_000_000, seed=32), synth.tiny(seed=33)]
    Gs = [folty.Graph(g.n, g.src, g.dst, g.t).build() for g in gs]
    rng = np.random.default_rng(9)
    qs = [(int(rng.integers(0, 2)), dict(delta=int(rng.choice([600, 86400, 10**6])), theta=(1, 4),
                                         variant=int(rng.choice([0, 3])), counts=False)) for _ in range(40)]
    alone = [Gs[gi].query(**q).pairs() for gi, q in qs]
    # what one worker keeps after a request on the largest graph
    probe = folty.Server(workers=1, hbm_budget_bytes=1 << 40)
    probe.wait(probe.submit(Gs[0], delta=10**6, counts=False))
    kept = probe.info()["kept_bytes"]
    probe.close()
    budget = int(2.5 * kept)
    folty.release_cached_memory()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    srv = folty.Server(workers=4, max_batch=4, hbm_budget_bytes=budget)
    say("bounded server: budget", budget, "kept by one worker", kept)
    tickets = [srv.submit(Gs[gi], **q) for gi, q in qs]
    growth = 0
    for (gi, q), a, t in zip(qs, alone, tickets):
        s = srv.wait(t)
        assert s.pairs() == a
        growth = max(growth, free0 - torch.cuda.mem_get_info()[0])
    info = srv.info()
    say("bounded info", info, "largest growth", growth)
    assert info["peak_in_use_bytes"] <= budget
    assert growth <= budget + (32 << 20)
    srv.close()
    folty.release_cached_memory()


def test_poll_and_ticket_errors():
    gs, Gs = _graphs()
    srv = folty.Server(workers=2)
    t = srv.submit(Gs[0], delta=86400, theta=(1, 4))
    r = None
    for _ in range(2000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.001)
    assert r is not None
    assert r.pairs() == Gs[0].query(86400, (1, 4)).pairs()
    with pytest.raises(folty.FoltyError):
        srv.wait(t)  # a ticket is taken once
    with pytest.raises(folty.FoltyError):
        srv.wait(12345)
    srv.close()
