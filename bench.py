"""Benchmark: the thresholded exists-exists-forall query on a 70M-edge temporal graph.

One step is the whole hot path over device-resident inputs: load + validate the
edge list, build the index (grouping sort, static edge table, degrees, core
numbers and the degeneracy rank, orientation, triangle counts), then one query
(wedge enumeration + closing probe, temporal tests, threshold, pair reduction)
ending with the sorted solution pairs on the host.

Prints ONE JSON line.  `value` is wedge checks per second over the whole step.
Outside the timed steps it checks every per-edge count, the pair list, the
certificate counts and |Sol| of the timed query against the CPU oracle run over
all edges, and reports that oracle run's wall time as the CPU baseline; checks
the small and medium workloads, the batched plans and served requests against
the oracle; and times the batched and served forms against the same queries run
one at a time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "wedge-checks/sec & query wall-time at 70M edges (bit-exact); batched queries/sec, p99"
HBM_PEAK_GBS = 8000.0
# vector ALU issue of the whole chip: 256 CUs x 4 SIMDs, one wave64 instruction
# every 4 cycles per SIMD, 2.4 GHz
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
# the query's dominant kernel, the sources it is compiled from, and the committed
# counter summary (FETCH_SIZE / WRITE_SIZE per dispatch and the copy-kernel
# calibration, SQ_INSTS_VALU) that gives its measured HBM traffic and issue rate
ROOF_KERNEL = "k_tri_enum<FilterSink<0, 0, false> >"
ROOF_SOURCES = ("paper_2507_17215_amd/csrc/tri_device.h", "paper_2507_17215_amd/csrc/query.hip")
TRAFFIC_SUMMARY = "profiles/k_tri_enum_filter_large_70M_pmc.md"
COPY_PROBE_BYTES = 1 << 30


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=float, default=1.0,
                   help="fraction of the 70M-edge workload (for quick local runs)")
    p.add_argument("--delta", type=int, default=3600)
    p.add_argument("--no-cpu-baseline", action="store_true",
                   help="skip the oracle run over all edges (and with it the full parity check)")
    p.add_argument("--no-parity", action="store_true", help="skip every check against the oracle")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the vertex, exists-exists-exists and smaller-side sections")
    p.add_argument("--no-configs", action="store_true", help="skip the small and medium workloads")
    p.add_argument("--parity-sample", type=int, default=4000)
    p.add_argument("--cache-dir", default=None,
                   help="keep the generated graph here as .npy files and reuse it")
    p.add_argument("--no-batch", action="store_true", help="skip the batched section")
    p.add_argument("--no-serve", action="store_true", help="skip the serving section")
    p.add_argument("--serve-small", action="store_true",
                   help="serving on the five smaller graphs at two rates only")
    p.add_argument("--copy-probe", action="store_true",
                   help="only copy a 1 GiB device buffer three times (calibrates HBM byte counters)")
    p.add_argument("--profile-queries", action="store_true",
                   help="after the timed steps, run a fixed sequence of queries on the 70M-edge graph "
                        "(no oracle) for profilers, print the JSON line and stop")
    return p.parse_args()


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ROOF_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_summary():
    """The dominant kernel's counters from the committed summary: HBM bytes per
    launch (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter reads
    for a plain copy of known size) and VALU instructions per launch; None when
    the summary is missing or the kernel's sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None, "no counter summary"
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json:"):
                rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None, "summary without traffic_json line"
    if rec.get("sources_sha256_16") != sources_hash():
        return None, "kernel sources changed since the counters were taken"
    f_fetch = rec["copy_bytes"] / (rec["copy_fetch_kib"] * 1024.0)
    f_write = rec["copy_bytes"] / (rec["copy_write_kib"] * 1024.0)
    out = {"traffic": rec["fetch_kib"] * 1024.0 * f_fetch + rec["write_kib"] * 1024.0 * f_write,
           "valu_insts": rec.get("valu_insts")}
    return out, "ok"


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def profile_queries(folty, synth, n, src, dst, tt, theta):
    """A fixed sequence for profilers, in order: on a fresh index, one day and one
    year with predicate 0 (two filter passes each; the one-year query's second
    pass re-enumerates most triangles, so later wide windows filter in one
    pass), then one year with predicates 0 and 3 (one pass), the smaller-side
    evaluation at one year, and the exists-exists-exists query at one year
    (counting only, then with temporal triangles, per-edge counts and listing)."""
    Y = synth.YEAR_S
    G = folty.Graph(n, src, dst, tt).build()
    seq = []

    def note(name, st):
        row = {"query": name}
        row.update({k: st[k] for k in ("query_ms", "wedge_ms", "temporal_ms", "tests", "filter_passes")})
        seq.append(row)
        log(f"profile {name}: query {st['query_ms']:.2f} ms, filter {st['wedge_ms']:.2f} ms, temporal "
            f"{st['temporal_ms']:.2f} ms, {st['tests']} tests, {st['filter_passes']} filter passes")

    for name, d, v, ss in (("1 day, predicate 0", 86_400, 0, False), ("1 year, predicate 0", Y, 0, False),
                           ("1 year, predicate 0, again", Y, 0, False), ("1 year, predicate 3", Y, 3, False),
                           ("1 year, predicate 0, smaller side", Y, 0, True)):
        note(name, G.query(d, theta, v, counts=False, smaller_side=ss).stats)
    for name, kw in (("triads 1 year, counting", dict(triples=False, instances=False)),
                     ("triads 1 year, triangles and listing", dict(triples=True, instances=True,
                                                                    edge_instances=True))):
        note(name, G.triad_query(Y, 0, **kw).stats)
    return seq


def copy_probe():
    import torch
    x = torch.empty(COPY_PROBE_BYTES, dtype=torch.uint8, device="cuda:0").fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for i in range(3):
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"copy probe {i}: {COPY_PROBE_BYTES} bytes")


def load_or_generate(synth, n, m, comm, cache_dir):
    if cache_dir:
        base = os.path.join(cache_dir, f"large_{n}_{m}_{comm}")
        if os.path.exists(base + "_t.npy"):
            return synth.TemporalGraph(n=n, src=np.load(base + "_src.npy"), dst=np.load(base + "_dst.npy"),
                                       t=np.load(base + "_t.npy"))
    g = synth.large(n=n, m=m, communities=comm)
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        for k in ("src", "dst", "t"):
            np.save(f"{base}_{k}.npy", getattr(g, k))
    return g


def check_against(res, want):
    """Mismatches between a GPU result and an oracle answer (pairs, certificate
    counts, |Sol|)."""
    u, v, k = res.pair_u, res.pair_v, res.n_cert
    same = (np.array_equal(u, want["pair_u"]) and np.array_equal(v, want["pair_v"])
            and np.array_equal(k, want["n_cert"]) and res.n_certificates == want["n_certificates"])
    return 0 if same else 1


def batched_section(folty, synth, steps, oracle_check, threads, rng):
    """64 mixed queries on one resident 10M-edge graph, and one query on each of
    32 graphs of 1e3..1e6 edges: plans (one launch sequence each, replayed from a
    HIP graph) against the same queries run one at a time.  The plans' results are
    checked against the oracle: on the 32 graphs every edge, pair and certificate;
    on the 10M-edge graph every pair and certificate count (from the oracle's
    counts over all edges in its many-window pass) and the per-edge counts of
    sampled edges plus edges the GPU counts as non-zero."""
    import torch
    from oracle.oracle import Oracle
    out = {}
    g = synth.c1_family(10_000_000, seed=0)
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    qs = [dict(q, counts=False) for q in synth.query_pool(4, 64, variants=(0, 3))]
    graphs = [synth.c1_family(int(round(10 ** (3 + 3 * i / 31))), seed=i) for i in range(32)]
    Gs = [folty.Graph(x.n, x.src, x.dst, x.t).build() for x in graphs]
    q32 = [dict(synth.query_pool(100 + i, 1)[0], counts=False) for i in range(32)]
    log(f"batched: resident graph m={g.m}, {len(graphs)} graphs with {sum(x.m for x in graphs)} edges")
    for name, plan_graphs, plan_queries, singles in (
            ("one_graph_64_queries", [G], [(0, q) for q in qs], [(G, q) for q in qs]),
            ("graphs_32_one_query_each", Gs, [(i, q) for i, q in enumerate(q32)], list(zip(Gs, q32)))):
        plan = folty.Plan(plan_graphs, plan_queries)
        first = plan.run()  # tunes the temporal launch shape, then captures
        plan.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = plan.run()
        plan_s = (time.perf_counter() - t0) / steps
        # the same queries one at a time through the single-query path
        seq = [gr.query(**q) for gr, q in singles]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            seq = [gr.query(**q) for gr, q in singles]
        seq_s = (time.perf_counter() - t0) / steps
        same = all(r.pairs() == s_.pairs() and r.n_certificates == s_.n_certificates
                   for r, s_ in zip(res, seq))
        n = len(plan_queries)
        out[name] = {"queries": n, "plan_ms": plan_s * 1e3, "queries_per_s": n / plan_s,
                     "sequential_ms": seq_s * 1e3, "sequential_queries_per_s": n / seq_s,
                     "speedup": seq_s / plan_s, "same_as_single_queries": same, "plan": plan.info()}
        log(f"batched {name}: plan {plan_s * 1e3:.2f} ms ({n / plan_s:.0f} q/s), sequential "
            f"{seq_s * 1e3:.2f} ms ({n / seq_s:.0f} q/s), identical results: {same}")
        plan.close()
    if oracle_check:
        # the same plans with per-edge counts kept, against the oracle
        t0 = time.perf_counter()
        plan = folty.Plan([G], [(0, dict(q, counts=True)) for q in qs])
        res = plan.run()
        o = Oracle(g.n, g.src, g.dst, g.t, threads=threads)
        bad_pairs = bad_edges = checked = 0
        for variant in (0, 3):
            ds = sorted({q["delta"] for q in qs if q["variant"] == variant})
            pool = o.counts_pool(ds, variant)
            for q, r in zip(qs, res):
                if q["variant"] != variant:
                    continue
                col = pool[:, ds.index(q["delta"])]
                want = o.query(q["delta"], q["theta"][0], q["theta"][1], variant, counts=col)
                bad_pairs += check_against(r, want)
                got = r.counts()
                nz = np.nonzero((got != 0xFFFFFFFF) & (got > 0))[0]
                idx = np.union1d(rng.choice(g.m, size=4000, replace=False),
                                 rng.choice(nz, size=min(4000, nz.size), replace=False) if nz.size else nz)
                bad_edges += int((got[idx] != col[idx]).sum())
                checked += int(idx.size)
        o.close()
        plan.close()
        plan = folty.Plan(Gs, [(i, dict(q, counts=True)) for i, q in enumerate(q32)])
        res32 = plan.run()
        bad32 = 0
        for x, q, r in zip(graphs, q32, res32):
            ox = Oracle(x.n, x.src, x.dst, x.t, threads=threads)
            want = ox.query(q["delta"], q["theta"][0], q["theta"][1], q["variant"])
            bad32 += check_against(r, want) + int((r.counts() != want["counts"]).sum())
            ox.close()
        plan.close()
        out["oracle_check"] = {"one_graph_64_queries": {"queries": len(qs), "pair_mismatches": bad_pairs,
                                                        "edges_checked": checked, "edge_mismatches": bad_edges,
                                                        "pairs_from": "oracle counts over all 10M edges"},
                               "graphs_32_one_query_each": {"graphs": len(graphs), "mismatches": bad32,
                                                            "checked": "every edge, pair and certificate"},
                               "bit_exact": bad_pairs + bad_edges + bad32 == 0,
                               "seconds": time.perf_counter() - t0}
        log(f"batched vs oracle: {bad_pairs} pair and {bad_edges} edge mismatches on the 10M graph "
            f"(64 queries), {bad32} on the 32 graphs ({time.perf_counter() - t0:.1f}s)")
    G.close()
    for x in Gs:
        x.close()
    return out


SERVE_REQUESTS = {10: 100, 30: 300, 100: 1000, 300: 2000, 1000: 2000}


def serving_section(folty, synth, big, small, oracle_check, threads, rng):
    """Poisson arrivals of queries on eight resident graphs (five of the tiny-graph
    generator, 1e5..1e7 edges; two of the large-graph generator, 2e7 and 4e7
    edges; and the 70M-edge graph itself) through the continuous-batching server;
    per-request latency is submit to result on the host.  Every served result is
    compared with the same query run alone, a sample of them with the oracle;
    then all requests of one mix are submitted at once and the served rate is
    compared with the same queries run one at a time; then the same under a
    16 GiB budget."""
    import threading
    import torch
    from oracle.oracle import Oracle
    sizes = [100_000, 300_000, 1_000_000, 3_000_000, 10_000_000]
    gs = [synth.c1_family(m, seed=10 + i) for i, m in enumerate(sizes)]
    if not small:
        gs += [synth.large_family(m, seed=20 + i) for i, m in enumerate((20_000_000, 40_000_000))]
    Gs = [folty.Graph(x.n, x.src, x.dst, x.t).build() for x in gs]
    if not small:
        gs.append(big[0])
        Gs.append(big[1])
    for G in Gs:
        G.stats()
    pool = sorted({int(round(np.exp(rng.uniform(np.log(60), np.log(604800))))) for _ in range(16)})
    rates = (100, 1000) if small else (10, 30, 100, 300, 1000)
    srv = folty.Server(workers=4, max_batch=16)
    out = {"graphs_edges": [x.m for x in gs], "delta_pool": pool, "rates": {}}
    oracles, pools = {}, {}

    def oracle_answer(gi, q):
        # five tiny-generator graphs: every window of the pool in one oracle pass
        x = gs[gi]
        if gi not in oracles:
            oracles[gi] = Oracle(x.n, x.src, x.dst, x.t, threads=threads)
        key = (gi, q["variant"])
        if key not in pools:
            pools[key] = oracles[gi].counts_pool(pool, q["variant"])
        col = pools[key][:, pool.index(q["delta"])]
        return oracles[gi].query(q["delta"], q["theta"][0], q["theta"][1], q["variant"], counts=col)

    def mix(k):
        return [(int(rng.integers(0, len(Gs))),
                 dict(delta=int(rng.choice(pool)), theta=(int(rng.integers(1, 10)), 10),
                      variant=int(rng.choice([0, 3])), counts=False)) for _ in range(k)]

    oracle_bad = oracle_checked = 0
    for rate in rates:
        per_rate = SERVE_REQUESTS[rate]
        reqs = mix(per_rate)
        gaps = rng.exponential(1.0 / rate, size=per_rate)
        tickets = [None] * per_rate

        def submit():
            t_next = time.perf_counter()
            for i, (gi, q) in enumerate(reqs):
                t_next += gaps[i]
                d = t_next - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(Gs[gi], **q)

        t0 = time.perf_counter()
        th = threading.Thread(target=submit)
        th.start()
        while th.is_alive():
            th.join(timeout=30.0)
            if th.is_alive():
                log(f"serving {rate} q/s: {sum(t is not None for t in tickets)} of {per_rate} submitted")
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - t0
        lat = np.array([r.stats["latency_ms"] for r in res])
        bs = np.array([r.stats["batch_size"] for r in res])
        # every request rerun alone must give the same answer; a sample against the oracle
        alone_bad = sum(1 for r, (gi, q) in zip(res, reqs) if r.pairs() != Gs[gi].query(**q).pairs())
        if oracle_check:
            small_idx = [i for i, (gi, q) in enumerate(reqs) if gi < len(sizes)]
            for i in rng.choice(small_idx, size=min(40, len(small_idx)), replace=False):
                gi, q = reqs[int(i)]
                oracle_bad += check_against(res[int(i)], oracle_answer(gi, q))
                oracle_checked += 1
        out["rates"][str(rate)] = {"requests": per_rate, "p50_ms": float(np.percentile(lat, 50)),
                                   "p99_ms": float(np.percentile(lat, 99)),
                                   "achieved_queries_per_s": per_rate / wall,
                                   "mean_batch": float(bs.mean()), "max_batch": int(bs.max()),
                                   "mismatches_vs_alone": alone_bad}
        log(f"serving {rate} q/s: p50 {np.percentile(lat, 50):.2f} ms, p99 {np.percentile(lat, 99):.2f} ms, "
            f"achieved {per_rate / wall:.0f} q/s, mean batch {bs.mean():.2f}, {alone_bad} differ from alone")
    # saturated: all requests at once, against the same queries one at a time
    reqs = mix(2000)
    for gi, q in reqs[:50]:
        Gs[gi].query(**q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = [Gs[gi].query(**q) for gi, q in reqs]
    seq_s = time.perf_counter() - t0
    info0 = srv.info()
    t0 = time.perf_counter()
    tickets = [srv.submit(Gs[gi], **q) for gi, q in reqs]
    res = [srv.wait(t) for t in tickets]
    sat_s = time.perf_counter() - t0
    info1 = srv.info()
    bad = sum(1 for r, a in zip(res, alone) if r.pairs() != a.pairs() or r.n_certificates != a.n_certificates)
    bs = np.array([r.stats["batch_size"] for r in res])
    out["saturated"] = {"requests": len(reqs), "served_queries_per_s": len(reqs) / sat_s,
                        "sequential_queries_per_s": len(reqs) / seq_s, "speedup": seq_s / sat_s,
                        "mean_batch": float(bs.mean()),
                        "passes_with_several_requests": info1["batches"] - info0["batches"],
                        "peak_concurrent_passes": info1["peak_concurrent_passes"],
                        "mismatches_vs_alone": bad}
    log(f"serving saturated: {len(reqs)} requests at once served at {len(reqs) / sat_s:.0f} q/s, one at a "
        f"time {len(reqs) / seq_s:.0f} q/s (x{seq_s / sat_s:.2f}); mean batch {bs.mean():.2f}, "
        f"{info1['batches'] - info0['batches']} shared passes, up to {info1['peak_concurrent_passes']} passes at "
        f"once, {bad} differ from alone")
    out["server"] = srv.info()
    srv.close()
    out["oracle_check"] = {"requests_checked": oracle_checked, "mismatches": oracle_bad,
                           "how": "sampled served requests on the five tiny-generator graphs: pairs, "
                                  "certificate counts and |Sol| from the oracle's counts over all edges"}
    if not small:
        # the same mix under a 16 GiB device budget: requests wait for admission
        srv = folty.Server(workers=4, max_batch=16, hbm_budget_bytes=16 << 30)
        n_req = 500
        reqs = mix(n_req)
        t0 = time.perf_counter()
        tickets = [srv.submit(Gs[gi], **q) for gi, q in reqs]
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - t0
        lat = np.array([r.stats["latency_ms"] for r in res])
        qwait = np.array([r.stats["queue_ms"] for r in res])
        bad = sum(1 for r, (gi, q) in zip(res, reqs) if r.pairs() != Gs[gi].query(**q).pairs())
        info = srv.info()
        srv.close()
        out["budget_16GiB"] = {"requests": n_req, "submitted_at_once": True,
                               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                               "queue_p50_ms": float(np.percentile(qwait, 50)),
                               "queue_p99_ms": float(np.percentile(qwait, 99)),
                               "achieved_queries_per_s": n_req / wall, "mismatches_vs_alone": bad, "server": info}
        log(f"serving under a 16 GiB budget: {n_req} requests at once, p50 {np.percentile(lat, 50):.2f} ms, "
            f"p99 {np.percentile(lat, 99):.2f} ms, queue p99 {np.percentile(qwait, 99):.2f} ms, "
            f"{n_req / wall:.0f} q/s, peak counted {info['peak_in_use_bytes'] / 2**30:.1f} GiB, "
            f"rejected {info['rejected']}, {bad} differ from alone")
    for o in oracles.values():
        o.close()
    for G in Gs[:len(Gs) - (0 if small else 1)]:
        G.close()
    return out


def configs_section(folty, synth, threads):
    """The small workload (n=2,000, m=20,000; delta 3600, theta 1/2) and the
    medium one (n=1M, m=10M; the nine queries delta in {600, 3600, 86400} x theta
    in {1/4, 1/2, 3/4}): every edge, pair and certificate against the oracle, and
    the oracle's time for the query (median of three runs on all host cores; the
    small workload also on one core)."""
    from oracle.oracle import Oracle
    out = {}
    g = synth.tiny()
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    r = G.query(3600, (1, 2), 0)
    o = Oracle(g.n, g.src, g.dst, g.t, threads=threads)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        w = o.query(3600, 1, 2, 0)
        times.append(time.perf_counter() - t0)
    o1 = Oracle(g.n, g.src, g.dst, g.t, threads=1)
    t0 = time.perf_counter()
    o1.query(3600, 1, 2, 0)
    t1 = time.perf_counter() - t0
    bad = check_against(r, w) + int((r.counts() != w["counts"]).sum())
    out["small"] = {"n": g.n, "m": g.m, "n_pairs": int(w["pair_u"].size), "n_certificates": w["n_certificates"],
                    "gpu_query_ms": r.stats["query_ms"], "oracle_s_median_of_3": float(np.median(times)),
                    "oracle_s_one_core": t1, "mismatches": bad}
    o.close()
    o1.close()
    G.close()
    log(f"small workload: {bad} mismatches; oracle {np.median(times) * 1e3:.1f} ms ({threads} cores), "
        f"{t1 * 1e3:.1f} ms (one core); GPU query {r.stats['query_ms']:.2f} ms")
    g = synth.medium()
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    o = Oracle(g.n, g.src, g.dst, g.t, threads=threads)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        o.query(3600, 1, 2, 0)
        times.append(time.perf_counter() - t0)
    deltas = [600, 3600, 86400]
    pool = o.counts_pool(deltas, 0)
    bad = 0
    qms = {}
    for j, d in enumerate(deltas):
        for th in ((1, 4), (1, 2), (3, 4)):
            r = G.query(d, th, 0)
            w = o.query(d, th[0], th[1], 0, counts=pool[:, j])
            bad += check_against(r, w) + int((r.counts() != pool[:, j]).sum())
            qms[f"{d}/{th[0]}/{th[1]}"] = r.stats["query_ms"]
    out["medium"] = {"n": g.n, "m": g.m, "queries": 9, "gpu_query_ms": qms,
                     "oracle_s_median_of_3": float(np.median(times)), "mismatches": bad,
                     "oracle_one_core": "not timed (about the all-core time times the core count)"}
    o.close()
    G.close()
    log(f"medium workload: {bad} mismatches over 9 queries; oracle {np.median(times):.2f} s ({threads} cores)")
    return out


def triads_section(folty, G, oracle, g, n, rng, deltas):
    """Exists-exists-exists queries (solution triples and temporal triangles) on
    the same index, predicate 0; sampled parity against the oracle: the third
    vertices of sampled directed pairs, and the temporal triangles of sampled
    first edges."""
    res = {}
    loop = g.src == g.dst
    for d in deltas:
        rc = G.triad_query(d, 0, triples=False, instances=False)  # the solution count alone
        r = G.triad_query(d, 0, triples=True, instances=True, edge_instances=True)
        t = r.triads()
        inst = r.edge_instances()
        trip = t["triples"]
        key = trip[:, 0].astype(np.int64) * n + trip[:, 1] if trip is not None else np.zeros(0, np.int64)
        # pairs: some with solutions, some uniform over the edges' pairs
        pk = np.unique(key)
        ek = g.src[~loop].astype(np.int64) * n + g.dst[~loop]
        pick = np.union1d(rng.choice(pk, size=min(200, pk.size), replace=False) if pk.size else pk,
                          rng.choice(ek, size=min(200, ek.size), replace=False))
        bad = 0
        for k in pick.tolist():
            lo, hi = np.searchsorted(key, k), np.searchsorted(key, k, side="right")
            want = oracle.triad_pair(k // n, k % n, d, 0)
            bad += int(not np.array_equal(trip[lo:hi, 2] if trip is not None else want[:0], want))
        # first edges: uniform plus ones the GPU counts as non-zero
        nz = np.nonzero(inst)[0]
        idx = np.union1d(rng.choice(g.m, size=min(2000, g.m), replace=False),
                         rng.choice(nz, size=min(2000, nz.size), replace=False) if nz.size else nz)
        ebad = int((oracle.triad_instances(d, 0, idx) != inst[idx]).sum())
        sums_ok = int(inst.sum()) == t["n_instances"] and (trip is None or trip.shape[0] == t["n_solutions"]) \
            and rc.triads()["n_solutions"] == t["n_solutions"]
        mism = bad + ebad + (0 if sums_ok else 1)
        res[str(d)] = {"predicate": 0, "solution_triples": t["n_solutions"], "temporal_triangles": t["n_instances"],
                       "count_only_query_ms": rc.stats["query_ms"], "count_only_temporal_ms": rc.stats["temporal_ms"],
                       "query_ms": r.stats["query_ms"], "wedge_ms": r.stats["wedge_ms"],
                       "temporal_ms": r.stats["temporal_ms"], "listing_ms": r.stats["threshold_ms"],
                       "tests": r.stats["tests"], "checked_pairs": int(pick.size), "pair_mismatches": bad,
                       "checked_edges": int(idx.size), "edge_mismatches": ebad, "totals_consistent": sums_ok,
                       "mismatches": mism}
        log(f"triads delta={d}: {t['n_solutions']} solution triples, {t['n_instances']} temporal triangles; "
            f"count only {rc.stats['query_ms']:.2f} ms, with triangles and listing {r.stats['query_ms']:.2f} ms "
            f"(listing {r.stats['threshold_ms']:.2f}); {bad} pair and {ebad} edge mismatches over "
            f"{pick.size} pairs and {idx.size} edges")
    return res


def smaller_side_section(folty, synth, G, oracle, g, rng, k):
    """The smaller-side evaluation (runs with a shorter L2 counted from the
    in-neighbour intervals) against the default one: identical counts over all
    edges, sampled edges against the oracle, and the temporal-step times; on this
    graph at one year and on a multiplicity-skewed graph."""
    from oracle.oracle import Oracle

    def compare(Gx, ox, gx, name, d, variant=0):
        r0 = Gx.query(d, (1, 10), variant)
        r1 = Gx.query(d, (1, 10), variant, smaller_side=True)
        c0, c1 = r0.counts(), r1.counts()
        diff = int((c0 != c1).sum())
        nz = np.nonzero((c1 != 0xFFFFFFFF) & (c1 > 0))[0]
        idx = np.union1d(rng.choice(gx.m, size=min(k, gx.m), replace=False),
                         rng.choice(nz, size=min(k, nz.size), replace=False) if nz.size else nz)
        bad = int((ox.counts(d, variant, idx) != c1[idx]).sum())
        same_pairs = r0.pairs() == r1.pairs() and r0.n_certificates == r1.n_certificates
        row = {"delta": d, "predicate": variant, "tests_default": r0.stats["tests"], "tests": r1.stats["tests"],
               "temporal_ms_default": r0.stats["temporal_ms"], "temporal_ms_smaller_side": r1.stats["temporal_ms"],
               "query_ms_default": r0.stats["query_ms"], "query_ms_smaller_side": r1.stats["query_ms"],
               "counts_differing_from_default": diff, "oracle_checked_edges": int(idx.size),
               "oracle_mismatches": bad, "mismatches": diff + bad + (0 if same_pairs else 1)}
        log(f"smaller side, {name} delta={d}: temporal {r0.stats['temporal_ms']:.2f} ms by E_ab, "
            f"{r1.stats['temporal_ms']:.2f} ms from the smaller side; {diff} counts differ, {bad} oracle "
            f"mismatches over {idx.size} edges")
        return row

    res = {"large/31536000": compare(G, oracle, g, "large", synth.YEAR_S)}
    gs = synth.skewed()
    os_ = Oracle(gs.n, gs.src, gs.dst, gs.t, threads=len(os.sched_getaffinity(0)))
    Gs = folty.Graph(gs.n, gs.src, gs.dst, gs.t).build()
    for d in (86_400, synth.YEAR_S):
        res[f"skewed/{d}"] = compare(Gs, os_, gs, "skewed", d)
    res["skewed_workload"] = {"n": gs.n, "m": gs.m, **gs.meta, "mismatches": 0}
    Gs.close()
    os_.close()
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process; there is no multi-GPU "
                                   "path, so --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    if a.copy_probe:
        copy_probe()
        return
    import torch

    from paper_2507_17215_amd import folty, synth

    n = int(round(4_000_000 * a.scale))
    m = int(round(70_000_000 * a.scale))
    comm = max(1, int(round(200 * a.scale)))
    t0 = time.time()
    g = load_or_generate(synth, n, m, comm, a.cache_dir)
    log(f"generated n={n} m={m} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    tt = torch.from_numpy(g.t).to(dev)
    torch.cuda.synchronize()
    theta = (1, 2)

    query_wall = []

    def step():
        G = folty.Graph(n, src, dst, tt, borrow=True)  # the resident inputs, read in place
        G.build()
        tq = time.perf_counter()
        r = G.query(a.delta, theta, 0, counts=False)  # returns with the sorted pairs on the host
        query_wall.append((time.perf_counter() - tq) * 1e3)
        st = G.stats()
        G.close()
        return r, st

    for i in range(a.warmup):
        r, st = step()
        log(f"warmup {i}: build {st['build_ms']:.1f} ms, query {r.stats['query_ms']:.1f} ms")
    torch.cuda.synchronize()
    times, qstats, bstats = [], [], []
    t_all = time.perf_counter()
    for i in range(a.steps):
        t1 = time.perf_counter()
        r, st = step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t1) * 1e3)
        qstats.append(r.stats)
        bstats.append(st)
        log(f"step {i}: {times[-1]:.1f} ms (build {st['build_ms']:.1f}, query {r.stats['query_ms']:.1f}, "
            f"wedge {r.stats['wedge_ms']:.2f}, temporal {r.stats['temporal_ms']:.2f}, "
            f"threshold {r.stats['threshold_ms']:.2f})")
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_all
    ms_per_step = total_s * 1e3 / a.steps
    qs = r.stats
    W, T, S = qs["wedges"], qs["triangles"], qs["tests"]
    P = qs["n_pairs"]
    med = lambda k, L: float(np.median([x[k] for x in L]))
    temporal_ms = med("temporal_ms", qstats)
    query_ms = med("query_ms", qstats)
    wedge_ms = med("wedge_ms", qstats)
    build_ms = med("build_ms", bstats)

    # The dominant kernel of the query: wedge enumeration, closing probe and the
    # per-triangle time-range filter; its duration comes from HIP events on the
    # graph's stream around that launch alone.  Its HBM traffic per launch is the
    # counter-measured one (FETCH_SIZE and WRITE_SIZE, calibrated on a copy of
    # known size); its algorithmic bytes are 12 B per wedge check (a neighbour id
    # and the closing-edge probe) and 48 B per static triangle (three
    # oriented-edge records' list bounds).  The counters show it limited by
    # vector-instruction issue, not by HBM.
    roof_bytes = 12 * W + 48 * T
    alg_gbs = roof_bytes / (wedge_ms * 1e-3) / 1e9 if wedge_ms > 0 else 0.0
    cs, cs_note = counter_summary()
    roofline = {"kernel": ROOF_KERNEL, "kernel_ms": round(wedge_ms, 4), "counters": cs_note,
                "algorithmic_bytes": int(roof_bytes), "algorithmic_gbs": round(alg_gbs, 2),
                "algorithmic_frac": round(alg_gbs / HBM_PEAK_GBS, 5)}
    if cs is not None and wedge_ms > 0:
        gbs = cs["traffic"] / (wedge_ms * 1e-3) / 1e9
        roofline.update({"bound": "alu", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": cs["traffic"],
                         "frac_basis": "HBM bytes from FETCH_SIZE + WRITE_SIZE per launch (calibrated)"})
        if cs.get("valu_insts"):
            roofline["valu_issue_frac"] = round(cs["valu_insts"] / (wedge_ms * 1e-3) / VALU_PEAK_WAVE_INSTS, 4)
    else:
        # no counters for these sources: the algorithmic figure, labelled as such
        roofline.update({"bound": "hbm", "achieved": round(alg_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(alg_gbs / HBM_PEAK_GBS, 5), "traffic": None,
                         "frac_basis": "algorithmic bytes (no counter summary for the current sources)"})

    out = {
        "metric": METRIC,
        "value": W / (ms_per_step * 1e-3),
        "unit": "wedge-checks/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"power-law temporal graph n={n} m={m} (gamma 2.0 + {comm} planted "
                               f"communities, Pareto multiplicity cap 1e4, 5-year renewal timestamps); "
                               f"one query delta={a.delta}, theta=1/2, predicate 0, universe N(b)",
                   "n": n, "m": m, "delta": a.delta, "theta": "1/2"},
        "step_wall_ms_median": float(np.median(times)) if times else None,
        # host wall time of the query call alone (index resident), pairs on the host
        "query_wall_ms_median": float(np.median(query_wall[-a.steps:])) if query_wall else None,
        "query_device_ms": query_ms, "build_device_ms": build_ms, "wedge_ms": wedge_ms,
        "temporal_ms": temporal_ms,
        "wedges": W, "triangles": T, "temporal_tests": S, "n_pairs": P,
        "n_certificates": qs["n_certificates"], "max_core": qs["max_core"],
        "max_out_degree": qs["max_out_degree"], "peel_rounds": qs["peel_rounds"],
        "core_sweeps": qs["core_sweeps"],
        "static_edges": qs["static_edges"], "directed_pairs": qs["directed_pairs"],
        "closing_probes": qs["closing_probes"], "enum_items": qs["enum_items"],
        "query_only_wedge_checks_per_s": W / (query_ms * 1e-3) if query_ms > 0 else None,
        "temporal_tests_per_s": S / (temporal_ms * 1e-3) if temporal_ms > 0 else None,
        "roofline": roofline,
    }

    from oracle.oracle import Oracle
    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(123)
    if a.profile_queries:
        out["profile_queries"] = profile_queries(folty, synth, n, src, dst, tt, theta)
        print(json.dumps(out), flush=True)
        return
    G = folty.Graph(n, src, dst, tt).build()  # resident: checks, extra sections, serving
    oracle = None
    ok = True
    if not a.no_parity and not a.no_cpu_baseline:
        # The timed query in full against the oracle run over every edge; that
        # run's wall time (index, per-edge counts, threshold and pairs) is the
        # CPU baseline of the whole job, measured, on all host cores.
        rq = G.query(a.delta, theta, 0)
        got = rq.counts()
        t1 = time.perf_counter()
        oracle = Oracle(n, g.src, g.dst, g.t, threads=threads)
        t2 = time.perf_counter()
        cnt = oracle.counts(a.delta, 0)
        t3 = time.perf_counter()
        want = oracle.query(a.delta, theta[0], theta[1], 0, counts=cnt)
        t4 = time.perf_counter()
        full_s = t4 - t1
        bad_edges = int((got != cnt).sum())
        bad_pairs = check_against(rq, want)
        # core numbers and the degeneracy rank of the same index, every vertex
        # (outside the CPU baseline: the oracle's counts do not need them)
        t5 = time.perf_counter()
        bad_core = int((G.core_numbers() != oracle.core_numbers()).sum())
        bad_rank = int((G.ranks() != oracle.degeneracy_rank()).sum())
        rank_s = time.perf_counter() - t5
        ok = ok and bad_edges == 0 and bad_pairs == 0 and bad_core == 0 and bad_rank == 0
        out["parity_full"] = {"bit_exact": bad_edges == 0 and bad_pairs == 0 and bad_core == 0 and bad_rank == 0,
                              "edges": int(got.size), "vertices": int(n),
                              "core_mismatches": bad_core, "rank_mismatches": bad_rank,
                              "edge_mismatches": bad_edges, "pair_list_equal": bad_pairs == 0,
                              "n_pairs": int(want["pair_u"].size), "n_certificates": int(want["n_certificates"]),
                              "nonzero_counts": int(((cnt > 0) & (cnt != 0xFFFFFFFF)).sum()),
                              "delta": a.delta, "theta": "1/2", "predicate": 0}
        out["cpu_baseline"] = {
            "value": W / full_s, "unit": "wedge-checks/s", "cores": threads, "kind": "oracle",
            "sample": f"none: the whole timed job on the CPU, measured once: oracle index over all {m} edges "
                      f"({t2 - t1:.1f}s), per-edge counts of all {m} edges ({t3 - t2:.1f}s), threshold and "
                      f"pairs ({t4 - t3:.1f}s); W from the GPU orientation",
            "full_job_s": full_s, "cpu_model": cpu_model()}
        log(f"full parity delta={a.delta}: {bad_edges} edge mismatches over {got.size} edges, pair list "
            f"{'equal' if bad_pairs == 0 else 'DIFFERENT'} ({want['pair_u'].size} pairs, "
            f"{want['n_certificates']} certificates); oracle {full_s:.1f}s on {threads} cores; "
            f"{bad_core} core and {bad_rank} rank mismatches over {n} vertices (oracle peel {rank_s:.1f}s)")
    elif not a.no_parity:
        oracle = Oracle(n, g.src, g.dst, g.t, threads=threads)
    if not a.no_parity:
        # other windows and predicates on the same index: a uniform sample of
        # edges, plus every edge the GPU counts as non-zero (so a wrongly
        # non-zero count cannot hide among the zeros)
        sample = np.sort(rng.choice(m, size=min(a.parity_sample, m), replace=False))
        checked = {}
        by_delta = {}
        for d, variant in ((86_400, 0), (synth.YEAR_S, 0), (synth.YEAR_S, 3), (synth.YEAR_S, 6)):
            rq = G.query(d, theta, variant)
            key = str(d) if variant == 0 else f"{d}/predicate{variant}"
            by_delta[key] = {k: rq.stats[k] for k in ("query_ms", "wedge_ms", "temporal_ms", "threshold_ms",
                                                      "tests", "n_pairs", "n_certificates", "filter_passes")}
            got = rq.counts()
            nz = np.nonzero((got != 0xFFFFFFFF) & (got > 0))[0]
            if nz.size > a.parity_sample:
                nz = np.sort(rng.choice(nz, size=a.parity_sample, replace=False))
            idx = np.union1d(sample, nz)
            want = oracle.counts(d, variant, idx)
            bad = int((got[idx] != want).sum())
            ok = ok and bad == 0
            checked[key] = {"edges": int(idx.size), "gpu_nonzero_checked": int(nz.size),
                            "oracle_nonzero": int((want > 0).sum()), "mismatches": bad}
            log(f"parity delta={d} predicate {variant}: {bad} mismatches over {idx.size} edges ({sample.size} "
                f"uniform + {nz.size} the GPU counts as non-zero; oracle non-zero: {int((want > 0).sum())})")
        out["parity_sampled"] = {"bit_exact": ok, "deltas": checked}
        out["query_by_delta"] = by_delta
        if not a.no_extras:
            # vertex queries (exists-forall-forall, exists-forall-exists) on the same
            # index, one-year window; checked against the oracle on sampled vertices
            # (each decided from the counts of its own outgoing edges)
            vq = {}
            outdeg = np.bincount(g.src[g.src != g.dst], minlength=n)
            small = np.nonzero((outdeg >= 1) & (outdeg <= 2000))[0]
            for name, inner in (("exists_forall_forall", folty.INNER_FORALL),
                                ("exists_forall_exists", folty.INNER_EXISTS)):
                rv = G.vertex_query(synth.YEAR_S, (1, 10), inner, (1, 10), 0, counts=False)
                verts, good = rv.vertices()
                sol_small = np.intersect1d(verts, small)
                pick = np.union1d(rng.choice(small, size=min(200, small.size), replace=False),
                                  rng.choice(sol_small, size=min(200, sol_small.size), replace=False)
                                  if verts.size else np.zeros(0, np.int64))
                w = oracle.vertex_query_at(pick, synth.YEAR_S, 1, 10, 0, inner == folty.INNER_FORALL, 1, 10)
                gpu_sol = np.isin(w["vertices"], verts)
                gmap = dict(zip(verts.tolist(), good.tolist()))
                bad = int((gpu_sol != w["solution"]).sum()) + sum(
                    1 for u, s_, gd in zip(w["vertices"].tolist(), w["solution"].tolist(), w["good"].tolist())
                    if s_ and gmap.get(u) != gd)
                ok = ok and bad == 0
                vq[name] = {"delta": synth.YEAR_S, "theta": "1/10",
                            "inner_theta": "1/10" if inner == folty.INNER_FORALL else None,
                            "solution_vertices": int(verts.size), "query_ms": rv.stats["query_ms"],
                            "threshold_ms": rv.stats["threshold_ms"], "checked_vertices": int(pick.size),
                            "oracle_edges_counted": w["edges_counted"], "mismatches": bad}
                log(f"{name}: {verts.size} solution vertices in {rv.stats['query_ms']:.2f} ms; "
                    f"{bad} mismatches over {pick.size} sampled vertices ({w['edges_counted']} edges counted "
                    f"by the oracle)")
            out["vertex_queries"] = vq
            out["triads"] = triads_section(folty, G, oracle, g, n, rng, (a.delta, 86_400, synth.YEAR_S))
            out["smaller_side"] = smaller_side_section(folty, synth, G, oracle, g, rng, a.parity_sample)
            ok = ok and all(v["mismatches"] == 0 for v in out["smaller_side"].values())
            ok = ok and all(v["mismatches"] == 0 for v in out["triads"].values())
        out["parity_sampled"]["bit_exact"] = ok
        if not a.no_configs:
            out["configs"] = configs_section(folty, synth, threads)
    if oracle is not None:
        oracle.close()
        oracle = None
    if not a.no_batch:
        out["batched"] = batched_section(folty, synth, max(3, a.steps), not a.no_parity, threads, rng)
    if not a.no_serve:
        out["serving"] = serving_section(folty, synth, (g, G), a.serve_small, not a.no_parity, threads, rng)
    G.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
