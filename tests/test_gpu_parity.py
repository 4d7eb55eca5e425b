"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything here is integer work, so the bar is bit-exact equality of the
per-edge counts, the solution pairs with their certificate counts, and |Sol|.
"""
import json
import os

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle.oracle import Oracle
from paper_2507_17215_amd import folty, synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")
INF = folty.DELTA_INF


def say(*a):
    print("[case]", *a, flush=True)


def gpu_graph(g, **build):
    return folty.Graph(g.n, g.src, g.dst, g.t).build(**build)


def assert_same(res, want, counts=True):
    if counts:
        got = res.counts()
        bad = np.nonzero(got != want["counts"])[0]
        assert bad.size == 0, f"{bad.size} count mismatches, first at {bad[:5]}: gpu {got[bad[:5]]} oracle {want['counts'][bad[:5]]}"
    assert res.n_certificates == want["n_certificates"]
    assert np.array_equal(res.pair_u, want["pair_u"])
    assert np.array_equal(res.pair_v, want["pair_v"])
    assert np.array_equal(res.n_cert, want["n_cert"])


def assert_vertices(res, want):
    v, good = res.vertices()
    assert np.array_equal(v, want["vertices"]), f"{v.size} vs {want['vertices'].size} solution vertices"
    assert np.array_equal(good, want["good"])
    assert np.array_equal(res.pair_u, want["pair_u"]) and np.array_equal(res.pair_v, want["pair_v"])


def test_hand_cases():
    d = json.load(open(GOLD))
    for g in d["graphs"]:
        e = np.array(g["edges"], dtype=np.int64)
        G = folty.Graph(g["n"], e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2]).build()
        for c in g["cases"]:
            say(g["name"], c)
            r = G.query(c["delta"], tuple(c["theta"]), c["variant"], c.get("universe", 0),
                        bool(c.get("exclude_other", 0)))
            assert r.counts().tolist() == c["counts"]
            assert [list(p) for p in r.pairs()] == c["pairs"]
            assert r.n_certificates == c["n_certificates"]


def test_random_tiny_graphs_all_variants():
    rng = np.random.default_rng(99)
    for it in range(60):
        g = synth.random_small(rng, n_max=14, m_max=120, t_max=25)
        o = Oracle(g.n, g.src, g.dst, g.t)
        G = gpu_graph(g)
        for variant in range(8):
            for delta in (0, 1, 5, INF):
                want = o.counts(delta, variant)
                r = G.query(delta, (1, 3), variant)
                say("tiny", it, variant, delta)
                assert np.array_equal(r.counts(), want)
                q = o.query(delta, 1, 3, variant, counts=want)
                assert_same(r, q, counts=False)


def test_bruteforce_sized_graph():
    g = synth.bruteforce_size()
    G = gpu_graph(g)
    for variant in (0, 3, 6):
        for delta in (3600, 200_000, 10**6):
            say("bf", variant, delta)
            want = np.array(bf.counts(g.n, g.src, g.dst, g.t, delta, variant), dtype=np.uint32)
            assert np.array_equal(G.query(delta, (1, 2), variant).counts(), want)


def test_tiny_workload_all_thetas_universes():
    g = synth.tiny()
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = gpu_graph(g)
    for delta in (3600, 86400, 10**6, INF):
        for variant in (0, 3):
            cnt = o.counts(delta, variant)
            for theta in ((0, 1), (1, 4), (1, 2), (3, 4), (1, 1)):
                for uni, ex in ((0, False), (1, False), (2, False), (0, True), (1, True)):
                    say("tiny-workload", delta, variant, theta, uni, ex)
                    r = G.query(delta, theta, variant, uni, ex)
                    assert_same(r, o.query(delta, theta[0], theta[1], variant, uni, ex, counts=cnt))


def test_index_matches_oracle_static_quantities():
    for g in (synth.tiny(), synth.bruteforce_size(),
              synth.generate(3000, 40000, 2.0, law="pareto", cap=50, times="uniform",
                             t_range=1000, seed=5, communities=3, c_min=40, c_max=80, c_p=0.5)):
        o = Oracle(g.n, g.src, g.dst, g.t)
        G = gpu_graph(g)
        st = G.stats()
        sz = o.sizes()
        say("static", g.meta)
        assert st["static_edges"] == sz["static_edges"]
        assert st["directed_pairs"] == sz["directed_pairs"]
        assert st["triangles"] == sz["triangles"]
        assert st["self_loops"] == int((g.src == g.dst).sum())
        assert np.array_equal(G.degrees(), o.degrees())
        core = o.core_numbers()
        assert np.array_equal(G.core_numbers(), core)
        assert st["max_core"] == core.max()
        # the rank is the order (core, round within the level, id) of level-synchronous
        # min-degree peeling, which leaves every vertex at most core(x) out-edges
        ranks = G.ranks()
        assert np.array_equal(ranks, o.degeneracy_rank())
        assert (G.out_degrees() <= core).all()
        assert st["max_out_degree"] <= st["max_core"]
        od = G.out_degrees()
        assert st["wedges"] == int((od.astype(np.int64) * (od - 1) // 2).sum())


def test_index_memory_from_torch_allocator():
    """folty_build_opts' allocator hook: the index (and parts made on first use)
    lives in PyTorch's caching allocator, results are unchanged, and freeing the
    graph hands the memory back to PyTorch."""
    import torch
    g = synth.tiny(seed=51)
    base = gpu_graph(g)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    G = folty.Graph(g.n, g.src, g.dst, g.t).build(allocator="torch")
    held = torch.cuda.memory_allocated() - before
    say("torch allocator: index", G.device_bytes(), "bytes, torch holds", held)
    assert held >= G.device_bytes() > 0
    G.stats()  # per-item triangle offsets, made on first use
    for delta, theta, variant, universe in ((10**6, (1, 4), 0, 0), (200_000, (1, 2), 3, 2), (3600, (0, 1), 6, 1)):
        a, b = G.query(delta, theta, variant, universe), base.query(delta, theta, variant, universe)
        assert a.pairs() == b.pairs() and np.array_equal(a.counts(), b.counts())
    assert torch.cuda.memory_allocated() - before >= G.device_bytes()
    G.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_borrowed_device_inputs_equal_copied_ones():
    """FOLTY_MEM_DEVICE_BORROWED: the build reads the caller's device arrays in
    place; index, counts and pairs equal those of a graph built from copies, the
    arrays are left unchanged, and they are read again by a second build.  An
    unknown mem_kind is rejected."""
    import ctypes
    import torch
    g = synth.generate(3000, 40000, 2.0, law="pareto", cap=50, times="uniform", t_range=100_000, seed=52,
                       communities=3, c_min=40, c_max=80, c_p=0.5)
    o = Oracle(g.n, g.src, g.dst, g.t)
    dev = torch.device("cuda:0")
    src, dst, tt = (torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.t))
    keep = [x.clone() for x in (src, dst, tt)]
    G = folty.Graph(g.n, src, dst, tt, borrow=True).build()
    C = folty.Graph(g.n, src, dst, tt).build()
    assert G.stats()["static_edges"] == C.stats()["static_edges"]
    assert np.array_equal(G.core_numbers(), o.core_numbers())
    cnt = o.counts(5000, 0)
    for rebuild in (False, True):
        if rebuild:
            G.build(rank_mode=folty.RANK_DEGREE)
        for delta, th, v in ((5000, (1, 2), 0), (20_000, (1, 4), 3)):
            say("borrowed", rebuild, delta, th, v)
            a, b = G.query(delta, th, v), C.query(delta, th, v)
            assert np.array_equal(a.counts(), b.counts()) and a.pairs() == b.pairs()
            if delta == 5000:
                assert np.array_equal(a.counts(), cnt)
    torch.cuda.synchronize()
    for x, y in zip((src, dst, tt), keep):
        assert torch.equal(x, y)
    G.close()
    C.close()
    lib = folty.load_library()
    h = ctypes.c_void_p()
    rc = lib.folty_load_temporal_graph(g.n, len(g.src), ctypes.c_void_p(src.data_ptr()),
                                       ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(tt.data_ptr()), 3, None,
                                       ctypes.byref(h))
    assert rc == folty.EINVAL and not h.value


def test_short_lists_on_and_off_agree():
    """Lists of one or two entries are read from their records' end timestamps
    when every timestamp is below 2^32; the tiny workload's clock scaled by 5,000
    (up to 5e9) turns that off.  Both graphs, at matching windows and all 8
    predicate codes, give the oracle's counts, pairs and certificate counts."""
    g = synth.tiny(seed=61)
    k = 5000
    t2 = g.t * k + 7
    assert g.t.max() < 2**32 <= t2.max()
    G1, G2 = gpu_graph(g), folty.Graph(g.n, g.src, g.dst, t2).build()
    o1, o2 = Oracle(g.n, g.src, g.dst, g.t), Oracle(g.n, g.src, g.dst, t2)
    for delta in (2000, 50_000, 400_000):
        for v in range(8):
            say("short lists", delta, v)
            want = o1.query(delta, 1, 2, v)
            assert_same(G1.query(delta, (1, 2), v), want)
            assert_same(G2.query(delta * k, (1, 2), v), o2.query(delta * k, 1, 2, v))
            assert np.array_equal(G2.query(delta * k, (1, 2), v).counts(), want["counts"])


def test_core_numbers_when_row_histograms_do_not_fit():
    """A 4,200-vertex clique makes the degree h-index 4,199, past the levels a
    long row's kept histogram may hold: its rows are evaluated from windowed
    block histograms and never reordered, and level counts come from row chunks.
    A path hangs off the clique and a few vertices join both, so cores 1, 2 and
    4,199 and several rounds occur.  Core numbers and ranks equal the oracle's."""
    k = 4200
    iu, ju = np.triu_indices(k, 1)
    path = np.arange(k, k + 300)
    src = np.concatenate([iu, path[:-1], [k + 5, k + 7, k + 9], path[:3]]).astype(np.int32)
    dst = np.concatenate([ju, path[1:], [0, 1, 2], [10, 11, 12]]).astype(np.int32)
    n = k + 300
    t = np.arange(len(src), dtype=np.int64)
    say("clique: edges", len(src))
    o = Oracle(n, src, dst, t)
    G = folty.Graph(n, src, dst, t).build()
    core = o.core_numbers()
    assert core.max() == k - 1
    assert np.array_equal(G.core_numbers(), core)
    assert np.array_equal(G.ranks(), o.degeneracy_rank())
    st = G.stats()
    assert st["max_core"] == k - 1 and st["max_out_degree"] <= k - 1
    G.close()


def test_orientation_does_not_change_results():
    g = synth.tiny(seed=3)
    base = gpu_graph(g).query(10**6, (1, 4), 0).counts()
    for mode, seed in ((folty.RANK_DEGREE, 0), (folty.RANK_RANDOM, 1), (folty.RANK_RANDOM, 2)):
        say("rank", mode, seed)
        assert np.array_equal(gpu_graph(g, rank_mode=mode, rank_seed=seed).query(10**6, (1, 4), 0).counts(), base)


def test_long_out_rows_under_other_orientations():
    """A hub with ~1500 neighbours: under a random order (seed 5 ranks it below
    most of them) its out-row is longer than the rows staged in LDS, so its
    items take the global-memory search.  Every orientation gives the oracle's
    counts."""
    rng = np.random.default_rng(17)
    g = synth.tiny(seed=23)
    hub_src = np.full(1500, 7, np.int32)
    hub_dst = rng.choice(np.arange(8, g.n, dtype=np.int32), size=1500, replace=False)
    flip = rng.random(1500) < 0.5
    src = np.concatenate([g.src, np.where(flip, hub_dst, hub_src)]).astype(np.int32)
    dst = np.concatenate([g.dst, np.where(flip, hub_src, hub_dst)]).astype(np.int32)
    t = np.concatenate([g.t, rng.integers(0, 1_000_000, 1500)]).astype(np.int64)
    o = Oracle(g.n, src, dst, t)
    want = {v: o.query(10**6, 1, 4, v) for v in (0, 3)}
    for mode, seed in ((folty.RANK_DEGENERACY, 0), (folty.RANK_DEGREE, 0), (folty.RANK_RANDOM, 5)):
        G = folty.Graph(g.n, src, dst, t).build(rank_mode=mode, rank_seed=seed)
        say("long rows", mode, "max out-degree", G.stats()["max_out_degree"])
        if mode == folty.RANK_RANDOM:
            assert G.stats()["max_out_degree"] > 512
        for v in (0, 3):
            assert_same(G.query(10**6, (1, 4), v), want[v])


def test_cached_triangles_and_determinism():
    g = synth.tiny(seed=4)
    G = gpu_graph(g)
    Gc = gpu_graph(g, cache_triangles=True)
    first = G.query(500_000, (1, 3), 3)
    for rep in range(5):
        say("repeat", rep)
        a = G.query(500_000, (1, 3), 3)
        b = Gc.query(500_000, (1, 3), 3)
        assert np.array_equal(a.counts(), first.counts())
        assert np.array_equal(b.counts(), first.counts())
        assert a.pairs() == first.pairs() == b.pairs()


def test_batch_equals_sequential():
    g = synth.tiny(seed=5)
    G = gpu_graph(g)
    qs = [dict(delta=d, theta=th, variant=v, universe=u)
          for d, th, v, u in ((3600, (1, 2), 0, 0), (86400, (1, 4), 0, 2), (10**6, (1, 10), 3, 0),
                              (86400, (3, 4), 3, 1), (10**6, (0, 1), 0, 0), (INF, (1, 2), 6, 0),
                              (0, (1, 2), 0, 0), (3600, (9, 10), 3, 0))]
    say("batch")
    rb = G.batch(qs)
    for q, r in zip(qs, rb):
        s = G.query(**q)
        assert np.array_equal(r.counts(), s.counts())
        assert r.pairs() == s.pairs() and r.n_certificates == s.n_certificates


def test_multi_graph_call():
    gs = [synth.c1_family(int(m), seed=i) for i, m in enumerate((1000, 3000, 10_000, 30_000))]
    Gs = [gpu_graph(g) for g in gs]
    qs = [dict(delta=d, theta=(1, 4), variant=v) for d, v in ((10**6, 0), (86400, 3), (10**5, 0), (INF, 3))]
    say("multi")
    rs = folty.run_multi(Gs, qs)
    for g, q, r in zip(gs, qs, rs):
        o = Oracle(g.n, g.src, g.dst, g.t)
        assert_same(r, o.query(q["delta"], 1, 4, q["variant"]))


def test_plan_replays_match_single_queries_and_oracle():
    """A plan over several graphs and mixed predicates: every replay (with other
    GPU work in between) equals the single-query path and the oracle."""
    gs = [synth.tiny(seed=11), synth.c1_family(5000, seed=12), synth.bruteforce_size(seed=13)]
    Gs = [gpu_graph(g) for g in gs]
    Gs[1] = gpu_graph(gs[1], cache_triangles=True)
    rng = np.random.default_rng(5)
    queries = []
    for i in range(24):
        gi = int(rng.integers(0, len(gs)))
        queries.append((gi, dict(delta=int(rng.choice([0, 600, 86400, 400_000, 10**6, INF])),
                                 theta=(int(rng.integers(0, 5)), 4), variant=int(rng.choice([0, 3, 6])),
                                 universe=int(rng.integers(0, 3)))))
    plan = folty.Plan(Gs, queries)
    oracles = [Oracle(g.n, g.src, g.dst, g.t) for g in gs]
    want = [oracles[gi].query(q["delta"], q["theta"][0], q["theta"][1], q["variant"], q["universe"])
            for gi, q in queries]
    for rep in range(4):
        say("plan replay", rep, plan.info())
        rs = plan.run()
        for (gi, q), r, w in zip(queries, rs, want):
            assert_same(r, w)
        # unrelated eager work between replays
        Gs[rep % 3].query(1000, (1, 2), 0)
    info = plan.info()
    assert info["n_queries"] == len(queries)
    assert info["n_jobs"] <= len(queries)


def test_tuning_table_persists_across_processes(tmp_path):
    """A plan's timed launch shape goes to the FOLTY_TUNE_CACHE file as JSON, and a
    fresh process takes it from there instead of timing again.  Plans with too
    little temporal work (under 2^20 tests) keep the default shape untimed; these
    short windows on a 16M-edge graph give about 1.7M tests."""
    import json
    import os
    import subprocess
    import sys
    path = str(tmp_path / "tune.json")
    os.environ["FOLTY_TUNE_CACHE"] = path
    template = ("from paper_2507_17215_amd import folty, synth\n"
                "g = synth.c1_family(16_000_000, seed=3)\n"
                "G = folty.Graph(g.n, g.src, g.dst, g.t).build()\n"
                "qs = [dict(delta=d, theta=(1, 4), variant=v) for d in (60, 300, 1800, 7200) for v in (0, 3)]\n"
                "p = folty.Plan([G], [(0, q) for q in qs])\n"
                "p.run()\n"
                "i = p.info()\n"
                "print(i['tests'], i['tune_source'], i['tests_per_chunk'], i['temporal_blocks'])\n")
    try:
        code = template
        ns = {}
        exec(compile(code, "plan", "exec"), ns)
        info = ns["i"]
        say("tuning workload", info["tests"], info["tune_source"])
        ns.clear()
        assert info["tests"] >= 1 << 20, "too little work for the tuner"
        with open(path) as fh:
            table = json.load(fh)
        say("tuning table", table)
        assert table["arch"] == "gfx950" and table["entries"]
        e = table["entries"][0]
        assert {"tests_log2", "edges_log2", "tests_per_chunk", "blocks", "ms"} <= set(e)
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                             env=dict(os.environ), cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        assert out.returncode == 0, out.stderr[-2000:]
        tests, source, ipt, blocks = map(int, out.stdout.split())
        say("fresh process", tests, source, ipt, blocks)
        assert tests == info["tests"] and source == 2
        assert any(x["tests_per_chunk"] == ipt and x["blocks"] == blocks for x in table["entries"])
    finally:
        del os.environ["FOLTY_TUNE_CACHE"]


def test_plan_with_empty_and_loop_only_graphs():
    e0 = folty.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64)).build()
    e1 = folty.Graph(3, np.array([1, 1], np.int32), np.array([1, 1], np.int32), np.array([0, 5])).build()
    g = synth.bruteforce_size(seed=3)
    G = gpu_graph(g)
    plan = folty.Plan([e0, e1, G], [(0, dict(delta=5)), (1, dict(delta=5, theta=(0, 1))), (2, dict(delta=10**6))])
    say("plan with empty graphs")
    for _ in range(2):
        r = plan.run()
        assert r[0].pairs() == [] and r[0].n_certificates == 0
        assert r[1].pairs() == [] and r[1].n_certificates == 0
        o = Oracle(g.n, g.src, g.dst, g.t)
        assert_same(r[2], o.query(10**6, 1, 2, 0))


def test_plan_buffers_larger_than_one_fill_grid():
    """64 mixed queries on a 1M-edge graph: the per-level histograms (levels x m)
    and the per-query pair slots (64 x 2S) exceed what one grid of the clearing
    kernel covers, so every run must clear them with a grid-stride loop.  Runs
    after the first (the autotuned one and the graph replays) must equal the
    single-query path; sampled counts must equal the oracle's."""
    g = synth.c1_family(1_000_000, seed=0)
    G = gpu_graph(g)
    qs = synth.query_pool(4, 64, variants=(0, 3))
    singles = [G.query(**q) for q in qs]
    plan = folty.Plan([G], [(0, q) for q in qs])
    o = Oracle(g.n, g.src, g.dst, g.t)
    idx = np.random.default_rng(9).choice(g.m, size=3000, replace=False)
    pool = {}
    for var in (0, 3):
        ds = sorted({q["delta"] for q in qs if q["variant"] == var})
        pool[var] = dict(zip(ds, o.counts_pool(ds, var, idx).T))
    for rep in range(3):
        rs = plan.run()
        say("plan 64 queries, run", rep, plan.info())
        for q, r, s in zip(qs, rs, singles):
            assert r.n_certificates == s.n_certificates, q
            assert r.pairs() == s.pairs(), q
            got = r.counts()
            assert np.array_equal(got, s.counts()), q
            assert np.array_equal(got[idx], pool[q["variant"]][q["delta"]]), q


def test_plan_without_counts_leaves_histograms_cleared():
    """Plans whose queries hand back no per-edge counts skip the per-run clear:
    the threshold step zeroes each histogram tile it read.  Replays (with other
    plans and queries on the same graph in between) must keep giving the
    single-query results, and so must a plan mixing both kinds on one job."""
    g = synth.c1_family(300_000, seed=3)
    G = gpu_graph(g)
    rng = np.random.default_rng(21)
    qs = [dict(delta=int(rng.choice([600, 3600, 86400, 400_000, 10**6])), theta=(int(rng.choice([1, 2, 5])), 20),
               variant=int(rng.choice([0, 3])), universe=int(rng.integers(0, 3))) for _ in range(24)]
    o = Oracle(g.n, g.src, g.dst, g.t)
    want = [o.query(q["delta"], q["theta"][0], q["theta"][1], q["variant"], q["universe"]) for q in qs]
    assert sum(w["n_certificates"] > 0 for w in want) >= 12
    lean = folty.Plan([G], [(0, dict(q, counts=False)) for q in qs])
    mixed = folty.Plan([G], [(0, dict(q, counts=(i % 3 == 0))) for i, q in enumerate(qs)])
    for rep in range(4):
        say("plan without counts, run", rep)
        for q, r, w in zip(qs, lean.run(), want):
            assert r.n_certificates == w["n_certificates"], q
            assert np.array_equal(r.pair_u, w["pair_u"]) and np.array_equal(r.pair_v, w["pair_v"]), q
            assert np.array_equal(r.n_cert, w["n_cert"]), q
        rs = mixed.run()
        for i, (q, r, w) in enumerate(zip(qs, rs, want)):
            if i % 3 == 0:
                assert_same(r, w)
            else:
                assert r.n_certificates == w["n_certificates"], q
                assert np.array_equal(r.n_cert, w["n_cert"]), q
        G.query(qs[rep]["delta"], (1, 2), 0, counts=False)


def test_vertex_queries_hand_cases():
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "vertex_cases.json")))
    e = np.array(d["graph"]["edges"], dtype=np.int64)
    G = folty.Graph(d["graph"]["n"], e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2]).build()
    for c in d["cases"]:
        say("vertex hand", c)
        inner = folty.INNER_FORALL if c["inner"] == "forall" else folty.INNER_EXISTS
        r = G.vertex_query(c["delta"], tuple(c["theta"]), inner, tuple(c.get("inner_theta", [1, 1])))
        v, good = r.vertices()
        assert v.tolist() == c["vertices"] and good.tolist() == c["good"]


def test_vertex_queries_match_oracle():
    """exists-forall-forall and exists-forall-exists: solution vertices, their
    qualifying-neighbour counts and the qualifying directed pairs equal the
    oracle's, over random tiny graphs (all predicate codes) and the tiny workload
    (every universe, several thresholds)."""
    rng = np.random.default_rng(17)
    for it in range(12):
        g = synth.random_small(rng, n_max=14, m_max=120, t_max=25)
        o = Oracle(g.n, g.src, g.dst, g.t)
        G = gpu_graph(g)
        for variant in range(8):
            for inner in (folty.INNER_FORALL, folty.INNER_EXISTS):
                delta = int(rng.choice([0, 2, 6, INF]))
                th, th2 = (int(rng.integers(0, 5)), 4), (int(rng.integers(0, 5)), 4)
                say("vertex tiny", it, variant, inner, delta, th, th2)
                r = G.vertex_query(delta, th, inner, th2, variant)
                cnt = o.counts(delta, variant)
                assert np.array_equal(r.counts(), cnt)
                assert_vertices(r, o.vertex_query(delta, th[0], th[1], variant, inner == folty.INNER_FORALL,
                                                  th2[0], th2[1], counts=cnt))
    g = synth.tiny()
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = gpu_graph(g)
    for delta in (3600, 10**6):
        cnt = o.counts(delta, 0)
        for uni, ex in ((0, False), (0, True), (1, False), (2, False)):
            for th in ((0, 1), (1, 10), (1, 2), (1, 1)):
                for inner in (folty.INNER_FORALL, folty.INNER_EXISTS):
                    say("vertex workload", delta, uni, ex, th, inner)
                    r = G.vertex_query(delta, th, inner, (1, 3), 0, uni, ex, counts=False)
                    assert_vertices(r, o.vertex_query(delta, th[0], th[1], 0, inner == folty.INNER_FORALL,
                                                      1, 3, uni, ex, counts=cnt))


def test_single_query_one_pass_and_two_pass_agree():
    """A fresh index filters in two passes (count, then emit only the items with
    survivors); with one_pass a query writes survivors into per-item triangle
    slots in one pass (the offsets are made on first use).  A plan that makes the
    offsets does not switch later queries by itself.  All equal the oracle."""
    g = synth.tiny(seed=21)
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = gpu_graph(g)
    qs = [(10**6, (1, 4), 0), (3600, (1, 2), 3), (0, (0, 1), 6), (INF, (1, 3), 0)]
    first = [G.query(d, th, v) for d, th, v in qs]
    say("two-pass stats", first[0].stats["triangles"], first[0].stats["tests"],
        [r.stats["filter_passes"] for r in first])
    assert first[0].stats["filter_passes"] == 2
    G2 = gpu_graph(g)
    folty.Plan([G2], [(0, dict(delta=qs[0][0], theta=qs[0][1], variant=qs[0][2]))])
    assert G2.query(*qs[1]).stats["filter_passes"] == 2
    for (d, th, v), r1 in zip(qs, first):
        r2 = G.query(d, th, v, one_pass=True)
        assert r2.stats["filter_passes"] == 1
        want = o.query(d, th[0], th[1], v)
        assert_same(r1, want)
        assert_same(r2, want)
        assert r2.stats["triangles"] == r1.stats["triangles"]
        assert r2.stats["tests"] == r1.stats["tests"]


def test_wide_window_switches_later_queries_to_one_pass():
    """A query whose second filter pass re-enumerates most items (every window
    at delta = INF) makes the per-item offsets from its own counting pass; later
    queries of at least an eighth of its window filter in one pass by
    themselves, narrower ones keep two.  Results equal the oracle throughout."""
    g = synth.tiny(seed=22)
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = gpu_graph(g)
    r0 = G.query(INF, (1, 4), 0)
    assert r0.stats["filter_passes"] == 2
    r1 = G.query(INF, (1, 4), 0)
    r2 = G.query(3600, (1, 4), 0)
    say("passes", r0.stats["filter_passes"], r1.stats["filter_passes"], r2.stats["filter_passes"])
    assert r1.stats["filter_passes"] == 1
    assert r2.stats["filter_passes"] == 2
    want = o.query(INF, 1, 4, 0)
    assert_same(r0, want)
    assert_same(r1, want)
    assert_same(r2, o.query(3600, 1, 4, 0))
    assert r1.stats["triangles"] == r0.stats["triangles"] and r1.stats["tests"] == r0.stats["tests"]


def test_heavy_list_capacity_does_not_change_results():
    """Surviving triangles with more than 64 tests are listed and their tests run
    in pieces of 4; those past the list's capacity run where they were found.
    With the capacity forced down to 3 triangles (FOLTY_MAX_HEAVY, read once per
    process, so in a child process) counts, pairs and exists-exists-exists
    results equal the oracle, in both filter modes."""
    import os
    import subprocess
    import sys
    code = r"""
import numpy as np
from oracle.oracle import Oracle
from paper_2507_17215_amd import folty
rng = np.random.default_rng(8)
n = 40
src = list(rng.integers(0, n, 3000)); dst = list(rng.integers(0, n, 3000)); t = list(rng.integers(0, 100_000, 3000))
for a, b in ((0, 1), (1, 0), (2, 3), (5, 9)):
    src += [a] * 4000; dst += [b] * 4000; t += list(rng.integers(0, 100_000, 4000))
src, dst, t = np.array(src, np.int32), np.array(dst, np.int32), np.array(t, np.int64)
o = Oracle(n, src, dst, t)
G = folty.Graph(n, src, dst, t).build()
for d, v, one in ((50, 0, False), (5000, 3, False), (30_000, 6, True), (folty.DELTA_INF, 0, True)):
    r = G.query(d, (1, 4), v, one_pass=one)
    want = o.query(d, 1, 4, v)
    assert np.array_equal(r.counts(), want["counts"]), (d, v)
    assert r.n_certificates == want["n_certificates"]
    assert np.array_equal(r.pair_u, want["pair_u"]) and np.array_equal(r.pair_v, want["pair_v"])
    assert r.stats["filter_passes"] == 1 or not one
    tr = G.triad_query(d, v, edge_instances=True)
    assert np.array_equal(tr.triads()["triples"], o.triad_solutions(d, v)), (d, v)
    assert np.array_equal(tr.edge_instances(), o.triad_instances(d, v)), (d, v)
print("ok")
"""
    env = dict(os.environ, FOLTY_MAX_HEAVY="3")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, env=env,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    say("capacity 3:", out.stdout.strip(), out.stderr[-1500:])
    assert out.returncode == 0 and out.stdout.strip() == "ok"


def test_device_tensor_inputs():
    import torch
    g = synth.tiny(seed=6)
    dev = torch.device("cuda:0")
    G1 = folty.Graph(g.n, torch.from_numpy(g.src).to(dev), torch.from_numpy(g.dst).to(dev),
                     torch.from_numpy(g.t).to(dev)).build()
    G2 = gpu_graph(g)
    say("torch inputs")
    assert np.array_equal(G1.query(10**6, (1, 4)).counts(), G2.query(10**6, (1, 4)).counts())


def test_edge_cases_and_errors():
    say("empty graph")
    G = folty.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64)).build()
    r = G.query(10, (1, 2))
    assert r.n_certificates == 0 and r.pairs() == [] and r.counts().size == 0
    say("only self-loops")
    G = folty.Graph(3, np.array([1, 1, 2], np.int32), np.array([1, 1, 2], np.int32), np.array([0, 5, 9])).build()
    r = G.query(10, (0, 1))
    assert r.n_certificates == 0 and r.counts().tolist() == [folty.U32_MAX] * 3
    say("no triangles")
    G = folty.Graph(4, np.array([0, 1, 2], np.int32), np.array([1, 2, 3], np.int32), np.array([0, 1, 2])).build()
    r = G.query(INF, (0, 1))
    assert r.n_certificates == 3 and r.pairs() == [(0, 1, 1), (1, 2, 1), (2, 3, 1)]
    say("errors")
    with pytest.raises(folty.FoltyError) as ei:
        folty.Graph(3, np.array([0, 3], np.int32), np.array([1, 1], np.int32), np.array([0, 0]))
    assert ei.value.code == folty.EINVAL
    with pytest.raises(folty.FoltyError) as ei:
        folty.Graph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([0, -4]))
    assert ei.value.code == folty.EINVAL
    G = folty.Graph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([0, 4]))
    with pytest.raises(folty.FoltyError) as ei:
        G.query(10, (1, 2))
    assert ei.value.code == folty.ENOTBUILT
    G.build()
    for bad in (dict(delta=-1), dict(delta=5, theta=(3, 2)), dict(delta=5, theta=(1, 0)),
                dict(delta=5, variant=8), dict(delta=5, universe=3),
                dict(delta=5, universe=2, exclude_other=True)):
        with pytest.raises(folty.FoltyError) as ei:
            G.query(**bad)
        assert ei.value.code == folty.EINVAL


def test_timestamps_at_extremes():
    # t near 2^62 and delta = INF must not overflow
    big = (1 << 62) - 10
    e = np.array([[0, 1, big - 5], [0, 2, big - 3], [1, 2, big - 1]], dtype=np.int64)
    G = folty.Graph(3, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2]).build()
    say("big timestamps")
    assert G.query(INF, (1, 2)).counts().tolist() == [1, 0, 0]
    assert G.query(4, (1, 2)).counts().tolist() == [1, 0, 0]
    assert G.query(3, (1, 2)).counts().tolist() == [0, 0, 0]


def test_unsorted_input_order():
    g = synth.tiny(seed=8)
    rng = np.random.default_rng(0)
    order = rng.permutation(g.m)
    G1 = gpu_graph(g)
    G2 = folty.Graph(g.n, g.src[order], g.dst[order], g.t[order]).build()
    say("shuffled input")
    a = G1.query(10**6, (1, 4)).counts()
    b = G2.query(10**6, (1, 4)).counts()
    assert np.array_equal(a[order], b)


@pytest.mark.timeout(900)
def test_medium_workload_full_counts():
    """n=1M, m=10M: the nine (delta, theta) queries plus a one-year window, full
    per-edge counts against the oracle's multi-window pass."""
    say("medium: generate")
    g = synth.medium()
    o = Oracle(g.n, g.src, g.dst, g.t)
    deltas = [600, 3600, 86400, synth.YEAR_S]
    say("medium: oracle pool")
    pool = o.counts_pool(deltas, 0)
    say("medium: gpu build")
    G = gpu_graph(g)
    st = G.stats()
    core = o.core_numbers()
    assert np.array_equal(G.core_numbers(), core)
    assert np.array_equal(G.ranks(), o.degeneracy_rank())
    assert (G.out_degrees() <= core).all()
    assert st["max_out_degree"] <= st["max_core"]
    for j, d in enumerate(deltas):
        for th in ((1, 4), (1, 2), (3, 4)):
            say("medium", d, th)
            r = G.query(d, th, 0)
            assert_same(r, o.query(d, th[0], th[1], 0, counts=pool[:, j]))
    say("medium: batch")
    rb = G.batch([dict(delta=d, theta=(1, 2), variant=0) for d in deltas])
    for j, r in enumerate(rb):
        assert np.array_equal(r.counts(), pool[:, j])
    say("medium: other predicate codes and universes")
    for variant in (3, 6):
        cnt = o.counts(86400, variant)
        for uni, ex in ((0, False), (1, True), (2, False)):
            say("medium variant", variant, uni, ex)
            r = G.query(86400, (1, 10), variant, uni, ex)
            assert_same(r, o.query(86400, 1, 10, variant, uni, ex, counts=cnt), counts=(uni == 0))
    say("medium: vertex queries")
    for j, d in ((1, 3600), (3, synth.YEAR_S)):
        for inner in (folty.INNER_FORALL, folty.INNER_EXISTS):
            r = G.vertex_query(d, (1, 10), inner, (1, 4), 0, counts=False)
            want = o.vertex_query(d, 1, 10, 0, inner == folty.INNER_FORALL, 1, 4, counts=pool[:, j])
            assert_vertices(r, want)


@pytest.mark.timeout(600)
def test_large_sparse_id_space():
    """n = 2^28 with a few hundred edges on ids spread over the whole range: every
    per-vertex array of the index spans 2^28 entries and the grouping keys use 57
    bits.  Results equal the oracle's on the same graph with its ids compacted in
    order (an order-preserving relabelling changes no count and no pair order)."""
    rng = np.random.default_rng(28)
    n = 1 << 28
    k = 24
    ids = np.sort(np.concatenate([[0, 1, n - 2, n - 1], rng.choice(np.arange(2, n - 2), k - 4, replace=False)]))
    m = 600
    cs = rng.integers(0, k, m)
    cd = rng.integers(0, k, m)
    t = rng.integers(0, 50, m).astype(np.int64)
    o = Oracle(k, cs.astype(np.int32), cd.astype(np.int32), t)
    G = folty.Graph(n, ids[cs].astype(np.int32), ids[cd].astype(np.int32), t).build()
    say("sparse ids: built", G.stats()["max_core"])
    for d, v in ((0, 0), (5, 3), (20, 6), (INF, 1)):
        say("sparse ids", d, v)
        want = o.query(d, 1, 3, v)
        r = G.query(d, (1, 3), v)
        assert np.array_equal(r.counts(), want["counts"])
        assert np.array_equal(r.pair_u, ids[want["pair_u"]].astype(np.int32))
        assert np.array_equal(r.pair_v, ids[want["pair_v"]].astype(np.int32))
        assert np.array_equal(r.n_cert, want["n_cert"])
        tr = G.triad_query(d, v).triads()
        ws = o.triad_solutions(d, v)
        assert np.array_equal(tr["triples"], ids[ws].astype(np.int32))
        vq = G.vertex_query(d, (1, 2), folty.INNER_EXISTS, variant=v).vertices()[0]
        wv = o.vertex_query(d, 1, 2, v, inner_forall=False)["vertices"]
        assert np.array_equal(vq, ids[wv].astype(np.int32))
    cores = G.core_numbers()
    assert np.array_equal(cores[ids], o.core_numbers())
    assert (np.delete(cores, ids) == 0).all()


def test_cached_memory_release_and_reuse():
    """Result arrays of 1 MiB or more come from cached pinned host blocks; freeing
    the result keeps its block, folty_release_cached_memory hands every cached
    device and host block back, and later queries allocate afresh with the same
    results."""
    rng = np.random.default_rng(3)
    n, m = 50_000, 600_000  # 2.4 MB of per-edge counts
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    t = rng.integers(0, 10**6, m).astype(np.int64)
    G = folty.Graph(n, src, dst, t).build()
    first = G.query(10**5, (1, 4), 0).counts()
    say("release cached memory")
    freed = folty.release_cached_memory()
    assert freed >= 4 * m  # at least the counts' pinned block
    again = G.query(10**5, (1, 4), 0).counts()
    assert np.array_equal(first, again)
    o = Oracle(n, src, dst, t)
    assert np.array_equal(again, o.counts(10**5, 0))
