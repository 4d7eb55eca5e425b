"""GPU parity of the smaller-side evaluation (FOLTY_QUERY_SMALLER_SIDE): runs
whose list L2 is shorter than E_{a,b} are counted from L2 through the
in-neighbour intervals and a per-edge difference array.  The counts, pairs and
|Sol| must equal the oracle's and the default evaluation's exactly.
"""
import ctypes

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2507_17215_amd import folty, synth

pytestmark = pytest.mark.gpu

INF = folty.DELTA_INF


def say(*a):
    print("[case]", *a, flush=True)


def check(G, o, delta, theta, variant, cnt=None):
    want = o.counts(delta, variant) if cnt is None else cnt
    r = G.query(delta, theta, variant, smaller_side=True)
    got = r.counts()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} count mismatches, first {bad[:5]}: {got[bad[:5]]} vs {want[bad[:5]]}"
    q = o.query(delta, theta[0], theta[1], variant, counts=want)
    assert r.n_certificates == q["n_certificates"]
    assert np.array_equal(r.pair_u, q["pair_u"]) and np.array_equal(r.pair_v, q["pair_v"])
    assert np.array_equal(r.n_cert, q["n_cert"])
    return r


def test_smaller_side_random_tiny_all_variants():
    rng = np.random.default_rng(555)
    for it in range(40):
        g = synth.random_small(rng, n_max=14, m_max=120, t_max=25)
        o = Oracle(g.n, g.src, g.dst, g.t)
        G = folty.Graph(g.n, g.src, g.dst, g.t).build()
        for variant in range(8):
            for delta in (0, 1, 5, INF):
                say("tiny", it, variant, delta)
                check(G, o, delta, (1, 3), variant)


def test_smaller_side_skewed_multigraph():
    """Long E_{a,b} lists closed by short ones: a few heavy pairs with thousands
    of parallel edges among light ones, so most heavy runs go through L2."""
    rng = np.random.default_rng(8)
    n = 40
    src = list(rng.integers(0, n, 3000))
    dst = list(rng.integers(0, n, 3000))
    t = list(rng.integers(0, 100_000, 3000))
    for a, b in ((0, 1), (1, 0), (2, 3), (5, 9)):
        k = 4000
        src += [a] * k
        dst += [b] * k
        t += list(rng.integers(0, 100_000, k))
    src, dst, t = np.array(src, np.int32), np.array(dst, np.int32), np.array(t, np.int64)
    o = Oracle(n, src, dst, t)
    G = folty.Graph(n, src, dst, t).build()
    for d, v in ((0, 0), (50, 0), (500, 1), (5000, 3), (30_000, 6), (INF, 0)):
        say("skewed", d, v)
        r = check(G, o, d, (1, 4), v)
        assert np.array_equal(r.counts(), G.query(d, (1, 4), v).counts())


def test_smaller_side_modes_and_orientations():
    g = synth.tiny(seed=13)
    o = Oracle(g.n, g.src, g.dst, g.t)
    cases = [(3600, 0), (86400, 3), (10**6, 6), (INF, 1)]
    cnt = {c: o.counts(c[0], c[1]) for c in cases}
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    for d, v in cases:
        say("two-pass", d, v)
        check(G, o, d, (1, 4), v, cnt[(d, v)])
    folty.Plan([G], [(0, dict(delta=3600, theta=(1, 2), variant=0))])
    for d, v in cases:
        say("one-pass", d, v)
        check(G, o, d, (1, 4), v, cnt[(d, v)])
    for kw in (dict(cache_triangles=True), dict(rank_mode=folty.RANK_RANDOM, rank_seed=4)):
        Gk = folty.Graph(g.n, g.src, g.dst, g.t).build(**kw)
        for d, v in cases:
            say(kw, d, v)
            check(Gk, o, d, (1, 4), v, cnt[(d, v)])


@pytest.mark.timeout(900)
def test_smaller_side_medium_workload():
    """n=1M, m=10M at a one-year window (over a million tests per query, so the
    chunks hold several tests and a run's L2 entries split between chunks)."""
    say("medium: generate")
    g = synth.medium()
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    for d, v in ((synth.YEAR_S, 0), (10**6, 6)):
        say("medium", d, v)
        r = check(G, o, d, (1, 10), v)
        r0 = G.query(d, (1, 10), v)
        say("medium", d, v, "tests", r.stats["tests"], "temporal ms: default", r0.stats["temporal_ms"],
            "smaller side", r.stats["temporal_ms"])


def test_smaller_side_flag_in_vertex_queries_and_plans():
    """The flag changes no result: vertex queries evaluated from the smaller side
    equal the default ones, and plans (which always walk E_{a,b}) accept it."""
    g = synth.tiny(seed=17)
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    for inner in (folty.INNER_FORALL, folty.INNER_EXISTS):
        vq = folty.VertexQuery()
        vq.edge = folty.make_query(10**6, (1, 4) if inner == folty.INNER_FORALL else (1, 1), 0,
                                   smaller_side=True)
        vq.theta_num, vq.theta_den = 1, 5
        vq.inner = inner
        out = ctypes.c_void_p()
        lib = folty.load_library()
        assert lib.folty_run_vertex_query(G._h, ctypes.byref(vq), ctypes.byref(out)) == 0
        a = folty.Result(out)
        b = G.vertex_query(10**6, (1, 5), inner, (1, 4), 0)
        say("vertex", inner)
        assert np.array_equal(a.vertices()[0], b.vertices()[0])
        assert np.array_equal(a.counts(), b.counts())
    q = folty.make_query(86400, (1, 3), 3, smaller_side=True)
    plan = folty.Plan([G], [(0, q)])
    r = plan.run()[0]
    ref = G.query(86400, (1, 3), 3)
    assert r.pairs() == ref.pairs() and np.array_equal(r.counts(), ref.counts())
