"""GPU parity at scale for the parts that small graphs do not reach.

* Predicate codes 1, 2, 4, 5 and 7 on the 10M-edge medium workload: full
  per-edge counts, pairs, certificate counts and |Sol| against the oracle
  (codes 0, 3 and 6 are covered in test_gpu_parity.py).
* Timestamps that need more than 32 bits.  The index keeps each list's first
  and last timestamp shifted right by tshift = bitlen(t_max) - 32 so that they
  fit 32 bits, and the time-range filter compares them with a slack.  Here the
  medium workload's timestamps become t * 4096 + 2^40 (tshift 9), and the tiny
  workload's a millisecond clock t * 1000 + 1.7e12 (tshift 9); windows are
  scaled ones and ones that are no multiple of 2^tshift.  Single queries (both
  filter modes), a plan, the smaller-side evaluation, the vertex queries and
  the exists-exists-exists query are compared with the oracle on the same
  timestamps.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2507_17215_amd import folty, synth

pytestmark = pytest.mark.gpu
YEAR = synth.YEAR_S


def say(*a):
    print("[case]", *a, flush=True)


def assert_same(res, want, counts=True):
    if counts:
        got = res.counts()
        bad = np.nonzero(got != want["counts"])[0]
        assert bad.size == 0, f"{bad.size} count mismatches, first at {bad[:5]}: gpu {got[bad[:5]]} oracle {want['counts'][bad[:5]]}"
    assert res.n_certificates == want["n_certificates"]
    assert np.array_equal(res.pair_u, want["pair_u"])
    assert np.array_equal(res.pair_v, want["pair_v"])
    assert np.array_equal(res.n_cert, want["n_cert"])


@pytest.fixture(scope="module")
def medium():
    say("medium: generate")
    return synth.medium()


@pytest.mark.timeout(900)
def test_other_predicate_codes_full_counts_at_scale(medium):
    g = medium
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    for variant in (1, 2, 4, 5, 7):
        say("medium predicate", variant)
        cnt = o.counts(86400, variant)
        assert int((cnt > 0).sum() - (cnt == 0xFFFFFFFF).sum()) > 0, "the window leaves no non-zero count"
        for theta in ((1, 10), (1, 2)):
            assert_same(G.query(86400, theta, variant), o.query(86400, theta[0], theta[1], variant, counts=cnt))


def shifted(g, scale, offset):
    return synth.TemporalGraph(n=g.n, src=g.src, dst=g.dst, t=g.t * scale + offset, meta=dict(g.meta))


@pytest.mark.timeout(900)
def test_wide_timestamps_medium_workload(medium):
    g = shifted(medium, 4096, 1 << 40)
    assert int(g.t.max()).bit_length() - 32 >= 8
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    deltas = [3600 * 4096, 86400 * 4096, YEAR * 4096, 86400 * 4096 + 12345, 1_000_003]
    say("wide medium: oracle pool")
    pool = o.counts_pool(deltas, 0)
    for j, d in enumerate(deltas):
        say("wide medium", d)
        assert_same(G.query(d, (1, 4), 0), o.query(d, 1, 4, 0, counts=pool[:, j]))
    say("wide medium: predicate 3")
    d = 86400 * 4096 + 777
    assert_same(G.query(d, (1, 2), 3), o.query(d, 1, 2, 3))
    say("wide medium: plan")
    plan = folty.Plan([G], [(0, dict(delta=d_, theta=(1, 4))) for d_ in deltas])
    for r, j in zip(plan.run(), range(len(deltas))):
        assert np.array_equal(r.counts(), pool[:, j])
    plan.close()


@pytest.mark.timeout(600)
def test_wide_timestamps_tiny_workload_all_query_kinds():
    g = shifted(synth.tiny(seed=4), 1000, 1_700_000_000_000)
    assert int(g.t.max()).bit_length() - 32 >= 8
    o = Oracle(g.n, g.src, g.dst, g.t)
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    deltas = [0, 1, 511, 3_600_000, 3_600_001, 86_400_000 + 123, 10**9 + 7, folty.DELTA_INF]
    for d in deltas:
        for variant in (0, 3, 6):
            say("wide tiny", d, variant)
            want = o.query(d, 1, 4, variant)
            assert_same(G.query(d, (1, 4), variant), want)
            assert_same(G.query(d, (1, 4), variant, smaller_side=True), want)
        tr = G.triad_query(d, 0, edge_instances=True)
        assert np.array_equal(tr.triads()["triples"], o.triad_solutions(d, 0))
        assert np.array_equal(tr.edge_instances(), o.triad_instances(d, 0))
        vq = G.vertex_query(d, (1, 10), folty.INNER_EXISTS, (1, 2), 0)
        wv = o.vertex_query(d, 1, 10, 0, False)
        v, good = vq.vertices()
        assert np.array_equal(v, wv["vertices"]) and np.array_equal(good, wv["good"])
    say("wide tiny: plan")
    qs = [(0, dict(delta=d, theta=(1, 4), variant=v)) for d in deltas for v in (0, 3)]
    plan = folty.Plan([G], qs)
    for rep in range(2):
        for (gi, q), r in zip(qs, plan.run()):
            assert_same(r, o.query(q["delta"], 1, 4, q["variant"]))
    plan.close()
    # the one-pass filter (per-item triangle slots) on the same timestamps
    for d in (3_600_001, 10**9 + 7):
        r = G.query(d, (1, 4), 0, one_pass=True)
        assert r.stats["filter_passes"] == 1
        assert_same(r, o.query(d, 1, 4, 0))
