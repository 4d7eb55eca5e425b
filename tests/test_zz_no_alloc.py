"""The entry point that allocates nothing (folty_run_fol_query_noalloc) against
the ordinary query entry point: identical per-edge counts, pairs, certificate
counts and |Sol|, on two calls in a row (the second on a smaller graph), and a
clear error when the fixed scratch is too small."""
import numpy as np
import pytest
import torch

from paper_2507_17215_amd import folty, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def outputs(G, cap):
    dev = torch.device("cuda:0")
    z = lambda k: torch.full((k,), -7, dtype=torch.int32, device=dev)
    return dict(pair_u=z(cap), pair_v=z(cap), n_cert=z(cap), edge_count=z(G.m))


def same_as_query(G, delta, theta, variant, universe=0, smaller_side=False):
    want = G.query(delta, theta, variant, universe, smaller_side=smaller_side)
    out = outputs(G, max(1, want.pair_u.size + 5))
    got = G.query_noalloc(delta, theta, variant, universe, smaller_side=smaller_side, **out)
    torch.cuda.synchronize()
    assert got["n_pairs"] == want.pair_u.size
    assert got["n_certificates"] == want.n_certificates
    assert np.array_equal(got["pair_u"].cpu().numpy(), want.pair_u)
    assert np.array_equal(got["pair_v"].cpu().numpy(), want.pair_v)
    assert np.array_equal(got["n_cert"].cpu().numpy().view(np.uint32), want.n_cert)
    assert np.array_equal(got["edge_count"].cpu().numpy().view(np.uint32), want.counts())
    return got


def test_noalloc_equals_query_two_calls_then_smaller():
    torch.cuda.set_device(0)
    big = synth.tiny(seed=41)
    small = synth.bruteforce_size(seed=42)
    Gb = folty.Graph(big.n, big.src, big.dst, big.t).build()
    Gs = folty.Graph(small.n, small.src, small.dst, small.t).build()
    for delta, theta, variant in ((200_000, (1, 4), 0), (10**6, (1, 2), 3), (3600, (0, 1), 6)):
        say("noalloc", delta, theta, variant)
        same_as_query(Gb, delta, theta, variant)   # first call
        same_as_query(Gs, delta, theta, variant)   # second call, smaller input
    same_as_query(Gb, 10**6, (1, 4), 0, smaller_side=True)
    # the universe N(a) & N(b) once its per-edge triangle counts exist
    Gb.query(10**6, (1, 4), 0, folty.UNIVERSE_COMMON)
    same_as_query(Gb, 10**6, (1, 4), 0, folty.UNIVERSE_COMMON)
    with pytest.raises(folty.FoltyError) as ei:
        Gs.query_noalloc(10**6, (1, 4), 0, folty.UNIVERSE_COMMON, **outputs(Gs, 4096))
    assert ei.value.code == folty.EINVAL


def test_noalloc_pair_capacity_and_scratch_limit():
    g = synth.tiny(seed=43)
    G = folty.Graph(g.n, g.src, g.dst, g.t).build()
    want = G.query(10**6, (0, 1), 0)  # theta = 0: every pair is a solution
    out = outputs(G, 3)
    with pytest.raises(folty.FoltyError) as ei:
        G.query_noalloc(10**6, (0, 1), 0, **out)
    assert ei.value.code == folty.EOVERFLOW
    assert str(want.pair_u.size) in str(ei.value)
    big = synth.c1_family(4_000_000, seed=44)
    Gbig = folty.Graph(big.n, big.src, big.dst, big.t).build()
    with pytest.raises(folty.FoltyError) as ei:
        Gbig.query_noalloc(10**6, (1, 2), 0, **outputs(Gbig, 16))
    assert ei.value.code == folty.ENOMEM
    assert "scratch" in str(ei.value)
    # the scratch is still fine for the next call
    same_as_query(G, 10**6, (1, 4), 3)
