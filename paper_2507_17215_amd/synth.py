"""Seeded synthetic temporal multigraphs.

This module only draws inputs: vertex pairs, multiplicities and timestamps.  It
holds none of the query's arithmetic, and it is the one piece of code that both
the CPU oracle's tests and the GPU path use.

Every graph is a list of directed temporal edges ``(src[i], dst[i], t[i])``
returned in non-decreasing timestamp order (the paper assumes its input stream
is time-sorted, Section "Main Ideas", Preliminaries), as
``src``/``dst`` int32 and ``t`` int64 numpy arrays.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``):

* Static pairs follow Chung-Lu: vertex ``i`` has weight ``(i+1)**(-1/(gamma-1))``;
  an ordered pair ``(u, v)``, ``u != v``, is drawn with ``u`` and ``v``
  independently proportional to weight (inverse CDF on the cumulative sum).
  Repeated ordered pairs are merged.  Vertex labels are then scrambled by a
  seeded permutation so that hub ids are spread over ``[0, n)``.
* Each distinct ordered pair receives a multiplicity ``k``: geometric with
  mean 3 (capped), or discrete Pareto ``floor(X)``, ``X ~ Pareto(alpha, x_m=1)``
  (capped).  Pairs are taken in draw order until ``m`` temporal edges exist; the
  last pair is truncated so that exactly ``m`` edges are emitted.
* Timestamps are either uniform integers in ``[0, t_range)`` per edge, or a
  per-pair renewal process: start ``~ U[0, Y)``, gaps ``ceil(60 * X)`` seconds with
  ``X ~ Pareto(1.5, x_m=1)``, wrapped modulo ``Y``.
* Optional planted communities: disjoint vertex sets of sizes drawn uniformly
  from ``[c_min, c_max]``; each unordered pair inside a community is an edge with
  probability ``p`` and gets a random direction and a multiplicity from the same
  law.  Community pairs come first; Chung-Lu background pairs fill up to ``m``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

YEAR_S = 31_536_000


@dataclass
class TemporalGraph:
    n: int
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    t: np.ndarray    # int64[m]
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _multiplicity(rng: np.random.Generator, size: int, law: str, cap: int) -> np.ndarray:
    if law == "geometric":
        k = rng.geometric(1.0 / 3.0, size=size)
    elif law == "pareto":
        # rng.pareto draws X - 1 for a classical Pareto(alpha, x_m = 1)
        k = np.floor(1.0 + rng.pareto(1.5, size=size))
    else:
        raise ValueError(law)
    return np.minimum(k, cap).astype(np.int64)


def _chung_lu_draw(rng, cum, n, size):
    u = np.searchsorted(cum, rng.random(size), side="right")
    v = np.searchsorted(cum, rng.random(size), side="right")
    np.minimum(u, n - 1, out=u)
    np.minimum(v, n - 1, out=v)
    return u.astype(np.int64), v.astype(np.int64)


def _first_occurrence_unique(keys: np.ndarray) -> np.ndarray:
    uk, first = np.unique(keys, return_index=True)
    return keys[np.sort(first)]


def generate(n: int, m: int, gamma: float, *, law: str, cap: int, times: str,
             t_range: int, seed: int, communities: int = 0, c_min: int = 300,
             c_max: int = 800, c_p: float = 0.3) -> TemporalGraph:
    """Draw a temporal multigraph with exactly ``m`` temporal edges."""
    if n < 2 or m < 0:
        raise ValueError("need n >= 2 and m >= 0")
    rng = _rng(seed)
    label = rng.permutation(n).astype(np.int64)
    key_parts, k_parts = [], []
    have = np.empty(0, dtype=np.int64)
    total = 0

    if communities:
        order = rng.permutation(n)
        pos = 0
        for _ in range(communities):
            s = int(rng.integers(c_min, c_max + 1))
            if pos + s > n:
                break
            members = order[pos:pos + s].astype(np.int64)
            pos += s
            iu, ju = np.triu_indices(s, 1)
            keep = rng.random(iu.shape[0]) < c_p
            a, b = members[iu[keep]], members[ju[keep]]
            flip = rng.random(a.shape[0]) < 0.5
            a, b = np.where(flip, b, a), np.where(flip, a, b)
            keys = a * n + b
            k = _multiplicity(rng, keys.shape[0], law, cap)
            key_parts.append(keys)
            k_parts.append(k)
            total += int(k.sum())
        if key_parts:
            have = np.sort(np.concatenate(key_parts))

    if total < m:
        w = (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))
        cum = np.cumsum(w)
        cum /= cum[-1]
        mean_k = 3.0
        while total < m:
            want = m - total
            batch = max(4096, int(want / mean_k * 1.3) + 64)
            u, v = _chung_lu_draw(rng, cum, n, batch)
            ok = u != v
            keys = label[u[ok]] * n + label[v[ok]]
            keys = _first_occurrence_unique(keys)
            if have.size:
                keys = keys[~np.isin(keys, have, assume_unique=True)]
            if keys.size == 0:
                continue
            k = _multiplicity(rng, keys.shape[0], law, cap)
            csum = np.cumsum(k)
            stop = int(np.searchsorted(csum, want, side="left"))
            if stop < keys.shape[0]:
                keys, k = keys[:stop + 1], k[:stop + 1]
            key_parts.append(keys)
            k_parts.append(k)
            total += int(k.sum())
            have = np.union1d(have, keys)

    keys = np.concatenate(key_parts) if key_parts else np.empty(0, np.int64)
    ks = np.concatenate(k_parts) if k_parts else np.empty(0, np.int64)
    csum = np.cumsum(ks)
    if csum.size and csum[-1] > m:
        last = int(np.searchsorted(csum, m, side="left"))
        keys, ks = keys[:last + 1].copy(), ks[:last + 1].copy()
        ks[-1] -= int(csum[last] - m)
        csum = np.cumsum(ks)
    npairs = keys.shape[0]
    src_p = (keys // n).astype(np.int32)
    dst_p = (keys % n).astype(np.int32)
    src = np.repeat(src_p, ks)
    dst = np.repeat(dst_p, ks)

    if times == "uniform":
        t = rng.integers(0, t_range, size=m, dtype=np.int64)
    elif times == "renewal":
        start = rng.integers(0, t_range, size=npairs, dtype=np.int64)
        gap = np.ceil(60.0 * (1.0 + rng.pareto(1.5, size=m)))
        gap = np.minimum(gap, float(t_range)).astype(np.int64)
        first = np.zeros(npairs, dtype=np.int64)
        if npairs:
            first[1:] = csum[:-1]
        gap[first] = start
        c = np.cumsum(gap)
        base = c[first] - gap[first]
        t = c - np.repeat(base, ks)
        t %= t_range
    else:
        raise ValueError(times)

    order = np.argsort(t, kind="stable")
    g = TemporalGraph(n=n, src=np.ascontiguousarray(src[order]),
                      dst=np.ascontiguousarray(dst[order]),
                      t=np.ascontiguousarray(t[order]))
    g.meta = dict(n=n, m=m, gamma=gamma, law=law, cap=cap, times=times,
                  t_range=t_range, seed=seed, communities=communities,
                  directed_pairs=int(npairs), max_multiplicity=int(ks.max()) if npairs else 0)
    return g


# ---------------------------------------------------------------------------
# Named workloads.  Shapes follow the paper's SNAP graphs (Table of the
# exists-exists-forall runtimes): a CollegeMsg-sized graph, a wiki-talk-sized
# graph and an sx-stackoverflow-sized graph.  The datasets themselves are not
# used; these generators stand in for them.
# ---------------------------------------------------------------------------

def tiny(seed: int = 0) -> TemporalGraph:
    """n=2,000, m=20,000; Chung-Lu gamma 2.5; geometric multiplicity (mean 3, cap 64);
    uniform timestamps in [0, 1e6)."""
    return generate(2000, 20000, 2.5, law="geometric", cap=64, times="uniform",
                    t_range=1_000_000, seed=seed)


def bruteforce_size(seed: int = 1) -> TemporalGraph:
    """n=200, m=2,000 with the tiny-graph generator (small enough for brute force)."""
    return generate(200, 2000, 2.5, law="geometric", cap=64, times="uniform",
                    t_range=1_000_000, seed=seed)


def medium(seed: int = 0, n: int = 1_000_000, m: int = 10_000_000) -> TemporalGraph:
    """n=1M, m=10M; gamma 2.1; discrete Pareto(1.5) multiplicity capped at 1,000;
    per-pair renewal timestamps over one year."""
    return generate(n, m, 2.1, law="pareto", cap=1000, times="renewal",
                    t_range=YEAR_S, seed=seed)


def large(seed: int = 0, n: int = 4_000_000, m: int = 70_000_000,
          communities: int = 200) -> TemporalGraph:
    """n=4M, m=70M; gamma 2.0 background plus planted dense communities
    (sizes 300-800, p=0.3); discrete Pareto(1.5) multiplicity capped at 1e4;
    renewal timestamps over five years."""
    return generate(n, m, 2.0, law="pareto", cap=10_000, times="renewal",
                    t_range=5 * YEAR_S, seed=seed, communities=communities)


def c1_family(m: int, seed: int) -> TemporalGraph:
    """Tiny-graph generator at another size: n = max(20, m // 10)."""
    return generate(max(20, m // 10), m, 2.5, law="geometric", cap=64,
                    times="uniform", t_range=1_000_000, seed=seed)


def large_family(m: int, seed: int) -> TemporalGraph:
    """Large-graph generator at another size: n = m / 17.5, communities scaled
    to max(1, round(200 * m / 7e7))."""
    return generate(max(20, int(m / 17.5)), m, 2.0, law="pareto", cap=10_000,
                    times="renewal", t_range=5 * YEAR_S, seed=seed,
                    communities=max(1, round(200 * m / 7e7)))


def skewed(seed: int = 0, n: int = 1_000_000, m_background: int = 5_000_000, heavy: int = 200,
           heavy_k: int = 5_000, fan: int = 100, light_k: int = 4) -> TemporalGraph:
    """A multiplicity-skewed graph: the medium generator's background (n vertices,
    m_background edges) plus ``heavy`` planted pairs a -> b with ``heavy_k``
    parallel edges each, every pair closed by ``fan`` third vertices w with
    ``light_k`` edges a -> w and ``light_k`` edges b -> w (vertices drawn without
    replacement per pair; uniform timestamps over one year).  Each heavy list
    then meets ``fan`` short closing lists.  Edges are returned in timestamp
    order."""
    base = generate(n, m_background, 2.1, law="pareto", cap=1000, times="renewal",
                    t_range=YEAR_S, seed=seed)
    rng = _rng(seed + 7919)
    pick = np.stack([rng.choice(n, size=fan + 2, replace=False) for _ in range(heavy)]).astype(np.int32)
    a, b, w = pick[:, 0], pick[:, 1], pick[:, 2:]
    src = np.concatenate([base.src, np.repeat(a, heavy_k), np.repeat(np.repeat(a, fan), light_k),
                          np.repeat(np.repeat(b, fan), light_k)])
    dst = np.concatenate([base.dst, np.repeat(b, heavy_k), np.repeat(w.reshape(-1), light_k),
                          np.repeat(w.reshape(-1), light_k)])
    extra = heavy * (heavy_k + 2 * fan * light_k)
    t = np.concatenate([base.t, rng.integers(0, YEAR_S, size=extra)]).astype(np.int64)
    order = np.argsort(t, kind="stable")
    return TemporalGraph(n=n, src=src[order].astype(np.int32), dst=dst[order].astype(np.int32), t=t[order],
                         meta=dict(kind="skewed", heavy=heavy, heavy_k=heavy_k, fan=fan, light_k=light_k))


def random_small(rng: np.random.Generator, n_max: int = 12, m_max: int = 80,
                 t_max: int = 20) -> TemporalGraph:
    """Tiny random multigraph with many timestamp ties (for exhaustive checks).
    Self-loops are allowed on purpose: the query must ignore them."""
    n = int(rng.integers(2, n_max + 1))
    m = int(rng.integers(0, m_max + 1))
    src = rng.integers(0, n, size=m).astype(np.int32)
    dst = rng.integers(0, n, size=m).astype(np.int32)
    t = rng.integers(0, t_max, size=m).astype(np.int64)
    return TemporalGraph(n=n, src=src, dst=dst, t=t, meta=dict(kind="random_small"))


def query_pool(seed: int, count: int, variants=(0, 3)):
    """Mixed queries: delta log-uniform integers in [60, 604800], theta in
    {1/10, ..., 9/10}, variant drawn from ``variants``."""
    rng = _rng(seed)
    out = []
    for _ in range(count):
        d = int(round(math.exp(rng.uniform(math.log(60), math.log(604800)))))
        th = int(rng.integers(1, 10))
        var = int(variants[int(rng.integers(0, len(variants)))])
        out.append(dict(delta=d, theta=(th, 10), variant=var))
    return out
