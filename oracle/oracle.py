"""Python front of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It loads ``libfolty_oracle.so`` built from ``folty_oracle.c`` in
this directory with plain ``gcc`` (compiled on first use if missing or older
than the source) and adds the threshold step and the pair reduction with numpy.

Threshold step (paper, Algorithm ExistExistForAll, final loop): a temporal edge
e = (a, b, t) is a certificate when count[e] >= theta * |U(e)|, with the
universe U(e) = N(b) by default.  theta is an exact rational num/den, so the
comparison is count * den >= num * |U| in integers.  Other universes: N(a), and
N(a) intersect N(b) (Section "Insights"); ``exclude_other`` removes the other
endpoint from N(b) / N(a).

Solutions (paper, Definition of a solution): the pairs (a, b) with at least one
certificate on them, listed in (a, b) order with their certificate counts;
n_certificates is |Sol|.

Vertex queries (paper, Section on the exists-forall-forall and exists-forall-
exists queries): exists u forall_{theta1} v in N(u) forall_{theta2} w, and
exists u forall_{theta} v in N(u) exists w.  ``vertex_query`` follows the
section's algorithm step by step: the edge-level solutions L (certificates of the
exists-exists-forall query at theta2, or the edges with count >= 1 for the
inner exists), the per-vertex marks L_u[v] for every e = (u, v, t) in L, their
sums over N(u), and the threshold sum >= theta1 * |N(u)| for the vertices whose
neighbourhood is not empty (the last step runs over N(u)).

Exists-exists-exists queries (paper, Definition of a solution; Section 1: for
this prefix the problem is temporal triangle counting): the solution triples
(a, b, w) with at least one temporal triangle e1 in E_{a,b}, e2, e3 in the
lists the predicate code picks and t(e1) <= t(e2) <= t(e3) <= t(e1) + delta,
and the number of such edge triples per first edge (``triad_instances``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "folty_oracle.c")
_LIB = os.path.join(_HERE, "libfolty_oracle.so")
U32_MAX = np.uint32(0xFFFFFFFF)

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.og_build.restype = P
        lib.og_build.argtypes = [i32, i64, P, P, P]
        lib.og_free.argtypes = [P]
        lib.og_counts.restype = ctypes.c_int
        lib.og_counts.argtypes = [P, i64, P, i64, ctypes.c_int, P, ctypes.c_int]
        lib.og_counts_pool.restype = ctypes.c_int
        lib.og_counts_pool.argtypes = [P, i64, P, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int]
        lib.og_degrees.argtypes = [P, P]
        lib.og_common_counts.argtypes = [P, i64, P, P, ctypes.c_int]
        lib.og_sizes.argtypes = [P, P, ctypes.c_int]
        lib.og_core_numbers.argtypes = [P, P]
        lib.og_peel_levels.argtypes = [P, P, P]
        lib.og_num_threads.restype = ctypes.c_int
        lib.og_triad_instances.restype = ctypes.c_int
        lib.og_triad_instances.argtypes = [P, i64, P, i64, ctypes.c_int, P, ctypes.c_int]
        lib.og_pair_table.restype = i64
        lib.og_pair_table.argtypes = [P, P, P]
        lib.og_triad_pair_counts.restype = ctypes.c_int
        lib.og_triad_pair_counts.argtypes = [P, i64, ctypes.c_int, P, ctypes.c_int]
        lib.og_triad_fill.restype = ctypes.c_int
        lib.og_triad_fill.argtypes = [P, i64, ctypes.c_int, P, P, ctypes.c_int]
        lib.og_triad_pair.restype = i64
        lib.og_triad_pair.argtypes = [P, i32, i32, i64, ctypes.c_int, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Oracle:
    """The plain CPU statement of the query for one temporal graph."""

    def __init__(self, n: int, src, dst, t, threads: int = 0):
        lib = _load()
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.t = np.ascontiguousarray(t, dtype=np.int64)
        self.m = int(self.src.shape[0])
        self.threads = int(threads)
        if self.m and (self.src.min() < 0 or self.dst.min() < 0
                       or self.src.max() >= n or self.dst.max() >= n):
            raise ValueError("vertex id out of range")
        self._h = lib.og_build(self.n, self.m, _ptr(self.src), _ptr(self.dst), _ptr(self.t))
        if not self._h:
            raise MemoryError("oracle build failed")
        self._deg = None

    def close(self):
        if self._h:
            _load().og_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- counts ---------------------------------------------------------------
    def counts(self, delta: int, variant: int = 0, idx=None) -> np.ndarray:
        """count[e] for the edges ``idx`` (input positions) or for all edges.
        Self-loops read 0xFFFFFFFF."""
        lib = _load()
        if idx is None:
            out = np.zeros(self.m, dtype=np.uint32)
            rc = lib.og_counts(self._h, 0, None, int(delta), int(variant), _ptr(out), self.threads)
        else:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            out = np.zeros(idx.shape[0], dtype=np.uint32)
            rc = lib.og_counts(self._h, idx.shape[0], _ptr(idx), int(delta), int(variant),
                               _ptr(out), self.threads)
        if rc != 0:
            raise ValueError("bad delta or variant")
        return out

    def counts_pool(self, deltas, variant: int = 0, idx=None) -> np.ndarray:
        """count[e] for several windows at once, shape (edges, len(deltas))."""
        lib = _load()
        d = np.ascontiguousarray(deltas, dtype=np.int64)
        k = self.m if idx is None else len(idx)
        out = np.zeros((k, d.shape[0]), dtype=np.uint32)
        if idx is None:
            rc = lib.og_counts_pool(self._h, 0, None, int(variant), d.shape[0], _ptr(d), _ptr(out),
                                    self.threads)
        else:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            rc = lib.og_counts_pool(self._h, k, _ptr(idx), int(variant), d.shape[0], _ptr(d),
                                    _ptr(out), self.threads)
        if rc != 0:
            raise ValueError("bad variant or pool")
        return out

    # -- static quantities ------------------------------------------------------
    def degrees(self) -> np.ndarray:
        if self._deg is None:
            out = np.zeros(self.n, dtype=np.int32)
            _load().og_degrees(self._h, _ptr(out))
            self._deg = out
        return self._deg

    def common_counts(self, idx) -> np.ndarray:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros(idx.shape[0], dtype=np.int64)
        _load().og_common_counts(self._h, idx.shape[0], _ptr(idx), _ptr(out), self.threads)
        return out

    def sizes(self) -> dict:
        out = np.zeros(4, dtype=np.int64)
        _load().og_sizes(self._h, _ptr(out), self.threads)
        return dict(directed_pairs=int(out[0]), static_edges=int(out[1]),
                    triangles=int(out[2]), max_degree=int(out[3]))

    def core_numbers(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int32)
        _load().og_core_numbers(self._h, _ptr(out))
        return out

    def peel_levels(self):
        """Level and round of each vertex in level-synchronous min-degree
        peeling: (core numbers, round within the level)."""
        core = np.zeros(self.n, dtype=np.int32)
        rnd = np.zeros(self.n, dtype=np.int32)
        _load().og_peel_levels(self._h, _ptr(core), _ptr(rnd))
        return core, rnd

    def degeneracy_rank(self) -> np.ndarray:
        """Position of each vertex when ordered by (core, round within the level, id)."""
        core, rnd = self.peel_levels()
        order = np.lexsort((np.arange(self.n), rnd, core))
        rank = np.empty(self.n, dtype=np.int32)
        rank[order] = np.arange(self.n, dtype=np.int32)
        return rank

    # -- threshold step and solutions ----------------------------------------------
    def universe_sizes(self, idx=None, universe: int = 0, exclude_other: bool = False):
        idx = np.arange(self.m, dtype=np.int64) if idx is None else np.asarray(idx, np.int64)
        a, b = self.src[idx], self.dst[idx]
        deg = self.degrees()
        if universe == 0:
            u = deg[b].astype(np.int64) - (1 if exclude_other else 0)
        elif universe == 1:
            u = deg[a].astype(np.int64) - (1 if exclude_other else 0)
        elif universe == 2:
            if exclude_other:
                raise ValueError("exclude_other applies to universes 0 and 1 only")
            u = self.common_counts(idx)
        else:
            raise ValueError("universe")
        return u

    def query(self, delta: int, theta_num: int, theta_den: int, variant: int = 0,
              universe: int = 0, exclude_other: bool = False, counts=None) -> dict:
        if theta_den <= 0 or theta_num < 0 or theta_num > theta_den:
            raise ValueError("theta must be num/den in [0, 1]")
        cnt = self.counts(delta, variant) if counts is None else counts
        loop = self.src == self.dst
        keep = ~loop
        idx = np.nonzero(keep)[0]
        u = self.universe_sizes(idx, universe, exclude_other)
        lhs = cnt[idx].astype(np.uint64) * np.uint64(theta_den)
        rhs = u.astype(np.uint64) * np.uint64(theta_num)
        cert = lhs >= rhs
        ci = idx[cert]
        keys = self.src[ci].astype(np.int64) * self.n + self.dst[ci].astype(np.int64)
        uk, nc = np.unique(keys, return_counts=True)
        return dict(pair_u=(uk // self.n).astype(np.int32), pair_v=(uk % self.n).astype(np.int32),
                    n_cert=nc.astype(np.uint32), n_certificates=int(cert.sum()),
                    counts=cnt, self_loops=int(loop.sum()))

    def vertex_query(self, delta: int, theta_num: int, theta_den: int, variant: int = 0,
                     inner_forall: bool = True, inner_num: int = 0, inner_den: int = 1,
                     universe: int = 0, exclude_other: bool = False, counts=None) -> dict:
        """Solution vertices of exists u forall_{theta} v (forall_{inner} | exists) w."""
        if theta_den <= 0 or theta_num < 0 or theta_num > theta_den:
            raise ValueError("theta must be num/den in [0, 1]")
        cnt = self.counts(delta, variant) if counts is None else counts
        # step 1: the edge-level solutions L
        if inner_forall:
            q = self.query(delta, inner_num, inner_den, variant, universe, exclude_other, counts=cnt)
            head, tail = q["pair_u"], q["pair_v"]
        else:
            keep = (self.src != self.dst) & (cnt != U32_MAX) & (cnt >= 1)
            keys = np.unique(self.src[keep].astype(np.int64) * self.n + self.dst[keep].astype(np.int64))
            head, tail = (keys // self.n).astype(np.int32), (keys % self.n).astype(np.int32)
        # steps 2-4: L_u[v] = 1 for every (u, v) with an edge of L from u to v; sums per u
        good = np.zeros(self.n, dtype=np.int64)
        np.add.at(good, head, 1)
        # step 5: threshold against |N(u)| over non-empty neighbourhoods
        deg = self.degrees().astype(np.int64)
        sol = (deg >= 1) & (good * theta_den >= theta_num * deg)
        v = np.nonzero(sol)[0].astype(np.int32)
        return dict(vertices=v, good=good[v].astype(np.uint32), n_vertices=int(v.size),
                    pair_u=head, pair_v=tail, counts=cnt)

    def vertex_query_at(self, us, delta: int, theta_num: int, theta_den: int, variant: int = 0,
                        inner_forall: bool = True, inner_num: int = 0, inner_den: int = 1,
                        universe: int = 0, exclude_other: bool = False) -> dict:
        """The vertex query decided for the vertices us only: a vertex's answer
        depends on the counts of its own outgoing edges alone, so those are the
        only edges counted (for checks on graphs too large to count whole)."""
        us = np.unique(np.asarray(us, dtype=np.int64))
        idx = np.nonzero(np.isin(self.src, us) & (self.src != self.dst))[0]
        cnt = self.counts(delta, variant, idx)
        if inner_forall:
            if theta_den <= 0 or inner_den <= 0 or inner_num > inner_den:
                raise ValueError("theta")
            ok = cnt.astype(np.uint64) * np.uint64(inner_den) >= \
                self.universe_sizes(idx, universe, exclude_other).astype(np.uint64) * np.uint64(inner_num)
        else:
            ok = cnt >= 1
        keys = np.unique(self.src[idx[ok]].astype(np.int64) * self.n + self.dst[idx[ok]].astype(np.int64))
        good = np.zeros(self.n, dtype=np.int64)
        np.add.at(good, keys // self.n, 1)
        deg = self.degrees().astype(np.int64)
        sol = (deg[us] >= 1) & (good[us] * theta_den >= theta_num * deg[us])
        return dict(vertices=us.astype(np.int32), solution=sol, good=good[us].astype(np.uint32),
                    edges_counted=int(idx.size))

    # -- exists-exists-exists ---------------------------------------------------------
    def triad_instances(self, delta: int, variant: int = 0, idx=None) -> np.ndarray:
        """Temporal triangles whose first edge is each edge of ``idx`` (input
        positions; all edges by default), over every third vertex; self-loops 0."""
        lib = _load()
        if idx is None:
            out = np.zeros(self.m, dtype=np.uint64)
            rc = lib.og_triad_instances(self._h, 0, None, int(delta), int(variant), _ptr(out),
                                        self.threads)
        else:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            out = np.zeros(idx.shape[0], dtype=np.uint64)
            rc = lib.og_triad_instances(self._h, idx.shape[0], _ptr(idx), int(delta), int(variant),
                                        _ptr(out), self.threads)
        if rc != 0:
            raise ValueError("bad delta or variant")
        return out

    def pair_table(self):
        """The directed pairs (x, y) with at least one temporal edge x -> y, ascending."""
        lib = _load()
        k = lib.og_pair_table(self._h, None, None)
        x = np.zeros(k, dtype=np.int32)
        y = np.zeros(k, dtype=np.int32)
        lib.og_pair_table(self._h, _ptr(x), _ptr(y))
        return x, y

    def triad_pair_counts(self, delta: int, variant: int = 0) -> np.ndarray:
        """Solution triples of each directed pair of ``pair_table``."""
        lib = _load()
        x, _ = self.pair_table()
        cnt = np.zeros(x.shape[0], dtype=np.int64)
        if lib.og_triad_pair_counts(self._h, int(delta), int(variant), _ptr(cnt), self.threads) != 0:
            raise ValueError("bad delta or variant")
        return cnt

    def triad_solutions(self, delta: int, variant: int = 0) -> np.ndarray:
        """All solution triples (a, b, w), shape (k, 3), ascending by (a, b, w)."""
        lib = _load()
        cnt = self.triad_pair_counts(delta, variant)
        off = np.zeros(cnt.shape[0] + 1, dtype=np.int64)
        np.cumsum(cnt, out=off[1:])
        out = np.zeros((int(off[-1]), 3), dtype=np.int32)
        if lib.og_triad_fill(self._h, int(delta), int(variant), _ptr(off), _ptr(out), self.threads) != 0:
            raise ValueError("bad delta or variant")
        return out

    def triad_pair(self, a: int, b: int, delta: int, variant: int = 0) -> np.ndarray:
        """The third vertices w (ascending) of the solution triples (a, b, w)."""
        lib = _load()
        deg = self.degrees()
        out = np.zeros(int(min(deg[a], deg[b])) + 1, dtype=np.int32)
        c = lib.og_triad_pair(self._h, int(a), int(b), int(delta), int(variant), _ptr(out))
        if c < 0:
            raise ValueError("bad arguments")
        return out[:c].copy()
