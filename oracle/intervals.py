"""The paper's in-neighbour mechanism, written out (test infrastructure only).

Only the tests may use this module.  It restates, for small inputs, how the
paper computes in-count[e] without walking E_{a,b} once per third vertex:

* ``interval_list(L2, L3, delta)`` - the intervals of the in-neighbour theorem
  (Section 3, "Dealing with In-Neighbours"): for every t2 in L2 whose first
  entry t3 of L3 at or after t2 satisfies t3 <= t2 + delta, the interval
  [max(0, t3 - delta), t2].  An edge at time t forms a delta-temporal triangle
  with the third vertex iff one of these intervals contains t.
* ``SegmentTree`` - the per-list structure of the appendix ("Segment-Trees to
  deal with in-neighbours"): a balanced tree over the distinct timestamps of
  one directed list, nodes with a Color, a Counter and a Vertex field, the
  three-phase lazy insertion of one vertex's interval list (Phase 1 marks
  canonical nodes grey unless a grey node lies above, Phase 2 turns grey nodes
  with a grey ancestor back to white, Phase 3 counts the remaining grey nodes
  once for the vertex), and the lookup that sums the counters on the path of t.
  An interval is clipped to the list's timestamps by binary search before
  insertion (appendix, "How to build the Segment Tree?").  Lookups only ever
  ask for timestamps of the list itself, so the tree's leaves are its distinct
  timestamps; the open gaps between them hold no query point.
* ``counts_via_intervals`` and ``counts_via_segment_trees`` - count[e] for every
  edge from these pieces (every common neighbour's intervals for the list of e,
  the union checked directly, or counted by the list's segment tree).
"""
from __future__ import annotations

import bisect

WHITE, GREY = 0, 1


def interval_list(L2, L3, delta):
    """The intervals of the in-neighbour theorem for sorted lists L2, L3."""
    out = []
    for t2 in L2:
        k = bisect.bisect_left(L3, t2)  # L23[e]: the first entry of L3 at or after t(e)
        if k == len(L3):
            continue
        t3 = L3[k]
        if t3 <= t2 + delta:
            out.append((max(0, t3 - delta), t2))
    return out


class SegmentTree:
    """Segment tree over the sorted distinct timestamps ts of one directed list."""

    def __init__(self, ts):
        self.ts = sorted(set(int(x) for x in ts))
        self.r = len(self.ts)
        size = 1
        while size < max(1, self.r):
            size *= 2
        self.size = size
        self.color = [WHITE] * (2 * size)
        self.counter = [0] * (2 * size)
        self.vertex = [-1] * (2 * size)

    # node k covers leaf positions [lo, hi]; the root is 1 over [0, size - 1]
    def _clip(self, a, b):
        """The leaf range of the timestamps inside [a, b] (None if there are none)."""
        i = bisect.bisect_left(self.ts, a)
        j = bisect.bisect_right(self.ts, b) - 1
        return (i, j) if i <= j else None

    def _walk(self, k, lo, hi, i, j, visit):
        """Depth-first over the canonical nodes of [i, j]: visit(k, at_canonical)
        is called on every node of the search; it returns False to stop below."""
        if j < lo or hi < i:
            return
        canonical = i <= lo and hi <= j
        if not visit(k, canonical) or canonical:
            return
        mid = (lo + hi) // 2
        self._walk(2 * k, lo, mid, i, j, visit)
        self._walk(2 * k + 1, mid + 1, hi, i, j, visit)

    def insert_list(self, intervals, z):
        """The three phases for the interval list of vertex z."""
        ranges = [c for c in (self._clip(a, b) for a, b in intervals) if c is not None]
        if not ranges:
            return

        # Phase 1: a canonical node turns grey unless a grey node was met above it
        def phase1(k, canonical):
            if self.color[k] == GREY:
                return False
            if canonical:
                self.color[k] = GREY
            return True

        # Phase 3: count the grey nodes that are left, once for z
        def phase3(k, canonical):
            if canonical:
                if self.color[k] == GREY:
                    self.color[k] = WHITE
                    self.counter[k] += 1
                    self.vertex[k] = z
                return True
            if self.color[k] == GREY:
                return False
            if self.counter[k] > 0 and self.vertex[k] == z:
                return False
            return True

        for i, j in ranges:
            self._walk(1, 0, self.size - 1, i, j, phase1)
        # Phase 2: a canonical node with a grey node above it turns white again
        for i, j in ranges:
            self._phase2(i, j)
        for i, j in ranges:
            self._walk(1, 0, self.size - 1, i, j, phase3)

    def _phase2(self, i, j):
        """Phase 2 for one interval: whether a grey node lies above is per root path."""
        def rec(k, lo, hi, grey_above):
            if j < lo or hi < i:
                return
            if i <= lo and hi <= j:
                if grey_above and self.color[k] == GREY:
                    self.color[k] = WHITE
                return
            g = grey_above or self.color[k] == GREY
            mid = (lo + hi) // 2
            rec(2 * k, lo, mid, g)
            rec(2 * k + 1, mid + 1, hi, g)
        rec(1, 0, self.size - 1, False)

    def lookup(self, t):
        """Sum of the counters on the path of timestamp t (0 if t is not a leaf)."""
        p = bisect.bisect_left(self.ts, t)
        if p == self.r or self.ts[p] != t:
            return 0
        k, lo, hi, s = 1, 0, self.size - 1, 0
        while True:
            s += self.counter[k]
            if lo == hi:
                return s
            mid = (lo + hi) // 2
            if p <= mid:
                k, hi = 2 * k, mid
            else:
                k, lo = 2 * k + 1, mid + 1


def _lists_and_neighbours(n, src, dst, t):
    by_pair = {}
    nb = [set() for _ in range(n)]
    for a, b, x in zip(src, dst, t):
        a, b, x = int(a), int(b), int(x)
        if a == b:
            continue
        by_pair.setdefault((a, b), []).append(x)
        nb[a].add(b)
        nb[b].add(a)
    for k in by_pair:
        by_pair[k].sort()
    return by_pair, nb


def _pick(by_pair, variant, a, b, w):
    X, Y = (b, a) if variant & 4 else (a, b)
    L2 = by_pair.get((w, X) if variant & 1 else (X, w), [])
    L3 = by_pair.get((w, Y) if variant & 2 else (Y, w), [])
    return L2, L3


def counts_via_intervals(n, src, dst, t, delta, variant=0):
    """count[e]: third vertices w with an interval of I(w) containing t(e)."""
    by_pair, nb = _lists_and_neighbours(n, src, dst, t)
    out = []
    for a, b, x in zip(src, dst, t):
        a, b, x = int(a), int(b), int(x)
        if a == b:
            out.append(0xFFFFFFFF)
            continue
        c = 0
        for w in nb[a] & nb[b]:
            L2, L3 = _pick(by_pair, variant, a, b, w)
            if any(lo <= x <= hi for lo, hi in interval_list(L2, L3, delta)):
                c += 1
        out.append(c)
    return out


def counts_via_segment_trees(n, src, dst, t, delta, variant=0):
    """count[e] from one segment tree per directed list: every common neighbour
    w of (a, b) inserts its interval list for E_{a,b}, then each edge looks up
    its timestamp."""
    by_pair, nb = _lists_and_neighbours(n, src, dst, t)
    trees = {}
    for (a, b), L1 in by_pair.items():
        T = SegmentTree(L1)
        for w in sorted(nb[a] & nb[b]):
            L2, L3 = _pick(by_pair, variant, a, b, w)
            T.insert_list(interval_list(L2, L3, delta), w)
        trees[(a, b)] = T
    return [0xFFFFFFFF if int(a) == int(b) else trees[(int(a), int(b))].lookup(int(x))
            for a, b, x in zip(src, dst, t)]
