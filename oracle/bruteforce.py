"""Literal brute force for the exists-exists-forall triadic query (tiny graphs).

Test infrastructure only.  Independent of ``folty_oracle.c``: it reads the
quantifiers off the definitions (paper, Definition of a thresholded FOL triadic
query and the delta-temporal triangle of Section "Main Ideas") with no
adjacency shortcut, no sorting and no greedy step:

    count[e] = #{ w in V \\ {a, b} : exists e2 in L2(w), e3 in L3(w) with
                  t(e) <= t(e2) <= t(e3) <= t(e) + delta }

where, for the 3-bit predicate code, edge 2 hangs off a (bit 2 clear) or b,
edge 3 off the other endpoint, and bits 0/1 flip edge 2/edge 3 to point at that
endpoint instead of away from it.  Cost O(m * n * m^2) in the worst case: use
n <= 200 and m <= 2,000.
"""
from __future__ import annotations


def counts(n, src, dst, t, delta, variant=0):
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    t = [int(x) for x in t]
    m = len(src)
    by_pair = {}
    for i in range(m):
        if src[i] != dst[i]:
            by_pair.setdefault((src[i], dst[i]), []).append(t[i])
    out = []
    for i in range(m):
        a, b, te = src[i], dst[i], t[i]
        if a == b:
            out.append(0xFFFFFFFF)
            continue
        X, Y = (b, a) if variant & 4 else (a, b)
        c = 0
        for w in range(n):
            if w == a or w == b:
                continue
            L2 = by_pair.get((w, X) if variant & 1 else (X, w), [])
            L3 = by_pair.get((w, Y) if variant & 2 else (Y, w), [])
            if any(te <= t2 <= t3 <= te + delta for t2 in L2 for t3 in L3):
                c += 1
        out.append(c)
    return out


def neighbours(n, src, dst):
    nb = [set() for _ in range(n)]
    for a, b in zip(src, dst):
        a, b = int(a), int(b)
        if a != b:
            nb[a].add(b)
            nb[b].add(a)
    return nb


def query(n, src, dst, t, delta, theta_num, theta_den, variant=0, universe=0,
          exclude_other=False):
    """Certificates and solution pairs, all by the definitions."""
    cnt = counts(n, src, dst, t, delta, variant)
    nb = neighbours(n, src, dst)
    pairs = {}
    ncert = 0
    for i, (a, b) in enumerate(zip(src, dst)):
        a, b = int(a), int(b)
        if a == b:
            continue
        if universe == 0:
            U = len(nb[b]) - (1 if exclude_other else 0)
        elif universe == 1:
            U = len(nb[a]) - (1 if exclude_other else 0)
        else:
            U = len(nb[a] & nb[b])
        if cnt[i] * theta_den >= theta_num * U:
            ncert += 1
            pairs[(a, b)] = pairs.get((a, b), 0) + 1
    keys = sorted(pairs)
    return dict(pairs=[(a, b, pairs[(a, b)]) for a, b in keys], n_certificates=ncert,
                counts=cnt)


def vertex_query(n, src, dst, t, delta, theta_num, theta_den, variant=0, inner_forall=True,
                 inner_num=0, inner_den=1, universe=0, exclude_other=False):
    """exists u forall_theta v in N(u) (forall_inner | exists) w, by the definitions:
    u is a solution when N(u) is not empty and at least theta * |N(u)| of its
    neighbours v have a temporal edge (u, v, t) that certifies the inner query
    (count >= inner * |U(e)|, or count >= 1 for an inner exists)."""
    cnt = counts(n, src, dst, t, delta, variant)
    nb = neighbours(n, src, dst)
    ok_pairs = set()
    for i, (a, b) in enumerate(zip(src, dst)):
        a, b = int(a), int(b)
        if a == b:
            continue
        if inner_forall:
            if universe == 0:
                U = len(nb[b]) - (1 if exclude_other else 0)
            elif universe == 1:
                U = len(nb[a]) - (1 if exclude_other else 0)
            else:
                U = len(nb[a] & nb[b])
            ok = cnt[i] * inner_den >= inner_num * U
        else:
            ok = cnt[i] >= 1
        if ok:
            ok_pairs.add((a, b))
    out = []
    for u in range(n):
        if not nb[u]:
            continue
        good = sum(1 for v in nb[u] if (u, v) in ok_pairs)
        if good * theta_den >= theta_num * len(nb[u]):
            out.append((u, good))
    return out


def triads(n, src, dst, t, delta, variant=0):
    """The exists-exists-exists query by its definition (paper, Definition of a
    solution): every ordered triple (a, b, w) of distinct vertices with an edge
    triple e1 = (a, b, t1), e2 in L2(w), e3 in L3(w), t1 <= t2 <= t3 <= t1 + delta
    is a solution; inst[e1] counts those edge triples per first edge."""
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    t = [int(x) for x in t]
    m = len(src)
    by_pair = {}
    for i in range(m):
        if src[i] != dst[i]:
            by_pair.setdefault((src[i], dst[i]), []).append(t[i])
    inst = [0] * m
    sols = set()
    for i in range(m):
        a, b, te = src[i], dst[i], t[i]
        if a == b:
            continue
        X, Y = (b, a) if variant & 4 else (a, b)
        for w in range(n):
            if w == a or w == b:
                continue
            L2 = by_pair.get((w, X) if variant & 1 else (X, w), [])
            L3 = by_pair.get((w, Y) if variant & 2 else (Y, w), [])
            c = sum(1 for t2 in L2 for t3 in L3 if te <= t2 <= t3 <= te + delta)
            if c:
                inst[i] += c
                sols.add((a, b, w))
    return dict(triples=sorted(sols), instances=inst, n_instances=sum(inst))
