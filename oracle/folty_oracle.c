/*
 * CPU oracle for the thresholded exists-exists-forall triadic query on a
 * temporal multigraph.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain statement of what the
 * GPU library computes.  It shares no code, header, table or helper with the
 * GPU library, and nothing in the product path may link or call it: only the
 * tests, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * What it computes (paper, Section "Main Ideas"):
 *   - The static graph G_S drops directions, parallel edges and self-loops;
 *     N(x) is the static neighbourhood of x.
 *   - E_{x,y} is the time-sorted list of temporal edges from x to y.
 *   - A temporal edge e = (a, b, t) forms a delta-temporal triangle with a
 *     third vertex w when temporal edges e2 in L2 and e3 in L3 exist with
 *     t <= t(e2) <= t(e3) <= t + delta.  For the paper's predicate (the
 *     temporal triangle of its Figure "Predicate for FOL queries") L2 = E_{a,w}
 *     and L3 = E_{b,w}.
 *   - count[e] is the number of distinct w that form at least one such
 *     triangle with e (Section 3, the in-count/out-count arrays, whose sum is
 *     what the threshold step compares).
 *   - Other edge-direction predicates are selected by a 3-bit code:
 *       bit 2 = 0: edge 2 hangs off a and edge 3 off b; 1: the reverse;
 *       bit 0 = 0: edge 2 points away from its endpoint (X -> w); 1: towards it;
 *       bit 1 = 0: edge 3 points away from its endpoint (Y -> w); 1: towards it.
 *     Code 0 is the paper's predicate.
 *
 * Every test here is the definition written out: the existence of (e2, e3) is
 * checked by looking at pairs, not by the greedy first-entry search of the
 * paper's Theorems 3.1 and 3.2 (those are what the GPU path uses).  The only
 * shortcuts rely on the lists being sorted by time (stop scanning once a
 * timestamp leaves the window).
 *
 * Core numbers follow the bucket form of the min-degree peeling the paper
 * cites for its degeneracy ordering (Section "Main Ideas", Preliminaries).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t key; /* x * n + y */
    int64_t t;
    int64_t idx; /* input position */
} og_rec;

typedef struct {
    int32_t n;
    int64_t m;
    int32_t *src, *dst;
    int64_t *t;
    /* static graph */
    int64_t *adj_off; /* n + 1 */
    int32_t *adj;     /* sorted neighbour ids */
    int64_t n_static;
    /* directed lists E_{x,y}, pair-major, time-sorted inside a pair */
    int64_t np;
    int64_t *pkey;    /* np, sorted */
    int64_t *poff;    /* np + 1 */
    int64_t *pt;      /* m' */
    int64_t *pidx;    /* m' */
} og_graph;

static int cmp_rec(const void *A, const void *B) {
    const og_rec *a = (const og_rec *)A, *b = (const og_rec *)B;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->t != b->t) return a->t < b->t ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

static int cmp_i64(const void *A, const void *B) {
    int64_t a = *(const int64_t *)A, b = *(const int64_t *)B;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int cmp_i32(const void *A, const void *B) {
    int32_t a = *(const int32_t *)A, b = *(const int32_t *)B;
    return a < b ? -1 : (a > b ? 1 : 0);
}

void og_free(og_graph *g) {
    if (!g) return;
    free(g->src); free(g->dst); free(g->t);
    free(g->adj_off); free(g->adj);
    free(g->pkey); free(g->poff); free(g->pt); free(g->pidx);
    free(g);
}

og_graph *og_build(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                   const int64_t *t) {
    og_graph *g = (og_graph *)calloc(1, sizeof(og_graph));
    if (!g) return NULL;
    g->n = n;
    g->m = m;
    g->src = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    g->dst = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    g->t = (int64_t *)malloc(sizeof(int64_t) * (m ? m : 1));
    memcpy(g->src, src, sizeof(int32_t) * m);
    memcpy(g->dst, dst, sizeof(int32_t) * m);
    memcpy(g->t, t, sizeof(int64_t) * m);

    /* E_{x,y}: sort the non-loop edges by (x, y, t, input index) */
    og_rec *r = (og_rec *)malloc(sizeof(og_rec) * (m ? m : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < m; i++) {
        if (src[i] == dst[i]) continue; /* self-loops are not in G_S */
        r[k].key = (int64_t)src[i] * n + dst[i];
        r[k].t = t[i];
        r[k].idx = i;
        k++;
    }
    qsort(r, (size_t)k, sizeof(og_rec), cmp_rec);
    int64_t np = 0;
    for (int64_t i = 0; i < k; i++)
        if (i == 0 || r[i].key != r[i - 1].key) np++;
    g->np = np;
    g->pkey = (int64_t *)malloc(sizeof(int64_t) * (np ? np : 1));
    g->poff = (int64_t *)malloc(sizeof(int64_t) * (np + 1));
    g->pt = (int64_t *)malloc(sizeof(int64_t) * (k ? k : 1));
    g->pidx = (int64_t *)malloc(sizeof(int64_t) * (k ? k : 1));
    int64_t p = -1;
    for (int64_t i = 0; i < k; i++) {
        if (i == 0 || r[i].key != r[i - 1].key) {
            p++;
            g->pkey[p] = r[i].key;
            g->poff[p] = i;
        }
        g->pt[i] = r[i].t;
        g->pidx[i] = r[i].idx;
    }
    g->poff[np] = k;
    free(r);

    /* G_S: unordered pairs {min, max}, deduplicated */
    int64_t *uk = (int64_t *)malloc(sizeof(int64_t) * (np ? np : 1));
    for (int64_t i = 0; i < np; i++) {
        int64_t x = g->pkey[i] / n, y = g->pkey[i] % n;
        int64_t lo = x < y ? x : y, hi = x < y ? y : x;
        uk[i] = lo * n + hi;
    }
    qsort(uk, (size_t)np, sizeof(int64_t), cmp_i64);
    int64_t ns = 0;
    for (int64_t i = 0; i < np; i++)
        if (i == 0 || uk[i] != uk[i - 1]) uk[ns++] = uk[i];
    g->n_static = ns;
    g->adj_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < ns; i++) {
        g->adj_off[uk[i] / n + 1]++;
        g->adj_off[uk[i] % n + 1]++;
    }
    for (int32_t x = 0; x < n; x++) g->adj_off[x + 1] += g->adj_off[x];
    g->adj = (int32_t *)malloc(sizeof(int32_t) * (2 * ns + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, g->adj_off, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < ns; i++) {
        int32_t lo = (int32_t)(uk[i] / n), hi = (int32_t)(uk[i] % n);
        g->adj[fill[lo]++] = hi;
        g->adj[fill[hi]++] = lo;
    }
    free(fill);
    free(uk);
    for (int32_t x = 0; x < n; x++)
        qsort(g->adj + g->adj_off[x], (size_t)(g->adj_off[x + 1] - g->adj_off[x]),
              sizeof(int32_t), cmp_i32);
    return g;
}

/* E_{x,y} as (times, input indices, length); length 0 when absent */
static int64_t og_list(const og_graph *g, int32_t x, int32_t y, const int64_t **times,
                       const int64_t **idx) {
    int64_t key = (int64_t)x * g->n + y;
    const int64_t *hit = (const int64_t *)bsearch(&key, g->pkey, (size_t)g->np,
                                                  sizeof(int64_t), cmp_i64);
    if (!hit) { *times = NULL; if (idx) *idx = NULL; return 0; }
    int64_t p = hit - g->pkey;
    *times = g->pt + g->poff[p];
    if (idx) *idx = g->pidx + g->poff[p];
    return g->poff[p + 1] - g->poff[p];
}

static int og_adjacent(const og_graph *g, int32_t x, int32_t y) {
    const int32_t *b = g->adj + g->adj_off[x];
    size_t len = (size_t)(g->adj_off[x + 1] - g->adj_off[x]);
    return bsearch(&y, b, len, sizeof(int32_t), cmp_i32) != NULL;
}

/* N(a) and N(b) intersected: walk the shorter list, look each id up in the other. */
static int64_t og_common(const og_graph *g, int32_t a, int32_t b, int32_t *out) {
    int64_t da = g->adj_off[a + 1] - g->adj_off[a];
    int64_t db = g->adj_off[b + 1] - g->adj_off[b];
    int32_t x = da <= db ? a : b, y = da <= db ? b : a;
    int64_t c = 0;
    for (int64_t i = g->adj_off[x]; i < g->adj_off[x + 1]; i++) {
        int32_t w = g->adj[i];
        if (og_adjacent(g, y, w)) {
            if (out) out[c] = w;
            c++;
        }
    }
    return c;
}

/* The two lists a predicate code picks for edge e = (a, b, t) and third vertex w. */
static void og_pick(const og_graph *g, int variant, int32_t a, int32_t b, int32_t w,
                    const int64_t **L2, int64_t *n2, const int64_t **L3, int64_t *n3) {
    int32_t X = (variant & 4) ? b : a; /* endpoint that edge 2 hangs off */
    int32_t Y = (variant & 4) ? a : b; /* endpoint that edge 3 hangs off */
    *n2 = (variant & 1) ? og_list(g, w, X, L2, NULL) : og_list(g, X, w, L2, NULL);
    *n3 = (variant & 2) ? og_list(g, w, Y, L3, NULL) : og_list(g, Y, w, L3, NULL);
}

/* Is there (t2, t3) in L2 x L3 with t <= t2 <= t3 and t3 - t <= delta? */
static int og_exists(int64_t t, int64_t delta, const int64_t *L2, int64_t n2,
                     const int64_t *L3, int64_t n3) {
    for (int64_t i = 0; i < n2; i++) {
        int64_t t2 = L2[i];
        if (t2 < t) continue;
        if (t2 - t > delta) break;
        for (int64_t j = 0; j < n3; j++) {
            int64_t t3 = L3[j];
            if (t3 < t2) continue;
            if (t3 - t > delta) break;
            return 1;
        }
    }
    return 0;
}

/* Smallest window t3 - t over all (t2, t3) with t <= t2 <= t3; INT64_MAX if none. */
static int64_t og_min_window(int64_t t, const int64_t *L2, int64_t n2, const int64_t *L3,
                             int64_t n3) {
    int64_t best = INT64_MAX;
    for (int64_t i = 0; i < n2; i++) {
        int64_t t2 = L2[i];
        if (t2 < t) continue;
        for (int64_t j = 0; j < n3; j++) {
            int64_t t3 = L3[j];
            if (t3 < t2) continue;
            if (t3 - t < best) best = t3 - t;
            break; /* sorted: the first t3 >= t2 is this t2's smallest window */
        }
    }
    return best;
}

/* count[e] for one temporal edge, given the common neighbours of its endpoints */
static uint32_t og_count_one(const og_graph *g, int64_t i, int64_t delta, int variant,
                             const int32_t *common, int64_t nc) {
    int32_t a = g->src[i], b = g->dst[i];
    uint32_t c = 0;
    for (int64_t j = 0; j < nc; j++) {
        const int64_t *L2, *L3;
        int64_t n2, n3;
        og_pick(g, variant, a, b, common[j], &L2, &n2, &L3, &n3);
        if (og_exists(g->t[i], delta, L2, n2, L3, n3)) c++;
    }
    return c;
}

/*
 * count[] for the edges idx[0..k) (input positions), or for all m edges when
 * idx is NULL (then out is indexed by input position).  Self-loops get
 * UINT32_MAX.  Returns 0, or -1 on bad arguments.
 *
 * For all edges the common neighbours of a pair are found once and serve every
 * temporal edge of its list E_{a,b}, as the paper's practical algorithm does
 * per static edge (Algorithm PRACTICAL-EEA); the per-edge test is the same.
 */
int og_counts(const og_graph *g, int64_t k, const int64_t *idx, int64_t delta, int variant,
              uint32_t *out, int threads) {
    if (delta < 0 || variant < 0 || variant > 7) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    if (!idx) {
        for (int64_t i = 0; i < g->m; i++)
            if (g->src[i] == g->dst[i]) out[i] = UINT32_MAX;
#pragma omp parallel
        {
            int32_t *buf = NULL;
            int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < g->np; p++) {
                int32_t a = (int32_t)(g->pkey[p] / g->n), b = (int32_t)(g->pkey[p] % g->n);
                int64_t need = g->adj_off[a + 1] - g->adj_off[a];
                int64_t nb = g->adj_off[b + 1] - g->adj_off[b];
                if (nb < need) need = nb;
                if (need + 1 > cap) { free(buf); cap = need + 1; buf = (int32_t *)malloc(sizeof(int32_t) * cap); }
                int64_t nc = og_common(g, a, b, buf);
                for (int64_t j = g->poff[p]; j < g->poff[p + 1]; j++)
                    out[g->pidx[j]] = og_count_one(g, g->pidx[j], delta, variant, buf, nc);
            }
            free(buf);
        }
        return 0;
    }
#pragma omp parallel
    {
        int32_t *buf = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < k; q++) {
            int64_t i = idx[q];
            int32_t a = g->src[i], b = g->dst[i];
            if (a == b) { out[q] = UINT32_MAX; continue; }
            int64_t need = g->adj_off[a + 1] - g->adj_off[a];
            int64_t nb = g->adj_off[b + 1] - g->adj_off[b];
            if (nb < need) need = nb;
            if (need + 1 > cap) { free(buf); cap = need + 1; buf = (int32_t *)malloc(sizeof(int32_t) * cap); }
            int64_t nc = og_common(g, a, b, buf);
            out[q] = og_count_one(g, i, delta, variant, buf, nc);
        }
        free(buf);
    }
    return 0;
}

/*
 * One pass for many windows: out[q * nd + j] = number of w whose smallest
 * window for edge idx[q] is <= deltas[j].  Same convention for idx == NULL.
 */
int og_counts_pool(const og_graph *g, int64_t k, const int64_t *idx, int variant, int nd,
                   const int64_t *deltas, uint32_t *out, int threads) {
    if (variant < 0 || variant > 7 || nd <= 0) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    int64_t cnt = idx ? k : g->m;
#pragma omp parallel
    {
        int32_t *buf = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < cnt; q++) {
            int64_t i = idx ? idx[q] : q;
            int32_t a = g->src[i], b = g->dst[i];
            uint32_t *o = out + q * nd;
            if (a == b) { for (int j = 0; j < nd; j++) o[j] = UINT32_MAX; continue; }
            for (int j = 0; j < nd; j++) o[j] = 0;
            int64_t need = g->adj_off[a + 1] - g->adj_off[a];
            int64_t nb = g->adj_off[b + 1] - g->adj_off[b];
            if (nb < need) need = nb;
            if (need + 1 > cap) { free(buf); cap = need + 1; buf = (int32_t *)malloc(sizeof(int32_t) * cap); }
            int64_t nc = og_common(g, a, b, buf);
            for (int64_t c = 0; c < nc; c++) {
                const int64_t *L2, *L3;
                int64_t n2, n3;
                og_pick(g, variant, a, b, buf[c], &L2, &n2, &L3, &n3);
                int64_t win = og_min_window(g->t[i], L2, n2, L3, n3);
                if (win == INT64_MAX) continue;
                for (int j = 0; j < nd; j++)
                    if (win <= deltas[j]) o[j]++;
            }
        }
        free(buf);
    }
    return 0;
}

/* |N(x)| for every vertex */
void og_degrees(const og_graph *g, int32_t *out) {
    for (int32_t x = 0; x < g->n; x++) out[x] = (int32_t)(g->adj_off[x + 1] - g->adj_off[x]);
}

/* |N(src[i]) intersect N(dst[i])| for the given input positions (self-loops: -1) */
void og_common_counts(const og_graph *g, int64_t k, const int64_t *idx, int64_t *out,
                      int threads) {
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < k; q++) {
        int64_t i = idx[q];
        out[q] = g->src[i] == g->dst[i] ? -1 : og_common(g, g->src[i], g->dst[i], NULL);
    }
}

/* static sizes: directed pairs, static edges, static triangles, max degree */
void og_sizes(const og_graph *g, int64_t *out4, int threads) {
    int64_t tri3 = 0, maxdeg = 0;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : tri3) reduction(max : maxdeg)
    for (int32_t x = 0; x < g->n; x++) {
        int64_t d = g->adj_off[x + 1] - g->adj_off[x];
        if (d > maxdeg) maxdeg = d;
        for (int64_t i = g->adj_off[x]; i < g->adj_off[x + 1]; i++) {
            int32_t y = g->adj[i];
            if (y > x) tri3 += og_common(g, x, y, NULL);
        }
    }
    out4[0] = g->np;
    out4[1] = g->n_static;
    out4[2] = tri3 / 3;
    out4[3] = maxdeg;
}

/*
 * Core numbers by min-degree peeling with degree buckets (Batagelj and
 * Zaversnik's O(m) form of the Matula-Beck ordering): repeatedly remove a
 * vertex of smallest remaining degree; its core number is the largest
 * smallest-degree seen so far.
 */
void og_core_numbers(const og_graph *g, int32_t *core) {
    int32_t n = g->n;
    int64_t maxd = 0;
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    for (int32_t x = 0; x < n; x++) {
        deg[x] = g->adj_off[x + 1] - g->adj_off[x];
        if (deg[x] > maxd) maxd = deg[x];
    }
    int64_t *bin = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t *vert = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    for (int32_t x = 0; x < n; x++) bin[deg[x]]++;
    int64_t start = 0;
    for (int64_t d = 0; d <= maxd; d++) { int64_t c = bin[d]; bin[d] = start; start += c; }
    for (int32_t x = 0; x < n; x++) { pos[x] = bin[deg[x]]; vert[pos[x]] = x; bin[deg[x]]++; }
    for (int64_t d = maxd; d >= 1; d--) bin[d] = bin[d - 1];
    bin[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t v = vert[i];
        for (int64_t j = g->adj_off[v]; j < g->adj_off[v + 1]; j++) {
            int32_t u = g->adj[j];
            if (deg[u] > deg[v]) {
                int64_t du = deg[u], pu = pos[u], pw = bin[du];
                int32_t w = vert[pw];
                if (u != w) { pos[u] = pw; vert[pu] = w; pos[w] = pu; vert[pw] = u; }
                bin[du]++;
                deg[u]--;
            }
        }
    }
    for (int32_t x = 0; x < n; x++) core[x] = (int32_t)deg[x];
    free(deg); free(bin); free(pos); free(vert);
}

/*
 * The degeneracy ordering as level-synchronous min-degree peeling (Section
 * "Main Ideas", Preliminaries: repeatedly remove a vertex of minimum degree).
 * Level k starts once no remaining vertex has degree below k; each round of
 * the level removes, all at once, every remaining vertex whose degree among the
 * remaining vertices is at most k, until a round finds none.  core[x] = k is
 * the level of x and rnd[x] the round of that level in which x went (0 for the
 * first).  Ordering vertices by (core, rnd, id) leaves each vertex at most k
 * neighbours after it: they were all still there when its round began.
 * Vertices whose degree passes above the current level wait in a bucket of
 * their degree (stale bucket entries are skipped).
 */
void og_peel_levels(const og_graph *g, int32_t *core, int32_t *rnd) {
    int32_t n = g->n;
    int64_t maxd = 0;
    int64_t *dc = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    for (int32_t x = 0; x < n; x++) {
        dc[x] = g->adj_off[x + 1] - g->adj_off[x];
        if (dc[x] > maxd) maxd = dc[x];
    }
    int64_t cap = (int64_t)n + g->adj_off[n] + 1;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * ((size_t)maxd + 1));
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    int32_t *val = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int64_t used = 0;
    for (int64_t d = 0; d <= maxd; d++) head[d] = -1;
    for (int32_t x = 0; x < n; x++) {
        val[used] = x; next[used] = head[dc[x]]; head[dc[x]] = used; used++;
    }
    char *gone = (char *)calloc((size_t)n + 1, 1);
    char *queued = (char *)calloc((size_t)n + 1, 1);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    for (int64_t k = 0; k <= maxd; k++) {
        int64_t nc = 0;
        for (int64_t e = head[k]; e >= 0; e = next[e]) {
            int32_t x = val[e];
            if (!gone[x] && !queued[x] && dc[x] == k) { queued[x] = 1; cur[nc++] = x; }
        }
        for (int32_t r = 0; nc > 0; r++) {
            for (int64_t i = 0; i < nc; i++) { gone[cur[i]] = 1; core[cur[i]] = (int32_t)k; rnd[cur[i]] = r; }
            int64_t nn = 0;
            for (int64_t i = 0; i < nc; i++) {
                int32_t x = cur[i];
                for (int64_t j = g->adj_off[x]; j < g->adj_off[x + 1]; j++) {
                    int32_t u = g->adj[j];
                    if (gone[u]) continue;
                    dc[u]--;
                    if (dc[u] == k) { if (!queued[u]) { queued[u] = 1; nxt[nn++] = u; } }
                    else if (dc[u] > k) { val[used] = u; next[used] = head[dc[u]]; head[dc[u]] = used; used++; }
                }
            }
            int32_t *t = cur; cur = nxt; nxt = t;
            nc = nn;
        }
    }
    free(dc); free(head); free(next); free(val); free(gone); free(queued); free(cur); free(nxt);
}

int og_num_threads(void) { return omp_get_max_threads(); }

/*
 * ---------------------------------------------------------------------------
 * Exists-exists-exists queries (paper, Definition of a solution: with three
 * existential quantifiers a solution is a vertex triple; Section 1 and the
 * problem statement: counting them is temporal triangle counting).
 *
 * For a predicate code, the temporal triangle on the ordered triple (a, b, w)
 * is three temporal edges e1 in E_{a,b}, e2 in L2 and e3 in L3 (the lists the
 * code picks, as above) with t(e1) <= t(e2) <= t(e3) <= t(e1) + delta.
 *   - (a, b, w) is a solution when at least one such edge triple exists;
 *   - inst[e1] is the number of such edge triples whose first edge is e1,
 *     summed over every third vertex w; their sum over all edges is the number
 *     of temporal triangles.
 * Both are computed from the definition: pairs are looked at one by one.
 * ---------------------------------------------------------------------------
 */

/* Number of (t2, t3) in L2 x L3 with t <= t2 <= t3 and t3 - t <= delta. */
static uint64_t og_pairs(int64_t t, int64_t delta, const int64_t *L2, int64_t n2,
                         const int64_t *L3, int64_t n3) {
    uint64_t c = 0;
    for (int64_t i = 0; i < n2; i++) {
        int64_t t2 = L2[i];
        if (t2 < t) continue;
        if (t2 - t > delta) break;
        for (int64_t j = 0; j < n3; j++) {
            int64_t t3 = L3[j];
            if (t3 < t2) continue;
            if (t3 - t > delta) break;
            c++;
        }
    }
    return c;
}

/*
 * inst[] for the edges idx[0..k) (input positions), or for all m edges when idx
 * is NULL.  Self-loops get 0.  Returns 0, or -1 on bad arguments.
 */
int og_triad_instances(const og_graph *g, int64_t k, const int64_t *idx, int64_t delta,
                       int variant, uint64_t *out, int threads) {
    if (delta < 0 || variant < 0 || variant > 7) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    int64_t cnt = idx ? k : g->m;
#pragma omp parallel
    {
        int32_t *buf = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < cnt; q++) {
            int64_t i = idx ? idx[q] : q;
            int32_t a = g->src[i], b = g->dst[i];
            out[q] = 0;
            if (a == b) continue;
            int64_t need = g->adj_off[a + 1] - g->adj_off[a];
            int64_t nb = g->adj_off[b + 1] - g->adj_off[b];
            if (nb < need) need = nb;
            if (need + 1 > cap) { free(buf); cap = need + 1; buf = (int32_t *)malloc(sizeof(int32_t) * cap); }
            int64_t nc = og_common(g, a, b, buf);
            uint64_t s = 0;
            for (int64_t c = 0; c < nc; c++) {
                const int64_t *L2, *L3;
                int64_t n2, n3;
                og_pick(g, variant, a, b, buf[c], &L2, &n2, &L3, &n3);
                s += og_pairs(g->t[i], delta, L2, n2, L3, n3);
            }
            out[q] = s;
        }
        free(buf);
    }
    return 0;
}

/*
 * The third vertices w, ascending, that make (a, b, w) a solution: some e1 in
 * E_{a,b} has a temporal triangle with w.  buf holds at least
 * min(|N(a)|, |N(b)|) ids; out may be NULL.  Returns how many.
 */
static int64_t og_triad_ws(const og_graph *g, int32_t a, int32_t b, int64_t delta, int variant,
                           int32_t *buf, int32_t *out) {
    const int64_t *L1;
    int64_t n1 = og_list(g, a, b, &L1, NULL);
    if (n1 == 0 || a == b) return 0;
    int64_t nc = og_common(g, a, b, buf); /* ascending: og_common walks a sorted row */
    int64_t c = 0;
    for (int64_t j = 0; j < nc; j++) {
        const int64_t *L2, *L3;
        int64_t n2, n3;
        og_pick(g, variant, a, b, buf[j], &L2, &n2, &L3, &n3);
        for (int64_t i = 0; i < n1; i++) {
            if (og_exists(L1[i], delta, L2, n2, L3, n3)) {
                if (out) out[c] = buf[j];
                c++;
                break;
            }
        }
    }
    return c;
}

/* the directed pairs (x, y) with E_{x,y} non-empty, ascending by (x, y) */
int64_t og_pair_table(const og_graph *g, int32_t *x, int32_t *y) {
    for (int64_t p = 0; p < g->np; p++) {
        if (x) x[p] = (int32_t)(g->pkey[p] / g->n);
        if (y) y[p] = (int32_t)(g->pkey[p] % g->n);
    }
    return g->np;
}

static int32_t *og_buf_for(const og_graph *g, int32_t a, int32_t b, int32_t **buf, int64_t *cap) {
    int64_t need = g->adj_off[a + 1] - g->adj_off[a];
    int64_t nb = g->adj_off[b + 1] - g->adj_off[b];
    if (nb < need) need = nb;
    if (need + 1 > *cap) { free(*buf); *cap = need + 1; *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)*cap); }
    return *buf;
}

/* cnt[p] = number of solution triples (x_p, y_p, w) of every directed pair p */
int og_triad_pair_counts(const og_graph *g, int64_t delta, int variant, int64_t *cnt, int threads) {
    if (delta < 0 || variant < 0 || variant > 7) return -1;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
    {
        int32_t *buf = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < g->np; p++) {
            int32_t a = (int32_t)(g->pkey[p] / g->n), b = (int32_t)(g->pkey[p] % g->n);
            cnt[p] = og_triad_ws(g, a, b, delta, variant, og_buf_for(g, a, b, &buf, &cap), NULL);
        }
        free(buf);
    }
    return 0;
}

/* the solution triples (a, b, w), three ids each, pair p's from out + 3 off[p] */
int og_triad_fill(const og_graph *g, int64_t delta, int variant, const int64_t *off, int32_t *out,
                  int threads) {
    if (delta < 0 || variant < 0 || variant > 7) return -1;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
    {
        int32_t *buf = NULL, *ws = NULL;
        int64_t cap = 0, wcap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < g->np; p++) {
            if (off[p + 1] == off[p]) continue;
            int32_t a = (int32_t)(g->pkey[p] / g->n), b = (int32_t)(g->pkey[p] % g->n);
            og_buf_for(g, a, b, &buf, &cap);
            if (cap > wcap) { free(ws); wcap = cap; ws = (int32_t *)malloc(sizeof(int32_t) * (size_t)wcap); }
            int64_t c = og_triad_ws(g, a, b, delta, variant, buf, ws);
            for (int64_t j = 0; j < c; j++) {
                int32_t *o = out + 3 * (off[p] + j);
                o[0] = a;
                o[1] = b;
                o[2] = ws[j];
            }
        }
        free(buf);
        free(ws);
    }
    return 0;
}

/* the solution third vertices of one directed pair (a, b); out holds min(|N(a)|, |N(b)|) */
int64_t og_triad_pair(const og_graph *g, int32_t a, int32_t b, int64_t delta, int variant,
                      int32_t *out) {
    if (delta < 0 || variant < 0 || variant > 7 || a < 0 || b < 0 || a >= g->n || b >= g->n) return -1;
    int32_t *buf = NULL;
    int64_t cap = 0;
    int64_t c = og_triad_ws(g, a, b, delta, variant, og_buf_for(g, a, b, &buf, &cap), out);
    free(buf);
    return c;
}
