/*
 * A plain C99 client of include/folty.h, for the tests: it checks that the
 * header compiles as C and that the library is usable without Python.
 *
 * stdin:  n m, then m lines "src dst t", then query lines:
 *           Q delta theta_num theta_den variant universe exclude_other
 *           T delta variant flags
 *           V delta theta_num theta_den inner inner_num inner_den variant
 * stdout: for Q: "COUNTS" and the m per-edge counts, "PAIRS k" and k lines
 *         "u v n_cert", "NCERT |Sol|"; for T: "TRIADS n_solutions n_instances",
 *         the listed triples one per line, and "INST" with the per-edge counts
 *         when asked for; for V: "VERTICES k" and k lines "vertex good".
 * On an error it prints "ERROR code message" to stderr and exits with 2.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "folty.h"

static int check(int rc, const char *what) {
    if (rc != FOLTY_OK) {
        fprintf(stderr, "ERROR %d %s: %s\n", rc, what, folty_last_error());
        exit(2);
    }
    return rc;
}

int main(void) {
    int32_t n;
    long long m;
    if (scanf("%d %lld", &n, &m) != 2) return 1;
    int32_t *src = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    int32_t *dst = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    int64_t *t = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    for (long long i = 0; i < m; i++) {
        long long tt;
        if (scanf("%d %d %lld", &src[i], &dst[i], &tt) != 3) return 1;
        t[i] = (int64_t)tt;
    }
    folty_graph *g = NULL;
    check(folty_load_temporal_graph(n, (int64_t)m, src, dst, t, FOLTY_MEM_HOST, NULL, &g), "load");
    check(folty_build_index(g, NULL), "build");
    char kind[4];
    while (scanf("%3s", kind) == 1) {
        folty_result *r = NULL;
        if (strcmp(kind, "Q") == 0) {
            long long delta;
            unsigned num, den, variant, universe, excl;
            if (scanf("%lld %u %u %u %u %u", &delta, &num, &den, &variant, &universe, &excl) != 6) return 1;
            folty_query q;
            memset(&q, 0, sizeof q);
            q.delta = (int64_t)delta;
            q.theta_num = num;
            q.theta_den = den;
            q.variant = (uint8_t)variant;
            q.universe = (uint8_t)universe;
            q.exclude_other = (uint8_t)excl;
            check(folty_run_fol_query(g, &q, &r), "query");
            int64_t ncert = 0, np = 0;
            const uint32_t *cnt = NULL, *nc = NULL;
            const int32_t *u = NULL, *v = NULL;
            check(folty_result_counts(r, &ncert, &cnt), "counts");
            printf("COUNTS");
            for (long long i = 0; i < m; i++) printf(" %u", cnt[i]);
            check(folty_result_pairs(r, &np, &u, &v, &nc), "pairs");
            printf("\nPAIRS %lld\n", (long long)np);
            for (int64_t i = 0; i < np; i++) printf("%d %d %u\n", u[i], v[i], nc[i]);
            printf("NCERT %lld\n", (long long)ncert);
        } else if (strcmp(kind, "T") == 0) {
            long long delta;
            unsigned variant, flags;
            if (scanf("%lld %u %u", &delta, &variant, &flags) != 3) return 1;
            folty_triad_query q;
            memset(&q, 0, sizeof q);
            q.delta = (int64_t)delta;
            q.variant = (uint8_t)variant;
            q.flags = (uint8_t)flags;
            check(folty_run_triad_query(g, &q, &r), "triad query");
            int64_t ns = 0, ni = 0;
            const int32_t *trip = NULL;
            check(folty_result_triads(r, &ns, &ni, &trip), "triads");
            printf("TRIADS %lld %lld\n", (long long)ns, (long long)ni);
            for (int64_t i = 0; trip && i < ns; i++) printf("%d %d %d\n", trip[3 * i], trip[3 * i + 1], trip[3 * i + 2]);
            if (flags & FOLTY_TRIAD_EDGE_INSTANCES) {
                const uint64_t *inst = NULL;
                check(folty_result_edge_instances(r, &inst), "edge instances");
                printf("INST");
                for (long long i = 0; i < m; i++) printf(" %llu", (unsigned long long)inst[i]);
                printf("\n");
            }
        } else if (strcmp(kind, "V") == 0) {
            long long delta;
            unsigned num, den, inner, inum, iden, variant;
            if (scanf("%lld %u %u %u %u %u %u", &delta, &num, &den, &inner, &inum, &iden, &variant) != 7) return 1;
            folty_vertex_query q;
            memset(&q, 0, sizeof q);
            q.edge.delta = (int64_t)delta;
            q.edge.theta_num = inum;
            q.edge.theta_den = iden;
            q.edge.variant = (uint8_t)variant;
            q.theta_num = num;
            q.theta_den = den;
            q.inner = (uint8_t)inner;
            check(folty_run_vertex_query(g, &q, &r), "vertex query");
            int64_t nv = 0;
            const int32_t *vs = NULL;
            const uint32_t *good = NULL;
            check(folty_result_vertices(r, &nv, &vs, &good), "vertices");
            printf("VERTICES %lld\n", (long long)nv);
            for (int64_t i = 0; i < nv; i++) printf("%d %u\n", vs[i], good[i]);
        } else {
            return 1;
        }
        folty_result_free(r);
    }
    folty_graph_free(g);
    free(src);
    free(dst);
    free(t);
    return 0;
}
