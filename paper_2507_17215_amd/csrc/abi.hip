// extern "C" entry points of include/folty.h: argument checks, error codes,
// handle lifetimes.  Every call catches internal errors and turns them into a
// return code plus a thread-local message.
#include <cstdarg>
#include <cstring>
#include <cstdlib>
#include <new>

#include "folty_internal.h"

struct folty_graph {
    folty::Graph g;
};
struct folty_result {
    folty::Result r;
};
struct folty_workspace {
    folty::Workspace ws;
};
struct folty_plan {
    folty::Plan *p;
};
struct folty_server {
    folty::Server *s;
};

namespace folty {

static thread_local std::string g_last_error;

void set_last_error(const char *msg) { g_last_error = msg ? msg : ""; }

void fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error(code, buf);
}

Graph::~Graph() {
    if (own_stream && stream) {
        // the index's buffers are freed after this body, with no stream of
        // their own; blocks freed on this stream before lose their events here
        (void)hipStreamSynchronize(stream);
        dev_forget_stream(stream);
        (void)hipStreamDestroy(stream);
    }
}

template <class F> static int guarded(F &&f) {
    try {
        f();
        return FOLTY_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return FOLTY_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return FOLTY_EDEVICE;
    }
}

} // namespace folty

using namespace folty;

extern "C" {

const char *folty_last_error(void) { return g_last_error.c_str(); }

const char *folty_version(void) { return "folty-gfx950 0.1"; }

int folty_load_temporal_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
                              int32_t mem_kind, void *stream, folty_graph **out) {
    return guarded([&] {
        if (!out) fail(FOLTY_EINVAL, "out is null");
        *out = nullptr;
        std::unique_ptr<folty_graph> h(new folty_graph());
        load_graph(&h->g, n, m, src, dst, t, mem_kind, stream);
        *out = h.release();
    });
}

int folty_build_index(folty_graph *g, const folty_build_opts *opts) {
    return guarded([&] {
        if (!g) fail(FOLTY_EINVAL, "graph is null");
        FOLTY_HIP(hipSetDevice(g->g.device));
        StreamScope sc(g->g.stream);
        build_index(&g->g, opts);
    });
}

int folty_run_fol_query(folty_graph *g, const folty_query *q, folty_result **out) {
    return guarded([&] {
        if (!g || !q || !out) fail(FOLTY_EINVAL, "null argument");
        *out = nullptr;
        StreamScope sc(g->g.stream);
        Result *r = run_query(&g->g, *q, g->g.ws);
        folty_result *h = new folty_result();
        h->r = std::move(*r);
        delete r;
        *out = h;
    });
}

int folty_run_fol_query_noalloc(folty_graph *g, const folty_query *q, int32_t *pair_u, int32_t *pair_v,
                                uint32_t *n_cert, int64_t pair_cap, uint32_t *edge_count, int64_t *n_pairs,
                                int64_t *n_certificates) {
    return guarded([&] {
        if (!g || !q || !n_pairs || !n_certificates) fail(FOLTY_EINVAL, "null argument");
        *n_pairs = 0;
        *n_certificates = 0;
        run_query_noalloc(&g->g, *q, pair_u, pair_v, n_cert, pair_cap, edge_count, n_pairs, n_certificates);
    });
}

int folty_run_vertex_query(folty_graph *g, const folty_vertex_query *q, folty_result **out) {
    return guarded([&] {
        if (!g || !q || !out) fail(FOLTY_EINVAL, "null argument");
        *out = nullptr;
        StreamScope sc(g->g.stream);
        Result *r = run_vertex_query(&g->g, *q, g->g.ws);
        folty_result *h = new folty_result();
        h->r = std::move(*r);
        delete r;
        *out = h;
    });
}

int folty_run_triad_query(folty_graph *g, const folty_triad_query *q, folty_result **out) {
    return guarded([&] {
        if (!g || !q || !out) fail(FOLTY_EINVAL, "null argument");
        *out = nullptr;
        StreamScope sc(g->g.stream);
        Result *r = run_triad_query(&g->g, *q, g->g.ws);
        folty_result *h = new folty_result();
        h->r = std::move(*r);
        delete r;
        *out = h;
    });
}

int folty_run_triad_query_ws(folty_graph *g, const folty_triad_query *q, folty_workspace *ws,
                             folty_result **out) {
    return guarded([&] {
        if (!g || !q || !ws || !out) fail(FOLTY_EINVAL, "null argument");
        *out = nullptr;
        StreamScope sc(g->g.stream);
        Result *r = run_triad_query(&g->g, *q, ws->ws);
        folty_result *h = new folty_result();
        h->r = std::move(*r);
        delete r;
        *out = h;
    });
}

int folty_result_triads(const folty_result *r, int64_t *n_solutions, int64_t *n_instances,
                        const int32_t **triples) {
    return guarded([&] {
        if (!r) fail(FOLTY_EINVAL, "result is null");
        if (!r->r.triad) fail(FOLTY_EINVAL, "not the result of an exists-exists-exists query");
        if (n_solutions) *n_solutions = r->r.n_triads;
        if (n_instances) *n_instances = r->r.n_tinst;
        if (triples) *triples = r->r.trip.empty() ? nullptr : r->r.trip.data();
    });
}

int folty_result_edge_instances(const folty_result *r, const uint64_t **instances) {
    return guarded([&] {
        if (!r || !instances) fail(FOLTY_EINVAL, "null argument");
        *instances = nullptr;
        if (!r->r.triad || r->r.tinst.size() != (size_t)r->r.stats.m_input)
            fail(FOLTY_EINVAL, "the query did not ask for FOLTY_TRIAD_EDGE_INSTANCES");
        *instances = r->r.tinst.data();
    });
}

int folty_workspace_create(folty_workspace **out) {
    return guarded([&] {
        if (!out) fail(FOLTY_EINVAL, "out is null");
        *out = new folty_workspace();
    });
}

void folty_workspace_free(folty_workspace *ws) { delete ws; }

int folty_run_fol_query_ws(folty_graph *g, const folty_query *q, folty_workspace *ws, folty_result **out) {
    return guarded([&] {
        if (!g || !q || !ws || !out) fail(FOLTY_EINVAL, "null argument");
        *out = nullptr;
        StreamScope sc(g->g.stream);
        Result *r = run_query(&g->g, *q, ws->ws);
        folty_result *h = new folty_result();
        h->r = std::move(*r);
        delete r;
        *out = h;
    });
}

int folty_run_batch(folty_graph *g, const folty_query *qs, int32_t nq, folty_result **outs) {
    return guarded([&] {
        if (!g || (nq > 0 && (!qs || !outs))) fail(FOLTY_EINVAL, "null argument");
        std::vector<Result *> rs(nq > 0 ? nq : 0, nullptr);
        StreamScope sc(g->g.stream);
        run_batch(&g->g, qs, nq, g->g.ws, rs.data());
        for (int i = 0; i < nq; i++) {
            folty_result *h = new folty_result();
            h->r = std::move(*rs[i]);
            delete rs[i];
            outs[i] = h;
        }
    });
}

int folty_run_multi(folty_graph *const *gs, const folty_query *qs, int32_t ng, folty_result **outs) {
    return guarded([&] {
        if (ng > 0 && (!gs || !qs || !outs)) fail(FOLTY_EINVAL, "null argument");
        std::vector<Graph *> g(ng > 0 ? ng : 0);
        for (int i = 0; i < ng; i++) {
            if (!gs[i]) fail(FOLTY_EINVAL, "graph %d is null", i);
            g[i] = &gs[i]->g;
        }
        std::vector<Result *> rs(ng > 0 ? ng : 0, nullptr);
        Workspace ws;
        run_multi(g.data(), qs, ng, ws, rs.data());
        for (int i = 0; i < ng; i++) {
            folty_result *h = new folty_result();
            h->r = std::move(*rs[i]);
            delete rs[i];
            outs[i] = h;
        }
    });
}

int folty_plan_create(folty_graph *const *graphs, int32_t n_graphs, const folty_query *qs,
                      const int32_t *query_graph, int32_t nq, folty_plan **out) {
    return guarded([&] {
        if (!out || !graphs || n_graphs <= 0 || nq < 0 || (nq > 0 && (!qs || !query_graph)))
            fail(FOLTY_EINVAL, "bad plan arguments");
        *out = nullptr;
        std::vector<Graph *> g(n_graphs);
        for (int i = 0; i < n_graphs; i++) {
            if (!graphs[i]) fail(FOLTY_EINVAL, "graph %d is null", i);
            g[i] = &graphs[i]->g;
        }
        std::unique_ptr<folty_plan> h(new folty_plan{nullptr});
        h->p = plan_create(g.data(), n_graphs, qs, query_graph, nq);
        *out = h.release();
    });
}

int folty_plan_run(folty_plan *p, folty_result **outs) {
    return guarded([&] {
        if (!p || !p->p || !outs) fail(FOLTY_EINVAL, "null argument");
        folty_plan_info info{};
        plan_info(p->p, &info);
        std::vector<Result *> rs(info.n_queries, nullptr);
        plan_run(p->p, rs.data());
        for (int i = 0; i < info.n_queries; i++) {
            folty_result *h = new folty_result();
            h->r = std::move(*rs[i]);
            delete rs[i];
            outs[i] = h;
        }
    });
}

int folty_plan_get_info(const folty_plan *p, folty_plan_info *info) {
    return guarded([&] {
        if (!p || !p->p || !info) fail(FOLTY_EINVAL, "null argument");
        plan_info(p->p, info);
    });
}

void folty_plan_free(folty_plan *p) {
    if (!p) return;
    if (p->p) plan_free(p->p);
    delete p;
}

int folty_server_create(const folty_server_opts *opts, folty_server **out) {
    return guarded([&] {
        if (!out) fail(FOLTY_EINVAL, "out is null");
        *out = nullptr;
        folty_server_opts o{};
        if (opts) o = *opts;
        if (o.hbm_budget_bytes <= 0) {
            const char *env = getenv("FOLTY_HBM_BUDGET");
            if (env && *env) o.hbm_budget_bytes = strtoll(env, nullptr, 10);
        }
        std::unique_ptr<folty_server> h(new folty_server{nullptr});
        h->s = server_create(&o);
        *out = h.release();
    });
}

int folty_server_submit(folty_server *s, folty_graph *g, const folty_query *q, int64_t *ticket) {
    return guarded([&] {
        if (!s || !g || !q || !ticket) fail(FOLTY_EINVAL, "null argument");
        *ticket = server_submit(s->s, &g->g, *q);
    });
}

static int server_take_abi(folty_server *s, int64_t ticket, folty_result **out, bool wait) {
    return guarded([&] {
        if (!s || !out) fail(FOLTY_EINVAL, "null argument");
        *out = nullptr;
        Result *r = server_take(s->s, ticket, wait);
        folty_result *h = new folty_result();
        h->r = std::move(*r);
        delete r;
        *out = h;
    });
}

int folty_server_poll(folty_server *s, int64_t ticket, folty_result **out) { return server_take_abi(s, ticket, out, false); }

int folty_server_wait(folty_server *s, int64_t ticket, folty_result **out) { return server_take_abi(s, ticket, out, true); }

int folty_server_get_info(folty_server *s, folty_server_info *info) {
    return guarded([&] {
        if (!s || !info) fail(FOLTY_EINVAL, "null argument");
        server_info(s->s, info);
    });
}

void folty_server_destroy(folty_server *s) {
    if (!s) return;
    if (s->s) server_destroy(s->s);
    delete s;
}

int folty_result_pairs(const folty_result *r, int64_t *n_pairs, const int32_t **u, const int32_t **v,
                       const uint32_t **n_cert) {
    return guarded([&] {
        if (!r) fail(FOLTY_EINVAL, "result is null");
        if (n_pairs) *n_pairs = (int64_t)r->r.u.size();
        if (u) *u = r->r.u.data();
        if (v) *v = r->r.v.data();
        if (n_cert) *n_cert = r->r.n_cert.data();
    });
}

int folty_result_vertices(const folty_result *r, int64_t *n_vertices, const int32_t **vertices,
                          const uint32_t **good) {
    return guarded([&] {
        if (!r) fail(FOLTY_EINVAL, "result is null");
        if (n_vertices) *n_vertices = (int64_t)r->r.vert.size();
        if (vertices) *vertices = r->r.vert.data();
        if (good) *good = r->r.vgood.data();
    });
}

int folty_result_counts(folty_result *r, int64_t *n_certificates, const uint32_t **edge_count) {
    return guarded([&] {
        if (!r) fail(FOLTY_EINVAL, "result is null");
        if (n_certificates) *n_certificates = r->r.n_certificates;
        if (!edge_count) return;
        *edge_count = nullptr;
        if (r->r.triad) fail(FOLTY_EINVAL, "an exists-exists-exists result has no per-edge certificate counts "
                                           "(folty_result_edge_instances gives its per-edge numbers)");
        if (!r->r.has_counts) fail(FOLTY_EINVAL, "query ran with FOLTY_QUERY_NO_COUNTS");
        if (!r->r.counts_fetched) {
            FOLTY_HIP(hipSetDevice(r->r.device));
            size_t n = (size_t)r->r.stats.m_input;
            r->r.counts_host.resize(n);
            if (n) FOLTY_HIP(hipMemcpy(r->r.counts_host.data(), r->r.counts_dev.p, 4 * n, hipMemcpyDeviceToHost));
            r->r.counts_fetched = true;
            r->r.counts_dev.release();
        }
        *edge_count = r->r.counts_host.data();
    });
}

int folty_result_stats(const folty_result *r, folty_stats *s) {
    return guarded([&] {
        if (!r || !s) fail(FOLTY_EINVAL, "null argument");
        *s = r->r.stats;
    });
}

void folty_result_free(folty_result *r) { delete r; }

int folty_graph_stats(const folty_graph *g, folty_stats *s) {
    return guarded([&] {
        if (!g || !s) fail(FOLTY_EINVAL, "null argument");
        *s = folty_stats{};
        if (g->g.ix.built && g->g.ix.T < 0) ensure_triangles(const_cast<Graph *>(&g->g));
        fill_stats_from_index(g->g.ix, s);
    });
}

int folty_graph_vertex_array(const folty_graph *g, int32_t what, int32_t *out) {
    return guarded([&] {
        if (!g || !out) fail(FOLTY_EINVAL, "null argument");
        const Index &ix = g->g.ix;
        if (!ix.built) fail(FOLTY_ENOTBUILT, "index not built");
        const DevBuf *b = what == 0 ? &ix.deg : what == 1 ? &ix.core : what == 2 ? &ix.rank : what == 3 ? &ix.outdeg : nullptr;
        if (!b) fail(FOLTY_EINVAL, "unknown vertex array %d", what);
        FOLTY_HIP(hipSetDevice(g->g.device));
        FOLTY_HIP(hipStreamSynchronize(g->g.stream));
        FOLTY_HIP(hipMemcpy(out, b->p, 4 * (size_t)ix.n, hipMemcpyDeviceToHost));
    });
}

int folty_graph_device_bytes(const folty_graph *g, int64_t *bytes) {
    return guarded([&] {
        if (!g || !bytes) fail(FOLTY_EINVAL, "null argument");
        *bytes = (int64_t)g->g.ix.device_bytes();
    });
}

int folty_release_cached_memory(int64_t *bytes) {
    return guarded([&] {
        size_t b = dev_trim() + host_trim();
        if (bytes) *bytes = (int64_t)b;
    });
}

void folty_graph_free(folty_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->g.device);
    if (g->g.stream) (void)hipStreamSynchronize(g->g.stream);
    delete g;
}

} // extern "C"
