/*
 * folty.h - C ABI of the MI355X (gfx950) library for thresholded
 * exists-exists-forall triadic queries on temporal multigraphs.
 *
 * The query (paper: Definition of a thresholded FOL triadic query; Section
 * "Main Ideas"; Algorithm ExistExistForAll):
 *
 *   A temporal edge e = (a, b, t) forms a delta-temporal triangle with a third
 *   vertex w when temporal edges e2 and e3 exist, on the lists the predicate
 *   picks, with t <= t(e2) <= t(e3) <= t + delta.  For the paper's predicate
 *   e2 runs a -> w and e3 runs b -> w.  count[e] is the number of distinct such
 *   w.  e is a certificate when count[e] >= theta * |U(e)|, where the universe
 *   U(e) is N(b) by default (N(x) = neighbours of x in the static graph that
 *   drops directions, parallel edges and self-loops).  A solution is a pair
 *   (a, b) with at least one certificate on it.
 *
 * The same index also answers the other query shapes of the paper's Definition
 * of a solution: exists u forall v forall w and exists u forall v exists w
 * (folty_run_vertex_query, one solution vertex u at a time), and exists u exists
 * v exists w (folty_run_triad_query: solution triples and temporal triangle
 * counts).
 *
 * Conventions for every call:
 *   - Every call returns FOLTY_OK (0) or a negative FOLTY_E* code; on error
 *     folty_last_error() returns a message for the calling thread.
 *   - Pointers marked "host" are CPU memory; "device" are HIP device memory of
 *     the current device.  Input arrays are only read during the call and are
 *     copied; the library never keeps a caller pointer.
 *   - Handles belong to the caller until the matching *_free call.  Result
 *     arrays returned by accessors stay valid until folty_result_free.
 *   - A built graph is read-only: several threads may query one graph at the
 *     same time, each with its own folty_workspace (see folty_run_fol_query_ws).
 *   - All work runs on the HIP stream given at load time (NULL = the library
 *     creates one stream per graph).
 *   - The library needs a HIP device; without one every call that touches the
 *     GPU fails with FOLTY_EDEVICE.  There is no CPU fallback.
 */
#ifndef FOLTY_H
#define FOLTY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FOLTY_OK = 0,
    FOLTY_EINVAL = -1,    /* bad argument: id out of range, t out of [0, 2^62), delta < 0,
                             theta not in [0, 1], den = 0, unknown variant or universe */
    FOLTY_ENOTBUILT = -2, /* query on a graph whose index was not built */
    FOLTY_ENOMEM = -3,    /* device allocation failed or an admission budget was exceeded */
    FOLTY_EDEVICE = -4,   /* a HIP call failed (no device, launch failure, ...) */
    FOLTY_EOVERFLOW = -5, /* m >= 2^31 or a count that does not fit the index types */
    FOLTY_EBUSY = -6      /* server: result not ready yet */
};

/* Where the arrays handed to folty_load_temporal_graph live.  HOST and DEVICE
 * arrays are copied; DEVICE_BORROWED arrays are read where they are, and the
 * caller keeps them allocated and unchanged until folty_graph_free. */
enum { FOLTY_MEM_HOST = 0, FOLTY_MEM_DEVICE = 1, FOLTY_MEM_DEVICE_BORROWED = 2 };

/* delta meaning "no window" */
#define FOLTY_DELTA_INF INT64_MAX

/* Universe of the thresholded universal quantifier */
enum {
    FOLTY_UNIVERSE_DST = 0,    /* N(b): Algorithm ExistExistForAll, the paper's default */
    FOLTY_UNIVERSE_SRC = 1,    /* N(a) */
    FOLTY_UNIVERSE_COMMON = 2  /* N(a) intersect N(b): Section "Insights" */
};

/* Ordering used to orient the static graph (result-neutral; only speed changes) */
enum {
    FOLTY_RANK_DEGENERACY = 0, /* min-degree peeling (core, peel round, id): out-degree <= degeneracy */
    FOLTY_RANK_DEGREE = 1,     /* (degree, id) */
    FOLTY_RANK_RANDOM = 2      /* hash of (id, seed); for orientation-independence tests */
};

typedef struct folty_graph folty_graph;
typedef struct folty_result folty_result;
typedef struct folty_workspace folty_workspace;

/* A caller-supplied device allocator (PyTorch's, say).  alloc returns `bytes` of
 * device memory to be used on `stream` (NULL when it cannot: FOLTY_ENOMEM); free
 * hands such memory back, after which only later work on that stream may use it
 * again.  ctx is passed through. */
typedef void *(*folty_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*folty_free_fn)(void *p, size_t bytes, void *stream, void *ctx);

typedef struct {
    int32_t rank_mode;       /* FOLTY_RANK_*; default FOLTY_RANK_DEGENERACY */
    int32_t cache_triangles; /* 1: keep the static triangle list in the index, so queries
                                skip wedge enumeration; 0 (default): enumerate per query */
    uint64_t rank_seed;      /* seed for FOLTY_RANK_RANDOM */
    /* Device memory of the index (every array it keeps, the build's temporaries and
     * index parts made later on first use) comes from alloc/free, on the graph's
     * stream, when both are set; NULL: the library's caching allocator.  They are
     * called on the threads that call into the library for this graph, and must
     * stay valid until folty_graph_free. */
    folty_alloc_fn alloc;
    folty_free_fn free;
    void *alloc_ctx;
} folty_build_opts;

/*
 * One query.  theta = theta_num / theta_den, compared exactly in integers:
 * count[e] * theta_den >= theta_num * |U(e)|.
 *
 * variant: 3-bit predicate code.  With X, Y the endpoints edge 2 and edge 3
 * hang off (X = a, Y = b when bit 2 is clear; X = b, Y = a when set):
 *   bit 0 clear: e2 runs X -> w; set: w -> X.
 *   bit 1 clear: e3 runs Y -> w; set: w -> Y.
 * 0 is the paper's temporal triangle (a->w, b->w); 3 has both closing edges
 * leave w (w->a, w->b); 6 is the cyclic triangle a->b, b->w, w->a.
 */
typedef struct {
    int64_t delta;          /* >= 0, seconds (same unit as t); FOLTY_DELTA_INF = no window */
    uint32_t theta_num;     /* theta_num <= theta_den */
    uint32_t theta_den;     /* > 0 */
    uint8_t variant;        /* 0..7 */
    uint8_t universe;       /* FOLTY_UNIVERSE_* */
    uint8_t exclude_other;  /* 1: |U| - 1 (drop the other endpoint); universes DST/SRC only */
    uint8_t flags;          /* FOLTY_QUERY_* bits; other bits must be 0 */
} folty_query;

/* Query flag: do not keep per-edge counts in the result (folty_result_counts then
 * gives |Sol| only).  Saves 4 bytes per input edge of device memory and a pass. */
#define FOLTY_QUERY_NO_COUNTS 1u

/* Query flag: evaluate each run (triangle, list E_{a,b}) from the shorter of
 * E_{a,b} and the list L2 of edge 2.  From L2 the run uses the paper's in-neighbour
 * intervals (an edge e on E_{a,b} forms a triangle with w iff some entry t2 of L2,
 * whose first L3 entry t3 >= t2 lies within delta, has t3 - delta <= t(e) <= t2),
 * marking their union as edge ranges in a difference array that is prefix-summed
 * into the counts.  Results are identical; it pays on graphs whose E_{a,b} lists
 * are much longer than the lists that close them, and costs 4 bytes per edge of
 * scratch and one scan.  Batched plans and the server ignore it. */
#define FOLTY_QUERY_SMALLER_SIDE 2u

/* Query flag: filter in one enumeration pass that writes surviving triangles
 * into per-item slots sized for every static triangle (12 bytes of workspace per
 * triangle; the graph's per-item triangle offsets are made first if missing,
 * one enumeration pass, kept with the graph).  Without it a query counts
 * survivors in one pass and enumerates the items that have any a second time,
 * unless an earlier query on the graph found that second pass re-enumerating
 * half of the items or triangles (a wide window): then queries of at least an
 * eighth of that window filter in one pass by themselves.  Results are
 * identical either way.  Single and vertex queries (plans always use the
 * slots; exists-exists-exists queries follow the graph's switch). */
#define FOLTY_QUERY_ONE_PASS 4u

/* Sizes and timings of a graph's index (folty_graph_stats) or of one query
 * (folty_result_stats; then the graph fields are copied in as well). */
typedef struct {
    int64_t n;                /* vertices */
    int64_t m_input;          /* temporal edges given */
    int64_t m;                /* temporal edges kept (self-loops dropped) */
    int64_t self_loops;
    int64_t static_edges;     /* |E(G_S)| */
    int64_t directed_pairs;   /* non-empty lists E_{x,y} */
    int64_t max_core;         /* degeneracy (largest core number) */
    int64_t max_out_degree;   /* largest |N+(x)| of the orientation used */
    int64_t wedges;           /* sum over x of C(|N+(x)|, 2): oriented wedges, one closing probe each */
    int64_t triangles;        /* static triangles (counted by the first query or stats call) */
    int64_t max_multiplicity; /* sigma_max: longest list E_{x,y} */
    int64_t peel_rounds;      /* rounds of the min-degree peeling within a level: the levels peel
                                 at once, so this is the most rounds any one level needs */
    int64_t closing_probes;   /* membership probes of the enumeration: sum over oriented edges
                                 (u,v) of min(|N+(u)|, |N+(v)|) */
    int64_t enum_items;       /* work items the enumeration is split into */
    int64_t batch_size;       /* server: requests that shared this request's pass */
    /* query only */
    int64_t tests;            /* temporal tests: sum over (triangle, list E_{a,b} with both
                                 closing lists non-empty) of |E_{a,b}| */
    int64_t n_pairs;          /* solution pairs */
    int64_t n_certificates;   /* |Sol| */
    double build_ms;          /* device time of folty_build_index */
    double wedge_ms;          /* device time of the counting enumeration pass alone: wedges,
                                 closing probes and the time-range filter of each triangle */
    double temporal_ms;       /* device time of the survivor scans, the emitting pass over the
                                 items with survivors, and the temporal tests */
    double threshold_ms;      /* device time of threshold, pair reduction and compaction */
    double query_ms;          /* device time of the whole query */
    double latency_ms;        /* server: submit to result ready on the host */
    double queue_ms;          /* server: submit to start of its pass */
    int64_t filter_passes;    /* query: enumeration passes of its filter (1, or 2 when the
                                 survivors are written by a second pass; 0 without items) */
    int64_t core_sweeps;      /* h-index sweeps that settled the core numbers */
} folty_stats;

/* Message for the last failed call on this thread ("" if none).  Valid until the
 * thread's next failing call. */
const char *folty_last_error(void);

/* Library version string. */
const char *folty_version(void);

/*
 * Load a temporal edge list (paper, Section "Main Ideas": a list of triples
 * (u, v, t), u the head, v the destination; a multigraph).
 *   n         vertices; ids must lie in [0, n); 1 <= n < 2^31.
 *   m         edges; 0 <= m < 2^31 (FOLTY_EOVERFLOW otherwise).
 *   src, dst  int32[m], t int64[m] with 0 <= t < 2^62; host or device memory as
 *             mem_kind says.  Order is free (the paper assumes time order; this
 *             library sorts).  Self-loops are accepted and ignored by the query.
 *   mem_kind  FOLTY_MEM_HOST or FOLTY_MEM_DEVICE: the arrays are copied (the
 *             caller may free them once this returns); FOLTY_MEM_DEVICE_BORROWED:
 *             device arrays read in place by this call and every build, which
 *             the caller keeps allocated and unchanged until folty_graph_free
 *             (saves a device copy of 16 bytes per edge).  Any other value:
 *             FOLTY_EINVAL.
 *   stream    hipStream_t to run on, or NULL.
 *   out       receives the graph handle.
 * Validates ids and timestamps on the device (FOLTY_EINVAL with the first bad
 * position in the message).
 */
int folty_load_temporal_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                              const int64_t *t, int32_t mem_kind, void *stream,
                              folty_graph **out);

/*
 * Build the index (paper, Section "Main Ideas" and Section 3 preamble):
 * group edges into time-sorted lists E_{x,y} and static edges, compute degrees
 * and core numbers, orient G_S by the chosen ordering, count static
 * triangles.  opts may be NULL (defaults).  Calling it again rebuilds.
 */
int folty_build_index(folty_graph *g, const folty_build_opts *opts);

/*
 * Run one query and wait for it (paper, Algorithm ExistExistForAll).  *out
 * receives a result holding the sorted solution pairs; per-edge counts are
 * fetched on demand by folty_result_counts.
 *
 * The filter of a query normally enumerates the graph's triangles twice: once to
 * count survivors, then again over the work items that have any.  After a query
 * (of any kind) whose second enumeration covered at least half of the items or
 * half of the triangles, the library keeps the per-item triangle offsets (from
 * the counts of its first pass), when 12 bytes per triangle fit in a quarter of
 * the free device memory.  Later queries on the graph whose delta is at least an
 * eighth of that query's then filter in one pass, with 12 bytes per triangle of
 * survivor slots in their workspace (FOLTY_QUERY_ONE_PASS asks for that on any
 * query).  The choice depends only on the graph and the queries run before.
 *
 * The temporal tests of surviving triangles with up to 64 tests run 64
 * triangles to a wavefront, one test per lane; a triangle with more is listed
 * and its tests run in pieces of 4, one piece per thread.  The list holds at
 * most 2^22 triangles (16 bytes each; the environment variable FOLTY_MAX_HEAVY
 * lowers the limit); triangles beyond it run where they were found, with the
 * same results.
 */
int folty_run_fol_query(folty_graph *g, const folty_query *q, folty_result **out);

/*
 * Vertex queries (paper, Section on the exists-forall-forall and
 * exists-forall-exists queries; a solution is a single vertex, Definition of a
 * solution):
 *   inner = FOLTY_INNER_FORALL:  exists u  forall_theta v in N(u)  forall_theta2 w  phi(u, v, w)
 *   inner = FOLTY_INNER_EXISTS:  exists u  forall_theta v in N(u)  exists w  phi(u, v, w)
 * A vertex u with at least one neighbour is a solution when at least
 * theta * |N(u)| of its neighbours v (compared exactly: good * theta_den >=
 * theta_num * |N(u)|) have a temporal edge e = (u, v, t), from u to v, that
 * solves the inner query on the edges: a certificate of the exists-exists-forall
 * query `edge` (its theta = theta2, universe and exclude_other), or, for the
 * inner exists, an edge with count[e] >= 1.  edge.delta and edge.variant give
 * the window and the predicate; with FOLTY_INNER_EXISTS edge.theta_* are not
 * read.  Vertices without neighbours are never solutions (the section's last
 * step runs over N(u)).
 * The result holds the solution vertices (folty_result_vertices), the directed
 * pairs (u, v) with a qualifying edge from u to v and the number of such edges
 * on each (folty_result_pairs), their total (folty_result_counts) and, unless
 * edge.flags has FOLTY_QUERY_NO_COUNTS, the per-edge counts.
 */
enum { FOLTY_INNER_FORALL = 0, FOLTY_INNER_EXISTS = 1 };

typedef struct {
    folty_query edge;      /* the query on the edges (see above) */
    uint32_t theta_num;    /* outer threshold over N(u): theta_num <= theta_den */
    uint32_t theta_den;    /* > 0 */
    uint8_t inner;         /* FOLTY_INNER_* */
    uint8_t reserved[7];   /* must be 0 */
} folty_vertex_query;

int folty_run_vertex_query(folty_graph *g, const folty_vertex_query *q, folty_result **out);

/*
 * Exists-exists-exists query (paper, Definition of a solution: with three
 * existential quantifiers a solution is a vertex triple; Section 1: for this
 * prefix the problem is temporal triangle counting).
 *
 * For the predicate code `variant` (the lists L2, L3 as for folty_query), the
 * ordered triple (a, b, w) is a solution when some temporal edges e1 on a -> b,
 * e2 in L2 and e3 in L3 satisfy t(e1) <= t(e2) <= t(e3) <= t(e1) + delta.  A
 * temporal triangle is one such edge triple (e1, e2, e3); the number of them is
 * the temporal triangle count for the code.
 *
 * flags (other bits must be 0):
 *   FOLTY_TRIAD_TRIPLES         list the solution triples (a, b, w), sorted;
 *                               otherwise only their number is kept;
 *   FOLTY_TRIAD_INSTANCES       count the temporal triangles as well (each test
 *                               then counts every (e2, e3), not just the first);
 *   FOLTY_TRIAD_EDGE_INSTANCES  also keep the count per first edge e1 (implies
 *                               FOLTY_TRIAD_INSTANCES; 8 bytes per input edge).
 * FOLTY_EOVERFLOW when the temporal triangles number 2^63 or more, or when more
 * than 2^31 - 1 solution triples are to be listed (their number is still
 * reported by a run without FOLTY_TRIAD_TRIPLES).
 */
#define FOLTY_TRIAD_TRIPLES 1u
#define FOLTY_TRIAD_INSTANCES 2u
#define FOLTY_TRIAD_EDGE_INSTANCES 4u

typedef struct {
    int64_t delta;         /* >= 0, same unit as t; FOLTY_DELTA_INF = no window */
    uint8_t variant;       /* predicate code 0..7 */
    uint8_t flags;         /* FOLTY_TRIAD_* bits */
    uint8_t reserved[6];   /* must be 0 */
} folty_triad_query;

int folty_run_triad_query(folty_graph *g, const folty_triad_query *q, folty_result **out);

/* The same with caller-owned scratch memory (see folty_workspace_create), for
 * exists-exists-exists queries on one graph from several threads at once. */
int folty_run_triad_query_ws(folty_graph *g, const folty_triad_query *q, folty_workspace *ws,
                             folty_result **out);

/*
 * Exists-exists-exists result: the number of solution triples, the number of
 * temporal triangles (-1 unless FOLTY_TRIAD_INSTANCES was asked) and, with
 * FOLTY_TRIAD_TRIPLES, the triples as 3 x n_solutions ids (a, b, w), ascending
 * by (a, b, w) (else NULL).  Host pointers, valid until folty_result_free.
 * FOLTY_EINVAL for a result of another query kind.
 */
int folty_result_triads(const folty_result *r, int64_t *n_solutions, int64_t *n_instances,
                        const int32_t **triples);

/*
 * Temporal triangles per first edge e1, in input order (m_input entries; 0 for
 * a self-loop), from a run with FOLTY_TRIAD_EDGE_INSTANCES (FOLTY_EINVAL
 * otherwise).  Host pointer, valid until folty_result_free.
 */
int folty_result_edge_instances(const folty_result *r, const uint64_t **instances);

/* The same with caller-owned scratch memory, for concurrent queries on one
 * graph from several threads (one workspace per thread). */
int folty_workspace_create(folty_workspace **out);
void folty_workspace_free(folty_workspace *ws);
int folty_run_fol_query_ws(folty_graph *g, const folty_query *q, folty_workspace *ws,
                           folty_result **out);

/*
 * Several queries on one graph in one pass (paper, proof of Theorem 3.1: the
 * greedy pair (first t2 >= t, then first t3 >= t2) gives the smallest window
 * t3 - t, so each (e, w) is resolved once for every delta).  Queries may mix
 * delta, theta, universe and variant.  outs[i] receives the result of qs[i].
 */
int folty_run_batch(folty_graph *g, const folty_query *qs, int32_t nq, folty_result **outs);

/*
 * One query on each of several graphs in one launch sequence (graphs of
 * uneven size share one load-balanced pass).  outs[i] is the result of qs[i]
 * on gs[i].  All graphs must be built and loaded on the same device.
 */
int folty_run_multi(folty_graph *const *gs, const folty_query *qs, int32_t ng,
                    folty_result **outs);

/*
 * Batched plans: a fixed set of queries over a fixed set of resident graphs,
 * prepared once and run many times.  query_graph[i] is the graph (index into
 * graphs) that qs[i] runs on.  A run executes one launch sequence for all
 * queries (queries sharing a graph and a predicate code share one pass; see
 * folty_run_batch); its launches are captured in a HIP graph on the first run
 * and replayed afterwards.  The graphs must stay alive and unchanged while the
 * plan exists.  One thread at a time may run a given plan.
 */
typedef struct folty_plan folty_plan;
typedef struct {
    int32_t n_jobs;          /* (graph, predicate code) passes */
    int32_t n_queries;
    int64_t items;           /* enumeration items over all jobs */
    int64_t tests;           /* temporal tests that survived the time-range filter */
    int32_t tests_per_chunk; /* temporal launch shape chosen by timing candidates */
    int32_t temporal_blocks;
    int32_t captured;        /* 1 if runs replay a captured HIP graph */
    int32_t records;         /* certificate records of the last run (one per run of a directed
                                pair within a wavefront, before merging) */
    double last_run_ms;      /* device time of the last run (launch sequence to sorted pairs) */
    int32_t tune_source;     /* 0: default launch shape (little work), 1: timed on this plan's
                                first run, 2: taken from the tuning table */
    int32_t reserved;
} folty_plan_info;

/* The launch shapes timed by plans are kept per workload bucket (log2 of the
 * test and edge counts) for the life of the process and, when the environment
 * variable FOLTY_TUNE_CACHE names a file, in that file as JSON, read on first
 * use and rewritten when an entry is added. */
int folty_plan_create(folty_graph *const *graphs, int32_t n_graphs, const folty_query *qs,
                      const int32_t *query_graph, int32_t nq, folty_plan **out);
int folty_plan_run(folty_plan *p, folty_result **outs);
int folty_plan_get_info(const folty_plan *p, folty_plan_info *info);
void folty_plan_free(folty_plan *p);

/*
 * Query server (continuous batching).  Worker threads, each with its own HIP
 * stream, take the oldest waiting request together with the other waiting
 * requests on the same graph (up to max_batch) and run them as one pass, so
 * requests that arrive while others run join the next pass.  A request is
 * started only when its device memory (estimated from its graph's index sizes)
 * fits in the budget beside the requests in flight and the workspace buffers
 * the workers keep (a worker gives its buffers back when the oldest request
 * does not fit; the library's cache of freed blocks is handed back to the
 * driver when it would push the device past the budget); requests whose
 * estimate exceeds the whole budget are rejected at submit with FOLTY_ENOMEM.
 *   workers           concurrent passes (streams); 0 = 4
 *   max_batch         requests per pass; 0 = 16
 *   hbm_budget_bytes  0 = the FOLTY_HBM_BUDGET environment variable (bytes) if
 *                     set, else 80% of the free device memory at creation
 * Graphs must outlive the requests that name them.  Results are taken with
 * folty_server_poll (FOLTY_EBUSY while not ready) or folty_server_wait; each
 * ticket can be taken once.  folty_server_destroy finishes the queued requests
 * first.  All calls are thread-safe.
 */
typedef struct folty_server folty_server;
typedef struct {
    int32_t workers;
    int32_t max_batch;
    int64_t hbm_budget_bytes;
} folty_server_opts;
typedef struct {
    int64_t submitted, completed, rejected, queued;
    int64_t batches;          /* passes that served more than one request */
    int64_t batched_requests; /* requests served in such passes */
    int64_t budget_bytes;
    int64_t in_use_bytes;     /* counted against the budget: estimates of the requests in
                                 flight plus the workspace buffers workers keep */
    int64_t peak_in_use_bytes;
    int64_t kept_bytes;       /* of in_use_bytes: workspace buffers kept between passes */
    int64_t peak_concurrent_passes; /* most passes running on the device at once */
    int64_t trimmed_bytes;    /* cached device blocks handed back to stay within the budget */
} folty_server_info;

int folty_server_create(const folty_server_opts *opts, folty_server **out);
int folty_server_submit(folty_server *s, folty_graph *g, const folty_query *q, int64_t *ticket);
int folty_server_poll(folty_server *s, int64_t ticket, folty_result **out);
int folty_server_wait(folty_server *s, int64_t ticket, folty_result **out);
int folty_server_get_info(folty_server *s, folty_server_info *info);
void folty_server_destroy(folty_server *s);

/*
 * Solution pairs of a result, sorted by (u, v), with the number of
 * certificates on each pair.  Host pointers, valid until folty_result_free.
 */
int folty_result_pairs(const folty_result *r, int64_t *n_pairs, const int32_t **u,
                       const int32_t **v, const uint32_t **n_cert);

/*
 * |Sol| and, if edge_count is not NULL, the per-temporal-edge counts in input
 * order (host, m_input entries; 0xFFFFFFFF marks a dropped self-loop).  The
 * counts are copied from the device on the first call.
 */
int folty_result_counts(folty_result *r, int64_t *n_certificates, const uint32_t **edge_count);

/*
 * The query of folty_run_fol_query for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  It calls no hipMalloc or hipFree and no allocating library
 * routine.  Its scratch (per-edge counts, survivors, per-pair certificate counts,
 * pair keys, sort and scan scratch) is a fixed device array of
 * FOLTY_NOALLOC_SCRATCH_BYTES that every device the library runs on holds until
 * the process ends; a query needing more fails with FOLTY_ENOMEM and a message
 * giving the size.  That is enough for graphs of about a million temporal edges.
 *   g, q            as for folty_run_fol_query; FOLTY_QUERY_NO_COUNTS is ignored
 *                   (edge_count decides), and the universe N(a) & N(b) needs the
 *                   graph's per-edge triangle counts to exist already (built by a
 *                   folty_run_fol_query with that universe), else FOLTY_EINVAL;
 *                   so does FOLTY_QUERY_ONE_PASS the per-item triangle offsets.
 *   pair_u, pair_v, n_cert  device arrays of pair_cap entries (caller-owned):
 *                   the solution pairs sorted by (u, v) and their certificate
 *                   counts.  More than pair_cap pairs: FOLTY_EOVERFLOW, with
 *                   *n_pairs set (then the arrays are not written).
 *   edge_count      device uint32[m_input] (caller-owned) for the per-edge counts in
 *                   input order (0xFFFFFFFF: self-loop), or NULL.
 *   n_pairs, n_certificates  host outputs: pairs and |Sol|.
 * Runs on the graph's stream and returns when the outputs are written.  All
 * calls on one device share its scratch, so the library runs them one at a
 * time (the first call on a device also sets the scratch up).
 */
#define FOLTY_NOALLOC_SCRATCH_BYTES (64u << 20)
int folty_run_fol_query_noalloc(folty_graph *g, const folty_query *q, int32_t *pair_u, int32_t *pair_v,
                                uint32_t *n_cert, int64_t pair_cap, uint32_t *edge_count, int64_t *n_pairs,
                                int64_t *n_certificates);

/*
 * Solution vertices of a vertex query in ascending id order, and for each the
 * number of its neighbours v with a qualifying edge from it to v.  Host
 * pointers, valid until folty_result_free; *n_vertices = 0 for a pair query.
 */
int folty_result_vertices(const folty_result *r, int64_t *n_vertices, const int32_t **vertices,
                          const uint32_t **good);

int folty_result_stats(const folty_result *r, folty_stats *s);
void folty_result_free(folty_result *r);

/* Index sizes and build timing.  The build does not count triangles (a query
 * does, in its own filter pass); if no query has run yet this call counts them
 * with one enumeration pass on the graph's stream, once. */
int folty_graph_stats(const folty_graph *g, folty_stats *s);

/*
 * Copies of index arrays, indexed by original vertex id (host int32[n]):
 *   what = 0: |N(x)|; 1: core number; 2: rank of x in the orientation order;
 *          3: |N+(x)| under that orientation.
 */
int folty_graph_vertex_array(const folty_graph *g, int32_t what, int32_t *out);

/* Device memory held by the index, in bytes. */
int folty_graph_device_bytes(const folty_graph *g, int64_t *bytes);

void folty_graph_free(folty_graph *g);

/* The library keeps freed device blocks for reuse (allocation and release are
 * slow and a release waits for the whole device), and the pinned host blocks of
 * freed results' large arrays (up to 4 GiB).  This hands every cached device
 * block of the current device, and every cached pinned block, back to the
 * driver; *bytes (if not NULL) receives the amount.  Call it when other code
 * needs the memory. */
int folty_release_cached_memory(int64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* FOLTY_H */
