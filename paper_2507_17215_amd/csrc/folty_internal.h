// Internal declarations of the gfx950 library behind include/folty.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <atomic>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "folty.h"

namespace folty {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

[[noreturn]] void fail(int code, const char *fmt, ...);
void set_last_error(const char *msg);

#define FOLTY_HIP(expr)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            ::folty::fail(e_ == hipErrorOutOfMemory ? FOLTY_ENOMEM : FOLTY_EDEVICE,          \
                          "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define FOLTY_LAUNCHED()                                                                     \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess)                                                                \
            ::folty::fail(FOLTY_EDEVICE, "kernel launch: %s (%s:%d)", hipGetErrorString(e_),  \
                          __FILE__, __LINE__);                                               \
    } while (0)

// ---------------------------------------------------------------------------
// device memory: a caching allocator (alloc.hip) and a growable buffer on it
// ---------------------------------------------------------------------------
// The stream that buffers allocated or freed on this thread are used with.
struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s);
    ~StreamScope();
};
void *dev_alloc(size_t bytes, size_t *got);
void dev_free(void *p, size_t bytes);
size_t dev_trim();   // give every cached block back to the driver; returns bytes
size_t dev_trim_to(size_t keep); // give back cached blocks, largest first, until at most keep bytes stay
size_t dev_cached(); // bytes held in the cache
void dev_forget_stream(hipStream_t s); // call before destroying a stream blocks were freed on
// pinned host blocks for large result arrays (alloc.hip); host_alloc returns
// nullptr when pinned memory is not available, host_free false for a pointer
// it did not hand out
void *host_alloc(size_t bytes);
bool host_free(void *p);
size_t host_trim();  // give the cached pinned blocks back; returns bytes

// A caller's allocator (folty_build_opts) and the scope in which the device
// buffers a thread asks for come from it; a buffer remembers where its memory
// came from and hands it back there.
struct AllocHook {
    folty_alloc_fn alloc = nullptr;
    folty_free_fn free = nullptr;
    void *ctx = nullptr;
    hipStream_t stream = nullptr;
    bool set() const { return alloc && free; }
};
struct HookScope {
    const AllocHook *prev;
    explicit HookScope(const AllocHook *h);
    ~HookScope();
};
const AllocHook *current_hook();

// While an ArenaScope is alive, the device buffers its thread asks for are
// carved one after another from [base, base + cap) instead of the allocator
// (FOLTY_ENOMEM, naming the size, when the next one does not fit) and handing
// them back does nothing.  Nothing else allocates device memory on that thread
// meanwhile.
struct ArenaScope {
    char *base;
    size_t cap, off = 0;
    ArenaScope *prev;
    ArenaScope(void *b, size_t c);
    ~ArenaScope();
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    AllocHook hook; // the caller's allocator p came from (unset: the library's)
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), hook(o.hook) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; hook = o.hook; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (hook.set()) hook.free(p, bytes, hook.stream, hook.ctx);
            else dev_free(p, bytes);
        }
        p = nullptr;
        bytes = 0;
        hook = AllocHook{};
    }
    // grow to at least b bytes; contents are not kept
    void ensure(size_t b) {
        if (b <= bytes && p) return;
        release();
        const AllocHook *h = current_hook();
        if (h) {
            const size_t want = ((b ? b : 256) + 255) & ~size_t(255);
            p = h->alloc(want, h->stream, h->ctx);
            if (!p) fail(FOLTY_ENOMEM, "the caller's allocator returned no memory for %zu bytes", want);
            bytes = want;
            hook = *h;
        } else {
            p = dev_alloc(b ? b : 256, &bytes);
        }
    }
    // drop the pointer without handing the memory back (memory an ArenaScope lent)
    void forget() {
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// pinned host scratch for small read-backs
struct PinnedBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool own = true; // false: p is host memory lent by the owner of this buffer, never freed here
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    ~PinnedBuf() { if (p && own) (void)hipHostFree(p); }
    void lend(void *q, size_t b) {
        if (p && own) (void)hipHostFree(p);
        p = q;
        bytes = b;
        own = false;
    }
    void ensure(size_t b) {
        if (b <= bytes && p) return;
        if (!own) fail(FOLTY_EINVAL, "a lent host buffer of %zu bytes cannot grow to %zu", bytes, b);
        if (p) (void)hipHostFree(p);
        p = nullptr;
        FOLTY_HIP(hipHostMalloc(&p, b ? b : 64, hipHostMallocDefault));
        bytes = b ? b : 64;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// the index of one temporal graph (all device arrays)
//
// Temporal edges without self-loops are sorted by (lo, hi, dir, t, input
// position) where lo < hi are the endpoints and dir = 1 for hi -> lo.  Static
// edge s owns the sorted range [soff[s], soff[s+1]); its lo -> hi list is
// [soff[s], smid[s]) and its hi -> lo list [smid[s], soff[s+1]).
//
// Vertices are renumbered by the orientation order ("new ids").  The oriented
// CSR holds, for each new id x, the heads y > x of its out-edges in ascending
// order; oeid packs the static edge id with bit 31 set when the tail of the
// oriented edge is the static edge's lo endpoint.  rec[p] describes oriented
// edge p: both of its directed lists with their first and last timestamps.
// Triangle enumeration: every triangle u < v < x (orientation order) is found
// from its lowest edge (u, v) by probing the members x of one endpoint's out-row
// for membership in the other's.  The edge is owned by the endpoint with the
// longer out-row, which is staged in LDS; the shorter row is scanned ("probe
// segment"):
//   mode A, |N+(v)| <= |N+(u)|: owner u, segment = row of v (x in N+(v)),
//   mode B, |N+(u)| <  |N+(v)|: owner v, segment = row of u (x in N+(u)).
// seg[j] = (row start, row length, oriented edge (u, v) | mode B << 31, owner),
// grouped by owner and mode.  Items are runs of at most ITEM_SEGS segments and
// about CHUNK probes of one owner; the triangles found by item it occupy slots
// [tri_base[it], tri_base[it+1]).
// ---------------------------------------------------------------------------
struct alignas(32) EnumItem {
    int32_t g0, ng; // segments [g0, g0 + ng) of the owner
    int32_t nq;     // probes: the total length of those segments' rows
    int32_t b, d;   // the owner's out-row: start and length
    int32_t pad[3];
};

// Histogram layout over sorted window levels (nls = levels rounded up to 4):
// tiles of 64 consecutive edges, each tile nls / 4 blocks of 64 x 4 counters
// (edge-minor within a block, four levels per edge), so a wavefront reading
// four levels of its 64 edges reads 1 KB contiguous.
__host__ __device__ inline int64_t hist_at(int64_t e, int32_t l, int32_t nls) {
    return ((((e >> 6) * (nls >> 2) + (l >> 2)) << 6) + (e & 63)) * 4 + (l & 3);
}
// counters of a histogram over m edges (whole tiles)
__host__ __device__ inline int64_t hist_words(int64_t m, int32_t nls) { return ((m + 63) & ~(int64_t)63) * nls; }

struct alignas(32) EdgeRec {
    int32_t fn, bn;   // lengths of E_{tail,head} and E_{head,tail}
    int32_t fs, bs;   // their starts in ts
    uint32_t flo, fhi; // first and last timestamp of E_{tail,head} >> tshift (0 if empty)
    uint32_t blo, bhi; // the same for E_{head,tail}
};
static_assert(sizeof(EdgeRec) == 32, "two records per cache line");

struct Index {
    int32_t n = 0;
    int64_t m_input = 0;
    int32_t m = 0;           // kept temporal edges
    int64_t self_loops = 0;
    int32_t S = 0;           // static edges
    int64_t P = 0;           // non-empty directed lists
    int64_t sigma_max = 0;
    std::atomic<int64_t> T{-1}; // static triangles (-1 until a query or ensure_tri_base counted them)
    // tri_base holds per-item triangle offsets; stored (release) after tri_base and
    // T are final, so a reader that loads it (acquire) sees them
    std::atomic<bool> tri_base_ready{false};
    // single queries of delta >= this filter in one pass (INT64_MAX: none, until
    // a query's second filter pass re-enumerated half of the items or triangles)
    std::atomic<int64_t> one_pass_from{INT64_MAX};
    int64_t W = 0;           // oriented wedges: sum of C(|N+(x)|, 2)
    int64_t probes = 0;      // closing probes the enumeration makes: sum over (u,v) of |N+(v)|
    int32_t NI = 0;          // enumeration items
    int32_t max_core = 0;
    int32_t max_out = 0;
    int64_t peel_rounds = 0;  // rounds of the all-levels peel (the most any one level needs)
    int64_t core_sweeps = 0;  // h-index sweeps until the core numbers settled
    int32_t rank_mode = 0;
    bool built = false;
    bool tri_cached = false;
    bool tcnt_ready = false;
    double build_ms = 0;
    int32_t tshift = 0; // timestamps >> tshift fit 32 bits (0 for t < 2^32)

    DevBuf ts;       // int64[m]
    DevBuf perm;     // int32[m]  input position of each sorted edge
    DevBuf sid;      // int32[m]  static edge of each sorted edge
    DevBuf soff;     // int32[S+1]
    DevBuf smid;     // int32[S]
    DevBuf slo;      // int32[S]
    DevBuf shi;      // int32[S]
    DevBuf deg;      // int32[n]  |N(x)|, original ids
    DevBuf core;     // int32[n]  core number, original ids
    DevBuf rank;     // int32[n]  original id -> new id
    DevBuf outdeg;   // int32[n]  |N+(x)|, original ids
    DevBuf ooff;     // int32[n+1] oriented CSR rows (new ids)
    DevBuf oadj;     // int32[S]  heads (new ids)
    DevBuf oeid;     // uint32[S] static edge id | direction bit
    DevBuf rec;      // EdgeRec[S]
    DevBuf erng;     // uint2[S]  first and last timestamp >> tshift over both lists of each oriented edge
    DevBuf otail;    // int32[S]  tail of each oriented edge (new id; released after the build)
    DevBuf seg;      // int4[S]   probe segments grouped by owner (see EnumItem)
    DevBuf item;     // EnumItem[NI]
    DevBuf tri_base; // int64[NI+1]
    DevBuf tcnt;     // int32[S]  triangles on each static edge = |N(lo) & N(hi)| (computed on first use)
    DevBuf tri;      // int32[3T] cached triangle list (optional): oriented edges (u,v), (u,w), (v,w)

    size_t device_bytes() const;
};

// per-query scratch; one per concurrent caller
struct Workspace {
    DevBuf count;   // uint32[m]
    DevBuf sv;      // int32[3 x slots] surviving triangles (oriented edges), in their item's slots
    DevBuf su;      // int32[NI]   survivors per item
    DevBuf wu;      // int64[NI+1] tests per item
    DevBuf wbase;   // int64[NI+1] exclusive offsets of wu
    DevBuf sbase;   // int64[NI+1] exclusive offsets of su: the dense index of each item's first survivor
    DevBuf tri_it;  // int32[NI+1] triangles per item, from the last counting filter pass
    DevBuf pieces;  // Heavy[]     the temporal step's survivors with many tests
    DevBuf gitem;   // int32[]     per group of 64 survivors, the item of its first (sparse slots)
    const int64_t *slots = nullptr; // first slot of each item's survivors in sv: sbase (dense) or the index's tri_base
    bool emit_timed = false;        // the last filter's second pass is bracketed by ev[6], ev[7]
    bool counted_items = false;     // tri_it holds every item's triangles (a counting pass ran)
    const Index *tri_it_of = nullptr; // the index that counting pass enumerated
    int32_t emit_items = 0;         // items the last filter's second pass enumerated again
    int64_t emit_triangles = 0;     // triangles those items hold
    int32_t filter_passes = 0;      // enumeration passes of the last filter
    DevBuf ncert;   // uint32[2S]
    DevBuf pairs_k; // uint64[2S]
    DevBuf pairs_v; // uint32[2S]
    DevBuf pairs_k2;
    DevBuf pairs_v2;
    DevBuf scal;    // small device scalars
    DevBuf cub;     // library scan/sort temporaries
    DevBuf ilist;   // int32[NI] items with survivors
    DevBuf vtmp;    // vertex queries: per-vertex counts, flags, offsets, output
    DevBuf diff;    // int32[2m+1] interval marks of the smaller-side evaluation and their prefix sum
    DevBuf tflag;   // exists-exists-exists: uint32[(survivor slots + 3) / 4] solution bits
    DevBuf tinst;   // exists-exists-exists: uint64[m_input] temporal triangles per first edge, input order
    PinnedBuf host;
    hipEvent_t ev[8] = {};
    bool events = false;
    ~Workspace();
    void ensure_events();
    size_t device_bytes() const; // device memory its buffers hold
    void forget_buffers();       // forget every device buffer (memory an ArenaScope lent)
};

struct Graph {
    int device = 0;
    hipStream_t stream = nullptr;
    AllocHook hook; // the caller's allocator for the index (folty_build_opts), if any
    bool own_stream = false;
    // inputs: device copies, or the caller's device arrays (borrowed); in_* point
    // at whichever holds them
    DevBuf src, dst, t;
    const int32_t *in_src = nullptr, *in_dst = nullptr;
    const int64_t *in_t = nullptr;
    bool sorted_by_time = false;
    int64_t tmax = 0;
    Index ix;
    Workspace ws;          // default workspace for the synchronous API
    std::mutex lazy_mu;    // guards index parts computed on first use
    ~Graph();
};

// Host arrays of a result are filled by device copies: their elements are left
// uninitialised on resize instead of being zeroed first, and arrays of 1 MiB and
// more live in cached pinned blocks (host_alloc).
template <class T> struct NoInitAlloc : std::allocator<T> {
    template <class U> struct rebind { using other = NoInitAlloc<U>; };
    NoInitAlloc() = default;
    template <class U> NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    T *allocate(size_t n) {
        if (n * sizeof(T) >= (size_t(1) << 20))
            if (void *p = host_alloc(n * sizeof(T))) return static_cast<T *>(p);
        return std::allocator<T>::allocate(n);
    }
    void deallocate(T *p, size_t n) {
        if (!host_free(p)) std::allocator<T>::deallocate(p, n);
    }
    template <class U> void construct(U *p) noexcept { ::new (static_cast<void *>(p)) U; }
    template <class U, class... A> void construct(U *p, A &&...a) { ::new (static_cast<void *>(p)) U(std::forward<A>(a)...); }
};
template <class T> using HostVec = std::vector<T, NoInitAlloc<T>>;

struct Result {
    HostVec<int32_t> u, v;
    HostVec<uint32_t> n_cert;
    HostVec<int32_t> vert;  // vertex queries: solution vertices, ascending
    HostVec<uint32_t> vgood; // and their neighbours with a qualifying edge
    bool triad = false;                // an exists-exists-exists result
    int64_t n_triads = 0;              // its solution triples
    int64_t n_tinst = -1;              // its temporal triangles (-1: not counted)
    HostVec<int32_t> trip;             // 3 per listed triple (a, b, w)
    HostVec<uint64_t> tinst;           // temporal triangles per first edge, input order
    int64_t n_certificates = 0;
    folty_stats stats{};
    bool has_counts = false;
    DevBuf counts_dev;                // uint32[m_input], input order
    HostVec<uint32_t> counts_host;
    bool counts_fetched = false;
    int device = 0;
};

// ---------------------------------------------------------------------------
// entry points used by the C ABI layer
// ---------------------------------------------------------------------------
void load_graph(Graph *g, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                const int64_t *t, int32_t mem_kind, void *stream);
void build_index(Graph *g, const folty_build_opts *opts);
void check_query(const Graph *g, const folty_query &q);
Result *run_query(Graph *g, const folty_query &q, Workspace &ws);
Result *run_query_on(Graph *g, const folty_query &q, Workspace &ws, hipStream_t stream);
Result *run_vertex_query(Graph *g, const folty_vertex_query &q, Workspace &ws);
Result *run_triad_query(Graph *g, const folty_triad_query &q, Workspace &ws);
// The time-range filter of one query (query.hip): surviving triangles in their
// slots (ws.slots), tests per item and their offsets (ws.wbase).  Returns the
// number of survivor slots; *tests is the test count, or -1 when the one-pass
// filter left it on the device.  e0, e1 bracket the counting pass.  ss: a run
// has min(|L1|, |L2|) tests (the smaller-side evaluation), else |L1|.
// one_pass: write survivors into the per-item triangle slots in one pass (when
// the index has them), else count first and emit the items with survivors.
int64_t find_survivors(const Index &ix, int variant, int64_t dmax, Workspace &ws, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1, int64_t *tri, int64_t *tests, bool ss, bool one_pass);
// whether query q on g filters in one pass; with FOLTY_QUERY_ONE_PASS the
// per-item triangle offsets are made first if missing
bool use_one_pass(Graph *g, const folty_query &q);
double ev_ms(hipEvent_t a, hipEvent_t b);
// The single query with its outputs in the caller's device memory: the sorted
// pairs (at most pair_cap; FOLTY_EOVERFLOW beyond, with *n_pairs set), and
// per-edge counts in input order when edge_count is not null.  Uses ws and
// nothing else, and builds no lazy index part (FOLTY_EINVAL for a universe
// whose per-edge triangle counts do not exist yet).
void run_query_into(Graph *g, const folty_query &q, Workspace &ws, int32_t *pair_u, int32_t *pair_v,
                    uint32_t *n_cert, int64_t pair_cap, uint32_t *edge_count, int64_t *n_pairs,
                    int64_t *n_certificates);
void run_query_noalloc(Graph *g, const folty_query &q, int32_t *pair_u, int32_t *pair_v, uint32_t *n_cert,
                       int64_t pair_cap, uint32_t *edge_count, int64_t *n_pairs, int64_t *n_certificates);
void run_batch(Graph *g, const folty_query *qs, int nq, Workspace &ws, Result **outs);
void run_multi(Graph *const *gs, const folty_query *qs, int ng, Workspace &ws, Result **outs);
void fill_stats_from_index(const Index &ix, folty_stats *s);
void ensure_tcnt(Index &ix, hipStream_t s); // per-static-edge triangle counts on first use

// batched plans (batch.hip)
struct Plan;
// oneshot: the plan runs once (no capture, no timing of launch shapes)
Plan *plan_create(Graph *const *gs, int ng, const folty_query *qs, const int32_t *qgraph, int nq,
                  bool oneshot = false);
void plan_run(Plan *p, Result **outs);
int64_t plan_footprint(const Graph *g, const folty_query *qs, int nq); // device bytes of such a plan
int64_t query_footprint(const Graph *g, const folty_query &q);         // of one single query
void plan_free(Plan *p);
void plan_info(const Plan *p, folty_plan_info *info);

// query server (server.hip)
struct Server;
Server *server_create(const folty_server_opts *o);
int64_t server_submit(Server *s, Graph *g, const folty_query &q);
Result *server_take(Server *s, int64_t ticket, bool wait);
void server_info(Server *s, folty_server_info *info);
void server_destroy(Server *s);
// oriented-edge records, triangle counts per lowest vertex, optional triangle cache
void index_triangles(Index &ix, bool cache, DevBuf &cub, hipStream_t s);
void ensure_tri_base(Index &ix, hipStream_t s); // caller holds Graph::lazy_mu once the graph is shared
void ensure_triangles(Graph *g);                 // ensure_tri_base on the graph's stream, under lazy_mu
// after a two-pass filter whose second pass enumerated half of the items or of
// the triangles again (a wide window), make the per-item triangle offsets (from
// the counting pass's per-item triangles) so later wide queries filter in one pass
void maybe_one_pass(Graph *g, const Workspace &ws, int64_t delta);

// library-primitive wrappers (rocPRIM), all on `stream`
size_t sort_pairs_u64_i32(void *tmp, size_t tmp_bytes, const uint64_t *kin, uint64_t *kout,
                          const int32_t *vin, int32_t *vout, int64_t n, int end_bit,
                          hipStream_t stream);
size_t sort_pairs_u64_u32(void *tmp, size_t tmp_bytes, const uint64_t *kin, uint64_t *kout,
                          const uint32_t *vin, uint32_t *vout, int64_t n, int end_bit,
                          hipStream_t stream);
size_t sort_pairs_u32_i32(void *tmp, size_t tmp_bytes, const uint32_t *kin, uint32_t *kout,
                          const int32_t *vin, int32_t *vout, int64_t n, int end_bit,
                          hipStream_t stream);
size_t exclusive_scan_i64(void *tmp, size_t tmp_bytes, const int64_t *in, int64_t *out, int64_t n,
                          hipStream_t stream);
size_t exclusive_scan_i32_to_i64(void *tmp, size_t tmp_bytes, const int32_t *in, int64_t *out,
                                 int64_t n, hipStream_t stream);
size_t inclusive_scan_i32(void *tmp, size_t tmp_bytes, const int32_t *in, int32_t *out, int64_t n,
                          hipStream_t stream);
size_t inclusive_scan_pair_starts(void *tmp, size_t tb, const uint64_t *key, int32_t *out, int64_t n,
                                  hipStream_t s);
size_t exclusive_scan_i32(void *tmp, size_t tmp_bytes, const int32_t *in, int32_t *out, int64_t n,
                          hipStream_t stream);

// core numbers and degeneracy rank keys (core.hip)
struct CoreStats {
    int32_t sweeps = 0;   // h-index sweeps with work
    int32_t rounds = 0;   // rounds of the all-levels peel
    int32_t global_h = 0; // h-index of the degree sequence (the starting bound)
};
int core_rank_keys(int32_t n, const int64_t *uoff, const int32_t *uadj, const int32_t *deg, int32_t *core,
                   uint32_t *key, hipStream_t s, CoreStats *out);

inline int bit_length(uint64_t x) {
    int b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

// Blocks for a launch over `items`.  With cap = 0 the kernel handles one item
// per thread, so the grid must cover every item; a dispatch holds fewer than
// 2^32 work-items, and a larger range is an error rather than a silently
// truncated grid.  With cap > 0 the kernel is grid-stride and at most cap
// blocks are launched.
inline unsigned grid_for(int64_t items, int block, int64_t cap = 0) {
    int64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    if (cap > 0) {
        if (g > cap) g = cap;
    } else if (g * (int64_t)block > (int64_t)UINT32_MAX) {
        fail(FOLTY_EOVERFLOW, "a launch over %lld items exceeds one dispatch", (long long)items);
    }
    return (unsigned)g;
}

} // namespace folty
