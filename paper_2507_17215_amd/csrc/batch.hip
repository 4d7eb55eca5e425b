// Batched queries: many queries over many resident graphs in one fixed launch
// sequence.
//
// Queries sharing a graph and a predicate code form a job.  A job resolves each
// (temporal edge e, third vertex w) once: by the proof of Theorem 3.1 the
// greedy pair (first t2 >= t, then first t3 >= t2) gives the smallest window
// t3 - t, so the job records that window in a histogram over its sorted
// distinct deltas, and a running sum over the levels yields count[e] for every
// delta of the job.  theta and the universe only enter the threshold step.
//
// One plan runs, whatever the number of queries and graphs:
//   filter   one grid over the enumeration items of all graphs (wave per
//            item); up to two jobs of a graph share each enumeration
//   scan     one exclusive scan over all items' test counts
//   temporal one persistent grid over all surviving tests of all jobs
//   threshold one grid over the edges of all jobs: running sum over the levels
//            and every query of the job at its level, each edge read once
//   pairs    one grid over all queries' pair slots
//   sort     one radix sort of (query, u, v) keys
// The launches from filter to pairs are captured once in a hipGraph and
// replayed.  The temporal kernel's chunk size and grid are picked by timing a
// few candidates on the plan's own work and remembered per workload size.
#include <algorithm>
#include <cstring>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "tri_device.h"

namespace folty {

namespace {

struct JobDev {
    // filter and temporal tests
    const int64_t *tri_base, *ts;
    const EdgeRec *rec;
    int32_t variant;
    int64_t dq; // range slack of the job's largest delta
    const int64_t *lv;
    int32_t nl, nls, m;
    uint32_t *hist;  // hist_words(m, nls) counters, tiled (see hist_at)
    unsigned long long *tmask; // per tile of 64 edges: which edges have a non-zero counter
    int32_t *sv;
    int64_t *sw;
    int32_t *su;
    int64_t *wu; // this job's slice of the concatenated per-item test counts
    // threshold step: the graph's static edge table and degrees, and the job's
    // queries: positions [q0, q1) of the plan's query list (job order, each job's by level)
    const int32_t *sid, *smid, *slo, *shi, *deg, *tcnt;
    int32_t q0, q1;
    int32_t keep_prefix; // some query of the job hands back its per-edge counts
    int32_t reset;       // the threshold step clears the tiles it read (reused plans)
};

// a plan's queries in job order, each job's by level (one scalar load each)
struct alignas(32) QueryDev {
    int32_t level; // index of the query's delta among its job's levels
    uint32_t num, den;
    int32_t universe;
    int32_t excl;  // 1: the other endpoint is left out of the universe (never for the common one)
    int32_t q;     // the query's index in the plan
    int32_t pad[2];
};

// the largest index i in [0, n) with base[i] <= x (base ascending, base[0] <= x)
__device__ inline int32_t owner_of(const int64_t *__restrict__ base, int32_t n, int64_t x) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// up to two jobs (predicate codes) of one graph share one enumeration
struct GroupDev {
    const EnumItem *item;
    const int4 *seg;
    const int32_t *oadj, *tri;
    const int64_t *tri_base;
    const EdgeRec *rec;
    const uint2 *rng;
    int32_t nj;
    int32_t job[2];
};

// NJ jobs per group: the groups of two come first in the plan's group list,
// so each instantiation covers one contiguous range of group items
template <int NJ>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(4))) void k_multi_filter(const GroupDev *__restrict__ groups, int32_t ngr,
                                                      const int64_t *__restrict__ group_item_base, int64_t g0,
                                                      int64_t g1, const JobDev *__restrict__ jobs) {
    __shared__ EnumLds lds[WPB];
    const int w = wave_id();
    for (int64_t g = g0 + (int64_t)blockIdx.x * WPB + w; g < g1; g += (int64_t)gridDim.x * WPB) {
        const int32_t gi = owner_of(group_item_base, ngr, g);
        const GroupDev &G = groups[gi];
        const int64_t it = g - group_item_base[gi];
        using Sink = std::conditional_t<NJ == 2, PairFilterSink, FilterSink<-1, FILTER_BOTH> >;
        Sink sink;
        sink.base = global_ptr(G.tri_base);
        sink.rec = global_ptr(G.rec);
        sink.rng = global_ptr(G.rng);
        if constexpr (NJ == 2) {
            for (int jj = 0; jj < 2; jj++) {
                const JobDev &J = jobs[G.job[jj]];
                sink.f[jj] = JobFilter{J.dq, J.variant, global_ptr(J.sv), global_ptr(J.sw), global_ptr(J.su),
                                       global_ptr(J.wu)};
            }
        } else {
            const JobDev &J = jobs[G.job[0]];
            sink.dq = J.dq;
            sink.variant = J.variant;
            sink.sv = global_ptr(J.sv);
            sink.sw = global_ptr(J.sw);
            sink.su = global_ptr(J.su);
            sink.wu = global_ptr(J.wu);
        }
        const int32_t *tri = global_ptr(G.tri);
        if (tri) cached_item(sink.base, tri, it, sink);
        else {
            const int32_t *oadj = global_ptr(G.oadj);
            const int4 *seg = global_ptr(G.seg);
            const EnumItem item = global_ptr(G.item)[it];
            enum_item(item, stage_ahead(item, oadj, seg), oadj, seg, it, sink, lds[w]);
        }
    }
}

__global__ __launch_bounds__(BLK) void k_multi_temporal(const JobDev *__restrict__ jobs, int32_t nj,
                                                        const int64_t *__restrict__ job_item_base, int64_t items,
                                                        const int64_t *__restrict__ wbase, int ipt) {
    const int64_t total = wbase[items];
    const int64_t nchunks = (total + ipt - 1) / ipt;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchunks; c += stride) {
        int64_t k = c * ipt;
        const int64_t k1 = k + ipt < total ? k + ipt : total;
        while (k < k1) {
            const int64_t k_start = k;
            // the global item whose tests contain k, its job, the survivor
            int64_t a = 0, b = items;
            while (a < b) {
                int64_t mid = (a + b) >> 1;
                if (wbase[mid + 1] <= k) a = mid + 1;
                else b = mid;
            }
            const int64_t g = a;
            const int32_t j = owner_of(job_item_base, nj, g);
            const JobDev &J = jobs[j];
            const int64_t it = g - job_item_base[j];
            const int32_t *sv = global_ptr(J.sv);
            const int64_t *sw = global_ptr(J.sw);
            int64_t r = k - wbase[g];
            const int64_t s0 = global_ptr(J.tri_base)[it];
            const int32_t ns = global_ptr(J.su)[it];
            if (ns <= 0) break; // cannot happen when the offsets are consistent
            int32_t lo = 0, hi = ns - 1;
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (sw[s0 + mid] <= r) lo = mid;
                else hi = mid - 1;
            }
            r -= sw[s0 + lo];
            PoolOp op{global_ptr(J.lv), J.nl, J.nls, global_ptr(J.hist), global_ptr(J.tmask)};
            const EdgeRec *rec = global_ptr(J.rec);
            const int64_t *ts = global_ptr(J.ts);
            for (int32_t s = lo; s < ns && k < k1; s++) {
                const int64_t p = s0 + s;
                TriLists L = load_lists(rec, sv[3 * p], sv[3 * p + 1], sv[3 * p + 2]);
                chunk_runs_rt(J.variant, L, run_slack(J.dq), ts, r, k, k1, op);
                r = 0;
            }
            if (k == k_start) break; // every survivor has tests, so this never triggers
        }
    }
}

// the plan's query at position qi, or one with no level past the job's last
// (qi is the same in every lane; saying so keeps the load scalar, all eight
// words at once)
__device__ inline QueryDev next_query(const QueryDev *__restrict__ qs, int32_t qi, int32_t q1) {
    QueryDev Q{};
    if (qi < q1) Q = qs[__builtin_amdgcn_readfirstlane(qi)];
    else Q.level = INT32_MAX;
    return Q;
}

// Certificates of one query over a wavefront of edges: per run of equal
// (static edge, direction) keys, the number of certifying edges.  The tail lane
// of each run with certificates appends one record (query, a, b) -> count.
__device__ inline void wave_run_records(int64_t key, bool in, bool cert, uint64_t rec_key,
                                        uint64_t *__restrict__ rk, uint32_t *__restrict__ rv,
                                        int32_t *__restrict__ nrec, int64_t cap) {
    const int lane = lane_id();
    const int64_t prev = __shfl_up(key, 1);
    const int64_t next = __shfl_down(key, 1);
    const bool head = lane == 0 || prev != key;
    const bool tail = lane == 63 || next != key;
    const unsigned long long heads = __ballot(head && in);
    const unsigned long long flags = __ballot(cert);
    int c = 0;
    if (in && tail) {
        const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const int start = 63 - __clzll((long long)(heads & upto));
        c = __popcll(flags & upto & ~((1ull << start) - 1ull));
    }
    const int32_t slot = wave_append(nrec, c > 0);
    if (slot >= 0 && slot < cap) {
        rk[slot] = rec_key;
        rv[slot] = (uint32_t)c;
    }
}

// Threshold step of every query, one pass per job: each temporal edge is read
// once, its histogram over the job's window levels (edge-major, four levels per
// load) is summed level by level in a register (count[e] at each delta of the
// job), and at each level the job's queries of that delta test
// count * den >= num * |U|.  Certificates are counted per query and emitted as
// (query, a, b) records, one per run of a wavefront.  Every wavefront lies
// inside one job (job slices are padded to 64 edges), so the per-query loop and
// its ballots are uniform.
__global__ __launch_bounds__(BLK) void k_job_threshold(const JobDev *__restrict__ jobs, int32_t nj,
                                                       const int64_t *__restrict__ job_w_base, int64_t total_w,
                                                       const QueryDev *__restrict__ qs, int nbits,
                                                       uint64_t *__restrict__ rk, uint32_t *__restrict__ rv,
                                                       int32_t *__restrict__ nrec, int64_t cap) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x0 = (int64_t)blockIdx.x * blockDim.x + 64 * wave_id(); x0 < total_w; x0 += stride) {
        const int32_t j = owner_of(job_w_base, nj, x0);
        const JobDev &J = jobs[j];
        const int64_t e = x0 - job_w_base[j] + lane;
        const bool in = e < J.m;
        int32_t s = 0, dir = 0, du = 0, da = 0, tc = 0;
        uint64_t ab = 0;
        const int32_t *tcnt = global_ptr(J.tcnt);
        if (in) {
            const int32_t *slo = global_ptr(J.slo), *shi = global_ptr(J.shi), *deg = global_ptr(J.deg);
            s = global_ptr(J.sid)[e];
            dir = e >= global_ptr(J.smid)[s] ? 1 : 0;
            const int32_t a = dir ? shi[s] : slo[s];
            const int32_t b = dir ? slo[s] : shi[s];
            du = deg[b];
            da = deg[a];
            if (tcnt) tc = tcnt[s];
            ab = ((uint64_t)(uint32_t)a << nbits) | (uint64_t)(uint32_t)b;
        }
        const int64_t run = in ? 2 * (int64_t)s + dir : -1;
        // this wavefront's tile: block c holds levels 4c..4c+3 of its 64 edges.
        // Edges no test added to hold zeros and are not read.
        const int64_t tile = (x0 - job_w_base[j]) >> 6;
        unsigned long long *tmask = global_ptr(J.tmask);
        const unsigned long long tm = tmask[tile];
        const bool touched = (tm >> lane) & 1ull;
        uint4 *hrow = reinterpret_cast<uint4 *>(global_ptr(J.hist) + hist_at(tile << 6, 0, J.nls)) + lane;
        uint32_t acc = 0;
        int32_t qi = J.q0;
        QueryDev Q = next_query(qs, qi, J.q1);
        const uint4 zero4 = make_uint4(0, 0, 0, 0);
        uint4 next = touched ? hrow[0] : zero4;
        for (int32_t l0 = 0; l0 < J.nl; l0 += 4) {
            const uint4 cur = next;
            if (touched && l0 + 4 < J.nl) next = hrow[((l0 >> 2) + 1) * 64]; // one block ahead
            uint32_t hv[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
            for (int jj = 0; jj < 4; jj++) {
                const int32_t l = l0 + jj;
                if (l >= J.nl) break;
                acc += hv[jj];
                hv[jj] = acc;
                while (Q.level == l) {
                    // |U| >= 0: an edge's endpoints have degree >= 1
                    const uint32_t U = (uint32_t)(Q.universe == FOLTY_UNIVERSE_DST   ? du
                                                  : Q.universe == FOLTY_UNIVERSE_SRC ? da
                                                                                     : tc) -
                                       (uint32_t)Q.excl;
                    const bool cert = in && (uint64_t)acc * Q.den >= (uint64_t)Q.num * U;
                    if (__ballot(cert))
                        wave_run_records(run, in, cert, ((uint64_t)Q.q << (2 * nbits)) | ab, rk, rv, nrec, cap);
                    Q = next_query(qs, ++qi, J.q1);
                }
            }
            // per-edge counts read back: the running sums stay; otherwise the
            // tile is left cleared for the next run
            if (touched) {
                if (J.keep_prefix) hrow[(l0 >> 2) * 64] = make_uint4(hv[0], hv[1], hv[2], hv[3]);
                else if (J.reset) hrow[(l0 >> 2) * 64] = zero4;
            }
        }
        if (tm && J.reset && lane == 0) tmask[tile] = 0ull;
    }
}

// level l of a histogram holding running sums is the count of sorted edge k at
// that level's delta; out is in input order
__global__ void k_scatter_counts(const uint32_t *__restrict__ hist, int32_t l, int32_t nls,
                                 const int32_t *__restrict__ perm, int32_t m, uint32_t *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) out[perm[k]] = hist[hist_at(k, l, nls)];
}

// histogram levels per edge, padded to whole blocks of four
int32_t padded_levels(size_t nl) { return (int32_t)((nl + 3) & ~(size_t)3); }

double ev_ms2(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    FOLTY_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
}

// Temporal-kernel launch shapes chosen by timing, per workload bucket: the
// log2 of the plan's test count and of its edge count.  The table is kept in
// memory and, when FOLTY_TUNE_CACHE names a file, in that file as JSON
//   {"arch": "gfx950", "entries": [{"tests_log2": T, "edges_log2": E,
//    "tests_per_chunk": I, "blocks": B, "ms": M}, ...]}
// read on first use and rewritten (through a temporary file and a rename)
// whenever an entry is added.  Entries of another arch are ignored.
struct TuneEntry {
    int ipt, blocks;
    double ms;
};
std::mutex g_tune_mu;
std::map<std::pair<int, int>, TuneEntry> g_tune;
std::string g_tune_loaded;  // file the table was last read from
std::string g_tune_written; // file the table was last written to

std::string tune_path() {
    const char *p = getenv("FOLTY_TUNE_CACHE");
    return p ? std::string(p) : std::string();
}

// numbers after "key": in one entry's text
bool tune_field(const std::string &e, const char *key, double *out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t i = e.find(k);
    if (i == std::string::npos) return false;
    i = e.find(':', i + k.size());
    if (i == std::string::npos) return false;
    char *end = nullptr;
    *out = strtod(e.c_str() + i + 1, &end);
    return end != e.c_str() + i + 1;
}

// caller holds g_tune_mu
void tune_load() {
    const std::string path = tune_path();
    if (path.empty() || path == g_tune_loaded) return;
    g_tune_loaded = path;
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    fclose(f);
    if (text.find("\"arch\": \"gfx950\"") == std::string::npos) return;
    size_t at = text.find("\"entries\"");
    while (at != std::string::npos) {
        const size_t a = text.find('{', at), b = a == std::string::npos ? a : text.find('}', a);
        if (a == std::string::npos || b == std::string::npos) break;
        const std::string e = text.substr(a, b - a + 1);
        double t, m, i, bl, ms = 0;
        if (tune_field(e, "tests_log2", &t) && tune_field(e, "edges_log2", &m) &&
            tune_field(e, "tests_per_chunk", &i) && tune_field(e, "blocks", &bl) && i >= 1 && i <= 64 &&
            bl >= 1 && bl <= (1 << 20)) {
            tune_field(e, "ms", &ms);
            g_tune[{(int)t, (int)m}] = TuneEntry{(int)i, (int)bl, ms};
        }
        at = b + 1;
    }
}

// caller holds g_tune_mu
void tune_save() {
    const std::string path = tune_path();
    if (path.empty()) return;
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [");
    bool first = true;
    for (auto &kv : g_tune) {
        fprintf(f, "%s\n  {\"tests_log2\": %d, \"edges_log2\": %d, \"tests_per_chunk\": %d, \"blocks\": %d, "
                   "\"ms\": %.4f}", first ? "" : ",", kv.first.first, kv.first.second, kv.second.ipt,
                kv.second.blocks, kv.second.ms);
        first = false;
    }
    fprintf(f, "\n]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0) remove(tmp.c_str());
    else g_tune_written = path;
}

int log2_ceil(int64_t x) {
    int b = 0;
    while ((1ll << b) < x && b < 62) b++;
    return b;
}

} // namespace

struct Plan {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<Graph *> graphs;
    std::vector<folty_query> queries;
    std::vector<int32_t> qgraph;
    // jobs
    struct Job {
        int32_t graph;
        int variant;
        std::vector<int64_t> levels;
        bool reset = false; // its threshold step leaves the histogram cleared
    };
    std::vector<Job> jobs;
    std::vector<int32_t> qjob, qlevel;
    std::vector<int64_t> job_item_base, job_w_base, group_item_base;
    int32_t ngroups = 0, npairs = 0; // groups; the first npairs hold two jobs
    int64_t gitems = 0;
    int64_t items = 0, total_w = 0, rec_cap = 0;
    int nbits = 0;
    // device memory
    DevBuf d_jobs, d_job_item_base, d_job_w_base, d_queries, d_groups, d_group_item_base;
    std::vector<DevBuf> hist, tmask, lv, sv, sw, su;
    bool dirty = true; // some histogram may hold counts (fresh, tuned, or a run did not finish)
    DevBuf wu, wbase, nrec, keys, vals, keys2, vals2, cub;
    size_t scan_bytes = 0;
    // launch shape and capture
    int ipt = 1, tblocks = 4096;
    bool tuned = false;
    int tune_source = 0; // 0: default shape, 1: timed by this plan, 2: from the tuning table
    bool eager = false; // capture refused: launch directly
    bool oneshot = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[4] = {};
    double last_ms = 0, last_compute_ms = 0;
    int64_t last_tests = 0;
    int32_t last_records = 0;
    ~Plan();
};

Plan::~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (stream) {
        (void)hipStreamSynchronize(stream);
        StreamScope sc(stream);
        hist.clear();
        tmask.clear();
        lv.clear();
        sv.clear();
        sw.clear();
        su.clear();
        d_jobs.release();
        d_job_item_base.release();
        d_groups.release();
        d_group_item_base.release();
        d_job_w_base.release();
        d_queries.release();
        wu.release();
        wbase.release();
        nrec.release();
        keys.release();
        vals.release();
        keys2.release();
        vals2.release();
        cub.release();
        (void)hipStreamSynchronize(stream);
        dev_forget_stream(stream);
        (void)hipStreamDestroy(stream);
    }
}

// zero job j's histogram and tile masks
static void clear_hist(Plan &P, int j, hipStream_t s) {
    const Index &ix = P.graphs[P.jobs[j].graph]->ix;
    const int64_t hn = hist_words(ix.m, padded_levels(P.jobs[j].levels.size()));
    if (hn > 0) k_fill<uint32_t><<<grid_for(hn, BLK, 1 << 16), BLK, 0, s>>>(P.hist[j].as<uint32_t>(), 0u, hn);
    const int64_t nt = ((int64_t)ix.m + 63) / 64;
    if (nt > 0)
        k_fill<unsigned long long><<<grid_for(nt, BLK, 1 << 16), BLK, 0, s>>>(P.tmask[j].as<unsigned long long>(), 0ull, nt);
    FOLTY_LAUNCHED();
}

static void enqueue_compute(Plan &P, hipStream_t s) {
    const int nj = (int)P.jobs.size();
    // clear what accumulates: the histograms of jobs whose threshold step does
    // not leave them cleared, the record count, the test total
    for (int j = 0; j < nj; j++)
        if (!P.jobs[j].reset) clear_hist(P, j, s);
    k_fill<int32_t><<<1, 1, 0, s>>>(P.nrec.as<int32_t>(), 0, 1);
    k_fill<int64_t><<<1, 1, 0, s>>>(P.wu.as<int64_t>() + P.items, (int64_t)0, 1);
    FOLTY_LAUNCHED();
    // groups of two jobs, then groups of one
    const int64_t gsplit = P.group_item_base[P.npairs];
    if (gsplit > 0) {
        unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((gsplit + WPB - 1) / WPB, ENUM_BLOCKS));
        k_multi_filter<2><<<g, BLK, 0, s>>>(P.d_groups.as<GroupDev>(), P.ngroups, P.d_group_item_base.as<int64_t>(),
                                            0, gsplit, P.d_jobs.as<JobDev>());
        FOLTY_LAUNCHED();
    }
    if (P.gitems > gsplit) {
        unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((P.gitems - gsplit + WPB - 1) / WPB, ENUM_BLOCKS));
        k_multi_filter<1><<<g, BLK, 0, s>>>(P.d_groups.as<GroupDev>(), P.ngroups, P.d_group_item_base.as<int64_t>(),
                                            gsplit, P.gitems, P.d_jobs.as<JobDev>());
        FOLTY_LAUNCHED();
    }
    exclusive_scan_i64(P.cub.p, P.scan_bytes, P.wu.as<int64_t>(), P.wbase.as<int64_t>(), P.items + 1, s);
    if (P.items > 0) {
        k_multi_temporal<<<P.tblocks, BLK, 0, s>>>(P.d_jobs.as<JobDev>(), nj, P.d_job_item_base.as<int64_t>(), P.items,
                                                   P.wbase.as<int64_t>(), P.ipt);
        FOLTY_LAUNCHED();
    }
    if (P.total_w > 0) {
        k_job_threshold<<<grid_for(P.total_w, BLK, 8192), BLK, 0, s>>>(
            P.d_jobs.as<JobDev>(), nj, P.d_job_w_base.as<int64_t>(), P.total_w, P.d_queries.as<QueryDev>(),
            P.nbits, P.keys.as<uint64_t>(), P.vals.as<uint32_t>(), P.nrec.as<int32_t>(),
            P.rec_cap);
        FOLTY_LAUNCHED();
    }
}

// time a few temporal launch shapes on the plan's own work (histograms are
// cleared before each try), keep the fastest
static void tune(Plan &P) {
    const int nj = (int)P.jobs.size();
    hipStream_t s = P.stream;
    int64_t tests = 0;
    FOLTY_HIP(hipMemcpyAsync(&tests, P.wbase.as<int64_t>() + P.items, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    P.last_tests = tests;
    const std::pair<int, int> bucket{log2_ceil(tests), log2_ceil(P.total_w)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load();
        auto it = g_tune.find(bucket);
        if (it != g_tune.end()) {
            P.ipt = it->second.ipt;
            P.tblocks = it->second.blocks;
            P.tuned = true;
            P.tune_source = 2;
            if (tune_path() != g_tune_written) tune_save(); // a file named since the entry was made
            return;
        }
    }
    if (tests < (1 << 20)) { // too little work to measure; the default shape
        P.tuned = true;
        return;
    }
    const int ipts[] = {1, 2, 4, 8, 16};
    const int blocks[] = {1024, 2048, 4096, 8192};
    double best = 1e30;
    int bi = P.ipt, bb = P.tblocks;
    for (int ip : ipts)
        for (int bl : blocks) {
            for (int j = 0; j < nj; j++) clear_hist(P, j, s);
            FOLTY_HIP(hipEventRecord(P.ev[1], s));
            k_multi_temporal<<<bl, BLK, 0, s>>>(P.d_jobs.as<JobDev>(), nj, P.d_job_item_base.as<int64_t>(), P.items,
                                                P.wbase.as<int64_t>(), ip);
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipEventRecord(P.ev[2], s));
            FOLTY_HIP(hipEventSynchronize(P.ev[2]));
            double ms = ev_ms2(P.ev[1], P.ev[2]);
            if (ms < best) {
                best = ms;
                bi = ip;
                bb = bl;
            }
        }
    P.ipt = bi;
    P.tblocks = bb;
    P.tuned = true;
    P.tune_source = 1;
    P.dirty = true; // the tries left counts behind
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[bucket] = TuneEntry{bi, bb, best};
    tune_save();
}

// Device bytes plan_create and plan_run take for these queries on one graph
// (the buffers of each job, one per predicate code: window histogram, touched
// mask, survivor slots; the certificate records of every query, their sorted
// copies and the sort's scratch; per-edge counts handed back), so that a
// server can admit a batch by what its plan will hold.
int64_t plan_footprint(const Graph *g, const folty_query *qs, int nq) {
    const Index &ix = g->ix;
    std::map<int, std::vector<int64_t>> lv; // predicate code -> windows
    int64_t b = 0;
    for (int q = 0; q < nq; q++) {
        lv[qs[q].variant].push_back(qs[q].delta);
        b += 24 * (2 * (int64_t)ix.S + (int64_t)ix.m / 64 + 2); // records, sorted copies, sort scratch
        if (!(qs[q].flags & FOLTY_QUERY_NO_COUNTS)) b += 4 * ix.m_input;
    }
    const int64_t T = std::max<int64_t>(0, ix.T.load());
    for (auto &kv : lv) {
        auto &d = kv.second;
        std::sort(d.begin(), d.end());
        d.erase(std::unique(d.begin(), d.end()), d.end());
        b += 4 * hist_words(ix.m, padded_levels(d.size())) + 8 * ((int64_t)ix.m / 64 + 1) + 8 * (int64_t)d.size();
        b += 20 * T + 4 * (int64_t)ix.NI + 16 * ((int64_t)ix.NI + 1);
    }
    // library scratch: the scan over the jobs' items and the sort of up to
    // 2 S certificate records per query (sizes only)
    const int64_t items = (int64_t)lv.size() * ((int64_t)ix.NI + 1);
    const int64_t recs = std::min<int64_t>((int64_t)nq * 2 * (int64_t)ix.S, INT32_MAX); // the sort's limit
    const int kb = bit_length((uint64_t)std::max(1, nq)) + 2 * bit_length((uint64_t)ix.n);
    b += (int64_t)std::max(exclusive_scan_i64(nullptr, 0, nullptr, nullptr, items + 1, nullptr),
                           sort_pairs_u64_u32(nullptr, 0, nullptr, nullptr, nullptr, nullptr, recs, kb, nullptr));
    return b + (1 << 20);
}

Plan *plan_create(Graph *const *gs, int ng, const folty_query *qs, const int32_t *qgraph, int nq, bool oneshot) {
    if (ng <= 0 || nq < 0) fail(FOLTY_EINVAL, "a plan needs at least one graph");
    for (int i = 0; i < ng; i++)
        if (!gs[i]) fail(FOLTY_EINVAL, "graph %d is null", i);
    int dev = gs[0]->device;
    for (int i = 0; i < ng; i++)
        if (gs[i]->device != dev) fail(FOLTY_EINVAL, "all graphs of a plan must be on one device");
    for (int q = 0; q < nq; q++) {
        if (qgraph[q] < 0 || qgraph[q] >= ng) fail(FOLTY_EINVAL, "query %d names graph %d", q, qgraph[q]);
        check_query(gs[qgraph[q]], qs[q]);
    }
    FOLTY_HIP(hipSetDevice(dev));
    std::unique_ptr<Plan> P(new Plan());
    P->device = dev;
    P->oneshot = oneshot;
    FOLTY_HIP(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
    for (auto &e : P->ev) FOLTY_HIP(hipEventCreate(&e));
    hipStream_t s = P->stream;
    StreamScope sc(s);
    // the graphs' own streams may still hold work; the one-pass filter writes
    // survivors into per-item triangle slots
    for (int i = 0; i < ng; i++) {
        FOLTY_HIP(hipStreamSynchronize(gs[i]->stream));
        ensure_triangles(gs[i]);
    }
    P->graphs.assign(gs, gs + ng);
    P->queries.assign(qs, qs + nq);
    P->qgraph.assign(qgraph, qgraph + nq);
    for (int q = 0; q < nq; q++)
        if (qs[q].universe == FOLTY_UNIVERSE_COMMON) {
            std::lock_guard<std::mutex> lk(gs[qgraph[q]]->lazy_mu);
            HookScope hs(&gs[qgraph[q]]->hook);
            ensure_tcnt(gs[qgraph[q]]->ix, s);
            FOLTY_HIP(hipStreamSynchronize(s));
        }
    // jobs: (graph, predicate code) with their distinct windows
    std::map<std::pair<int, int>, int> jid;
    P->qjob.resize(nq);
    P->qlevel.resize(nq);
    for (int q = 0; q < nq; q++) {
        auto key = std::make_pair((int)qgraph[q], (int)qs[q].variant);
        auto it = jid.find(key);
        if (it == jid.end()) {
            it = jid.emplace(key, (int)P->jobs.size()).first;
            P->jobs.push_back({key.first, key.second, {}});
        }
        P->qjob[q] = it->second;
        P->jobs[it->second].levels.push_back(qs[q].delta);
    }
    for (auto &J : P->jobs) {
        std::sort(J.levels.begin(), J.levels.end());
        J.levels.erase(std::unique(J.levels.begin(), J.levels.end()), J.levels.end());
    }
    for (int q = 0; q < nq; q++) {
        const auto &lv = P->jobs[P->qjob[q]].levels;
        P->qlevel[q] = (int32_t)(std::lower_bound(lv.begin(), lv.end(), qs[q].delta) - lv.begin());
    }
    const int nj = (int)P->jobs.size();
    // per-job buffers and descriptors
    P->hist.resize(nj);
    P->tmask.resize(nj);
    P->lv.resize(nj);
    P->sv.resize(nj);
    P->sw.resize(nj);
    P->su.resize(nj);
    std::vector<JobDev> jd(nj);
    P->job_item_base.assign(nj + 1, 0);
    P->job_w_base.assign(nj + 1, 0);
    for (int j = 0; j < nj; j++) {
        P->job_item_base[j + 1] = P->job_item_base[j] + P->graphs[P->jobs[j].graph]->ix.NI;
        // each job's edges start on a wavefront boundary
        P->job_w_base[j + 1] = P->job_w_base[j] + (((int64_t)P->graphs[P->jobs[j].graph]->ix.m + 63) & ~63ll);
    }
    P->items = P->job_item_base[nj];
    P->total_w = P->job_w_base[nj];
    // the plan's queries grouped by job, each job's by level
    std::vector<int32_t> jq(nq);
    for (int q = 0; q < nq; q++) jq[q] = q;
    std::stable_sort(jq.begin(), jq.end(), [&](int32_t x, int32_t y) {
        return P->qjob[x] != P->qjob[y] ? P->qjob[x] < P->qjob[y] : P->qlevel[x] < P->qlevel[y];
    });
    std::vector<int32_t> qpos(nq);
    for (int i = 0; i < nq; i++) qpos[jq[i]] = i;
    std::vector<int32_t> jq0(nj, 0), jq1(nj, 0);
    for (int i = nq - 1; i >= 0; i--) jq0[P->qjob[jq[i]]] = i;
    for (int i = 0; i < nq; i++) jq1[P->qjob[jq[i]]] = i + 1;
    P->wu.ensure(8 * ((size_t)P->items + 1));
    P->wbase.ensure(8 * ((size_t)P->items + 1));
    for (int j = 0; j < nj; j++) {
        const Index &ix = P->graphs[P->jobs[j].graph]->ix;
        const auto &lvs = P->jobs[j].levels;
        P->hist[j].ensure(4 * (size_t)hist_words(ix.m, padded_levels(lvs.size())) + 16);
        P->tmask[j].ensure(8 * (((size_t)ix.m + 63) / 64) + 8);
        P->lv[j].ensure(8 * lvs.size());
        FOLTY_HIP(hipMemcpyAsync(P->lv[j].p, lvs.data(), 8 * lvs.size(), hipMemcpyHostToDevice, s));
        P->sv[j].ensure(12 * (size_t)ix.T + 12);
        P->sw[j].ensure(8 * (size_t)ix.T + 8);
        P->su[j].ensure(4 * (size_t)ix.NI + 4);
        JobDev &d = jd[j];
        d.tri_base = ix.tri_base.as<int64_t>();
        d.ts = ix.ts.as<int64_t>();
        d.rec = ix.rec.as<EdgeRec>();
        d.variant = P->jobs[j].variant;
        d.dq = range_slack(lvs.back(), ix.tshift);
        d.lv = P->lv[j].as<int64_t>();
        d.nl = (int32_t)lvs.size();
        d.nls = padded_levels(lvs.size());
        d.m = ix.m;
        d.hist = P->hist[j].as<uint32_t>();
        d.tmask = P->tmask[j].as<unsigned long long>();
        d.sv = P->sv[j].as<int32_t>();
        d.sw = P->sw[j].as<int64_t>();
        d.su = P->su[j].as<int32_t>();
        d.wu = P->wu.as<int64_t>() + P->job_item_base[j];
        d.sid = ix.sid.as<int32_t>();
        d.smid = ix.smid.as<int32_t>();
        d.slo = ix.slo.as<int32_t>();
        d.shi = ix.shi.as<int32_t>();
        d.deg = ix.deg.as<int32_t>();
        d.tcnt = nullptr;
        d.q0 = jq0[j];
        d.q1 = jq1[j];
        d.keep_prefix = 0;
        for (int i = d.q0; i < d.q1; i++) {
            if (qs[jq[i]].universe == FOLTY_UNIVERSE_COMMON) d.tcnt = ix.tcnt.as<int32_t>();
            if (!(qs[jq[i]].flags & FOLTY_QUERY_NO_COUNTS)) d.keep_prefix = 1;
        }
        d.reset = !d.keep_prefix && !oneshot;
        P->jobs[j].reset = d.reset != 0;
    }
    // groups: the jobs of each graph, two at a time, share one enumeration
    std::vector<GroupDev> gd, singles;
    for (int gi = 0; gi < ng; gi++) {
        std::vector<int> js;
        for (int j = 0; j < nj; j++)
            if (P->jobs[j].graph == gi) js.push_back(j);
        for (size_t k = 0; k < js.size(); k += 2) {
            const Index &ix = P->graphs[gi]->ix;
            GroupDev G{};
            G.item = ix.item.as<EnumItem>();
            G.seg = ix.seg.as<int4>();
            G.oadj = ix.oadj.as<int32_t>();
            G.tri = ix.tri_cached ? ix.tri.as<int32_t>() : nullptr;
            G.tri_base = ix.tri_base.as<int64_t>();
            G.rec = ix.rec.as<EdgeRec>();
            G.rng = ix.erng.as<uint2>();
            G.nj = k + 1 < js.size() ? 2 : 1;
            G.job[0] = js[k];
            G.job[1] = G.nj == 2 ? js[k + 1] : js[k];
            (G.nj == 2 ? gd : singles).push_back(G);
        }
    }
    P->npairs = (int32_t)gd.size();
    gd.insert(gd.end(), singles.begin(), singles.end());
    P->ngroups = (int32_t)gd.size();
    P->group_item_base.assign(gd.size() + 1, 0);
    for (size_t k = 0; k < gd.size(); k++)
        P->group_item_base[k + 1] = P->group_item_base[k] + P->graphs[P->jobs[gd[k].job[0]].graph]->ix.NI;
    P->gitems = P->group_item_base[gd.size()];
    P->d_groups.ensure(sizeof(GroupDev) * std::max<size_t>(1, gd.size()));
    P->d_group_item_base.ensure(8 * (gd.size() + 1));
    if (!gd.empty()) FOLTY_HIP(hipMemcpyAsync(P->d_groups.p, gd.data(), sizeof(GroupDev) * gd.size(), hipMemcpyHostToDevice, s));
    FOLTY_HIP(hipMemcpyAsync(P->d_group_item_base.p, P->group_item_base.data(), 8 * (gd.size() + 1),
                             hipMemcpyHostToDevice, s));
    // queries, in job order
    std::vector<QueryDev> qd(nq);
    int64_t cap = 0;
    int32_t nmax = 1;
    for (int q = 0; q < nq; q++) {
        const Graph *g = P->graphs[qgraph[q]];
        const Index &ix = g->ix;
        QueryDev d{};
        d.q = q;
        d.level = P->qlevel[q];
        d.num = qs[q].theta_num;
        d.den = qs[q].theta_den;
        d.universe = qs[q].universe;
        d.excl = qs[q].exclude_other && qs[q].universe != FOLTY_UNIVERSE_COMMON ? 1 : 0;
        // records of this query: at most one per run of equal (static edge,
        // direction) keys within a wavefront, i.e. one per directed pair plus one
        // per wavefront boundary
        cap += 2 * (int64_t)ix.S + ix.m / 64 + 2;
        nmax = std::max(nmax, ix.n);
        qd[qpos[q]] = d;
    }
    P->rec_cap = cap;
    P->nbits = bit_length((uint64_t)nmax);
    if (bit_length((uint64_t)std::max(1, nq)) + 2 * P->nbits > 64)
        fail(FOLTY_EOVERFLOW, "too many queries for one plan at this graph size");
    P->d_jobs.ensure(sizeof(JobDev) * (size_t)std::max(1, nj));
    P->d_job_item_base.ensure(8 * ((size_t)nj + 1));
    P->d_job_w_base.ensure(8 * ((size_t)nj + 1));
    P->d_queries.ensure(sizeof(QueryDev) * (size_t)std::max(1, nq));
    if (nj) FOLTY_HIP(hipMemcpyAsync(P->d_jobs.p, jd.data(), sizeof(JobDev) * nj, hipMemcpyHostToDevice, s));
    FOLTY_HIP(hipMemcpyAsync(P->d_job_item_base.p, P->job_item_base.data(), 8 * (nj + 1), hipMemcpyHostToDevice, s));
    FOLTY_HIP(hipMemcpyAsync(P->d_job_w_base.p, P->job_w_base.data(), 8 * (nj + 1), hipMemcpyHostToDevice, s));
    if (nq) {
        FOLTY_HIP(hipMemcpyAsync(P->d_queries.p, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
    }
    P->nrec.ensure(4);
    P->keys.ensure(8 * (size_t)P->rec_cap + 8);
    P->vals.ensure(4 * (size_t)P->rec_cap + 4);
    P->scan_bytes = exclusive_scan_i64(nullptr, 0, P->wu.as<int64_t>(), P->wbase.as<int64_t>(), P->items + 1, s);
    P->cub.ensure(P->scan_bytes);
    FOLTY_HIP(hipStreamSynchronize(s));
    return P.release();
}

void plan_run(Plan *P, Result **outs) {
    FOLTY_HIP(hipSetDevice(P->device));
    hipStream_t s = P->stream;
    StreamScope sc(s);
    const int nq = (int)P->queries.size();
    if (P->oneshot) {
        // a shape already chosen for this much work, else the default; no capture
        P->eager = true;
        P->tuned = true;
    }
    // histograms that runs leave cleared must start cleared (jobs that keep
    // their counts are cleared at the start of every run)
    auto settle = [&] {
        if (!P->dirty) return;
        for (int j = 0; j < (int)P->jobs.size(); j++)
            if (P->jobs[j].reset) clear_hist(*P, j, s);
        P->dirty = false;
    };
    settle();
    if (!P->tuned) {
        // first run: eager, with the autotuner between the filter and the tests
        enqueue_compute(*P, s);
        tune(*P);
        settle();
    }
    if (!P->exec && !P->eager) {
        // capture once; if the runtime refuses, keep launching eagerly
        bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            try {
                enqueue_compute(*P, s);
            } catch (...) {
                ok = false;
            }
            hipGraph_t g = nullptr;
            ok = hipStreamEndCapture(s, &g) == hipSuccess && ok;
            if (ok && hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0) == hipSuccess) {
                P->graph = g;
            } else {
                if (g) (void)hipGraphDestroy(g);
                P->exec = nullptr;
                ok = false;
            }
        }
        if (!ok) {
            (void)hipGetLastError();
            P->eager = true;
        }
    }
    FOLTY_HIP(hipEventRecord(P->ev[0], s));
    P->dirty = true; // until the run is known to have finished
    if (P->exec) FOLTY_HIP(hipGraphLaunch(P->exec, s));
    else enqueue_compute(*P, s);
    FOLTY_HIP(hipEventRecord(P->ev[3], s));
    // read back how many records, then sort the (query, u, v) records; records
    // of one pair from several wavefronts are merged below, and a query's
    // certificates are the sum of its records
    int32_t npairs = 0;
    FOLTY_HIP(hipMemcpyAsync(&npairs, P->nrec.p, 4, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    P->dirty = false;
    if (npairs < 0 || npairs > P->rec_cap)
        fail(FOLTY_EDEVICE, "certificate records exceed their bound (%d > %lld)", npairs, (long long)P->rec_cap);
    P->last_records = npairs;
    HostVec<uint64_t> keys(npairs);
    HostVec<uint32_t> vals(npairs);
    if (npairs > 0) {
        P->keys2.ensure(8 * (size_t)npairs);
        P->vals2.ensure(4 * (size_t)npairs);
        int kb = bit_length((uint64_t)std::max(1, nq)) + 2 * P->nbits;
        size_t need = sort_pairs_u64_u32(nullptr, 0, P->keys.as<uint64_t>(), P->keys2.as<uint64_t>(),
                                         P->vals.as<uint32_t>(), P->vals2.as<uint32_t>(), npairs, kb, s);
        DevBuf tmp;
        tmp.ensure(need);
        sort_pairs_u64_u32(tmp.p, need, P->keys.as<uint64_t>(), P->keys2.as<uint64_t>(), P->vals.as<uint32_t>(),
                           P->vals2.as<uint32_t>(), npairs, kb, s);
        FOLTY_HIP(hipMemcpyAsync(keys.data(), P->keys2.p, 8 * (size_t)npairs, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(vals.data(), P->vals2.p, 4 * (size_t)npairs, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
    }
    P->last_ms = ev_ms2(P->ev[0], P->ev[3]);
    // split per query
    std::vector<std::unique_ptr<Result>> res(nq);
    for (int q = 0; q < nq; q++) res[q].reset(new Result());
    const uint64_t nmask = (1ull << P->nbits) - 1ull;
    {
        // distinct pairs per query first, so each query's arrays grow once
        std::vector<int64_t> per(nq, 0);
        for (int32_t i = 0; i < npairs; i++)
            if (i == 0 || keys[i] != keys[i - 1]) per[(size_t)(keys[i] >> (2 * P->nbits))]++;
        for (int q = 0; q < nq; q++) {
            res[q]->u.reserve((size_t)per[q]);
            res[q]->v.reserve((size_t)per[q]);
            res[q]->n_cert.reserve((size_t)per[q]);
        }
    }
    for (int32_t i = 0; i < npairs;) {
        uint32_t c = 0;
        int32_t e = i;
        while (e < npairs && keys[e] == keys[i]) c += vals[e++];
        int q = (int)(keys[i] >> (2 * P->nbits));
        Result *r = res[q].get();
        r->u.push_back((int32_t)((keys[i] >> P->nbits) & nmask));
        r->v.push_back((int32_t)(keys[i] & nmask));
        r->n_cert.push_back(c);
        r->n_certificates += c;
        i = e;
    }
    for (int q = 0; q < nq; q++) {
        Result *r = res[q].get();
        const Graph *g = P->graphs[P->qgraph[q]];
        fill_stats_from_index(g->ix, &r->stats);
        r->stats.filter_passes = 1; // plans filter once, into per-item triangle slots
        r->stats.n_pairs = (int64_t)r->u.size();
        r->stats.n_certificates = r->n_certificates;
        r->stats.query_ms = P->last_ms / std::max(1, nq);
        r->stats.temporal_ms = r->stats.query_ms;
        if (!(P->queries[q].flags & FOLTY_QUERY_NO_COUNTS)) {
            const Index &ix = g->ix;
            // the job's histogram holds running sums
            const int32_t nls = padded_levels(P->jobs[P->qjob[q]].levels.size());
            const uint32_t *hist = P->hist[P->qjob[q]].as<uint32_t>();
            r->counts_dev.ensure(4 * (size_t)ix.m_input + 4);
            if (ix.m_input > 0)
                k_fill<uint32_t><<<grid_for(ix.m_input, BLK), BLK, 0, s>>>(r->counts_dev.as<uint32_t>(),
                                                                                    0xffffffffu, ix.m_input);
            if (ix.m > 0)
                k_scatter_counts<<<grid_for(ix.m, BLK), BLK, 0, s>>>(hist, P->qlevel[q], nls, ix.perm.as<int32_t>(),
                                                                       ix.m, r->counts_dev.as<uint32_t>());
            FOLTY_LAUNCHED();
            r->has_counts = true;
            r->device = P->device;
        }
    }
    FOLTY_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < nq; q++) outs[q] = res[q].release();
}

void plan_free(Plan *P) { delete P; }

void plan_info(const Plan *P, folty_plan_info *info) {
    info->n_jobs = (int32_t)P->jobs.size();
    info->n_queries = (int32_t)P->queries.size();
    info->items = P->items;
    info->tests = P->last_tests;
    info->records = P->last_records;
    info->tests_per_chunk = P->ipt;
    info->temporal_blocks = P->tblocks;
    info->captured = P->exec != nullptr;
    info->last_run_ms = P->last_ms;
    info->tune_source = P->tune_source;
}

void run_batch(Graph *g, const folty_query *qs, int nq, Workspace &, Result **outs) {
    if (nq < 0) fail(FOLTY_EINVAL, "nq < 0");
    if (nq == 0) return;
    std::vector<int32_t> qg(nq, 0);
    std::unique_ptr<Plan> P(plan_create(&g, 1, qs, qg.data(), nq));
    plan_run(P.get(), outs);
}

void run_multi(Graph *const *gs, const folty_query *qs, int ng, Workspace &, Result **outs) {
    if (ng < 0) fail(FOLTY_EINVAL, "ng < 0");
    if (ng == 0) return;
    std::vector<int32_t> qg(ng);
    for (int i = 0; i < ng; i++) qg[i] = i;
    std::unique_ptr<Plan> P(plan_create(gs, ng, qs, qg.data(), ng));
    plan_run(P.get(), outs);
}

} // namespace folty
