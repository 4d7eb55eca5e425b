// Query kernels for the thresholded exists-exists-forall triadic query.
//
//  a.5  wedge enumeration + closing probe (paper, Algorithm OutNeighbours:
//       (u, v) in G->_pi and w in N+(u), test whether v and w are adjacent).
//       One wavefront per vertex u stages N+(u) in LDS, walks the wedges
//       u -> v -> x for every v in N+(u) and x in N+(v) with coalesced reads of
//       N+(v), and probes x in the staged N+(u).  Each static triangle is found
//       once, from its lowest-ranked vertex, as three oriented edges.
//  a.6  temporal tests (paper, Theorems 3.1 and 3.2): a temporal edge e on list
//       L1 forms a delta-temporal triangle with the third vertex w iff, with
//       t2 = the first entry of L2 at or after t(e) and t3 = the first entry of
//       L3 at or after t2, both exist and t3 - t(e) <= delta.  The first-entry
//       searches are binary searches over the time-sorted lists (the log
//       sigma_max factor).  A (triangle, directed list) pair is a run of tests.
//       A run is skipped when the time ranges of its three lists already rule
//       out t <= t2 <= t3 <= t + delta (a necessary condition, so no result
//       changes).  The surviving tests are cut into equal chunks over the grid.
//  a.7  threshold (paper, Algorithm ExistExistForAll, final loop) with the exact
//       rational theta, then per-pair certificate counts by a wavefront
//       segmented reduction and a ballot/prefix compaction of the pairs.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

#include "tri_device.h"

namespace folty {

namespace {

// ---------------------------------------------------------------------------
// index helpers
// ---------------------------------------------------------------------------
// The records of the static edges in their own order, lists lo -> hi first:
// soff, smid and the lists' end timestamps are read in the order they are
// stored, so this pass streams.
__global__ void k_static_recs(const int32_t *__restrict__ soff, const int32_t *__restrict__ smid,
                              const int64_t *__restrict__ ts, int32_t S, int32_t tshift,
                              EdgeRec *__restrict__ srec) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S) return;
    const int32_t a = soff[e], mid = smid[e], b = soff[e + 1];
    EdgeRec r;
    r.fs = a;
    r.fn = mid - a;
    r.bs = mid;
    r.bn = b - mid;
    r.flo = r.fn ? (uint32_t)(ts[a] >> tshift) : 0;
    r.fhi = r.fn ? (uint32_t)(ts[mid - 1] >> tshift) : 0;
    r.blo = r.bn ? (uint32_t)(ts[mid] >> tshift) : 0;
    r.bhi = r.bn ? (uint32_t)(ts[b - 1] >> tshift) : 0;
    srec[e] = r;
}

// Oriented edge p (static edge e, tail lo when bit 31 of its id is set): one
// 32-byte read of e's record, lists swapped when the tail is hi.
__global__ void k_edge_recs(const uint32_t *__restrict__ oeid, const EdgeRec *__restrict__ srec, int32_t S,
                            EdgeRec *__restrict__ rec, uint2 *__restrict__ erng) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S) return;
    const uint32_t id = oeid[p];
    const EdgeRec q = srec[id & 0x7fffffffu];
    EdgeRec r = q;
    if (!(id >> 31)) {
        r.fs = q.bs, r.fn = q.bn, r.flo = q.blo, r.fhi = q.bhi;
        r.bs = q.fs, r.bn = q.fn, r.blo = q.flo, r.bhi = q.fhi;
    }
    rec[p] = r;
    // a static edge has at least one temporal edge, so one of the lists is non-empty
    uint32_t lo = r.fn ? r.flo : r.blo, hi = r.fn ? r.fhi : r.bhi;
    if (r.fn && r.bn) {
        lo = r.blo < lo ? r.blo : lo;
        hi = r.bhi > hi ? r.bhi : hi;
    }
    erng[p] = make_uint2(lo, hi);
}

// Probe segments: the oriented edge (u, v) at position p goes to the endpoint
// with the longer out-row (mode A: u, scanning v's row; mode B: v, scanning
// u's row).  Sort key: owner * 2 + mode.
__global__ void k_seg_keys(const int32_t *__restrict__ ooff, const int32_t *__restrict__ oadj,
                           const int32_t *__restrict__ otail, int32_t S, uint32_t *__restrict__ key,
                           int32_t *__restrict__ val) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S) return;
    const int32_t u = otail[p], v = oadj[p];
    const int32_t du = ooff[u + 1] - ooff[u], dv = ooff[v + 1] - ooff[v];
    const bool mode_b = du < dv;
    key[p] = ((uint32_t)(mode_b ? v : u) << 1) | (mode_b ? 1u : 0u);
    val[p] = (int32_t)p;
}

// first sorted position of each key 0 .. 2n
__global__ void k_part_off(const uint32_t *__restrict__ key, int32_t S, int64_t nk, int32_t *__restrict__ off) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > nk) return;
    int32_t a = 0, b = S;
    while (a < b) {
        int32_t mid = (int32_t)(((int64_t)a + b) >> 1);
        if ((int64_t)key[mid] < x) a = mid + 1;
        else b = mid;
    }
    off[x] = a;
}

// seg[j] = (row start, row length, oriented edge | mode B << 31, owner)
__global__ void k_seg_recs(const uint32_t *__restrict__ key, const int32_t *__restrict__ val,
                           const int32_t *__restrict__ ooff, const int32_t *__restrict__ oadj,
                           const int32_t *__restrict__ otail, int32_t S, int4 *__restrict__ seg,
                           int32_t *__restrict__ len) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    const int32_t p = val[j];
    const bool mode_b = key[j] & 1u;
    const int32_t r = mode_b ? otail[p] : oadj[p]; // the vertex whose row is scanned
    const int32_t rs = ooff[r], rl = ooff[r + 1] - rs;
    seg[j] = make_int4(rs, rl, (int32_t)((uint32_t)p | (mode_b ? MODE_B : 0u)), (int32_t)(key[j] >> 1));
    len[j] = rl;
}

// An item starts at the first segment of each (owner, mode) run and wherever
// the run's probe count crosses a multiple of CHUNK or its segment count a
// multiple of ITEM_SEGS (both indices only grow, so runs of equal value are
// contiguous).
__global__ void k_item_flags(const uint32_t *__restrict__ key, const int64_t *__restrict__ P,
                             const int32_t *__restrict__ part_off, int32_t S, int32_t *__restrict__ flag) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    const int32_t p0 = part_off[key[j]];
    const int64_t cj = (P[j] - P[p0]) / CHUNK + (j - p0) / ITEM_SEGS;
    int f = j == p0;
    if (!f) f = cj != (P[j - 1] - P[p0]) / CHUNK + (j - 1 - p0) / ITEM_SEGS;
    flag[j] = f;
}

__global__ void k_item_starts(const int32_t *__restrict__ flag, const int32_t *__restrict__ fid, int32_t S,
                              int32_t *__restrict__ start) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < S && flag[j]) start[fid[j] - 1] = (int32_t)j;
}

__global__ void k_items(const int32_t *__restrict__ start, const int4 *__restrict__ seg, const int64_t *__restrict__ P,
                        const int32_t *__restrict__ ooff, int32_t NI, EnumItem *__restrict__ items) {
    int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= NI) return;
    const int32_t g0 = start[it], g1 = start[it + 1];
    const int32_t w = seg[g0].w;
    EnumItem e{};
    e.g0 = g0;
    e.ng = g1 - g0;
    e.nq = (int32_t)(P[g1] - P[g0]);
    e.b = ooff[w];
    e.d = ooff[w + 1] - e.b;
    items[it] = e;
}

// ---------------------------------------------------------------------------
// a.7 threshold + per-pair certificate counts
// ---------------------------------------------------------------------------
struct ThreshArgs {
    const uint32_t *count;
    const int32_t *sid, *smid, *slo, *shi, *deg, *tcnt;
    int32_t m;
    uint32_t num, den;
    int universe, excl;
    int zero_never;                  // theta > 0 and |U| >= 1 for every edge: count 0 never certifies
    int any;                         // the inner exists of a vertex query: count >= 1 qualifies
    uint32_t *ncert;                 // [2S]: 2 s + dir
    unsigned long long *total;       // certificates
};

__global__ __launch_bounds__(BLK) void k_threshold(ThreshArgs A) {
    __shared__ unsigned long long s_tot[BLK / 64];
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool in = k < A.m;
    int64_t key = -1;
    bool cert = false;
    const uint32_t cnt = in ? A.count[k] : 0u;
    // a wavefront whose edges all count 0 has no certificate when 0 cannot
    // reach theta * |U| (its lanes stay out of every run below)
    if (A.zero_never && !__ballot(cnt != 0u)) in = false;
    if (in) {
        int32_t s = A.sid[k];
        int dir = k >= A.smid[s] ? 1 : 0;
        int32_t a = dir ? A.shi[s] : A.slo[s];
        int32_t b = dir ? A.slo[s] : A.shi[s];
        if (A.any) {
            cert = cnt >= 1u;
        } else {
            int64_t U;
            if (A.universe == FOLTY_UNIVERSE_DST) U = (int64_t)A.deg[b] - A.excl;
            else if (A.universe == FOLTY_UNIVERSE_SRC) U = (int64_t)A.deg[a] - A.excl;
            else U = A.tcnt[s];
            cert = (uint64_t)cnt * A.den >= (uint64_t)A.num * (uint64_t)U;
        }
        key = 2 * (int64_t)s + dir;
    }
    // segmented count of certificates over runs of equal keys inside the wave
    int lane = lane_id();
    int64_t prev = __shfl_up(key, 1);
    int64_t next = __shfl_down(key, 1);
    bool head = lane == 0 || prev != key;
    bool tail = lane == 63 || next != key;
    unsigned long long heads = __ballot(head && in);
    unsigned long long certs = __ballot(cert);
    if (in && tail) {
        unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        unsigned long long h = heads & upto;
        int start = 63 - __clzll((long long)h);
        unsigned long long seg = upto & ~((1ull << start) - 1ull);
        int c = __popcll(certs & seg);
        if (c) atomicAdd(&A.ncert[key], (uint32_t)c);
    }
    if (lane == 0) s_tot[threadIdx.x >> 6] = (unsigned long long)__popcll(certs);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < BLK / 64; i++) t += s_tot[i];
        if (t) atomicAdd(A.total, t);
    }
}

// bits of a vertex id in a pair key (at least 1)
__host__ __device__ inline int pair_bits(int32_t n) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < (int64_t)n) b++;
    return b;
}

// Directed pairs with certificates, as keys (a << nbits) | b with their counts.
// Each block takes BLK x PAIR_ITEMS entries (2 s + dir) and claims its output
// range with one atomic, so a dense result does not serialise on the counter.
constexpr int PAIR_ITEMS = 8;
__global__ __launch_bounds__(BLK) void k_pairs_compact(const uint32_t *__restrict__ ncert, int32_t S,
                                                       const int32_t *__restrict__ slo, const int32_t *__restrict__ shi,
                                                       int nbits, uint64_t *__restrict__ keys,
                                                       uint32_t *__restrict__ vals, int32_t *__restrict__ npairs) {
    __shared__ int32_t s_wave[BLK / 64];
    __shared__ int32_t s_base;
    const int64_t n2 = 2 * (int64_t)S;
    const int64_t tile = (int64_t)blockIdx.x * BLK * PAIR_ITEMS;
    uint32_t c[PAIR_ITEMS];
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < PAIR_ITEMS; j++) {
        const int64_t i = tile + (int64_t)j * BLK + threadIdx.x;
        c[j] = i < n2 ? ncert[i] : 0u;
        mine += c[j] > 0;
    }
    const int w = threadIdx.x >> 6;
    const int32_t incl = wave_inclusive_sum(mine);
    if (lane_id() == 63) s_wave[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t tot = 0;
        for (int k = 0; k < BLK / 64; k++) {
            const int32_t x = s_wave[k];
            s_wave[k] = tot;
            tot += x;
        }
        s_base = tot ? atomicAdd(npairs, tot) : 0;
    }
    __syncthreads();
    int32_t pos = s_base + s_wave[w] + incl - mine;
#pragma unroll
    for (int j = 0; j < PAIR_ITEMS; j++) {
        if (!c[j]) continue;
        const int64_t i = tile + (int64_t)j * BLK + threadIdx.x;
        const int32_t e = (int32_t)(i >> 1);
        const uint64_t a = (uint64_t)((i & 1) ? shi[e] : slo[e]);
        const uint64_t b = (uint64_t)((i & 1) ? slo[e] : shi[e]);
        keys[pos] = (a << nbits) | b;
        vals[pos] = c[j];
        pos++;
    }
}

__global__ void k_pairs_unpack(const uint64_t *__restrict__ keys, int32_t np, int nbits, int32_t *__restrict__ u,
                               int32_t *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const uint64_t k = keys[i];
    u[i] = (int32_t)(k >> nbits);
    v[i] = (int32_t)(k & ((1ull << nbits) - 1));
}

// count[e] += the prefix sum of the interval marks at e
__global__ void k_add_counts(const int32_t *__restrict__ ps, int32_t m, uint32_t *__restrict__ count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        count[e] += (uint32_t)ps[e];
}

__global__ void k_counts_scatter(const uint32_t *__restrict__ count, const int32_t *__restrict__ perm, int32_t m,
                                 uint32_t *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) out[perm[k]] = count[k];
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

} // namespace

double ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    FOLTY_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
}

namespace {

unsigned enum_grid(int32_t n) {
    int64_t g = ((int64_t)n + WPB - 1) / WPB;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, ENUM_BLOCKS));
}

// a.5 for one predicate code and window bound, in two passes over the
// enumeration items.  The counting pass keeps, per item, how many triangles
// survive the time-range filter and how many tests they carry, and counts all
// triangles; exclusive scans give each item its first survivor slot (ws.sbase)
// and its first test (ws.wbase, total at [NI]); the emitting pass then
// enumerates only the items that have survivors and writes them.  When the
// index already holds per-item triangle offsets (after a plan, a server
// submission or a stats call) one pass writes survivors into those slots
// instead.  e0 and e1 bracket the (first) enumeration launch alone, so its
// duration is measured on the stream it runs on.  Returns the number of
// survivors (an upper bound in the one-pass case); *tri gets the triangle count.
// the items with at least one survivor (any order: each item writes its own
// slots), and the triangles those items hold
__global__ void k_item_list(const int32_t *__restrict__ su, const int32_t *__restrict__ tri_it, int32_t NI,
                            int32_t *__restrict__ list, int32_t *__restrict__ nlist,
                            unsigned long long *__restrict__ tri_listed) {
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool take = it < NI && su[it] > 0;
    const int32_t slot = wave_append(nlist, take);
    if (take) list[slot] = (int32_t)it;
    const int64_t t = wave_inclusive_sum((int64_t)(take ? tri_it[it] : 0));
    if (lane_id() == 63 && t > 0) atomicAdd(tri_listed, (unsigned long long)t);
}

} // namespace

namespace {
template <bool SS>
int64_t find_survivors_t(const Index &ix, int variant, int64_t dmax, Workspace &ws, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, int64_t *tri, int64_t *tests, bool one_pass) {
    *tests = -1; // known on the host only after the two-pass filter
    ws.emit_timed = false;
    ws.emit_items = 0;
    ws.emit_triangles = 0;
    ws.counted_items = false;
    ws.filter_passes = 1;
    const int32_t NI = ix.NI;
    ws.su.ensure(4 * ((size_t)NI + 1));
    ws.tri_it.ensure(4 * ((size_t)NI + 1));
    ws.wu.ensure(8 * ((size_t)NI + 1));
    ws.wbase.ensure(8 * ((size_t)NI + 1));
    ws.sbase.ensure(8 * ((size_t)NI + 1));
    ws.scal.ensure(128);
    ws.host.ensure(64);
    unsigned long long *hits = ws.scal.as<unsigned long long>() + 8; // [0, 8) belong to the threshold step
    k_fill<unsigned long long><<<1, 1, 0, s>>>(hits, 0ull, 1);
    FOLTY_LAUNCHED();
    auto sink_for = [&](auto V, auto M) {
        FilterSink<decltype(V)::value, decltype(M)::value, SS> sink{};
        sink.base = ws.sbase.as<int64_t>();
        sink.rec = ix.rec.as<EdgeRec>();
        sink.rng = ix.erng.as<uint2>();
        sink.dq = range_slack(dmax, ix.tshift);
        sink.variant = variant;
        sink.sv = ws.sv.as<int32_t>();
        sink.sw = nullptr; // the temporal step finds each survivor's tests itself
        sink.su = ws.su.as<int32_t>();
        sink.wu = ws.wu.as<int64_t>();
        sink.hits = hits;
        sink.tri_it = ws.tri_it.as<int32_t>();
        return sink;
    };
    // all items, or the nlist items of list
    auto run = [&](auto V, auto M, const int32_t *list, int32_t nlist) {
        auto sink = sink_for(V, M);
        const unsigned g = enum_grid(list ? nlist : NI);
        if (ix.tri_cached)
            k_filter_cached<<<g, BLK, 0, s>>>(ix.tri_base.as<int64_t>(), ix.tri.as<int32_t>(), NI, sink, list, nlist);
        else
            k_tri_enum<<<g, BLK, 0, s>>>(ix.item.as<EnumItem>(), ix.oadj.as<int32_t>(), ix.seg.as<int4>(), NI, sink,
                                         list, nlist);
        FOLTY_LAUNCHED();
    };
    using CountM = std::integral_constant<int, FILTER_COUNT>;
    using EmitM = std::integral_constant<int, FILTER_EMIT>;
    using BothM = std::integral_constant<int, FILTER_BOTH>;
    if (one_pass && ix.tri_base_ready.load(std::memory_order_acquire)) {
        // per-item triangle offsets exist: one pass writes survivors into them
        ws.sv.ensure(12 * ((size_t)ix.T + 1));
        FOLTY_HIP(hipEventRecord(e0, s));
        dispatch_variant(variant, [&](auto V) {
            auto sink = sink_for(V, BothM{});
            sink.base = ix.tri_base.as<int64_t>();
            if (ix.tri_cached)
                k_filter_cached<<<enum_grid(NI), BLK, 0, s>>>(ix.tri_base.as<int64_t>(), ix.tri.as<int32_t>(), NI,
                                                              sink);
            else
                k_tri_enum<<<enum_grid(NI), BLK, 0, s>>>(ix.item.as<EnumItem>(), ix.oadj.as<int32_t>(),
                                                         ix.seg.as<int4>(), NI, sink);
            FOLTY_LAUNCHED();
        });
        FOLTY_HIP(hipEventRecord(e1, s));
        // su[NI] = wu[NI] = 0 so that the exclusive scans leave the totals at [NI]
        k_fill<int32_t><<<1, 1, 0, s>>>(ws.su.as<int32_t>() + NI, 0, 1);
        k_fill<int64_t><<<1, 1, 0, s>>>(ws.wu.as<int64_t>() + NI, (int64_t)0, 1);
        FOLTY_LAUNCHED();
        size_t need = std::max(
            exclusive_scan_i64(nullptr, 0, ws.wu.as<int64_t>(), ws.wbase.as<int64_t>(), (int64_t)NI + 1, s),
            exclusive_scan_i32_to_i64(nullptr, 0, ws.su.as<int32_t>(), ws.sbase.as<int64_t>(), (int64_t)NI + 1, s));
        ws.cub.ensure(need);
        exclusive_scan_i64(ws.cub.p, need, ws.wu.as<int64_t>(), ws.wbase.as<int64_t>(), (int64_t)NI + 1, s);
        exclusive_scan_i32_to_i64(ws.cub.p, need, ws.su.as<int32_t>(), ws.sbase.as<int64_t>(), (int64_t)NI + 1, s);
        *tri = ix.T;
        ws.slots = ix.tri_base.as<int64_t>();
        return ix.T; // an upper bound: the temporal step reads the exact count
    }
    ws.slots = ws.sbase.as<int64_t>();
    FOLTY_HIP(hipEventRecord(e0, s));
    dispatch_variant(variant, [&](auto V) { run(V, CountM{}, nullptr, 0); });
    FOLTY_HIP(hipEventRecord(e1, s));
    // su[NI] = wu[NI] = 0 so that the exclusive scans leave the totals at [NI]
    k_fill<int32_t><<<1, 1, 0, s>>>(ws.su.as<int32_t>() + NI, 0, 1);
    k_fill<int64_t><<<1, 1, 0, s>>>(ws.wu.as<int64_t>() + NI, (int64_t)0, 1);
    FOLTY_LAUNCHED();
    size_t need = std::max(
        exclusive_scan_i64(nullptr, 0, ws.wu.as<int64_t>(), ws.wbase.as<int64_t>(), (int64_t)NI + 1, s),
        exclusive_scan_i32_to_i64(nullptr, 0, ws.su.as<int32_t>(), ws.sbase.as<int64_t>(), (int64_t)NI + 1, s));
    ws.cub.ensure(need);
    exclusive_scan_i64(ws.cub.p, need, ws.wu.as<int64_t>(), ws.wbase.as<int64_t>(), (int64_t)NI + 1, s);
    exclusive_scan_i32_to_i64(ws.cub.p, need, ws.su.as<int32_t>(), ws.sbase.as<int64_t>(), (int64_t)NI + 1, s);
    // the items with survivors, for the emitting pass
    ws.ilist.ensure(4 * ((size_t)NI + 1));
    unsigned long long *sc = ws.scal.as<unsigned long long>();
    int32_t *nlist = reinterpret_cast<int32_t *>(sc + 9);
    k_fill<unsigned long long><<<1, 2, 0, s>>>(sc + 9, 0ull, 2); // nlist, triangles of the listed items
    k_item_list<<<grid_for(NI, BLK), BLK, 0, s>>>(ws.su.as<int32_t>(), ws.tri_it.as<int32_t>(), NI,
                                                 ws.ilist.as<int32_t>(), nlist, sc + 10);
    FOLTY_LAUNCHED();
    int64_t *h = ws.host.as<int64_t>();
    h[3] = 0;
    FOLTY_HIP(hipMemcpyAsync(h, ws.sbase.as<int64_t>() + NI, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipMemcpyAsync(h + 3, nlist, 4, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipMemcpyAsync(h + 1, hits, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipMemcpyAsync(h + 2, ws.wbase.as<int64_t>() + NI, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipMemcpyAsync(h + 4, sc + 10, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    const int64_t survivors = h[0];
    *tri = h[1];
    *tests = h[2];
    ws.counted_items = true; // tri_it holds every item's triangles
    ws.tri_it_of = &ix;
    if (survivors > 0) {
        ws.sv.ensure(12 * (size_t)survivors);
        const int32_t nl = (int32_t)h[3];
        FOLTY_HIP(hipEventRecord(ws.ev[6], s));
        dispatch_variant(variant, [&](auto V) { run(V, EmitM{}, ws.ilist.as<int32_t>(), nl); });
        FOLTY_HIP(hipEventRecord(ws.ev[7], s));
        ws.emit_timed = true;
        ws.emit_items = nl;
        ws.emit_triangles = h[4];
        ws.filter_passes = 2;
    }
    return survivors;
}
} // namespace

int64_t find_survivors(const Index &ix, int variant, int64_t dmax, Workspace &ws, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1, int64_t *tri, int64_t *tests, bool ss, bool one_pass) {
    return ss ? find_survivors_t<true>(ix, variant, dmax, ws, s, e0, e1, tri, tests, one_pass)
              : find_survivors_t<false>(ix, variant, dmax, ws, s, e0, e1, tri, tests, one_pass);
}

bool use_one_pass(Graph *g, const folty_query &q) {
    if (q.flags & FOLTY_QUERY_ONE_PASS) {
        ensure_triangles(g);
        return true;
    }
    return q.delta >= g->ix.one_pass_from.load(std::memory_order_relaxed);
}

namespace {

// per-edge counts of the survivors' runs (a.6)
template <class Op, bool SS = false>
void launch_temporal(const Index &ix, int variant, int64_t dmax, Workspace &ws, const Op &op, int64_t tests,
                     int64_t survivors, hipStream_t s) {
    const uint32_t dq = run_slack(range_slack(dmax, ix.tshift));
    dispatch_variant(variant, [&](auto V) {
        launch_tests(ix, ws,
                     CountRunner<decltype(V)::value, Op, SS>{dq, ix.ts.as<int64_t>(), op, ws.sv.as<int32_t>(),
                                                             ix.rec.as<EdgeRec>()},
                     survivors, tests, s);
    });
}

// threshold + pairs for one query given device counts (sorted edge order)
// ---------------------------------------------------------------------------
// vertex queries: per vertex u, its neighbours v with a qualifying edge u -> v
// ---------------------------------------------------------------------------
// good[u] += 1 for every directed pair (u, v) (key 2 s + dir) with a qualifying edge
__global__ void k_vertex_good(const uint32_t *__restrict__ ncert, int32_t S, const int32_t *__restrict__ slo,
                              const int32_t *__restrict__ shi, uint32_t *__restrict__ good) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * (int64_t)S || ncert[k] == 0) return;
    const int32_t e = (int32_t)(k >> 1);
    atomicAdd(&good[(k & 1) ? shi[e] : slo[e]], 1u);
}

// u is a solution: |N(u)| >= 1 and good[u] * den >= num * |N(u)|
__global__ void k_vertex_flags(const uint32_t *__restrict__ good, const int32_t *__restrict__ deg, int32_t n,
                               uint32_t num, uint32_t den, int32_t *__restrict__ flag) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int32_t d = deg[u];
    flag[u] = d >= 1 && (uint64_t)good[u] * den >= (uint64_t)num * (uint64_t)d;
}

// the solutions in id order, at their exclusive-scan positions
__global__ void k_vertex_compact(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                                 const uint32_t *__restrict__ good, int32_t n, int32_t *__restrict__ vert,
                                 uint32_t *__restrict__ vgood) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n || !flag[u]) return;
    vert[pos[u]] = (int32_t)u;
    vgood[pos[u]] = good[u];
}

// the vertex step after the edge-level threshold (ncert holds its per-pair counts)
void finish_vertex(const Graph *g, const folty_vertex_query &vq, Workspace &ws, Result *res, hipStream_t s) {
    const Index &ix = g->ix;
    const int32_t n = ix.n, S = ix.S;
    ws.vtmp.ensure(20 * (size_t)n + 16);
    uint32_t *good = ws.vtmp.as<uint32_t>();
    int32_t *flag = reinterpret_cast<int32_t *>(good + n);
    int32_t *pos = flag + n;
    int32_t *vert = pos + n;
    uint32_t *vgood = reinterpret_cast<uint32_t *>(vert + n);
    k_fill<uint32_t><<<grid_for(n, BLK), BLK, 0, s>>>(good, 0u, n);
    FOLTY_LAUNCHED();
    if (S > 0 && ix.m > 0) {
        k_vertex_good<<<grid_for(2 * (int64_t)S, BLK), BLK, 0, s>>>(ws.ncert.as<uint32_t>(), S, ix.slo.as<int32_t>(),
                                                                  ix.shi.as<int32_t>(), good);
        FOLTY_LAUNCHED();
    }
    k_vertex_flags<<<grid_for(n, BLK), BLK, 0, s>>>(good, ix.deg.as<int32_t>(), n, vq.theta_num, vq.theta_den, flag);
    FOLTY_LAUNCHED();
    size_t need = exclusive_scan_i32(nullptr, 0, flag, pos, n, s);
    ws.cub.ensure(need);
    exclusive_scan_i32(ws.cub.p, need, flag, pos, n, s);
    k_vertex_compact<<<grid_for(n, BLK), BLK, 0, s>>>(flag, pos, good, n, vert, vgood);
    FOLTY_LAUNCHED();
    int32_t last[2] = {0, 0};
    FOLTY_HIP(hipMemcpyAsync(&last[0], pos + n - 1, 4, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipMemcpyAsync(&last[1], flag + n - 1, 4, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    const int32_t nv = last[0] + last[1];
    res->vert.resize(nv);
    res->vgood.resize(nv);
    if (nv > 0) {
        FOLTY_HIP(hipMemcpyAsync(res->vert.data(), vert, 4 * (size_t)nv, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(res->vgood.data(), vgood, 4 * (size_t)nv, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
    }
}

// any: qualify edges with count >= 1 (the inner exists of a vertex query)
// Threshold step: certificates, per-pair certificate counts and the compacted
// pair keys (unsorted, in ws).  Returns |Sol| and the number of pairs.
struct PairCounts {
    int64_t ncerts;
    int32_t npairs;
};

PairCounts threshold_pairs(const Graph *g, const folty_query &q, const uint32_t *count, Workspace &ws,
                           hipStream_t s, bool any) {
    const Index &ix = g->ix;
    const int32_t S = ix.S, m = ix.m;
    ws.ncert.ensure(8 * (size_t)S + 8);
    ws.scal.ensure(64);
    k_fill<unsigned long long><<<1, 8, 0, s>>>(ws.scal.as<unsigned long long>(), 0ull, 8);
    if (S > 0) {
        k_fill<uint32_t><<<grid_for(2 * (int64_t)S, BLK), BLK, 0, s>>>(ws.ncert.as<uint32_t>(), 0u,
                                                                               2 * (int64_t)S);
    }
    FOLTY_LAUNCHED();
    unsigned long long *total = ws.scal.as<unsigned long long>();
    int32_t *np = ws.scal.as<int32_t>() + 4;
    if (m > 0) {
        ThreshArgs A;
        A.count = count;
        A.sid = ix.sid.as<int32_t>();
        A.smid = ix.smid.as<int32_t>();
        A.slo = ix.slo.as<int32_t>();
        A.shi = ix.shi.as<int32_t>();
        A.deg = ix.deg.as<int32_t>();
        A.tcnt = ix.tcnt.as<int32_t>();
        A.m = m;
        A.num = q.theta_num;
        A.den = q.theta_den;
        A.universe = q.universe;
        A.excl = q.exclude_other ? 1 : 0;
        // N(b) and N(a) hold the other endpoint, so |U| >= 1 unless it is left out
        A.zero_never = any || (q.theta_num > 0 && !q.exclude_other &&
                               (q.universe == FOLTY_UNIVERSE_DST || q.universe == FOLTY_UNIVERSE_SRC));
        A.any = any ? 1 : 0;
        A.ncert = ws.ncert.as<uint32_t>();
        A.total = total;
        k_threshold<<<grid_for(m, BLK), BLK, 0, s>>>(A);
        FOLTY_LAUNCHED();
        ws.pairs_k.ensure(16 * (size_t)S + 16);
        ws.pairs_v.ensure(8 * (size_t)S + 8);
        k_pairs_compact<<<grid_for(2 * (int64_t)S, BLK * PAIR_ITEMS), BLK, 0, s>>>(
            ws.ncert.as<uint32_t>(), S, ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), pair_bits(ix.n),
            ws.pairs_k.as<uint64_t>(), ws.pairs_v.as<uint32_t>(), np);
        FOLTY_LAUNCHED();
    }
    ws.host.ensure(64);
    FOLTY_HIP(hipMemcpyAsync(ws.host.p, ws.scal.p, 32, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    unsigned long long ncerts;
    int32_t npairs;
    memcpy(&ncerts, ws.host.p, 8);
    memcpy(&npairs, ws.host.as<char>() + 16, 4);
    return PairCounts{(int64_t)ncerts, npairs};
}

// sort the pair keys of threshold_pairs and unpack them: u, v and the
// certificate counts, sorted by (u, v), in ws
void sort_pairs(const Graph *g, Workspace &ws, int32_t npairs, hipStream_t s, int32_t **du, int32_t **dv,
                uint32_t **dn) {
    const Index &ix = g->ix;
    ws.pairs_k2.ensure(8 * (size_t)npairs);
    ws.pairs_v2.ensure(4 * (size_t)npairs);
    const int nb = pair_bits(ix.n);
    size_t need = sort_pairs_u64_u32(nullptr, 0, ws.pairs_k.as<uint64_t>(), ws.pairs_k2.as<uint64_t>(),
                                     ws.pairs_v.as<uint32_t>(), ws.pairs_v2.as<uint32_t>(), npairs, 2 * nb, s);
    ws.cub.ensure(need);
    sort_pairs_u64_u32(ws.cub.p, need, ws.pairs_k.as<uint64_t>(), ws.pairs_k2.as<uint64_t>(),
                       ws.pairs_v.as<uint32_t>(), ws.pairs_v2.as<uint32_t>(), npairs, 2 * nb, s);
    // the unsorted keys are no longer needed: u and v go where they were
    *du = reinterpret_cast<int32_t *>(ws.pairs_k.p);
    *dv = *du + npairs;
    *dn = ws.pairs_v2.as<uint32_t>();
    k_pairs_unpack<<<grid_for(npairs, BLK), BLK, 0, s>>>(ws.pairs_k2.as<uint64_t>(), npairs, nb, *du, *dv);
    FOLTY_LAUNCHED();
}

void finish_query(const Graph *g, const folty_query &q, const uint32_t *count, Workspace &ws, Result *res,
                  hipStream_t s, bool any = false) {
    const PairCounts pc = threshold_pairs(g, q, count, ws, s, any);
    const int32_t npairs = pc.npairs;
    res->n_certificates = pc.ncerts;
    res->u.resize(npairs);
    res->v.resize(npairs);
    res->n_cert.resize(npairs);
    if (npairs > 0) {
        int32_t *du, *dv;
        uint32_t *dn;
        sort_pairs(g, ws, npairs, s, &du, &dv, &dn);
        FOLTY_HIP(hipMemcpyAsync(res->u.data(), du, 4 * (size_t)npairs, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(res->v.data(), dv, 4 * (size_t)npairs, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(res->n_cert.data(), dn, 4 * (size_t)npairs, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
    }
}

// per-edge counts in input order (0xFFFFFFFF for self-loops) into out
void scatter_counts(const Graph *g, const uint32_t *count, uint32_t *out, hipStream_t s) {
    const Index &ix = g->ix;
    if (ix.m_input > 0) {
        k_fill<uint32_t><<<grid_for(ix.m_input, BLK), BLK, 0, s>>>(out, 0xffffffffu, ix.m_input);
        FOLTY_LAUNCHED();
    }
    if (ix.m > 0) {
        k_counts_scatter<<<grid_for(ix.m, BLK), BLK, 0, s>>>(count, ix.perm.as<int32_t>(), ix.m, out);
        FOLTY_LAUNCHED();
    }
}

void keep_counts(const Graph *g, const uint32_t *count, Result *res, hipStream_t s) {
    res->counts_dev.ensure(4 * (size_t)g->ix.m_input + 4);
    scatter_counts(g, count, res->counts_dev.as<uint32_t>(), s);
    res->has_counts = true;
    res->device = g->device;
}

} // namespace

void index_triangles(Index &ix, bool cache, DevBuf &cub, hipStream_t s) {
    const int32_t n = ix.n, S = ix.S;
    ix.rec.ensure(sizeof(EdgeRec) * ((size_t)S + 1));
    ix.erng.ensure(sizeof(uint2) * ((size_t)S + 1));
    ix.tcnt_ready = false;
    if (S > 0) {
        DevBuf srec;
        srec.ensure(sizeof(EdgeRec) * (size_t)S);
        k_static_recs<<<grid_for(S, BLK), BLK, 0, s>>>(ix.soff.as<int32_t>(), ix.smid.as<int32_t>(),
                                                       ix.ts.as<int64_t>(), S, ix.tshift, srec.as<EdgeRec>());
        k_edge_recs<<<grid_for(S, BLK), BLK, 0, s>>>(ix.oeid.as<uint32_t>(), srec.as<EdgeRec>(), S,
                                                     ix.rec.as<EdgeRec>(), ix.erng.as<uint2>());
        FOLTY_LAUNCHED();
    }
    // probe segments grouped by (owner, mode), their probe prefix, and items
    ix.seg.ensure(sizeof(int4) * ((size_t)S + 1));
    int32_t ni = 0;
    int64_t probes = 0;
    {
        DevBuf key, key2, val, val2, part_off, len, P, flag, fid, start;
        key.ensure(4 * (size_t)S + 4);
        key2.ensure(4 * (size_t)S + 4);
        val.ensure(4 * (size_t)S + 4);
        val2.ensure(4 * (size_t)S + 4);
        len.ensure(4 * ((size_t)S + 1));
        P.ensure(8 * ((size_t)S + 1));
        flag.ensure(4 * (size_t)S + 4);
        fid.ensure(4 * (size_t)S + 4);
        start.ensure(4 * ((size_t)S + 1));
        const int64_t nk = 2 * (int64_t)n;
        part_off.ensure(4 * ((size_t)nk + 1));
        if (S > 0) {
            k_seg_keys<<<grid_for(S, BLK), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.oadj.as<int32_t>(),
                                                        ix.otail.as<int32_t>(), S, key.as<uint32_t>(), val.as<int32_t>());
            FOLTY_LAUNCHED();
            const int kb = bit_length((uint64_t)nk);
            size_t need = sort_pairs_u32_i32(nullptr, 0, key.as<uint32_t>(), key2.as<uint32_t>(), val.as<int32_t>(),
                                             val2.as<int32_t>(), S, kb, s);
            cub.ensure(need);
            sort_pairs_u32_i32(cub.p, need, key.as<uint32_t>(), key2.as<uint32_t>(), val.as<int32_t>(),
                               val2.as<int32_t>(), S, kb, s);
            k_part_off<<<grid_for(nk + 1, BLK), BLK, 0, s>>>(key2.as<uint32_t>(), S, nk, part_off.as<int32_t>());
            k_seg_recs<<<grid_for(S, BLK), BLK, 0, s>>>(key2.as<uint32_t>(), val2.as<int32_t>(), ix.ooff.as<int32_t>(),
                                                        ix.oadj.as<int32_t>(), ix.otail.as<int32_t>(), S,
                                                        ix.seg.as<int4>(), len.as<int32_t>());
            k_fill<int32_t><<<1, 1, 0, s>>>(len.as<int32_t>() + S, 0, 1);
            FOLTY_LAUNCHED();
            need = exclusive_scan_i32_to_i64(nullptr, 0, len.as<int32_t>(), P.as<int64_t>(), (int64_t)S + 1, s);
            cub.ensure(need);
            exclusive_scan_i32_to_i64(cub.p, need, len.as<int32_t>(), P.as<int64_t>(), (int64_t)S + 1, s);
            k_item_flags<<<grid_for(S, BLK), BLK, 0, s>>>(key2.as<uint32_t>(), P.as<int64_t>(), part_off.as<int32_t>(),
                                                          S, flag.as<int32_t>());
            FOLTY_LAUNCHED();
            need = inclusive_scan_i32(nullptr, 0, flag.as<int32_t>(), fid.as<int32_t>(), S, s);
            cub.ensure(need);
            inclusive_scan_i32(cub.p, need, flag.as<int32_t>(), fid.as<int32_t>(), S, s);
            k_item_starts<<<grid_for(S, BLK), BLK, 0, s>>>(flag.as<int32_t>(), fid.as<int32_t>(), S,
                                                           start.as<int32_t>());
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipMemcpyAsync(&ni, fid.as<int32_t>() + (S - 1), 4, hipMemcpyDeviceToHost, s));
            FOLTY_HIP(hipMemcpyAsync(&probes, P.as<int64_t>() + S, 8, hipMemcpyDeviceToHost, s));
            FOLTY_HIP(hipStreamSynchronize(s));
            k_fill<int32_t><<<1, 1, 0, s>>>(start.as<int32_t>() + ni, S, 1);
            FOLTY_LAUNCHED();
        }
        ix.item.ensure(sizeof(EnumItem) * ((size_t)ni + 1));
        if (ni > 0) {
            k_items<<<grid_for(ni, BLK), BLK, 0, s>>>(start.as<int32_t>(), ix.seg.as<int4>(), P.as<int64_t>(),
                                                      ix.ooff.as<int32_t>(), ni, ix.item.as<EnumItem>());
            FOLTY_LAUNCHED();
        }
        FOLTY_HIP(hipStreamSynchronize(s)); // the temporaries go back to the pool
    }
    ix.otail.release();
    ix.NI = ni;
    ix.probes = probes;
    // triangle slots per item are made on first use (plans, the server's memory
    // estimate, the cached list): a single query counts its survivors itself
    ix.T = -1;
    ix.tri_base_ready.store(false, std::memory_order_release);
    ix.tri_cached = false;
    ix.tri.release();
    if (cache) {
        ensure_tri_base(ix, s);
        if (ix.T > 0) {
            ix.tri.ensure(12 * (size_t)ix.T);
            CacheSink sink{ix.tri_base.as<int64_t>(), ix.tri.as<int32_t>(), 0};
            k_tri_enum<<<enum_grid(ni), BLK, 0, s>>>(ix.item.as<EnumItem>(), ix.oadj.as<int32_t>(),
                                                     ix.seg.as<int4>(), ni, sink);
            FOLTY_LAUNCHED();
            ix.tri_cached = true;
        }
    }
}


// per-item triangle offsets from per-item triangle counts tri_it[0, NI) (the
// counting filter's, or a CountSink pass); tri_it[NI] is set to 0 here
static void tri_base_from_counts(Index &ix, int32_t *tri_it, hipStream_t s) {
    const int32_t ni = ix.NI;
    ix.tri_base.ensure(8 * ((size_t)ni + 1));
    DevBuf cub;
    k_fill<int32_t><<<1, 1, 0, s>>>(tri_it + ni, 0, 1);
    FOLTY_LAUNCHED();
    size_t need = exclusive_scan_i32_to_i64(nullptr, 0, tri_it, ix.tri_base.as<int64_t>(), (int64_t)ni + 1, s);
    cub.ensure(need);
    exclusive_scan_i32_to_i64(cub.p, need, tri_it, ix.tri_base.as<int64_t>(), (int64_t)ni + 1, s);
    int64_t T = 0;
    FOLTY_HIP(hipMemcpyAsync(&T, ix.tri_base.as<int64_t>() + ni, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    ix.T = T;
    ix.tri_base_ready.store(true, std::memory_order_release);
}

// triangles of each enumeration item, their exclusive offsets (the slots of a
// one-pass filter and of the cached list) and the triangle count
void ensure_tri_base(Index &ix, hipStream_t s) {
    if (ix.tri_base_ready.load(std::memory_order_acquire)) return;
    const int32_t ni = ix.NI;
    DevBuf tri_it;
    tri_it.ensure(4 * ((size_t)ni + 1));
    if (ni > 0) {
        CountSink cs{tri_it.as<int32_t>(), 0};
        k_tri_enum<<<enum_grid(ni), BLK, 0, s>>>(ix.item.as<EnumItem>(), ix.oadj.as<int32_t>(),
                                                 ix.seg.as<int4>(), ni, cs);
        FOLTY_LAUNCHED();
    }
    tri_base_from_counts(ix, tri_it.as<int32_t>(), s);
}

// The two-pass filter enumerates the items with survivors a second time.  At a
// wide window those are the items that hold most triangles, and the second
// pass costs about as much as the first (70M edges, one year: 7.1 ms on top of
// the 6.9 ms counting pass).  When the second pass enumerated at least half of
// the items or half of the triangles again, later queries of about this window
// or wider (from an eighth of it) filter in one pass instead, writing survivors
// into per-item triangle slots: 12 bytes of workspace per static triangle, so
// only when that fits in a quarter of the free device memory.  The offsets come
// from the counting pass's per-item triangle counts (no extra enumeration).
// The rule depends only on the graph and the queries, never on timing.  Narrow
// windows keep the two passes: their second pass is short, and the one pass
// writes into slots sized for every triangle (70M edges: 5.4-5.6 ms for one
// pass against 5.0-5.2 ms for the counting pass at 1 hour and 1 day).
void maybe_one_pass(Graph *g, const Workspace &ws, int64_t delta) {
    Index &ix = g->ix;
    if (!ws.emit_timed || !ws.counted_items || ws.tri_it_of != &ix || ix.T <= 0) return;
    if (2 * (int64_t)ws.emit_items < (int64_t)ix.NI && 2 * ws.emit_triangles < ix.T) return;
    if (delta / 8 >= ix.one_pass_from.load(std::memory_order_relaxed)) return;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (!ix.tri_base_ready.load(std::memory_order_acquire) && (size_t)ix.T * 12 > fr / 4) return;
    std::lock_guard<std::mutex> lk(g->lazy_mu);
    if (!ix.tri_base_ready.load(std::memory_order_acquire)) {
        FOLTY_HIP(hipSetDevice(g->device));
        StreamScope sc(g->stream);
        HookScope hs(&g->hook);
        // the counting pass left its per-item triangles in the workspace, on a
        // stream the caller has synchronised
        tri_base_from_counts(ix, ws.tri_it.as<int32_t>(), g->stream);
    }
    if (delta / 8 < ix.one_pass_from.load(std::memory_order_relaxed))
        ix.one_pass_from.store(delta / 8, std::memory_order_relaxed);
}

void ensure_triangles(Graph *g) {
    std::lock_guard<std::mutex> lk(g->lazy_mu);
    if (g->ix.tri_base_ready.load(std::memory_order_acquire) || !g->ix.built) return;
    FOLTY_HIP(hipSetDevice(g->device));
    StreamScope sc(g->stream);
    HookScope hs(&g->hook);
    ensure_tri_base(g->ix, g->stream);
}

void ensure_tcnt(Index &ix, hipStream_t s) {
    if (ix.tcnt_ready) return;
    ix.tcnt.ensure(4 * (size_t)ix.S + 4);
    if (ix.S > 0) {
        k_fill<int32_t><<<grid_for(ix.S, BLK), BLK, 0, s>>>(ix.tcnt.as<int32_t>(), 0, ix.S);
        FOLTY_LAUNCHED();
        TcntSink sink{ix.oeid.as<uint32_t>(), ix.tcnt.as<int32_t>()};
        k_tri_enum<<<enum_grid(ix.NI), BLK, 0, s>>>(ix.item.as<EnumItem>(), ix.oadj.as<int32_t>(),
                                                    ix.seg.as<int4>(), ix.NI, sink);
        FOLTY_LAUNCHED();
    }
    ix.tcnt_ready = true;
}

void check_query(const Graph *g, const folty_query &q) {
    if (!g->ix.built) fail(FOLTY_ENOTBUILT, "folty_build_index has not been called for this graph");
    if (q.delta < 0) fail(FOLTY_EINVAL, "delta must be >= 0 (got %lld)", (long long)q.delta);
    if (q.theta_den == 0) fail(FOLTY_EINVAL, "theta_den must be > 0");
    if (q.theta_num > q.theta_den) fail(FOLTY_EINVAL, "theta must lie in [0, 1]");
    if (q.variant > 7) fail(FOLTY_EINVAL, "variant must be 0..7 (got %u)", (unsigned)q.variant);
    if (q.universe > 2) fail(FOLTY_EINVAL, "unknown universe %u", (unsigned)q.universe);
    if (q.exclude_other > 1) fail(FOLTY_EINVAL, "exclude_other must be 0 or 1");
    if (q.exclude_other && q.universe == FOLTY_UNIVERSE_COMMON)
        fail(FOLTY_EINVAL, "exclude_other applies to the N(a) and N(b) universes only");
    if (q.flags & ~(FOLTY_QUERY_NO_COUNTS | FOLTY_QUERY_SMALLER_SIDE | FOLTY_QUERY_ONE_PASS))
        fail(FOLTY_EINVAL, "unknown query flags 0x%x", (unsigned)q.flags);
}

Result *run_query(Graph *g, const folty_query &q, Workspace &ws) { return run_query_on(g, q, ws, g->stream); }

static Result *run_query_impl(Graph *g, const folty_query &q, Workspace &ws, hipStream_t s,
                              const folty_vertex_query *vq);

Result *run_query_on(Graph *g, const folty_query &q, Workspace &ws, hipStream_t s) {
    check_query(g, q);
    return run_query_impl(g, q, ws, s, nullptr);
}

Result *run_vertex_query(Graph *g, const folty_vertex_query &vq, Workspace &ws) {
    if (vq.inner > FOLTY_INNER_EXISTS) fail(FOLTY_EINVAL, "unknown inner quantifier %u", (unsigned)vq.inner);
    for (int i = 0; i < 7; i++)
        if (vq.reserved[i]) fail(FOLTY_EINVAL, "reserved fields of the vertex query must be 0");
    if (vq.theta_den == 0) fail(FOLTY_EINVAL, "theta_den must be > 0");
    if (vq.theta_num > vq.theta_den) fail(FOLTY_EINVAL, "theta must lie in [0, 1]");
    folty_query q = vq.edge;
    if (vq.inner == FOLTY_INNER_EXISTS) { // the edge threshold is not read
        q.theta_num = 1;
        q.theta_den = 1;
    }
    check_query(g, q);
    return run_query_impl(g, q, ws, g->stream, &vq);
}

// The counts of a query (paper, Algorithm ExistExistForAll, the out- and
// in-count arrays summed): filter, temporal tests, per-edge counts in sorted
// edge order in ws.count.  Events: ev[0] start, ev[4]/ev[5] around the counting
// filter pass, ev[2] after the tests.  *tests receives the number of temporal
// tests by a copy on the stream: read it after the stream is synchronised.
static const uint32_t *query_counts(Graph *g, const folty_query &q, Workspace &ws, hipStream_t s,
                                    int64_t *tests) {
    Index &ix = g->ix;
    ws.ensure_events();
    FOLTY_HIP(hipEventRecord(ws.ev[0], s));
    ws.count.ensure(4 * (size_t)ix.m + 4);
    uint32_t *count = ws.count.as<uint32_t>();
    if (ix.m > 0) {
        k_fill<uint32_t><<<grid_for(ix.m, BLK), BLK, 0, s>>>(count, 0u, ix.m);
        FOLTY_LAUNCHED();
    }
    int64_t tri = 0;
    *tests = 0;
    ws.filter_passes = 0;
    if (ix.NI > 0) {
        int64_t known = -1;
        const bool ss = (q.flags & FOLTY_QUERY_SMALLER_SIDE) != 0;
        const bool one = use_one_pass(g, q);
        const int64_t survivors =
            find_survivors(ix, q.variant, q.delta, ws, s, ws.ev[4], ws.ev[5], &tri, &known, ss, one);
        if (survivors > 0) {
            if (ss) {
                // runs with a shorter L2 mark edge ranges in diff; its prefix sum is added at the end
                ws.diff.ensure(4 * (2 * (size_t)ix.m + 1));
                int32_t *diff = ws.diff.as<int32_t>(), *ps = diff + ix.m + 1;
                k_fill<int32_t><<<grid_for(ix.m + 1, BLK, PERSIST_BLOCKS), BLK, 0, s>>>(diff, 0, ix.m + 1);
                FOLTY_LAUNCHED();
                DirectOp op{q.delta, count, diff};
                launch_temporal<DirectOp, true>(ix, q.variant, q.delta, ws, op, known, survivors, s);
                size_t need = inclusive_scan_i32(nullptr, 0, diff, ps, ix.m, s);
                ws.cub.ensure(need);
                inclusive_scan_i32(ws.cub.p, need, diff, ps, ix.m, s);
                k_add_counts<<<grid_for(ix.m, BLK, PERSIST_BLOCKS), BLK, 0, s>>>(ps, ix.m, count);
                FOLTY_LAUNCHED();
            } else {
                DirectShortOp op{q.delta, count};
                op.inl = ix.tshift == 0; // the records' end timestamps are exact
                launch_temporal(ix, q.variant, q.delta, ws, op, known, survivors, s);
            }
            FOLTY_HIP(hipMemcpyAsync(tests, ws.wbase.as<int64_t>() + ix.NI, 8, hipMemcpyDeviceToHost, s));
        }
    } else {
        FOLTY_HIP(hipEventRecord(ws.ev[4], s));
        FOLTY_HIP(hipEventRecord(ws.ev[5], s));
    }
    if (ix.T < 0) ix.T = tri; // every query enumerates every triangle once
    FOLTY_HIP(hipEventRecord(ws.ev[2], s));
    return count;
}

void run_query_into(Graph *g, const folty_query &q, Workspace &ws, int32_t *pair_u, int32_t *pair_v,
                    uint32_t *n_cert, int64_t pair_cap, uint32_t *edge_count, int64_t *n_pairs,
                    int64_t *n_certificates) {
    check_query(g, q);
    if (pair_cap < 0) fail(FOLTY_EINVAL, "pair_cap must be >= 0");
    if (pair_cap > 0 && (!pair_u || !pair_v || !n_cert)) fail(FOLTY_EINVAL, "null pair output array");
    if (hipSetDevice(g->device) != hipSuccess) fail(FOLTY_EDEVICE, "hipSetDevice failed");
    const Index &ix = g->ix;
    if (q.universe == FOLTY_UNIVERSE_COMMON && !ix.tcnt_ready)
        fail(FOLTY_EINVAL, "the universe N(a) & N(b) needs the graph's per-edge triangle counts, which this call "
                           "does not build: run one query with that universe through folty_run_fol_query first");
    if ((q.flags & FOLTY_QUERY_ONE_PASS) && !ix.tri_base_ready.load(std::memory_order_acquire))
        fail(FOLTY_EINVAL, "FOLTY_QUERY_ONE_PASS needs the graph's per-item triangle offsets, which this call does "
                           "not build: run one query with that flag through folty_run_fol_query first");
    hipStream_t s = g->stream;
    int64_t tests = 0;
    const uint32_t *count = query_counts(g, q, ws, s, &tests);
    const PairCounts pc = threshold_pairs(g, q, count, ws, s, false);
    *n_pairs = pc.npairs;
    *n_certificates = pc.ncerts;
    if (edge_count) scatter_counts(g, count, edge_count, s);
    if (pc.npairs > pair_cap) {
        FOLTY_HIP(hipStreamSynchronize(s));
        fail(FOLTY_EOVERFLOW, "%d solution pairs do not fit the %lld the caller's arrays hold", pc.npairs,
             (long long)pair_cap);
    }
    if (pc.npairs > 0) {
        int32_t *du, *dv;
        uint32_t *dn;
        sort_pairs(g, ws, pc.npairs, s, &du, &dv, &dn);
        FOLTY_HIP(hipMemcpyAsync(pair_u, du, 4 * (size_t)pc.npairs, hipMemcpyDeviceToDevice, s));
        FOLTY_HIP(hipMemcpyAsync(pair_v, dv, 4 * (size_t)pc.npairs, hipMemcpyDeviceToDevice, s));
        FOLTY_HIP(hipMemcpyAsync(n_cert, dn, 4 * (size_t)pc.npairs, hipMemcpyDeviceToDevice, s));
    }
    FOLTY_HIP(hipStreamSynchronize(s));
}

static Result *run_query_impl(Graph *g, const folty_query &q, Workspace &ws, hipStream_t s,
                              const folty_vertex_query *vq) {
    if (hipSetDevice(g->device) != hipSuccess) fail(FOLTY_EDEVICE, "hipSetDevice failed");
    Index &ix = g->ix;
    if (q.universe == FOLTY_UNIVERSE_COMMON) {
        std::lock_guard<std::mutex> lk(g->lazy_mu);
        HookScope hs(&g->hook);
        ensure_tcnt(ix, s);
        FOLTY_HIP(hipStreamSynchronize(s));
    }
    std::unique_ptr<Result> res(new Result());
    int64_t tests = 0;
    const uint32_t *count = query_counts(g, q, ws, s, &tests);
    finish_query(g, q, count, ws, res.get(), s, vq && vq->inner == FOLTY_INNER_EXISTS);
    if (vq) finish_vertex(g, *vq, ws, res.get(), s);
    FOLTY_HIP(hipEventRecord(ws.ev[3], s));
    if (!(q.flags & FOLTY_QUERY_NO_COUNTS)) keep_counts(g, count, res.get(), s);
    FOLTY_HIP(hipStreamSynchronize(s));
    fill_stats_from_index(ix, &res->stats);
    res->stats.tests = tests;
    res->stats.n_pairs = (int64_t)res->u.size();
    res->stats.n_certificates = res->n_certificates;
    res->stats.wedge_ms = ev_ms(ws.ev[4], ws.ev[5]);
    res->stats.temporal_ms = ev_ms(ws.ev[5], ws.ev[2]);
    res->stats.threshold_ms = ev_ms(ws.ev[2], ws.ev[3]);
    res->stats.query_ms = ev_ms(ws.ev[0], ws.ev[3]);
    res->stats.filter_passes = ws.filter_passes;
    maybe_one_pass(g, ws, q.delta);
    return res.release();
}

// Device bytes one single query takes beyond the resident index: per-edge
// counts, per-item survivor counts and offsets, survivor slots (at most one per
// triangle), the smaller-side difference array, per-pair certificate counts,
// pair keys and their sorted copies, sort and scan scratch, and the per-edge
// counts handed back.
int64_t query_footprint(const Graph *g, const folty_query &q) {
    const Index &ix = g->ix;
    const int64_t T = std::max<int64_t>(0, ix.T.load());
    // counts; per item su, tri_it, wu, wbase, sbase, ilist; survivors and their
    // groups; pieces; pair step
    int64_t b = 4 * (int64_t)ix.m + 36 * ((int64_t)ix.NI + 1) + 12 * (T + 1) + 4 * (T / 64 + 3) +
                (int64_t)sizeof(Heavy) * heavy_slots(T, -1) + 56 * (int64_t)ix.S;
    if (q.flags & FOLTY_QUERY_SMALLER_SIDE) b += 8 * (int64_t)ix.m + 4;
    if (!(q.flags & FOLTY_QUERY_NO_COUNTS)) b += 4 * ix.m_input;
    // the library scratch the query's sorts and scans ask for (sizes only)
    const int64_t S2 = 2 * (int64_t)ix.S, NI1 = (int64_t)ix.NI + 1;
    const size_t scratch = std::max({sort_pairs_u64_u32(nullptr, 0, nullptr, nullptr, nullptr, nullptr, S2,
                                                        2 * pair_bits(ix.n), nullptr),
                                     exclusive_scan_i64(nullptr, 0, nullptr, nullptr, NI1, nullptr),
                                     exclusive_scan_i32_to_i64(nullptr, 0, nullptr, nullptr, NI1, nullptr),
                                     inclusive_scan_i32(nullptr, 0, nullptr, nullptr, ix.m, nullptr),
                                     exclusive_scan_i32(nullptr, 0, nullptr, nullptr, ix.n, nullptr)});
    return b + (int64_t)scratch + (1 << 20);
}

void fill_stats_from_index(const Index &ix, folty_stats *s) {
    s->n = ix.n;
    s->m_input = ix.m_input;
    s->m = ix.m;
    s->self_loops = ix.self_loops;
    s->static_edges = ix.S;
    s->directed_pairs = ix.P;
    s->max_core = ix.max_core;
    s->max_out_degree = ix.max_out;
    s->wedges = ix.W;
    s->triangles = ix.T;
    s->max_multiplicity = ix.sigma_max;
    s->peel_rounds = ix.peel_rounds;
    s->core_sweeps = ix.core_sweeps;
    s->closing_probes = ix.probes;
    s->enum_items = ix.NI;
    s->build_ms = ix.build_ms;
}

Workspace::~Workspace() {
    if (events)
        for (auto &e : ev) (void)hipEventDestroy(e);
}

size_t Workspace::device_bytes() const {
    const DevBuf *b[] = {&count, &sv, &su, &wu, &wbase, &sbase, &tri_it, &pieces, &gitem, &ncert, &pairs_k, &pairs_v,
                         &pairs_k2, &pairs_v2, &scal, &cub, &ilist, &vtmp, &diff, &tflag, &tinst};
    size_t t = 0;
    for (auto *x : b) t += x->bytes;
    return t;
}

void Workspace::forget_buffers() {
    DevBuf *b[] = {&count, &sv, &su, &wu, &wbase, &sbase, &tri_it, &pieces, &gitem, &ncert, &pairs_k, &pairs_v,
                   &pairs_k2, &pairs_v2, &scal, &cub, &ilist, &vtmp, &diff, &tflag, &tinst};
    for (auto *x : b) x->forget();
}

void Workspace::ensure_events() {
    if (events) return;
    for (auto &e : ev) FOLTY_HIP(hipEventCreate(&e));
    events = true;
}

} // namespace folty
