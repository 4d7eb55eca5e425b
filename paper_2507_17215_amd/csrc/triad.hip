// The exists-exists-exists triadic query: solution triples and temporal
// triangles (paper, Definition of a solution; Section 1, where this prefix is
// identified with temporal triangle counting).
//
// It shares the index and the time-range filter of the exists-exists-forall
// query: the filter keeps the static triangles with a run (triangle, directed
// list E_{a,b}) whose three lists can hold t <= t2 <= t3 <= t + delta, and the
// runs' temporal edges are cut into equal chunks over the grid.  Per chunk:
//   - solutions: the first-entry search of Theorems 3.1 and 3.2 per edge of
//     E_{a,b}, stopping at the first edge with a triangle, sets the run's bit;
//     a run is the ordered triple (a, b, w), so the set bits are the solutions;
//   - temporal triangles (optional): for an edge at time t, with L2[lo, hi) the
//     entries of L2 in [t, t + delta], h3 the first entry of L3 after t + delta
//     and f(j) the first entry of L3 at or after L2[j], the edge closes
//     sum_{j in [lo, hi)} (h3 - f(j)) = (hi - lo) h3 - (F(hi) - F(lo)) pairs,
//     F the running sum of f.  lo, hi, h3 and the two search cursors for f only
//     move forward over a chunk's time-sorted edges, so a chunk costs its edges
//     plus the entries its windows pass, each with a search from the cursor.
// The set bits are then counted item by item over the survivor slots only, and
// listed as (a, b, w) in original ids, sorted by two stable radix sorts (w, then
// the pair key a n + b).
#include <algorithm>
#include <cstring>

#include "tri_device.h"

namespace folty {
namespace {

// first position p in [from, n) with L[p] - t > d (n if none); L ascending
__device__ inline int32_t past_window(const int64_t *__restrict__ L, int32_t from, int32_t n, int64_t t, int64_t d) {
    if (from >= n || L[from] - t > d) return from;
    int32_t a = from + 1, b = n;
    while (a < b) {
        int32_t mid = (a + b) >> 1;
        if (L[mid] - t <= d) a = mid + 1;
        else b = mid;
    }
    return a;
}

struct TriadOut {
    int64_t delta;
    uint32_t *flag;                // bit run of byte (slot & 3) of word slot >> 2
    unsigned long long *inst;      // temporal triangles per input edge, or null
    const int32_t *perm;           // input position of each sorted edge (with inst)
};

// edges [l1s, l1s + cnt) of one run against its lists (L2, L3)
template <bool INST>
__device__ inline void triad_chunk(const TriadOut &o, const int64_t *__restrict__ ts, int32_t l1s, int32_t cnt,
                                   const Span &l2, const Span &l3, int64_t slot, int run, unsigned long long &acc,
                                   bool &ovf) {
    const int64_t *L2 = ts + l2.s, *L3 = ts + l3.s;
    const int32_t n2 = l2.n, n3 = l3.n;
    const int64_t d = o.delta;
    bool any = false;
    if (!INST) {
        int32_t c2 = 0, c3 = 0;
        for (int32_t q = 0; q < cnt; q++) {
            const int64_t t = ts[l1s + q];
            c2 = lower_bound_from(L2, c2, n2, t);
            if (c2 == n2) break; // later edges are no earlier: no t2 for them either
            const int64_t t2 = L2[c2];
            if (t2 - t > d) continue;
            c3 = lower_bound_from(L3, c3, n3, t2);
            if (c3 == n3) break;
            if (L3[c3] - t <= d) {
                any = true;
                break;
            }
        }
    } else {
        int32_t lo = lower_bound_from(L2, 0, n2, ts[l1s]);
        int32_t hi = lo, flo = 0, fhi = 0, h3 = 0;
        unsigned long long Flo = 0, Fhi = 0; // sums of f over L2[lo0, lo) and L2[lo0, hi)
        for (int32_t q = 0; q < cnt; q++) {
            const int32_t e = l1s + q;
            const int64_t t = ts[e];
            while (hi < n2 && L2[hi] - t <= d) {
                fhi = lower_bound_from(L3, fhi, n3, L2[hi]);
                Fhi += (unsigned)fhi;
                hi++;
            }
            while (lo < hi && L2[lo] < t) {
                flo = lower_bound_from(L3, flo, n3, L2[lo]);
                Flo += (unsigned)flo;
                lo++;
            }
            if (lo == hi) {
                if (lo == n2) break; // no t2 at or after t for this or any later edge
                continue;
            }
            h3 = past_window(L3, h3, n3, t, d);
            const unsigned long long pairs = (unsigned long long)(hi - lo) * (unsigned)h3 - (Fhi - Flo);
            if (pairs) {
                any = true;
                if (o.inst) atomicAdd(&o.inst[o.perm[e]], pairs);
                const unsigned long long s = acc + pairs;
                ovf |= s < acc;
                acc = s;
            }
        }
    }
    if (any) atomicOr(&o.flag[slot >> 2], 1u << (((int)(slot & 3) << 3) + run));
}

// one run (I, J) of a surviving triangle inside the chunk [k, k1); r = tests of
// this triangle still to skip.  Returns false once the chunk is used up.
template <int VAR, int I, int J, int RUN, bool INST>
__device__ inline bool triad_run(const TriLists &T, uint32_t dq, const int64_t *ts, int64_t &r, int64_t &k,
                                 int64_t k1, const TriadOut &o, int64_t slot, unsigned long long &acc, bool &ovf) {
    Span l1, l2, l3;
    if (!run_lists<VAR, I, J>(T, dq, l1, l2, l3)) return true;
    if (r >= l1.n) {
        r -= l1.n;
        return true;
    }
    int64_t cnt = l1.n - r;
    if (cnt > k1 - k) cnt = k1 - k;
    triad_chunk<INST>(o, ts, l1.s + (int32_t)r, (int32_t)cnt, l2, l3, slot, RUN, acc, ovf);
    k += cnt;
    r = 0;
    return k < k1;
}

// run numbers: (x0, x1), (x1, x0), (x0, x2), (x2, x0), (x1, x2), (x2, x1)
template <int VAR, bool INST>
__device__ inline void triad_runs(const TriLists &L, uint32_t dq, const int64_t *ts, int64_t &r, int64_t &k,
                                  int64_t k1, const TriadOut &o, int64_t slot, unsigned long long &acc, bool &ovf) {
    if (triad_run<VAR, 0, 1, 0, INST>(L, dq, ts, r, k, k1, o, slot, acc, ovf) &&
        triad_run<VAR, 1, 0, 1, INST>(L, dq, ts, r, k, k1, o, slot, acc, ovf) &&
        triad_run<VAR, 0, 2, 2, INST>(L, dq, ts, r, k, k1, o, slot, acc, ovf) &&
        triad_run<VAR, 2, 0, 3, INST>(L, dq, ts, r, k, k1, o, slot, acc, ovf) &&
        triad_run<VAR, 1, 2, 4, INST>(L, dq, ts, r, k, k1, o, slot, acc, ovf))
        triad_run<VAR, 2, 1, 5, INST>(L, dq, ts, r, k, k1, o, slot, acc, ovf);
}

// The surviving runs' tests, scheduled as the count's (k_tests_light, then the
// pieces of survivors with many tests); total[0] += temporal triangles, total[1]
// = 1 on a 64-bit overflow.
template <int VAR, bool INST> struct TriadRunner {
    static constexpr bool kFlat = false; // a run's tests share their window bookkeeping
    using Flat = FlatLds<false>;
    using Surv = TriLists;
    uint32_t dq;
    const int64_t *ts;
    TriadOut o;
    unsigned long long *total;
    const int32_t *sv;  // survivors as three oriented edges
    const EdgeRec *rec;
    unsigned long long acc = 0;
    bool ovf = false;
    __device__ inline TriLists load(int64_t slot) const {
        return load_lists(rec, sv[3 * slot], sv[3 * slot + 1], sv[3 * slot + 2]);
    }
    __device__ inline int64_t work(const TriLists &L) const { return tri_work<VAR, false>(L, dq); }
    __device__ inline void run(const TriLists &L, int64_t slot, int64_t r, int64_t k1) {
        int64_t k = r;
        triad_runs<VAR, INST>(L, dq, ts, r, k, k1, o, slot, acc, ovf);
    }
    // every lane of the wavefront calls this once, at the end
    __device__ inline void finish() {
        if constexpr (INST) {
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned long long y = __shfl_xor(acc, off);
                const int oy = __shfl_xor((int)ovf, off);
                const unsigned long long s = acc + y;
                ovf = ovf || oy || s < acc;
                acc = s;
            }
            if (lane_id() == 0 && (acc || ovf)) {
                const unsigned long long old = atomicAdd(&total[0], acc);
                if (ovf || old + acc < old) atomicOr(&total[1], 1ull);
            }
        }
    }
};

// The survivors of item u sit in slots [base[u], base[u] + su[u]): per-item
// slots of the one-pass filter (sparse over all triangles) or the compact slots
// of the two-pass one.  The passes below touch only those slots; slot p's bits
// are byte p of the flag array.
__global__ __launch_bounds__(BLK) void k_triad_clear(const int64_t *__restrict__ base, const int32_t *__restrict__ su,
                                                     int32_t NI, uint8_t *__restrict__ flag8) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < NI; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p0 = base[u], p1 = p0 + su[u];
        for (int64_t p = p0; p < p1; p++) flag8[p] = 0;
    }
}

// solutions per item (optional) and their total
__global__ __launch_bounds__(BLK) void k_triad_count(const int64_t *__restrict__ base, const int32_t *__restrict__ su,
                                                     int32_t NI, const uint8_t *__restrict__ flag8,
                                                     int32_t *__restrict__ icnt, unsigned long long *total) {
    unsigned long long c = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < NI; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p0 = base[u], p1 = p0 + su[u];
        int32_t x = 0;
        for (int64_t p = p0; p < p1; p++) x += __popc(flag8[p] & 0x3fu);
        if (icnt) icnt[u] = x;
        c += (unsigned)x;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane_id() == 0 && c) atomicAdd(total, c);
}

// the endpoints (original ids) of oriented edge q: tail, head
__device__ inline void oriented_ends(const uint32_t *__restrict__ oeid, const int32_t *__restrict__ slo,
                                     const int32_t *__restrict__ shi, int32_t q, int32_t &tail, int32_t &head) {
    const uint32_t x = oeid[q];
    const uint32_t s = x & 0x7fffffffu;
    const int32_t lo = slo[s], hi = shi[s];
    tail = (x >> 31) ? lo : hi;
    head = (x >> 31) ? hi : lo;
}

// each set bit as (w, its index, pair key a n + b), from the item's offset
__global__ __launch_bounds__(BLK) void k_triad_emit(const int64_t *__restrict__ base, const int32_t *__restrict__ su,
                                                    int32_t NI, const int64_t *__restrict__ ioff,
                                                    const uint8_t *__restrict__ flag8, const int32_t *__restrict__ sv,
                                                    const uint32_t *__restrict__ oeid, const int32_t *__restrict__ slo,
                                                    const int32_t *__restrict__ shi, int64_t n,
                                                    uint32_t *__restrict__ wkey, int32_t *__restrict__ idx,
                                                    unsigned long long *__restrict__ pkey) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= NI) return;
    const int64_t p0 = base[u], p1 = p0 + su[u];
    int64_t o = ioff[u];
    for (int64_t p = p0; p < p1; p++) {
        const uint32_t bits = flag8[p] & 0x3fu;
        if (!bits) continue;
        int32_t x0, x1, x2, t;
        oriented_ends(oeid, slo, shi, sv[3 * p], x0, x1);
        oriented_ends(oeid, slo, shi, sv[3 * p + 1], t, x2);
        // run -> (a, b, w): (x0,x1,x2) (x1,x0,x2) (x0,x2,x1) (x2,x0,x1) (x1,x2,x0) (x2,x1,x0)
        const int32_t A[6] = {x0, x1, x0, x2, x1, x2};
        const int32_t B[6] = {x1, x0, x2, x0, x2, x1};
        const int32_t W[6] = {x2, x2, x1, x1, x0, x0};
#pragma unroll
        for (int run = 0; run < 6; run++) {
            if (!((bits >> run) & 1u)) continue;
            wkey[o] = (uint32_t)W[run];
            idx[o] = (int32_t)o;
            pkey[o] = (unsigned long long)A[run] * (unsigned long long)n + (unsigned long long)B[run];
            o++;
        }
    }
}

__global__ void k_gather_u64(const unsigned long long *__restrict__ in, const int32_t *__restrict__ idx, int64_t k,
                             unsigned long long *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) out[i] = in[idx[i]];
}

__global__ void k_triad_unpack(const unsigned long long *__restrict__ pkey, const uint32_t *__restrict__ w, int64_t k,
                               int64_t n, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const unsigned long long key = pkey[i];
    out[3 * i] = (int32_t)(key / (unsigned long long)n);
    out[3 * i + 1] = (int32_t)(key % (unsigned long long)n);
    out[3 * i + 2] = (int32_t)w[i];
}


void check_triad(const Graph *g, const folty_triad_query &q) {
    if (!g->ix.built) fail(FOLTY_ENOTBUILT, "folty_build_index has not been called for this graph");
    if (q.delta < 0) fail(FOLTY_EINVAL, "delta must be >= 0 (got %lld)", (long long)q.delta);
    if (q.variant > 7) fail(FOLTY_EINVAL, "variant must be 0..7 (got %u)", (unsigned)q.variant);
    if (q.flags & ~(FOLTY_TRIAD_TRIPLES | FOLTY_TRIAD_INSTANCES | FOLTY_TRIAD_EDGE_INSTANCES))
        fail(FOLTY_EINVAL, "unknown triad flags 0x%x", (unsigned)q.flags);
    for (int i = 0; i < 6; i++)
        if (q.reserved[i]) fail(FOLTY_EINVAL, "reserved fields of the triad query must be 0");
}

// the listed triples, sorted by (a, b, w), copied to res->trip
void list_triples(const Index &ix, const Workspace &ws, int64_t nsol, Result *res, hipStream_t s) {
    if (nsol > INT32_MAX) fail(FOLTY_EOVERFLOW, "%lld solution triples exceed the listing limit of 2^31 - 1",
                               (long long)nsol);
    const int32_t NI = ix.NI;
    DevBuf icnt, ioff, wk, ix0, pk, wk2, ix2, pk2, trip;
    icnt.ensure(4 * (size_t)NI + 4);
    ioff.ensure(8 * (size_t)NI + 8);
    unsigned long long *dummy = ws.scal.as<unsigned long long>() + 12;
    k_fill<unsigned long long><<<1, 1, 0, s>>>(dummy, 0ull, 1);
    k_triad_count<<<grid_for(NI, BLK, PERSIST_BLOCKS), BLK, 0, s>>>(ws.slots, ws.su.as<int32_t>(), NI,
                                                                     ws.tflag.as<uint8_t>(), icnt.as<int32_t>(), dummy);
    FOLTY_LAUNCHED();
    DevBuf cub;
    size_t need = exclusive_scan_i32_to_i64(nullptr, 0, icnt.as<int32_t>(), ioff.as<int64_t>(), NI, s);
    const size_t k = (size_t)nsol;
    const int endw = std::max(1, bit_length((uint64_t)ix.n - 1));
    const int endp = std::max(1, bit_length((uint64_t)ix.n * (uint64_t)ix.n - 1));
    need = std::max(need, sort_pairs_u32_i32(nullptr, 0, nullptr, nullptr, nullptr, nullptr, (int64_t)k, endw, s));
    need = std::max(need, sort_pairs_u64_i32(nullptr, 0, nullptr, nullptr, nullptr, nullptr, (int64_t)k, endp, s));
    cub.ensure(need);
    exclusive_scan_i32_to_i64(cub.p, need, icnt.as<int32_t>(), ioff.as<int64_t>(), NI, s);
    wk.ensure(4 * k);
    ix0.ensure(4 * k);
    pk.ensure(8 * k);
    wk2.ensure(4 * k);
    ix2.ensure(4 * k);
    pk2.ensure(8 * k);
    trip.ensure(12 * k);
    k_triad_emit<<<grid_for(NI, BLK), BLK, 0, s>>>(ws.slots, ws.su.as<int32_t>(), NI, ioff.as<int64_t>(),
                                                   ws.tflag.as<uint8_t>(), ws.sv.as<int32_t>(), ix.oeid.as<uint32_t>(),
                                                   ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), ix.n, wk.as<uint32_t>(),
                                                   ix0.as<int32_t>(), pk.as<unsigned long long>());
    FOLTY_LAUNCHED();
    // by w, then stably by the pair key: (a, b, w) order
    sort_pairs_u32_i32(cub.p, need, wk.as<uint32_t>(), wk2.as<uint32_t>(), ix0.as<int32_t>(), ix2.as<int32_t>(),
                       (int64_t)k, endw, s);
    k_gather_u64<<<grid_for((int64_t)k, BLK), BLK, 0, s>>>(pk.as<unsigned long long>(), ix2.as<int32_t>(),
                                                           (int64_t)k, pk2.as<unsigned long long>());
    FOLTY_LAUNCHED();
    sort_pairs_u64_i32(cub.p, need, pk2.as<uint64_t>(), pk.as<uint64_t>(), wk2.as<int32_t>(), wk.as<int32_t>(),
                       (int64_t)k, endp, s);
    k_triad_unpack<<<grid_for((int64_t)k, BLK), BLK, 0, s>>>(pk.as<unsigned long long>(), wk.as<uint32_t>(),
                                                             (int64_t)k, ix.n, trip.as<int32_t>());
    FOLTY_LAUNCHED();
    res->trip.resize(3 * k);
    FOLTY_HIP(hipMemcpyAsync(res->trip.data(), trip.p, 12 * k, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
}

} // namespace

Result *run_triad_query(Graph *g, const folty_triad_query &q, Workspace &ws) {
    check_triad(g, q);
    if (hipSetDevice(g->device) != hipSuccess) fail(FOLTY_EDEVICE, "hipSetDevice failed");
    Index &ix = g->ix;
    hipStream_t s = g->stream;
    const bool edge = (q.flags & FOLTY_TRIAD_EDGE_INSTANCES) != 0;
    const bool inst = edge || (q.flags & FOLTY_TRIAD_INSTANCES) != 0;
    std::unique_ptr<Result> res(new Result());
    res->triad = true;
    res->device = g->device;
    ws.ensure_events();
    ws.scal.ensure(128);
    ws.host.ensure(64);
    FOLTY_HIP(hipEventRecord(ws.ev[0], s));
    // [0] temporal triangles, [1] overflow, [2] solutions ([8, 12) belong to the filter)
    unsigned long long *tot = ws.scal.as<unsigned long long>();
    k_fill<unsigned long long><<<1, 4, 0, s>>>(tot, 0ull, 4);
    FOLTY_LAUNCHED();
    if (edge) {
        // counted straight into input order (self-loops keep their 0)
        ws.tinst.ensure(8 * (size_t)ix.m_input + 8);
        if (ix.m_input > 0) {
            k_fill<unsigned long long><<<grid_for(ix.m_input, BLK, PERSIST_BLOCKS), BLK, 0, s>>>(
                ws.tinst.as<unsigned long long>(), 0ull, ix.m_input);
            FOLTY_LAUNCHED();
        }
    }
    int64_t tests = 0, tri = 0, slots = 0;
    ws.filter_passes = 0;
    if (ix.NI > 0) {
        int64_t known = -1;
        const bool one = q.delta >= ix.one_pass_from.load(std::memory_order_relaxed);
        slots = find_survivors(ix, q.variant, q.delta, ws, s, ws.ev[4], ws.ev[5], &tri, &known, false, one);
        if (slots > 0) {
            const int64_t nw = (slots + 3) / 4;
            ws.tflag.ensure(4 * (size_t)nw);
            k_triad_clear<<<grid_for(ix.NI, BLK, PERSIST_BLOCKS), BLK, 0, s>>>(ws.slots, ws.su.as<int32_t>(), ix.NI,
                                                                                ws.tflag.as<uint8_t>());
            FOLTY_LAUNCHED();
            TriadOut o{q.delta, ws.tflag.as<uint32_t>(), edge ? ws.tinst.as<unsigned long long>() : nullptr,
                       ix.perm.as<int32_t>()};
            const uint32_t dq = run_slack(range_slack(q.delta, ix.tshift));
            dispatch_variant(q.variant, [&](auto V) {
                constexpr int VAR = decltype(V)::value;
                const int32_t *sv = ws.sv.as<int32_t>();
                const EdgeRec *rec = ix.rec.as<EdgeRec>();
                if (inst)
                    launch_tests(ix, ws, TriadRunner<VAR, true>{dq, ix.ts.as<int64_t>(), o, tot, sv, rec}, slots, known,
                                 s);
                else
                    launch_tests(ix, ws, TriadRunner<VAR, false>{dq, ix.ts.as<int64_t>(), o, tot, sv, rec}, slots,
                                 known, s);
            });
            FOLTY_LAUNCHED();
            k_triad_count<<<grid_for(ix.NI, BLK, PERSIST_BLOCKS), BLK, 0, s>>>(ws.slots, ws.su.as<int32_t>(), ix.NI,
                                                                                ws.tflag.as<uint8_t>(), nullptr, tot + 2);
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipMemcpyAsync(&tests, ws.wbase.as<int64_t>() + ix.NI, 8, hipMemcpyDeviceToHost, s));
        }
    } else {
        FOLTY_HIP(hipEventRecord(ws.ev[4], s));
        FOLTY_HIP(hipEventRecord(ws.ev[5], s));
    }
    if (ix.T < 0) ix.T = tri;
    FOLTY_HIP(hipEventRecord(ws.ev[2], s));
    unsigned long long *h = ws.host.as<unsigned long long>();
    FOLTY_HIP(hipMemcpyAsync(h, tot, 24, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    if (h[1] || h[0] > (unsigned long long)INT64_MAX)
        fail(FOLTY_EOVERFLOW, "the temporal triangles number 2^63 or more");
    res->n_triads = (int64_t)h[2];
    res->n_tinst = inst ? (int64_t)h[0] : -1;
    if ((q.flags & FOLTY_TRIAD_TRIPLES) && res->n_triads > 0)
        list_triples(ix, ws, res->n_triads, res.get(), s);
    FOLTY_HIP(hipEventRecord(ws.ev[3], s));
    if (edge) {
        res->tinst.resize((size_t)ix.m_input);
        if (ix.m_input > 0)
            FOLTY_HIP(hipMemcpyAsync(res->tinst.data(), ws.tinst.p, 8 * (size_t)ix.m_input, hipMemcpyDeviceToHost,
                                     s));
    }
    FOLTY_HIP(hipStreamSynchronize(s));
    fill_stats_from_index(ix, &res->stats);
    res->stats.tests = tests;
    res->stats.wedge_ms = ev_ms(ws.ev[4], ws.ev[5]);
    res->stats.temporal_ms = ev_ms(ws.ev[5], ws.ev[2]);
    res->stats.threshold_ms = ev_ms(ws.ev[2], ws.ev[3]);
    res->stats.query_ms = ev_ms(ws.ev[0], ws.ev[3]);
    res->stats.filter_passes = ws.filter_passes;
    maybe_one_pass(g, ws, q.delta);
    return res.release();
}

} // namespace folty
