// Device code shared by the single-query kernels (query.hip) and the batched
// engine (batch.hip): triangle enumeration, the exact run filter, the temporal
// tests.  See query.hip for what each step computes and where the paper says so.
#pragma once

#include <cstdlib>

#include "folty_internal.h"

namespace folty {
namespace {

constexpr int BLK = 256;
constexpr int WPB = BLK / 64;         // wavefronts per block
constexpr int CAP = 512;              // N+(u) staged in LDS up to this length
constexpr int PERSIST_BLOCKS = 4096;
constexpr int ENUM_BLOCKS = 32768; // 8 x the resident blocks: about a dozen items per wavefront, balanced by the dispatcher
constexpr int32_t CHUNK = 4096;       // closing probes per enumeration item (about; whole segments)

__device__ inline int lane_id() { return __lane_id(); }

// A pointer field of a table in device memory (a plan's per-job records), read
// as a pointer to global memory.  The compiler cannot tell where such a pointer
// points and would use flat instructions, whose completion shares one wait
// counter with LDS and scalar loads (so every LDS wait would also wait for the
// global loads in flight).
template <class T> __device__ inline T *global_ptr(T *const &field) {
    __attribute__((address_space(1))) T *g;
    __builtin_memcpy(&g, &field, sizeof g);
    return (T *)g;
}

// this wavefront's index in its block, as a value the compiler knows is uniform
// (so what is indexed by it is loaded into scalar registers)
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ inline unsigned long long lanes_below() { return (1ull << lane_id()) - 1ull; }

// make this wavefront's LDS writes visible to all of its lanes
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int32_t wave_append(int32_t *counter, bool pred) {
    unsigned long long mask = __ballot(pred);
    if (!mask) return -1;
    int lane = lane_id();
    int leader = __ffsll((long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (int32_t)__popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + (int32_t)__popcll(mask & lanes_below()) : -1;
}

template <class T> __device__ inline T wave_inclusive_sum(T x) {
    const int lane = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// the predicate code as a compile-time constant for kernel templates
template <class F> void dispatch_variant(int v, F &&f) {
    switch (v) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    default: f(std::integral_constant<int, 7>{}); break;
    }
}

template <class T> __global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// directed lists of a triangle
// ---------------------------------------------------------------------------
struct Span {
    int32_t s, n;     // start in ts, length
    uint32_t lo, hi;  // first and last timestamp >> tshift
};

// D[i][j] = E_{x_i, x_j} for the triangle's vertices x0 < x1 < x2 (by rank)
struct TriLists {
    Span d01, d10, d02, d20, d12, d21;
    template <int I, int J> __device__ inline const Span &get() const {
        static_assert(I != J, "");
        if constexpr (I == 0 && J == 1) return d01;
        else if constexpr (I == 1 && J == 0) return d10;
        else if constexpr (I == 0 && J == 2) return d02;
        else if constexpr (I == 2 && J == 0) return d20;
        else if constexpr (I == 1 && J == 2) return d12;
        else return d21;
    }
};

// STARTS: also the lists' starts in ts (the filter needs only lengths and ranges)
template <bool STARTS>
__device__ inline void rec_spans(const EdgeRec *__restrict__ rec, int32_t p, Span &fwd, Span &bwd) {
    const uint4 *q = reinterpret_cast<const uint4 *>(rec + p);
    if constexpr (STARTS) {
        const uint4 a = q[0];
        fwd.n = (int32_t)a.x;
        bwd.n = (int32_t)a.y;
        fwd.s = (int32_t)a.z;
        bwd.s = (int32_t)a.w;
    } else {
        const uint2 a = *reinterpret_cast<const uint2 *>(q);
        fwd.n = (int32_t)a.x;
        bwd.n = (int32_t)a.y;
        fwd.s = bwd.s = 0;
    }
    const uint4 b = q[1];
    fwd.lo = b.x;
    fwd.hi = b.y;
    bwd.lo = b.z;
    bwd.hi = b.w;
}

// the three oriented edges (x0,x1), (x0,x2), (x1,x2) of a triangle
template <bool STARTS = true>
__device__ inline TriLists load_lists(const EdgeRec *__restrict__ rec, int32_t p01, int32_t p02, int32_t p12) {
    TriLists L;
    rec_spans<STARTS>(rec, p01, L.d01, L.d10);
    rec_spans<STARTS>(rec, p02, L.d02, L.d20);
    rec_spans<STARTS>(rec, p12, L.d12, L.d21);
    return L;
}

// Slack of the run test below in timestamps >> tshift: the range slack of the
// window bound, saturated to 32 bits (no difference of two such values exceeds it).
__host__ __device__ inline uint32_t run_slack(int64_t dq) {
    return dq >= (int64_t)0xffffffffu ? 0xffffffffu : (uint32_t)dq;
}

// The predicate code picks, for L1 = E_{a,b} (a = x_I, b = x_J, third w = x_C),
// L2 between X and w and L3 between Y and w (see folty.h for the bits).
template <int VAR, int I, int J> struct Pick {
    static constexpr int C = 3 - I - J;
    static constexpr int X = (VAR & 4) ? J : I;
    static constexpr int Y = (VAR & 4) ? I : J;
    static constexpr int L2a = (VAR & 1) ? C : X, L2b = (VAR & 1) ? X : C;
    static constexpr int L3a = (VAR & 2) ? C : Y, L3b = (VAR & 2) ? Y : C;
};

// A run can only count if all three lists are non-empty and some t <= t2 <= t3
// <= t + dmax is possible given each list's first and last timestamp.  The test
// reads the timestamps shifted right by tshift with slack dq = run_slack(
// range_slack(dmax, tshift)): a run it drops has no such t, t2, t3 (floors keep
// order, and floors of two values differ by at most one more unit than the
// values do); with tshift = 0 it is exact.  A run it keeps without such a
// window only adds tests that find nothing.
template <int VAR, int I, int J>
__device__ inline bool run_lists(const TriLists &T, uint32_t dq, Span &l1, Span &l2, Span &l3) {
    using P = Pick<VAR, I, J>;
    l1 = T.template get<I, J>();
    l2 = T.template get<P::L2a, P::L2b>();
    l3 = T.template get<P::L3a, P::L3b>();
    if (l1.n == 0 || l2.n == 0 || l3.n == 0) return false;
    if (l2.hi < l1.lo || l3.hi < l2.lo) return false;
    if ((l2.lo > l1.hi && l2.lo - l1.hi > dq) || (l3.lo > l1.hi && l3.lo - l1.hi > dq)) return false;
    return true;
}

// Tests of a run: |L1|, or with SS the shorter of |L1| and |L2| (the side the
// run is evaluated from; see chunk_run).
template <bool SS> __device__ inline int32_t run_tests(const Span &l1, const Span &l2) {
    return SS && l2.n < l1.n ? l2.n : l1.n;
}

template <int VAR, int I, int J, bool SS = false> __device__ inline int64_t run_work(const TriLists &T, uint32_t dq) {
    Span a, b, c;
    return run_lists<VAR, I, J>(T, dq, a, b, c) ? run_tests<SS>(a, b) : 0;
}

template <int VAR, bool SS = false> __device__ inline int64_t tri_work(const TriLists &T, uint32_t dq) {
    return run_work<VAR, 0, 1, SS>(T, dq) + run_work<VAR, 1, 0, SS>(T, dq) + run_work<VAR, 0, 2, SS>(T, dq) +
           run_work<VAR, 2, 0, SS>(T, dq) + run_work<VAR, 1, 2, SS>(T, dq) + run_work<VAR, 2, 1, SS>(T, dq);
}

// runtime predicate code (one code per job in a batch)
__device__ inline int64_t tri_work_rt(int variant, const TriLists &T, uint32_t dq) {
    switch (variant) {
    case 0: return tri_work<0>(T, dq);
    case 1: return tri_work<1>(T, dq);
    case 2: return tri_work<2>(T, dq);
    case 3: return tri_work<3>(T, dq);
    case 4: return tri_work<4>(T, dq);
    case 5: return tri_work<5>(T, dq);
    case 6: return tri_work<6>(T, dq);
    default: return tri_work<7>(T, dq);
    }
}

// first position p in [from, n) with L[p] >= key (n if none)
__device__ inline int32_t lower_bound_from(const int64_t *__restrict__ L, int32_t from, int32_t n, int64_t key) {
    if (from >= n || L[from] >= key) return from;
    int32_t a = from + 1, b = n;
    while (a < b) {
        int32_t mid = (a + b) >> 1;
        if (L[mid] < key) a = mid + 1;
        else b = mid;
    }
    return a;
}

// Entry k of a list of at most two entries, from its record's first and last
// timestamps (exact when the timestamps fit 32 bits, tshift = 0).
__device__ inline int64_t short_at(const Span &l, int32_t k) { return (int64_t)(k == 0 ? l.lo : l.hi); }
__device__ inline int32_t short_lower_bound(const Span &l, int32_t from, int64_t key) {
    int32_t p = from;
    while (p < l.n && short_at(l, p) < key) p++;
    return p;
}

// cnt consecutive temporal edges of L1 starting at l1s against (L2, L3).  With
// SHORT and `inl` (timestamps below 2^32) a list of one or two entries is read
// from its span's first and last timestamps instead of ts: most lists are that
// short, and their entries are scattered reads that no neighbouring test
// shares.  (A compile-time switch: the branches cost registers where unused.)
template <bool SHORT> struct DirectOpT {
    static constexpr bool kShort = SHORT;
    int64_t delta;
    uint32_t *count;
    int32_t *diff = nullptr; // per sorted edge + 1: +1 / -1 at the ends of edge ranges (interval evaluation)
    bool inl = false;
    __device__ inline void operator()(const int64_t *__restrict__ ts, int32_t l1s, int32_t cnt, const Span &l2,
                                      const Span &l3) const {
        const int64_t *L2 = ts + l2.s, *L3 = ts + l3.s;
        const bool s2 = SHORT && inl && l2.n <= 2, s3 = SHORT && inl && l3.n <= 2;
        int32_t c2 = 0, c3 = 0;
        for (int32_t q = 0; q < cnt; q++) {
            int32_t e = l1s + q;
            int64_t t = ts[e];
            c2 = s2 ? short_lower_bound(l2, c2, t) : lower_bound_from(L2, c2, l2.n, t);
            if (c2 == l2.n) break; // later edges are no earlier: no t2 for them either
            int64_t t2 = s2 ? short_at(l2, c2) : L2[c2];
            if (t2 - t > delta) continue;
            c3 = s3 ? short_lower_bound(l3, c3, t2) : lower_bound_from(L3, c3, l3.n, t2);
            if (c3 == l3.n) break;
            if ((s3 ? short_at(l3, c3) : L3[c3]) - t <= delta) atomicAdd(&count[e], 1u);
        }
    }

    // The same run evaluated from L2 (paper, the in-neighbour theorem: e forms
    // a triangle with w iff some entry t2 of L2, with t3 the first entry of L3
    // at or after t2 and t3 - t2 <= delta, has t3 - delta <= t(e) <= t2).
    // Those intervals have non-decreasing ends, so entry j adds exactly the
    // times in [max(t3 - delta, t2' + 1), t2] (t2' the entry before it) to the
    // union of the earlier ones; each such piece is a range of L1 marked +1 / -1
    // in diff, whose prefix sum over the sorted edges adds one per third vertex.
    // Entries [j0, j0 + cnt) of L2.
    __device__ inline void iv(const int64_t *__restrict__ ts, const Span &l1, int32_t j0, int32_t cnt,
                              const Span &l2, const Span &l3) const {
        const int64_t *L1 = ts + l1.s, *L2 = ts + l2.s, *L3 = ts + l3.s;
        int32_t c3 = 0, a = 0, b = 0;
        for (int32_t q = 0; q < cnt; q++) {
            const int32_t j = j0 + q;
            const int64_t t2 = L2[j];
            c3 = lower_bound_from(L3, c3, l3.n, t2);
            if (c3 == l3.n) break; // no t3 for this or any later entry
            const int64_t t3 = L3[c3];
            if (t3 - t2 > delta) continue; // an empty interval
            int64_t lo = t3 - delta;
            if (j > 0 && L2[j - 1] + 1 > lo) lo = L2[j - 1] + 1;
            if (lo > t2) continue;
            a = lower_bound_from(L1, a, l1.n, lo);
            b = lower_bound_from(L1, a > b ? a : b, l1.n, t2 + 1);
            if (a < b) {
                atomicAdd(&diff[l1.s + a], 1);
                atomicAdd(&diff[l1.s + b], -1);
            }
        }
    }
};
using DirectOp = DirectOpT<false>;      // plain tests (also the interval evaluation)
using DirectShortOp = DirectOpT<true>;  // short lists from their spans' end timestamps

// the smallest window per (e, w) into a histogram over sorted window levels:
// level j counts w whose smallest window lies in (lv[j-1], lv[j]]
struct PoolOp {
    const int64_t *lv;
    int nl, nls;
    uint32_t *hist;
    unsigned long long *tmask; // per tile of 64 edges: bit e & 63 set once a counter of edge e is non-zero
    __device__ inline void operator()(const int64_t *__restrict__ ts, int32_t l1s, int32_t cnt, const Span &l2,
                                      const Span &l3) const {
        const int64_t *L2 = ts + l2.s, *L3 = ts + l3.s;
        const int64_t dmax = lv[nl - 1];
        int32_t c2 = 0, c3 = 0;
        for (int32_t q = 0; q < cnt; q++) {
            int32_t e = l1s + q;
            int64_t t = ts[e];
            c2 = lower_bound_from(L2, c2, l2.n, t);
            if (c2 == l2.n) break;
            int64_t t2 = L2[c2];
            if (t2 - t > dmax) continue;
            c3 = lower_bound_from(L3, c3, l3.n, t2);
            if (c3 == l3.n) break;
            int64_t win = L3[c3] - t;
            if (win > dmax) continue;
            int a = 0, b = nl;
            while (a < b) {
                int mid = (a + b) >> 1;
                if (lv[mid] < win) a = mid + 1;
                else b = mid;
            }
            if (atomicAdd(&hist[hist_at(e, a, nls)], 1u) == 0u) atomicOr(&tmask[e >> 6], 1ull << (e & 63));
        }
    }
};

// one run of a surviving triangle within the chunk [k, k1); r = tests of this
// triangle still to skip.  Returns false once the chunk is used up.  With SS (and
// a filter that counted tests the same way) a run whose L2 is shorter than L1
// has |L2| tests, the entries of L2, and is evaluated from them.
template <int VAR, int I, int J, class Op, bool SS = false>
__device__ inline bool chunk_run(const TriLists &T, uint32_t dq, const int64_t *ts, int64_t &r, int64_t &k,
                                 int64_t k1, const Op &op) {
    Span l1, l2, l3;
    if (!run_lists<VAR, I, J>(T, dq, l1, l2, l3)) return true;
    const int32_t w = run_tests<SS>(l1, l2);
    if (r >= w) {
        r -= w;
        return true;
    }
    int64_t cnt = w - r;
    if (cnt > k1 - k) cnt = k1 - k;
    if constexpr (SS) {
        if (w < l1.n) op.iv(ts, l1, (int32_t)r, (int32_t)cnt, l2, l3);
        else op(ts, l1.s + (int32_t)r, (int32_t)cnt, l2, l3);
    } else {
        op(ts, l1.s + (int32_t)r, (int32_t)cnt, l2, l3);
    }
    k += cnt;
    r = 0;
    return k < k1;
}

// ---------------------------------------------------------------------------
// a.5: triangle enumeration, one wavefront per lowest vertex u
// ---------------------------------------------------------------------------
// Sinks receive every probe: hit(h, p_uv, p_uw, p_vw) is called by all lanes of
// the wave together (h = this lane found a triangle), so sinks may use ballots.
struct CountSink {
    static constexpr bool kCompact = false;
    int32_t *tri_u;
    int32_t c;
    __device__ void begin(int64_t) { c = 0; }
    __device__ void hit(bool h, int32_t, int32_t, int32_t) { c += (int32_t)__popcll(__ballot(h)); }
    __device__ void end(int64_t u) {
        if (lane_id() == 0) tri_u[u] = c;
    }
    __device__ void prefetch(int32_t, int32_t, bool) {}
    __device__ void finish() {}
};

struct CacheSink {
    static constexpr bool kCompact = false;
    const int64_t *base;
    int32_t *tri;
    int64_t slot;
    __device__ void begin(int64_t u) { slot = base[u]; }
    __device__ void hit(bool h, int32_t a, int32_t b, int32_t c) {
        unsigned long long mask = __ballot(h);
        if (h) {
            int64_t pos = slot + __popcll(mask & lanes_below());
            tri[3 * pos] = a;
            tri[3 * pos + 1] = b;
            tri[3 * pos + 2] = c;
        }
        slot += __popcll(mask);
    }
    __device__ void end(int64_t) {}
    __device__ void prefetch(int32_t, int32_t, bool) {}
    __device__ void finish() {}
};

struct TcntSink {
    static constexpr bool kCompact = false;
    const uint32_t *oeid;
    int32_t *tcnt;
    __device__ void begin(int64_t) {}
    __device__ void hit(bool h, int32_t a, int32_t b, int32_t c) {
        if (h) {
            atomicAdd(&tcnt[oeid[a] & 0x7fffffffu], 1);
            atomicAdd(&tcnt[oeid[b] & 0x7fffffffu], 1);
            atomicAdd(&tcnt[oeid[c] & 0x7fffffffu], 1);
        }
    }
    __device__ void end(int64_t) {}
    __device__ void prefetch(int32_t, int32_t, bool) {}
    __device__ void finish() {}
};

// Slack of the range test on timestamps shifted right by `shift`: floors of two
// values differ by at most one unit more than their difference does.
__host__ __device__ inline int64_t range_slack(int64_t dmax, int32_t shift) {
    return shift ? (dmax >> shift) + 1 : dmax;
}

// two oriented edges can share a run only if their time ranges come within dmax
__device__ inline bool ranges_meet(uint2 x, uint2 y, int64_t dq) {
    return (int64_t)x.x - (int64_t)y.y <= dq && (int64_t)y.x - (int64_t)x.y <= dq;
}

// What a filter pass does with the triangles it keeps.
enum FilterMode {
    FILTER_COUNT = 0, // survivors and tests per item, triangles seen; writes no survivor
    FILTER_EMIT = 1,  // survivors into their item's slots (offsets from a counting pass)
    FILTER_BOTH = 2,  // both, into slots sized by the item's triangle count
};

// Keeps triangles with at least one run that can count, with each survivor's
// test offset inside its item.  Every run uses one list of each of the three
// edges, and its three timestamps lie within dmax of each other, so the edges'
// time ranges must pairwise come within dmax: the two ranges loaded before the
// exact search are tested first, the third edge's range is loaded only if they
// meet (8 bytes each), and only then are the three edge records read.  The enumeration order inside an item is fixed, so a
// counting pass and a later emitting pass agree on every survivor's position.
// VAR < 0: the predicate code is read from `variant` at run time
template <int VAR, int MODE, bool SS = false> struct FilterSink {
    // a run-time predicate code inlines all eight tests: keep the enumeration's
    // code small (one copy of the sink) for those
    static constexpr bool kCompact = VAR < 0;
    const int64_t *base; // EMIT, BOTH: first survivor slot of each item
    const EdgeRec *rec;
    const uint2 *rng; // per oriented edge: (first, last) timestamp >> shift
    int64_t dq;       // range_slack(dmax, shift)
    int variant;
    int32_t *sv;      // EMIT, BOTH: survivors (three oriented edges each)
    int64_t *sw;      // EMIT, BOTH: test offset of each survivor inside its item (null: not kept)
    int32_t *su;      // COUNT, BOTH: survivors per item
    int64_t *wu;      // COUNT, BOTH: tests per item
    unsigned long long *hits; // COUNT: triangles seen (added once per wavefront)
    int32_t *tri_it;  // COUNT: triangles of each item (null: not kept)
    int64_t slot;
    int32_t ns;
    int32_t nt;
    int64_t work;
    unsigned long long nhit;
    uint2 pra, prk; // ranges of edge (x0, x1) and of the known one of (x0, x2) / (x1, x2)
    bool pkb;       // the known one is (x0, x2)
    // called for every probe that may hit, before hit(): edge (x0, x1) and one of
    // the other two are known before the search that finds the third
    __device__ void prefetch(int32_t a, int32_t k, bool k_is_b) {
        pra = rng[a];
        prk = rng[k];
        pkb = k_is_b;
    }
    __device__ void begin(int64_t it) {
        if constexpr (MODE != FILTER_COUNT) slot = base[it];
        ns = 0;
        nt = 0;
        work = 0;
    }
    __device__ void hit(bool h, int32_t a, int32_t b, int32_t c) {
        if constexpr (MODE == FILTER_COUNT) nt += (int32_t)__popcll(__ballot(h));
        int64_t wk = 0;
        // the two ranges loaded ahead first; the third edge's only if they meet
        if (h && ranges_meet(pra, prk, dq)) {
            const uint2 r3 = rng[pkb ? c : b];
            if (ranges_meet(pra, r3, dq) && ranges_meet(prk, r3, dq)) {
                if constexpr (VAR >= 0) wk = tri_work<VAR, SS>(load_lists<false>(rec, a, b, c), run_slack(dq));
                else wk = tri_work_rt(variant, load_lists<false>(rec, a, b, c), run_slack(dq));
            }
        }
        bool keep = wk > 0;
        unsigned long long mask = __ballot(keep);
        if (!mask) return;
        int64_t incl = wave_inclusive_sum(wk);
        if constexpr (MODE != FILTER_COUNT) {
            if (keep) {
                int64_t pos = slot + ns + __popcll(mask & lanes_below());
                sv[3 * pos] = a;
                sv[3 * pos + 1] = b;
                sv[3 * pos + 2] = c;
                if (sw) sw[pos] = work + incl - wk;
            }
        }
        ns += (int32_t)__popcll(mask);
        work += __shfl(incl, 63);
    }
    __device__ void end(int64_t it) {
        if constexpr (MODE != FILTER_EMIT) {
            if (lane_id() == 0) {
                su[it] = ns;
                wu[it] = work;
            }
        }
        if constexpr (MODE == FILTER_COUNT) {
            nhit += (unsigned long long)nt;
            if (tri_it && lane_id() == 0) tri_it[it] = nt;
        }
    }
    __device__ void finish() {
        if constexpr (MODE == FILTER_COUNT) {
            if (lane_id() == 0 && nhit) atomicAdd(hits, nhit);
        }
    }
};

// What the filter needs of one predicate code and window bound.
struct JobFilter {
    int64_t dq;
    int variant;
    int32_t *sv;
    int64_t *sw;
    int32_t *su;
    int64_t *wu;
};

// FILTER_BOTH for two predicate codes over the same triangles (a plan's two
// jobs on one graph): one enumeration and one read of the edges' ranges per
// triangle; each code then reads the three edge records for itself (the second
// read hits the cache), so only one code's lists are live at a time, and keeps
// its survivors in its own slots.
struct PairFilterSink {
    static constexpr bool kCompact = true;
    const int64_t *base; // first slot of each item (the graph's triangle offsets)
    const EdgeRec *rec;
    const uint2 *rng;
    JobFilter f[2];
    int64_t slot;
    int32_t ns[2];
    int64_t work[2];
    uint2 pra, prk;
    bool pkb;
    __device__ void prefetch(int32_t a, int32_t k, bool k_is_b) {
        pra = rng[a];
        prk = rng[k];
        pkb = k_is_b;
    }
    __device__ void begin(int64_t it) {
        slot = base[it];
        ns[0] = ns[1] = 0;
        work[0] = work[1] = 0;
    }
    template <int J> __device__ void keep(bool pass, int32_t a, int32_t b, int32_t c) {
        const int64_t wk = pass ? tri_work_rt(f[J].variant, load_lists<false>(rec, a, b, c), run_slack(f[J].dq)) : 0;
        const bool kp = wk > 0;
        const unsigned long long mask = __ballot(kp);
        if (!mask) return;
        const int64_t incl = wave_inclusive_sum(wk);
        if (kp) {
            const int64_t pos = slot + ns[J] + __popcll(mask & lanes_below());
            f[J].sv[3 * pos] = a;
            f[J].sv[3 * pos + 1] = b;
            f[J].sv[3 * pos + 2] = c;
            f[J].sw[pos] = work[J] + incl - wk;
        }
        ns[J] += (int32_t)__popcll(mask);
        work[J] += __shfl(incl, 63);
    }
    __device__ void hit(bool h, int32_t a, int32_t b, int32_t c) {
        bool p0 = false, p1 = false;
        const int64_t dq = f[0].dq > f[1].dq ? f[0].dq : f[1].dq;
        if (h && ranges_meet(pra, prk, dq)) {
            const uint2 r3 = rng[pkb ? c : b];
            p0 = ranges_meet(pra, prk, f[0].dq) && ranges_meet(pra, r3, f[0].dq) && ranges_meet(prk, r3, f[0].dq);
            p1 = ranges_meet(pra, prk, f[1].dq) && ranges_meet(pra, r3, f[1].dq) && ranges_meet(prk, r3, f[1].dq);
        }
        keep<0>(p0, a, b, c);
        keep<1>(p1, a, b, c);
    }
    __device__ void end(int64_t it) {
        if (lane_id() == 0)
            for (int j = 0; j < 2; j++) {
                f[j].su[it] = ns[j];
                f[j].wu[it] = work[j];
            }
    }
    __device__ void finish() {}
};

// LDS of one wavefront's enumeration item: the owner's out-row N+(w), the
// item's probe segments, and a bitmap with one hash bit per vertex of N+(w), so
// a probe whose bit is clear misses without a search.  The other probes (the
// hits and a few collisions) wait in a queue until 64 of them fill a wavefront,
// which then searches N+(w) exactly and hands its triangles to the sink.  7 KB
// per wavefront.
constexpr int ITEM_SEGS = 128;              // probe segments per item
constexpr int BM_LOG = 12;                  // 4096 bits
constexpr int BM_WORDS = 1 << (BM_LOG - 5);
constexpr int QCAP = 128;                   // < 64 waiting + one step's 64
constexpr int ENUM_UNROLL = 4;              // probe steps whose loads overlap
constexpr int Q_SHIFT = 13;                 // probes of an item < CHUNK + CAP <= 2^13
struct EnumLds {
    int32_t nu[CAP];        // N+(w), ascending
    int32_t off[ITEM_SEGS]; // row start of segment i minus PRE[i]: probe q reads oadj[off[i] + q]
    int32_t pre[ITEM_SEGS]; // PRE[i+1] = total row length of segments j <= i
    int32_t pm[ITEM_SEGS];  // oriented edge (u, v) of segment i | mode B << 31
    uint32_t bm[BM_WORDS];
    int32_t qx[QCAP];       // waiting probes: x
    int32_t qr[QCAP];       // and q | i << Q_SHIFT
};
static_assert(CHUNK + CAP <= (1 << Q_SHIFT) && ITEM_SEGS <= (1 << (31 - Q_SHIFT)), "queue packing");

__device__ inline uint32_t bm_hash(int32_t x) { return ((uint32_t)x * 0x9E3779B1u) >> (32 - BM_LOG); }

constexpr uint32_t MODE_B = 0x80000000u;

// Hands the triangle of segment edge (u, v) = pm, probe position p and owner-row
// position pw to the sink as (edge (x0,x1), edge (x0,x2), edge (x1,x2)):
// mode A: p is in v's row, pw in u's;  mode B: p is in u's row, pw in v's.
__device__ inline void tri_edges(int32_t pm, int32_t p, int32_t pw, int32_t &e01, int32_t &e02, int32_t &e12) {
    e01 = (int32_t)((uint32_t)pm & ~MODE_B);
    if ((uint32_t)pm & MODE_B) {
        e02 = p;
        e12 = pw;
    } else {
        e02 = pw;
        e12 = p;
    }
}

// the first cnt waiting probes, one per lane: exact search of x in N+(w)
template <class Sink>
__device__ inline void enum_batch(int32_t b, int32_t d, const EnumLds &L, int32_t cnt, Sink &sink) {
    const int lane = lane_id();
    bool hit = false;
    int32_t e01 = 0, e02 = 0, e12 = 0;
    if (lane < cnt) {
        const int32_t x = L.qx[lane], r = L.qr[lane];
        const int32_t i = r >> Q_SHIFT;
        const int32_t pm = L.pm[i];
        const int32_t p = L.off[i] + (r & ((1 << Q_SHIFT) - 1));
        sink.prefetch((int32_t)((uint32_t)pm & ~MODE_B), p, ((uint32_t)pm & MODE_B) != 0);
        int32_t a = 0, c = d;
        while (a < c) {
            int32_t mid = (a + c) >> 1;
            if (L.nu[mid] < x) a = mid + 1;
            else c = mid;
        }
        hit = a < d && L.nu[a] == x;
        tri_edges(pm, p, b + a, e01, e02, e12);
    }
    sink.hit(hit, e01, e02, e12);
}

// The first 64 entries of an item's owner row and of its segments (this
// lane's), loaded one item ahead.
struct StageAhead {
    int32_t v;
    int4 sg;
};

__device__ inline StageAhead stage_ahead(const EnumItem &item, const int32_t *__restrict__ oadj,
                                         const int4 *__restrict__ seg) {
    StageAhead a{0, make_int4(0, 0, 0, 0)};
    const int lane = lane_id();
    if (item.d >= 1 && item.d <= CAP && item.nq > 0) {
        if (lane < item.d) a.v = oadj[item.b + lane];
        if (lane < item.ng) a.sg = seg[item.g0 + lane];
    }
    return a;
}

// One wavefront per item: the owner's out-row and the item's segments, whose
// rows are probed as one flat range q in [0, nq).  Sinks see the triangles of
// an item in a fixed order.
template <class Sink>
__device__ inline void enum_item(const EnumItem &item, const StageAhead &ahead, const int32_t *__restrict__ oadj,
                                 const int4 *__restrict__ seg, int64_t it, Sink &sink, EnumLds &L) {
    const int lane = lane_id();
    const int32_t b = item.b, d = item.d, ng = item.ng, nq = item.nq;
    sink.begin(it);
    if (d >= 1 && d <= CAP && nq > 0) {
        // stage N+(w) and its hash bits, then the segments with a prefix of
        // their row lengths
        for (int w = lane; w < BM_WORDS; w += 64) L.bm[w] = 0;
        for (int32_t i = lane; i < d; i += 64) L.nu[i] = i < 64 ? ahead.v : oadj[b + i];
        wave_sync();
        for (int32_t i = lane; i < d; i += 64) {
            const uint32_t h = bm_hash(L.nu[i]);
            atomicOr(&L.bm[h >> 5], 1u << (h & 31));
        }
        int32_t carry = 0;
        for (int32_t i0 = 0; i0 < ng; i0 += 64) {
            const int32_t i = i0 + lane;
            int4 sg = make_int4(0, 0, 0, 0);
            if (i < ng) sg = i0 == 0 ? ahead.sg : seg[item.g0 + i];
            const int32_t x = wave_inclusive_sum(sg.y);
            if (i < ng) {
                L.pre[i] = carry + x;
                L.off[i] = sg.x - (carry + x - sg.y);
                L.pm[i] = sg.z;
            }
            carry += __shfl(x, 63);
        }
        wave_sync();
        int32_t i = 0;  // this lane's segment; q only grows, so i only grows
        int32_t qn = 0; // waiting probes (wave-uniform)
        // one probe step's candidates into the queue; a full wavefront of them
        // (or, at the end, whatever waits) goes to the sink
        auto enqueue = [&](bool v, int32_t x, int32_t r, bool last) {
            bool cand = false;
            if (v) {
                const uint32_t h = bm_hash(x);
                cand = (L.bm[h >> 5] >> (h & 31)) & 1u;
            }
            const unsigned long long mask = __ballot(cand);
            if (cand) {
                const int32_t slot = qn + (int32_t)__popcll(mask & lanes_below());
                L.qx[slot] = x;
                L.qr[slot] = r;
            }
            qn += (int32_t)__popcll(mask);
            if (qn >= 64 || (last && qn > 0)) {
                const int32_t cnt = qn < 64 ? qn : 64;
                wave_sync();
                enum_batch(b, d, L, cnt, sink);
                const int32_t rest = qn - cnt;
                int32_t tx = 0, tr = 0;
                if (lane < rest) {
                    tx = L.qx[64 + lane];
                    tr = L.qr[64 + lane];
                }
                wave_sync();
                if (lane < rest) {
                    L.qx[lane] = tx;
                    L.qr[lane] = tr;
                }
                qn = rest;
                wave_sync();
            }
        };
        // ENUM_UNROLL steps of 64 probes at a time: their loads of x are all in
        // flight before the first is used.  A last pass without probes hands over
        // the probes still waiting.
        for (int32_t q0 = 0;; q0 += 64 * ENUM_UNROLL) {
            const bool more = q0 < nq;
            int32_t rk[ENUM_UNROLL], xk[ENUM_UNROLL];
            bool vk[ENUM_UNROLL];
#pragma unroll
            for (int k = 0; k < ENUM_UNROLL; k++) {
                const int32_t q = q0 + 64 * k + lane;
                vk[k] = q < nq;
                xk[k] = 0;
                rk[k] = 0;
                if (vk[k]) {
                    // the segment of q (the i with PRE[i] <= q < PRE[i+1]); walk a few
                    // segments forward before bisecting.  PRE[ng] = nq > q stops both.
                    for (int w = 0; w < 4 && L.pre[i] <= q; w++) i++;
                    if (L.pre[i] <= q) {
                        int32_t lo = i + 1, hi = ng;
                        while (lo < hi) {
                            int32_t mid = (lo + hi) >> 1;
                            if (L.pre[mid] <= q) lo = mid + 1;
                            else hi = mid;
                        }
                        i = lo;
                    }
                    xk[k] = L.off[i] + q; // position of x, replaced by x below
                    rk[k] = q | (i << Q_SHIFT);
                }
            }
#pragma unroll
            for (int k = 0; k < ENUM_UNROLL; k++) xk[k] = vk[k] ? oadj[xk[k]] : 0;
            if constexpr (Sink::kCompact) {
                // the steps enter the queue in a loop that is not unrolled (each
                // step's values move down one register), so the sink's code is
                // generated once
                const int steps = more ? ENUM_UNROLL : 1;
#pragma unroll 1
                for (int k = 0; k < steps; k++) {
                    enqueue(vk[0], xk[0], rk[0], !more);
#pragma unroll
                    for (int j = 0; j + 1 < ENUM_UNROLL; j++) {
                        xk[j] = xk[j + 1];
                        rk[j] = rk[j + 1];
                        vk[j] = vk[j + 1];
                    }
                }
            } else if (more) {
#pragma unroll
                for (int k = 0; k < ENUM_UNROLL; k++) enqueue(vk[k], xk[k], rk[k], false);
            } else {
                enqueue(false, 0, 0, true);
            }
            if (!more) break;
        }
        wave_sync(); // the next item overwrites this wave's LDS
    } else if (d > CAP && nq > 0) {
        // long owner rows (only for orientations without the degeneracy bound):
        // the same probes, searched in N+(w) in global memory
        for (int32_t g = item.g0; g < item.g0 + ng; g++) {
            const int4 sg = seg[g];
            for (int32_t p0 = sg.x; p0 < sg.x + sg.y; p0 += 64) {
                const int32_t p = p0 + lane;
                bool hit = false;
                int32_t e01 = 0, e02 = 0, e12 = 0;
                if (p < sg.x + sg.y) {
                    sink.prefetch((int32_t)((uint32_t)sg.z & ~MODE_B), p, ((uint32_t)sg.z & MODE_B) != 0);
                    const int32_t x = oadj[p];
                    int32_t a = 0, c = d;
                    while (a < c) {
                        int32_t mid = (a + c) >> 1;
                        if (oadj[b + mid] < x) a = mid + 1;
                        else c = mid;
                    }
                    hit = a < d && oadj[b + a] == x;
                    tri_edges(sg.z, p, b + a, e01, e02, e12);
                }
                sink.hit(hit, e01, e02, e12);
            }
        }
    }
    sink.end(it);
}

// the triangles a cached list holds for one item
template <class Sink>
__device__ inline void cached_item(const int64_t *__restrict__ base, const int32_t *__restrict__ tri, int64_t it,
                                   Sink &sink) {
    const int lane = lane_id();
    const int64_t b = base[it], e = base[it + 1];
    sink.begin(it);
    for (int64_t p0 = b; p0 < e; p0 += 64) {
        int64_t p = p0 + lane;
        bool valid = p < e;
        if (valid) sink.prefetch(tri[3 * p], tri[3 * p + 2], false);
        sink.hit(valid, valid ? tri[3 * p] : 0, valid ? tri[3 * p + 1] : 0, valid ? tri[3 * p + 2] : 0);
    }
    sink.end(it);
}

// Waves per SIMD the compiler must fit a sink's enumeration into (a floor): at
// least 7 (72 VGPRs) for the query's counting filter; the others keep their size.
template <class S> struct enum_waves { static constexpr int value = 4; };
template <int V> struct enum_waves<FilterSink<V, FILTER_COUNT> > { static constexpr int value = 7; };

// One wavefront per item; list != nullptr: only the nlist items list[0..nlist)
template <class Sink>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(enum_waves<Sink>::value))) void k_tri_enum(const EnumItem *__restrict__ items, const int32_t *__restrict__ oadj,
                                                  const int4 *__restrict__ seg, int32_t NI, Sink sink,
                                                  const int32_t *__restrict__ list = nullptr, int32_t nlist = 0) {
    __shared__ EnumLds lds[WPB];
    const int w = wave_id();
    const int64_t stride = (int64_t)gridDim.x * WPB;
    int64_t it = (int64_t)blockIdx.x * WPB + w;
    if (list) {
        // a pass over a few listed items
        for (; it < nlist; it += stride) {
            const int64_t li = list[it];
            const EnumItem item = items[li];
            enum_item(item, stage_ahead(item, oadj, seg), oadj, seg, li, sink, lds[w]);
        }
        sink.finish();
        return;
    }
    // item headers run two items ahead and the first row and segment chunks
    // one item ahead, so a wavefront starts each item with its data loaded
    const EnumItem none{};
    EnumItem h0 = it < NI ? items[it] : none;
    EnumItem h1 = it + stride < NI ? items[it + stride] : none;
    StageAhead a0 = stage_ahead(h0, oadj, seg);
    for (; it < NI; it += stride) {
        const EnumItem cur = h0;
        const StageAhead ca = a0;
        h0 = h1;
        a0 = stage_ahead(h0, oadj, seg);
        h1 = it + 2 * stride < NI ? items[it + 2 * stride] : none;
        enum_item(cur, ca, oadj, seg, it, sink, lds[w]);
    }
    sink.finish();
}

// cached triangle list: the same filter, one wavefront per item
template <int VAR, int MODE, bool SS>
__global__ __launch_bounds__(BLK) void k_filter_cached(const int64_t *__restrict__ base, const int32_t *__restrict__ tri,
                                                       int32_t NI, FilterSink<VAR, MODE, SS> sink,
                                                       const int32_t *__restrict__ list = nullptr, int32_t nlist = 0) {
    const int w = wave_id();
    const int64_t n = list ? nlist : NI;
    for (int64_t i = (int64_t)blockIdx.x * WPB + w; i < n; i += (int64_t)gridDim.x * WPB)
        cached_item(base, tri, list ? (int64_t)list[i] : i, sink);
    sink.finish();
}

template <int VAR, class Op, bool SS = false>
__device__ inline void chunk_runs(const TriLists &L, uint32_t dq, const int64_t *ts, int64_t &r, int64_t &k, int64_t k1,
                                  const Op &op) {
    if (chunk_run<VAR, 0, 1, Op, SS>(L, dq, ts, r, k, k1, op) && chunk_run<VAR, 1, 0, Op, SS>(L, dq, ts, r, k, k1, op) &&
        chunk_run<VAR, 0, 2, Op, SS>(L, dq, ts, r, k, k1, op) && chunk_run<VAR, 2, 0, Op, SS>(L, dq, ts, r, k, k1, op) &&
        chunk_run<VAR, 1, 2, Op, SS>(L, dq, ts, r, k, k1, op))
        chunk_run<VAR, 2, 1, Op, SS>(L, dq, ts, r, k, k1, op);
}

template <class Op>
__device__ inline void chunk_runs_rt(int variant, const TriLists &L, uint32_t dq, const int64_t *ts, int64_t &r,
                                     int64_t &k, int64_t k1, const Op &op) {
    switch (variant) {
    case 0: chunk_runs<0>(L, dq, ts, r, k, k1, op); break;
    case 1: chunk_runs<1>(L, dq, ts, r, k, k1, op); break;
    case 2: chunk_runs<2>(L, dq, ts, r, k, k1, op); break;
    case 3: chunk_runs<3>(L, dq, ts, r, k, k1, op); break;
    case 4: chunk_runs<4>(L, dq, ts, r, k, k1, op); break;
    case 5: chunk_runs<5>(L, dq, ts, r, k, k1, op); break;
    case 6: chunk_runs<6>(L, dq, ts, r, k, k1, op); break;
    default: chunk_runs<7>(L, dq, ts, r, k, k1, op); break;
    }
}

// ---------------------------------------------------------------------------
// a.6: scheduling the tests of the surviving triangles
// ---------------------------------------------------------------------------
// Survivors are reached through a dense index q in [0, sbase[NI]): item u holds
// q in [sbase[u], sbase[u + 1]), at slots slot_base[u] + (q - sbase[u]) of the
// filter's output (slot_base null: the slots are dense, slot = q).  A wavefront
// takes a group of 64 consecutive survivors, one per lane.  A survivor with at
// most LIGHT_TESTS tests is run by the group.  One with more (a heavy survivor)
// gets an entry in a list and a range of piece numbers, both from one packed
// counter, so entries are in the order of their pieces; a second kernel runs
// piece p (tests [4 i, 4 i + 4) of its survivor) per thread, finding its
// entry by binary search over the entries' first pieces and starting its L2 and
// L3 cursors with one binary search each (the merge-path split of a long run
// over neighbouring threads).  No test pays a search over items or survivors.
// Heavy survivors past the list's capacity run where they were found, so any
// capacity gives the same result.
//
// How a group runs its light tests depends on the runner.  Flat runners (the
// per-edge counts): the lanes stage their survivors' six list spans in LDS, and
// the group's tests, concatenated, go one per lane, so neighbouring lanes take
// neighbouring tests of one run and their loads coalesce; each test finds its
// survivor by a search over 64 prefix sums in LDS and its cursors by binary
// search.  Other runners (the exists-exists-exists counting, whose window
// bookkeeping is shared by the tests of a run): each lane runs its own
// survivor's tests in order.
// 70M-edge graph, one year (36.8M tests) and a graph of 5,000-edge lists closed
// by short ones (104M tests): light limit 16 / pieces of 32: 2.45 and 3.2 ms;
// 64 / 8: 1.97 and 1.74 ms; 64 / 4: 1.85 and 1.15 ms; 64 / 2: 1.83 and 1.30 ms
constexpr int64_t LIGHT_TESTS = 64;
constexpr int64_t PIECE_TESTS = 4;

struct Heavy {
    int64_t slot;  // survivor slot
    int64_t first; // its first piece number
};
// the counter of heavy survivors: entries in bits 40-63, piece numbers in 0-39
constexpr int HEAVY_SHIFT = 40;
constexpr unsigned long long PIECE_MASK = (1ull << HEAVY_SHIFT) - 1;

// the largest u in [a, b) with sbase[u] <= q (sbase ascending, sbase[a] <= q)
__device__ inline int32_t item_of(const int64_t *__restrict__ sbase, int32_t a, int32_t b, int64_t q) {
    int32_t lo = a, hi = b - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (sbase[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// For sparse slots: gitem[g] = the item of survivor 64 g, for every group g
// with 64 g < sbase[NI], and gitem[g] = NI - 1 for the group past the last.
__global__ __launch_bounds__(BLK) void k_group_items(const int64_t *__restrict__ sbase, int32_t NI, int64_t ngroups,
                                                     int32_t *__restrict__ gitem) {
    const int64_t nsurv = sbase[NI];
    for (int64_t g = (int64_t)blockIdx.x * BLK + threadIdx.x; g < ngroups; g += (int64_t)gridDim.x * BLK) {
        const int64_t q0 = g * 64;
        if (q0 >= nsurv) {
            if (q0 - 64 < nsurv) gitem[g] = NI - 1;
            break;
        }
        gitem[g] = item_of(sbase, 0, NI, q0);
    }
}

// The survivor slot of dense index q in group g (q < sbase[NI]).
__device__ inline int64_t survivor_slot(const int64_t *__restrict__ sbase, const int64_t *__restrict__ slot_base,
                                        const int32_t *__restrict__ gitem, int64_t g, int64_t q) {
    if (!slot_base) return q;
    const int32_t u = item_of(sbase, gitem[g], gitem[g + 1] + 1, q);
    return slot_base[u] + (q - sbase[u]);
}

// list index of E_{x_a, x_b} in TriLists order (d01, d10, d02, d20, d12, d21)
constexpr int list_id(int a, int b) { return a == 0 ? (b == 1 ? 0 : 2) : a == 1 ? (b == 0 ? 1 : 4) : (b == 0 ? 3 : 5); }

// One light group's survivors in LDS: start and length of each directed list,
// the runs that can count (bit k: run k in the order of chunk_runs), and the
// inclusive prefix of the survivors' tests.
// SHORT also keeps each list's first and last timestamp (3 KB more per
// wavefront), for tests that read short lists from them.
template <bool SHORT> struct FlatLds;
template <> struct FlatLds<false> {
    int32_t incl[64];
    int32_t ls[6][64];
    int32_t ln[6][64];
    uint32_t live[64];
};
template <> struct FlatLds<true> : FlatLds<false> {
    uint32_t lo[6][64]; // first and last timestamp >> tshift
    uint32_t hi[6][64];
};

// run k = (I, J) of survivor si holds test r (r < that run's tests): run it
template <int VAR, int I, int J, bool SS, class Op, bool SHORT>
__device__ inline bool flat_run(const FlatLds<SHORT> &F, int si, int k, int64_t &r, const int64_t *__restrict__ ts,
                                const Op &op) {
    if (!((F.live[si] >> k) & 1u)) return false;
    using P = Pick<VAR, I, J>;
    constexpr int i1 = list_id(I, J), i2 = list_id(P::L2a, P::L2b), i3 = list_id(P::L3a, P::L3b);
    const int32_t n1 = F.ln[i1][si], n2 = F.ln[i2][si];
    const int32_t nt = SS && n2 < n1 ? n2 : n1;
    if (r >= nt) {
        r -= nt;
        return false;
    }
    Span l1{}, l2{}, l3{};
    l1.s = F.ls[i1][si];
    l1.n = n1;
    l2.s = F.ls[i2][si];
    l2.n = n2;
    l3.s = F.ls[i3][si];
    l3.n = F.ln[i3][si];
    if constexpr (SHORT) {
        l2.lo = F.lo[i2][si];
        l2.hi = F.hi[i2][si];
        l3.lo = F.lo[i3][si];
        l3.hi = F.hi[i3][si];
    }
    if (SS && nt < n1) op.iv(ts, l1, (int32_t)r, 1, l2, l3);
    else op(ts, l1.s + (int32_t)r, 1, l2, l3);
    return true;
}

// Runs the tests of the per-edge counts: work() is a survivor's number of
// tests, run() takes tests [r, k1) of it in order, flat() its test r alone,
// from the spans stage() put in LDS.
template <int VAR, class Op, bool SS> struct CountRunner {
    static constexpr bool kFlat = true;
    static constexpr bool kShort = Op::kShort && !SS; // staging keeps the lists' end timestamps
    static_assert(!(Op::kShort && SS), "short lists are read only by the plain evaluation");
    using Flat = FlatLds<kShort>;
    using Surv = TriLists;
    uint32_t dq;
    const int64_t *ts;
    Op op;
    const int32_t *sv; // survivors as three oriented edges
    const EdgeRec *rec;
    __device__ inline TriLists load(int64_t slot) const {
        return load_lists(rec, sv[3 * slot], sv[3 * slot + 1], sv[3 * slot + 2]);
    }
    __device__ inline int64_t work(const TriLists &L) const { return tri_work<VAR, SS>(L, dq); }
    __device__ inline void run(const TriLists &L, int64_t, int64_t r, int64_t k1) {
        int64_t k = r;
        chunk_runs<VAR, Op, SS>(L, dq, ts, r, k, k1, op);
    }
    // the runs that can count, as bits in the order of chunk_runs
    __device__ inline uint32_t live(const TriLists &L) const {
        Span a, b, c;
        return (uint32_t)run_lists<VAR, 0, 1>(L, dq, a, b, c) | (uint32_t)run_lists<VAR, 1, 0>(L, dq, a, b, c) << 1 |
               (uint32_t)run_lists<VAR, 0, 2>(L, dq, a, b, c) << 2 | (uint32_t)run_lists<VAR, 2, 0>(L, dq, a, b, c) << 3 |
               (uint32_t)run_lists<VAR, 1, 2>(L, dq, a, b, c) << 4 | (uint32_t)run_lists<VAR, 2, 1>(L, dq, a, b, c) << 5;
    }
    __device__ inline void stage(Flat &F, int lane, const TriLists &T, bool light) const {
        const Span *sp[6] = {&T.d01, &T.d10, &T.d02, &T.d20, &T.d12, &T.d21};
#pragma unroll
        for (int k = 0; k < 6; k++) {
            F.ls[k][lane] = sp[k]->s;
            F.ln[k][lane] = sp[k]->n;
            if constexpr (kShort) {
                F.lo[k][lane] = sp[k]->lo;
                F.hi[k][lane] = sp[k]->hi;
            }
        }
        F.live[lane] = light ? live(T) : 0u;
    }
    __device__ inline void flat(const Flat &F, int si, int64_t r) const {
        flat_run<VAR, 0, 1, SS>(F, si, 0, r, ts, op) || flat_run<VAR, 1, 0, SS>(F, si, 1, r, ts, op) ||
            flat_run<VAR, 0, 2, SS>(F, si, 2, r, ts, op) || flat_run<VAR, 2, 0, SS>(F, si, 3, r, ts, op) ||
            flat_run<VAR, 1, 2, SS>(F, si, 4, r, ts, op) || flat_run<VAR, 2, 1, SS>(F, si, 5, r, ts, op);
    }
    __device__ inline void finish() {}
};

// Lanes with np > 0 (heavy survivors, np pieces each) take list entries and
// piece numbers for the whole wavefront with one atomic.  A survivor whose
// entry lies past cap runs here; the piece numbers it reserved follow every
// listed one.  `full` is set once this wavefront's atomic returned an entry
// count of cap or more, after which it lists nothing: each wavefront adds at
// most 64 entries past cap, so the entry count stays below cap + 64 x (the
// grid's wavefronts), far below 2^24.
template <class R>
__device__ inline void defer_heavy(R &runner, const typename R::Surv &S, int64_t slot, int64_t w, int64_t np,
                                   Heavy *__restrict__ heavy, unsigned long long *__restrict__ counter, int64_t cap,
                                   bool &full) {
    if (!__ballot(np > 0)) return;
    if (full) {
        if (np > 0) runner.run(S, slot, 0, w);
        return;
    }
    const unsigned long long add = np > 0 ? (1ull << HEAVY_SHIFT) | (unsigned long long)np : 0ull;
    const unsigned long long incl = wave_inclusive_sum(add);
    unsigned long long at = 0;
    if (lane_id() == 63) at = atomicAdd(counter, incl);
    at = __shfl(at, 63);
    full = (int64_t)(at >> HEAVY_SHIFT) + 64 >= cap;
    if (np == 0) return;
    const unsigned long long mine = at + incl - add;
    const int64_t e = (int64_t)(mine >> HEAVY_SHIFT);
    if (e < cap) heavy[e] = Heavy{slot, (int64_t)(mine & PIECE_MASK)};
    else runner.run(S, slot, 0, w);
}

template <class R>
__global__ __launch_bounds__(BLK) void k_tests_light(const int64_t *__restrict__ sbase,
                                                     const int64_t *__restrict__ slot_base,
                                                     const int32_t *__restrict__ gitem, int32_t NI, R runner,
                                                     Heavy *__restrict__ heavy,
                                                     unsigned long long *__restrict__ counter, int64_t cap) {
    __shared__ typename R::Flat flds[R::kFlat ? WPB : 1];
    const int w = wave_id();
    const int lane = lane_id();
    const int64_t nsurv = sbase[NI];
    const int64_t ng = (nsurv + 63) / 64;
    bool full = false;
    for (int64_t g = (int64_t)blockIdx.x * WPB + w; g < ng; g += (int64_t)gridDim.x * WPB) {
        const int64_t q = g * 64 + lane;
        const bool on = q < nsurv;
        int64_t slot = 0, wk = 0, np = 0;
        typename R::Surv S{};
        if (on) {
            slot = survivor_slot(sbase, slot_base, gitem, g, q);
            S = runner.load(slot);
            wk = runner.work(S);
            if (wk > LIGHT_TESTS) np = (wk + PIECE_TESTS - 1) / PIECE_TESTS;
        }
        defer_heavy(runner, S, slot, wk, np, heavy, counter, cap, full);
        const int64_t light = np ? 0 : wk;
        if constexpr (R::kFlat) {
            typename R::Flat &F = flds[w];
            const int32_t incl = (int32_t)wave_inclusive_sum(light);
            const int32_t total = __shfl(incl, 63);
            if (total == 0) continue;
            F.incl[lane] = incl;
            runner.stage(F, lane, S, light != 0);
            wave_sync();
            for (int32_t t = lane; t < total; t += 64) {
                // the survivor whose tests hold t: the first si with incl[si] > t
                int a = 0, b = 63;
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (F.incl[mid] > t) b = mid;
                    else a = mid + 1;
                }
                runner.flat(F, a, (int64_t)(t - (a ? F.incl[a - 1] : 0)));
            }
            wave_sync(); // the LDS is rewritten by the next group
        } else {
            if (light) runner.run(S, slot, 0, light);
        }
    }
    runner.finish();
}

template <class R>
__global__ __launch_bounds__(BLK) void k_tests_pieces(const Heavy *__restrict__ heavy,
                                                      const unsigned long long *__restrict__ counter, int64_t cap,
                                                      R runner) {
    const unsigned long long c = *counter;
    const int64_t ne = (int64_t)(c >> HEAVY_SHIFT) < cap ? (int64_t)(c >> HEAVY_SHIFT) : cap;
    const int64_t np = (int64_t)(c & PIECE_MASK);
    if (ne > 0) {
        for (int64_t p = (int64_t)blockIdx.x * BLK + threadIdx.x; p < np; p += (int64_t)gridDim.x * BLK) {
            // the last entry whose first piece is <= p (entry 0 starts at piece 0)
            int64_t a = 0, b = ne - 1;
            while (a < b) {
                const int64_t mid = (a + b + 1) >> 1;
                if (heavy[mid].first <= p) a = mid;
                else b = mid - 1;
            }
            const Heavy h = heavy[a];
            const int64_t k0 = (p - h.first) * PIECE_TESTS;
            // pieces past the last listed survivor's belong to ones that ran
            // where they were found: k0 lies past every run, nothing is tested
            runner.run(runner.load(h.slot), h.slot, k0, k0 + PIECE_TESTS);
        }
    }
    runner.finish();
}

constexpr int64_t MAX_HEAVY = 1 << 22; // 64 MB of heavy-survivor entries at most
constexpr int64_t MIN_HEAVY = 1 << 16; // room for this many whatever the survivors
constexpr int64_t LIGHT_BLOCKS = 16384;
constexpr int64_t PIECE_BLOCKS = 8192;

// the heavy list's capacity limit: MAX_HEAVY, or FOLTY_MAX_HEAVY (>= 1) when set
inline int64_t max_heavy() {
    static const int64_t v = [] {
        const char *e = getenv("FOLTY_MAX_HEAVY");
        const long long x = e ? atoll(e) : 0;
        return x >= 1 ? (int64_t)std::min<long long>(x, MAX_HEAVY) : MAX_HEAVY;
    }();
    return v;
}

// Entries a query's heavy list holds: no more than its tests can fill (when
// known), and at most one per survivor (at least MIN_HEAVY, at most the limit),
// so that 16 * heavy_slots(T, -1) bounds the list's memory on a graph of T
// triangles.
inline int64_t heavy_slots(int64_t survivors, int64_t tests) {
    int64_t b = std::max<int64_t>(survivors + 1, MIN_HEAVY);
    if (tests >= 0) b = std::min<int64_t>(b, tests / (LIGHT_TESTS + 1) + 1);
    return std::max<int64_t>(1, std::min<int64_t>(b, max_heavy()));
}

// The tests of the survivors of the last filter (see k_tests_light): survivors is
// their number, or an upper bound when the filter ran in one pass; tests is
// their number of tests, or < 0 when unknown on the host.
template <class R>
void launch_tests(const Index &ix, Workspace &ws, const R &runner, int64_t survivors, int64_t tests, hipStream_t s) {
    const int64_t cap = heavy_slots(survivors, tests);
    ws.pieces.ensure(sizeof(Heavy) * (size_t)cap);
    ws.scal.ensure(128);
    unsigned long long *np = ws.scal.as<unsigned long long>() + 14;
    k_fill<unsigned long long><<<1, 1, 0, s>>>(np, 0ull, 1);
    FOLTY_LAUNCHED();
    const int64_t groups = (survivors + 63) / 64; // an upper bound when survivors is one
    const int64_t *sparse = ws.slots == ws.sbase.as<int64_t>() ? nullptr : ws.slots;
    if (sparse) {
        ws.gitem.ensure(4 * ((size_t)groups + 2));
        const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((groups + 1 + BLK - 1) / BLK, LIGHT_BLOCKS));
        k_group_items<<<gb, BLK, 0, s>>>(ws.sbase.as<int64_t>(), ix.NI, groups + 1, ws.gitem.as<int32_t>());
        FOLTY_LAUNCHED();
    }
    const unsigned lb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((groups + WPB - 1) / WPB, LIGHT_BLOCKS));
    k_tests_light<<<lb, BLK, 0, s>>>(ws.sbase.as<int64_t>(), sparse, ws.gitem.as<int32_t>(), ix.NI, runner,
                                     ws.pieces.as<Heavy>(), np, cap);
    FOLTY_LAUNCHED();
    // the pieces are numbered on the device; with the tests known, no more
    // threads than pieces
    const int64_t most = tests >= 0 ? tests / PIECE_TESTS + std::min<int64_t>(cap, tests / (LIGHT_TESTS + 1)) + 1
                                    : (int64_t)PIECE_BLOCKS * BLK;
    const unsigned pb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((most + BLK - 1) / BLK, PIECE_BLOCKS));
    k_tests_pieces<<<pb, BLK, 0, s>>>(ws.pieces.as<Heavy>(), np, cap, runner);
    FOLTY_LAUNCHED();
}

} // namespace
} // namespace folty
