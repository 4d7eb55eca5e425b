// Query kernels for the thresholded exists-exists-forall triadic query.
//
//  a.5  wedge enumeration + closing probe (paper, Algorithm OutNeighbours'
//       double loop over (u, v) in G->_pi and w in N+(u), with the adjacency
//       test of v and w): every static triangle is found once, from its
//       lowest-ranked vertex, as three oriented edges.
//  a.6  temporal tests (paper, Theorems 3.1 and 3.2): for a temporal edge e on
//       list L1 and the third vertex w, e forms a delta-temporal triangle with w
//       iff, with t2 = the first entry of L2 at or after t(e) and t3 = the first
//       entry of L3 at or after t2, both exist and t3 - t(e) <= delta.  The two
//       first-entry searches are binary searches over the time-sorted lists
//       (the log sigma_max factor of the paper's bound).  Every (triangle,
//       directed list) pair is a run of tests; runs are cut into equal chunks
//       over the whole grid (a flat, degree- and multiplicity-blind split).
//  a.7  threshold (paper, Algorithm ExistExistForAll, final loop) with the
//       exact rational theta, then per-pair certificate counts by a wavefront
//       segmented reduction and a ballot/prefix compaction of the pairs.
#include <algorithm>
#include <cstring>
#include <map>

#include "folty_internal.h"

namespace folty {

namespace {

constexpr int BLK = 256;
constexpr int IPT = 8;          // temporal tests per chunk
constexpr int PERSIST_BLOCKS = 4096;

__device__ inline int lane_id() { return __lane_id(); }

__device__ inline int32_t wave_append(int32_t *counter, bool pred) {
    unsigned long long mask = __ballot(pred);
    if (!mask) return -1;
    int lane = lane_id();
    int leader = __ffsll((long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (int32_t)__popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + (int32_t)__popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

template <class T> __global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// directed lists of a triangle
// ---------------------------------------------------------------------------
struct Span {
    int32_t s, n;
};

// E_{tail,head} and E_{head,tail} of an oriented edge record
__device__ inline void edge_spans(uint32_t rec, const int32_t *__restrict__ soff,
                                  const int32_t *__restrict__ smid, Span &fwd, Span &bwd) {
    uint32_t e = rec & 0x7fffffffu;
    int32_t a = soff[e], mid = smid[e], b = soff[e + 1];
    if (rec >> 31) {
        fwd = {a, mid - a};
        bwd = {mid, b - mid};
    } else {
        fwd = {mid, b - mid};
        bwd = {a, mid - a};
    }
}

// D[i][j] = E_{x_i, x_j} for the triangle's vertices x0 < x1 < x2 (by rank)
struct TriLists {
    Span d01, d10, d02, d20, d12, d21;
    template <int I, int J> __device__ inline Span get() const {
        static_assert(I != J, "");
        if constexpr (I == 0 && J == 1) return d01;
        else if constexpr (I == 1 && J == 0) return d10;
        else if constexpr (I == 0 && J == 2) return d02;
        else if constexpr (I == 2 && J == 0) return d20;
        else if constexpr (I == 1 && J == 2) return d12;
        else return d21;
    }
};

__device__ inline TriLists load_tri(const uint32_t *__restrict__ tri, int64_t tau,
                                    const int32_t *__restrict__ soff, const int32_t *__restrict__ smid) {
    TriLists L;
    uint32_t r0 = tri[3 * tau], r1 = tri[3 * tau + 1], r2 = tri[3 * tau + 2];
    edge_spans(r0, soff, smid, L.d01, L.d10);
    edge_spans(r1, soff, smid, L.d02, L.d20);
    edge_spans(r2, soff, smid, L.d12, L.d21);
    return L;
}

// The predicate code picks, for L1 = E_{a,b} (a = x_I, b = x_J, third w = x_C),
// L2 between X and w and L3 between Y and w (see folty.h for the bits).
template <int VAR, int I, int J> struct Pick {
    static constexpr int C = 3 - I - J;
    static constexpr int X = (VAR & 4) ? J : I;
    static constexpr int Y = (VAR & 4) ? I : J;
    static constexpr int L2a = (VAR & 1) ? C : X, L2b = (VAR & 1) ? X : C;
    static constexpr int L3a = (VAR & 2) ? C : Y, L3b = (VAR & 2) ? Y : C;
    __device__ static inline void lists(const TriLists &T, Span &l1, Span &l2, Span &l3) {
        l1 = T.template get<I, J>();
        l2 = T.template get<L2a, L2b>();
        l3 = T.template get<L3a, L3b>();
    }
};

template <int VAR, int I, int J> __device__ inline int64_t list_work(const TriLists &T) {
    Span a, b, c;
    Pick<VAR, I, J>::lists(T, a, b, c);
    return (b.n > 0 && c.n > 0) ? a.n : 0;
}

template <int VAR> __device__ inline int64_t tri_work(const TriLists &T) {
    return list_work<VAR, 0, 1>(T) + list_work<VAR, 1, 0>(T) + list_work<VAR, 0, 2>(T) +
           list_work<VAR, 2, 0>(T) + list_work<VAR, 1, 2>(T) + list_work<VAR, 2, 1>(T);
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

// cnt consecutive temporal edges of L1 starting at l1s against (L2, L3)
__device__ inline void run_tests(const int64_t *__restrict__ ts, int32_t l1s, int32_t cnt, Span l2, Span l3,
                                 int64_t delta, uint32_t *__restrict__ count) {
    const int64_t *L2 = ts + l2.s, *L3 = ts + l3.s;
    int32_t c2 = 0, c3 = 0;
    for (int32_t q = 0; q < cnt; q++) {
        int32_t e = l1s + q;
        int64_t t = ts[e];
        c2 = lower_bound_from(L2, c2, l2.n, t);
        if (c2 == l2.n) break;           // later edges are no earlier: no t2 for them either
        int64_t t2 = L2[c2];
        if (t2 - t > delta) continue;
        c3 = lower_bound_from(L3, c3, l3.n, t2);
        if (c3 == l3.n) break;
        if (L3[c3] - t <= delta) atomicAdd(&count[e], 1u);
    }
}

// the same, recording the smallest window per (e, w) into a histogram over
// sorted window levels: level j counts w whose smallest window is in (lv[j-1], lv[j]]
__device__ inline void run_windows(const int64_t *__restrict__ ts, int32_t l1s, int32_t cnt, Span l2, Span l3,
                                   const int64_t *__restrict__ lv, int nl, int64_t m,
                                   uint32_t *__restrict__ hist) {
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
        atomicAdd(&hist[(int64_t)a * m + e], 1u);
    }
}

struct DirectOp {
    int64_t delta;
    uint32_t *count;
    __device__ inline void operator()(const int64_t *ts, int32_t l1s, int32_t cnt, Span l2, Span l3) const {
        run_tests(ts, l1s, cnt, l2, l3, delta, count);
    }
};

struct PoolOp {
    const int64_t *lv;
    int nl;
    int64_t m;
    uint32_t *hist;
    __device__ inline void operator()(const int64_t *ts, int32_t l1s, int32_t cnt, Span l2, Span l3) const {
        run_windows(ts, l1s, cnt, l2, l3, lv, nl, m, hist);
    }
};

// one list of the triangle within the chunk [k, k1); r = items of this
// triangle still to skip.  Returns false once the chunk is used up.
template <int VAR, int I, int J, class Op>
__device__ inline bool chunk_list(const TriLists &T, const int64_t *ts, int64_t &r, int64_t &k, int64_t k1,
                                  const Op &op) {
    Span l1, l2, l3;
    Pick<VAR, I, J>::lists(T, l1, l2, l3);
    if (l1.n == 0 || l2.n == 0 || l3.n == 0) return true;
    if (r >= l1.n) {
        r -= l1.n;
        return true;
    }
    int64_t cnt = l1.n - r;
    if (cnt > k1 - k) cnt = k1 - k;
    op(ts, l1.s + (int32_t)r, (int32_t)cnt, l2, l3);
    k += cnt;
    r = 0;
    return k < k1;
}

// Flat split of all tests into chunks of IPT; grid-stride over chunks.  The
// chunk's first triangle is found by binary search over the work offsets.
template <int VAR, class Op>
__global__ __launch_bounds__(BLK) void k_temporal(const uint32_t *__restrict__ tri, const int64_t *__restrict__ woff,
                                                  int64_t T, const int32_t *__restrict__ soff,
                                                  const int32_t *__restrict__ smid, const int64_t *__restrict__ ts,
                                                  Op op) {
    const int64_t total = woff[T];
    const int64_t nchunks = (total + IPT - 1) / IPT;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchunks; c += stride) {
        int64_t k = c * IPT;
        int64_t k1 = k + IPT < total ? k + IPT : total;
        int64_t a = 0, b = T;
        while (a < b) {
            int64_t mid = (a + b) >> 1;
            if (woff[mid] <= k) a = mid + 1;
            else b = mid;
        }
        int64_t tau = a - 1;
        int64_t r = k - woff[tau];
        while (k < k1 && tau < T) {
            TriLists L = load_tri(tri, tau, soff, smid);
            if (chunk_list<VAR, 0, 1>(L, ts, r, k, k1, op) && chunk_list<VAR, 1, 0>(L, ts, r, k, k1, op) &&
                chunk_list<VAR, 0, 2>(L, ts, r, k, k1, op) && chunk_list<VAR, 2, 0>(L, ts, r, k, k1, op) &&
                chunk_list<VAR, 1, 2>(L, ts, r, k, k1, op))
                chunk_list<VAR, 2, 1>(L, ts, r, k, k1, op);
            tau++;
            r = 0;
        }
    }
}

// a.5: wedges (u; v, w) with v < w in N+(u), closing probe w in N+(v) by a
// forward-moving binary search; writes the triangle at its precomputed slot
// and, if VAR >= 0, the triangle's test count for that predicate code.
template <int VAR>
__global__ __launch_bounds__(BLK) void k_wedges(const int32_t *__restrict__ osrc, const int32_t *__restrict__ oadj,
                                                const int32_t *__restrict__ ooff, const uint32_t *__restrict__ oeid,
                                                const int64_t *__restrict__ tri_off, int32_t S,
                                                const int32_t *__restrict__ soff, const int32_t *__restrict__ smid,
                                                uint32_t *__restrict__ tri, int64_t *__restrict__ work) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    int32_t u = osrc[j], v = oadj[j];
    int32_t end = ooff[u + 1];
    int32_t lo = ooff[v], hi = ooff[v + 1];
    int64_t slot = tri_off[j];
    const uint32_t r0 = oeid[j];
    for (int32_t j2 = (int32_t)j + 1; j2 < end && lo < hi; j2++) {
        int32_t w = oadj[j2];
        int32_t a = lo, b = hi;
        while (a < b) {
            int32_t mid = (a + b) >> 1;
            if (oadj[mid] < w) a = mid + 1;
            else b = mid;
        }
        lo = a;
        if (a < hi && oadj[a] == w) {
            uint32_t r1 = oeid[j2], r2 = oeid[a];
            tri[3 * slot] = r0;
            tri[3 * slot + 1] = r1;
            tri[3 * slot + 2] = r2;
            if constexpr (VAR >= 0) {
                TriLists L;
                edge_spans(r0, soff, smid, L.d01, L.d10);
                edge_spans(r1, soff, smid, L.d02, L.d20);
                edge_spans(r2, soff, smid, L.d12, L.d21);
                work[slot] = tri_work<VAR>(L);
            }
            slot++;
            lo = a + 1;
        }
    }
}

template <int VAR>
__global__ void k_tri_work(const uint32_t *__restrict__ tri, int64_t T, const int32_t *__restrict__ soff,
                           const int32_t *__restrict__ smid, int64_t *__restrict__ work) {
    int64_t tau = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tau >= T) return;
    work[tau] = tri_work<VAR>(load_tri(tri, tau, soff, smid));
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
    uint32_t *ncert;                 // [2S]: 2 s + dir
    unsigned long long *total;       // certificates
};

__global__ __launch_bounds__(BLK) void k_threshold(ThreshArgs A) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool in = k < A.m;
    int64_t key = -1;
    bool cert = false;
    if (in) {
        int32_t s = A.sid[k];
        int dir = k >= A.smid[s] ? 1 : 0;
        int32_t a = dir ? A.shi[s] : A.slo[s];
        int32_t b = dir ? A.slo[s] : A.shi[s];
        int64_t U;
        if (A.universe == FOLTY_UNIVERSE_DST) U = (int64_t)A.deg[b] - A.excl;
        else if (A.universe == FOLTY_UNIVERSE_SRC) U = (int64_t)A.deg[a] - A.excl;
        else U = A.tcnt[s];
        cert = (uint64_t)A.count[k] * A.den >= (uint64_t)A.num * (uint64_t)U;
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
    if (lane == 0 && certs) atomicAdd(A.total, (unsigned long long)__popcll(certs));
    if (in && tail) {
        unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        unsigned long long h = heads & upto;
        int start = 63 - __clzll((long long)h);
        unsigned long long seg = upto & ~((1ull << start) - 1ull);
        int c = __popcll(certs & seg);
        if (c) atomicAdd(&A.ncert[key], (uint32_t)c);
    }
}

__global__ void k_pairs_compact(const uint32_t *__restrict__ ncert, int32_t S, const int32_t *__restrict__ slo,
                                 const int32_t *__restrict__ shi, uint64_t *__restrict__ keys,
                                 uint32_t *__restrict__ vals, int32_t *__restrict__ npairs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool in = i < 2 * (int64_t)S;
    uint32_t c = in ? ncert[i] : 0;
    int32_t slot = wave_append(npairs, c > 0);
    if (slot >= 0) {
        int32_t s = (int32_t)(i >> 1);
        int dir = (int)(i & 1);
        uint64_t a = (uint64_t)(dir ? shi[s] : slo[s]);
        uint64_t b = (uint64_t)(dir ? slo[s] : shi[s]);
        keys[slot] = (a << 32) | b;
        vals[slot] = c;
    }
}

__global__ void k_counts_scatter(const uint32_t *__restrict__ count, const int32_t *__restrict__ perm, int32_t m,
                                 uint32_t *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) out[perm[k]] = count[k];
}

// running sum over window levels: hist[j][e] becomes #w with smallest window <= lv[j]
__global__ void k_hist_prefix(uint32_t *__restrict__ hist, int nl, int64_t m) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t acc = 0;
    for (int j = 0; j < nl; j++) {
        acc += hist[(int64_t)j * m + e];
        hist[(int64_t)j * m + e] = acc;
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
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

double ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    FOLTY_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
}

// Triangles (cached or enumerated now) and per-triangle test counts for one
// predicate code, then exclusive offsets in ws.work.  Returns the triangle list.
const uint32_t *prepare_work(const Index &ix, int variant, Workspace &ws, hipStream_t s, bool reuse_tri,
                             bool *enumerated) {
    const int64_t T = ix.T;
    ws.work.ensure(8 * ((size_t)T + 1));
    ws.aux.ensure(8 * ((size_t)T + 1));
    const uint32_t *tri;
    *enumerated = false;
    if (ix.tri_cached) {
        tri = ix.tri.as<uint32_t>();
        dispatch_variant(variant, [&](auto V) {
            k_tri_work<decltype(V)::value><<<grid_for(T, BLK, 1ll << 30), BLK, 0, s>>>(
                tri, T, ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), ws.work.as<int64_t>());
        });
    } else if (reuse_tri) {
        tri = ws.tri.as<uint32_t>();
        dispatch_variant(variant, [&](auto V) {
            k_tri_work<decltype(V)::value><<<grid_for(T, BLK, 1ll << 30), BLK, 0, s>>>(
                tri, T, ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), ws.work.as<int64_t>());
        });
    } else {
        ws.tri.ensure(12 * (size_t)T);
        tri = ws.tri.as<uint32_t>();
        dispatch_variant(variant, [&](auto V) {
            k_wedges<decltype(V)::value><<<grid_for(ix.S, BLK, 1ll << 30), BLK, 0, s>>>(
                ix.osrc.as<int32_t>(), ix.oadj.as<int32_t>(), ix.ooff.as<int32_t>(), ix.oeid.as<uint32_t>(),
                ix.tri_off.as<int64_t>(), ix.S, ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), ws.tri.as<uint32_t>(),
                ws.work.as<int64_t>());
        });
        *enumerated = true;
    }
    FOLTY_LAUNCHED();
    // work[T] = 0 so that the exclusive scan leaves the total in woff[T]
    FOLTY_HIP(hipMemsetAsync(ws.work.as<int64_t>() + T, 0, 8, s));
    size_t need = exclusive_scan_i64(nullptr, 0, ws.work.as<int64_t>(), ws.aux.as<int64_t>(), T + 1, s);
    ws.cub.ensure(need);
    exclusive_scan_i64(ws.cub.p, need, ws.work.as<int64_t>(), ws.aux.as<int64_t>(), T + 1, s);
    return tri;
}

template <class Op>
void launch_temporal(const Index &ix, int variant, const uint32_t *tri, const int64_t *woff, const Op &op,
                     hipStream_t s) {
    dispatch_variant(variant, [&](auto V) {
        k_temporal<decltype(V)::value, Op><<<PERSIST_BLOCKS, BLK, 0, s>>>(
            tri, woff, ix.T, ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), ix.ts.as<int64_t>(), op);
    });
    FOLTY_LAUNCHED();
}

// threshold + pairs for one query given device counts (sorted edge order)
void finish_query(const Graph *g, const folty_query &q, const uint32_t *count, Workspace &ws, Result *res,
                  hipStream_t s) {
    const Index &ix = g->ix;
    const int32_t S = ix.S, m = ix.m;
    ws.ncert.ensure(8 * (size_t)S + 8);
    ws.scal.ensure(64);
    FOLTY_HIP(hipMemsetAsync(ws.scal.p, 0, 64, s));
    if (S > 0) {
        k_fill<uint32_t><<<grid_for(2 * (int64_t)S, BLK, 1ll << 30), BLK, 0, s>>>(ws.ncert.as<uint32_t>(), 0u,
                                                                               2 * (int64_t)S);
        FOLTY_LAUNCHED();
    }
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
        A.ncert = ws.ncert.as<uint32_t>();
        A.total = total;
        k_threshold<<<grid_for(m, BLK, 1ll << 30), BLK, 0, s>>>(A);
        FOLTY_LAUNCHED();
        ws.pairs_k.ensure(16 * (size_t)S);
        ws.pairs_v.ensure(8 * (size_t)S);
        k_pairs_compact<<<grid_for(2 * (int64_t)S, BLK, 1ll << 30), BLK, 0, s>>>(
            ws.ncert.as<uint32_t>(), S, ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), ws.pairs_k.as<uint64_t>(),
            ws.pairs_v.as<uint32_t>(), np);
        FOLTY_LAUNCHED();
    }
    ws.host.ensure(64);
    FOLTY_HIP(hipMemcpyAsync(ws.host.p, ws.scal.p, 32, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    unsigned long long ncerts;
    int32_t npairs;
    memcpy(&ncerts, ws.host.p, 8);
    memcpy(&npairs, ws.host.as<char>() + 16, 4);
    res->n_certificates = (int64_t)ncerts;
    res->u.resize(npairs);
    res->v.resize(npairs);
    res->n_cert.resize(npairs);
    if (npairs > 0) {
        ws.pairs_k2.ensure(8 * (size_t)npairs);
        ws.pairs_v2.ensure(4 * (size_t)npairs);
        int kb = 32 + bit_length((uint64_t)ix.n);
        size_t need = sort_pairs_u64_u32(nullptr, 0, ws.pairs_k.as<uint64_t>(), ws.pairs_k2.as<uint64_t>(),
                                         ws.pairs_v.as<uint32_t>(), ws.pairs_v2.as<uint32_t>(), npairs, kb, s);
        ws.cub.ensure(need);
        sort_pairs_u64_u32(ws.cub.p, need, ws.pairs_k.as<uint64_t>(), ws.pairs_k2.as<uint64_t>(),
                           ws.pairs_v.as<uint32_t>(), ws.pairs_v2.as<uint32_t>(), npairs, kb, s);
        std::vector<uint64_t> keys(npairs);
        FOLTY_HIP(hipMemcpyAsync(keys.data(), ws.pairs_k2.p, 8 * (size_t)npairs, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(res->n_cert.data(), ws.pairs_v2.p, 4 * (size_t)npairs, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < npairs; i++) {
            res->u[i] = (int32_t)(keys[i] >> 32);
            res->v[i] = (int32_t)(keys[i] & 0xffffffffu);
        }
    }
}

void keep_counts(const Graph *g, const uint32_t *count, Result *res, hipStream_t s) {
    const Index &ix = g->ix;
    res->counts_dev.ensure(4 * (size_t)ix.m_input + 4);
    if (ix.m_input > 0) {
        k_fill<uint32_t><<<grid_for(ix.m_input, BLK, 1ll << 30), BLK, 0, s>>>(res->counts_dev.as<uint32_t>(),
                                                                            0xffffffffu, ix.m_input);
        FOLTY_LAUNCHED();
    }
    if (ix.m > 0) {
        k_counts_scatter<<<grid_for(ix.m, BLK, 1ll << 30), BLK, 0, s>>>(count, ix.perm.as<int32_t>(), ix.m,
                                                                       res->counts_dev.as<uint32_t>());
        FOLTY_LAUNCHED();
    }
    res->has_counts = true;
    res->device = g->device;
}

} // namespace

void enumerate_triangles(const Index &ix, uint32_t *tri, hipStream_t s) {
    if (ix.S == 0 || ix.T == 0) return;
    k_wedges<-1><<<grid_for(ix.S, BLK, 1ll << 30), BLK, 0, s>>>(
        ix.osrc.as<int32_t>(), ix.oadj.as<int32_t>(), ix.ooff.as<int32_t>(), ix.oeid.as<uint32_t>(),
        ix.tri_off.as<int64_t>(), ix.S, ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), tri, nullptr);
    FOLTY_LAUNCHED();
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
    if (q.flags & ~FOLTY_QUERY_NO_COUNTS) fail(FOLTY_EINVAL, "unknown query flags 0x%x", (unsigned)q.flags);
}

Result *run_query(Graph *g, const folty_query &q, Workspace &ws) {
    check_query(g, q);
    if (hipSetDevice(g->device) != hipSuccess) fail(FOLTY_EDEVICE, "hipSetDevice failed");
    const Index &ix = g->ix;
    hipStream_t s = g->stream;
    std::unique_ptr<Result> res(new Result());
    ws.ensure_events();
    FOLTY_HIP(hipEventRecord(ws.ev[0], s));
    ws.count.ensure(4 * (size_t)ix.m + 4);
    uint32_t *count = ws.count.as<uint32_t>();
    if (ix.m > 0) {
        k_fill<uint32_t><<<grid_for(ix.m, BLK, 1ll << 30), BLK, 0, s>>>(count, 0u, ix.m);
        FOLTY_LAUNCHED();
    }
    int64_t tests = 0;
    if (ix.T > 0) {
        bool enumerated = false;
        const uint32_t *tri = prepare_work(ix, q.variant, ws, s, false, &enumerated);
        FOLTY_HIP(hipEventRecord(ws.ev[1], s));
        DirectOp op{q.delta, count};
        launch_temporal(ix, q.variant, tri, ws.aux.as<int64_t>(), op, s);
        FOLTY_HIP(hipMemcpyAsync(&res->stats.tests, ws.aux.as<int64_t>() + ix.T, 8, hipMemcpyDeviceToHost, s));
    } else {
        FOLTY_HIP(hipEventRecord(ws.ev[1], s));
    }
    FOLTY_HIP(hipEventRecord(ws.ev[2], s));
    finish_query(g, q, count, ws, res.get(), s);
    FOLTY_HIP(hipEventRecord(ws.ev[3], s));
    if (!(q.flags & FOLTY_QUERY_NO_COUNTS)) keep_counts(g, count, res.get(), s);
    FOLTY_HIP(hipStreamSynchronize(s));
    tests = res->stats.tests;
    fill_stats_from_index(ix, &res->stats);
    res->stats.tests = tests;
    res->stats.n_pairs = (int64_t)res->u.size();
    res->stats.n_certificates = res->n_certificates;
    res->stats.wedge_ms = ev_ms(ws.ev[0], ws.ev[1]);
    res->stats.temporal_ms = ev_ms(ws.ev[1], ws.ev[2]);
    res->stats.threshold_ms = ev_ms(ws.ev[2], ws.ev[3]);
    res->stats.query_ms = ev_ms(ws.ev[0], ws.ev[3]);
    return res.release();
}

// Several queries on one graph: one pass per predicate code over the distinct
// windows of its queries, then a threshold per query.
void run_batch(Graph *g, const folty_query *qs, int nq, Workspace &ws, Result **outs) {
    if (nq < 0) fail(FOLTY_EINVAL, "nq < 0");
    for (int i = 0; i < nq; i++) check_query(g, qs[i]);
    if (hipSetDevice(g->device) != hipSuccess) fail(FOLTY_EDEVICE, "hipSetDevice failed");
    const Index &ix = g->ix;
    hipStream_t s = g->stream;
    std::map<int, std::vector<int>> by_var;
    for (int i = 0; i < nq; i++) by_var[qs[i].variant].push_back(i);
    std::vector<std::unique_ptr<Result>> res(nq);
    for (int i = 0; i < nq; i++) res[i].reset(new Result());
    ws.ensure_events();
    bool have_tri = false;
    for (auto &kv : by_var) {
        int variant = kv.first;
        std::vector<int64_t> lv;
        for (int i : kv.second) lv.push_back(qs[i].delta);
        std::sort(lv.begin(), lv.end());
        lv.erase(std::unique(lv.begin(), lv.end()), lv.end());
        const int nl = (int)lv.size();
        FOLTY_HIP(hipEventRecord(ws.ev[0], s));
        ws.hist.ensure(4 * (size_t)nl * (size_t)ix.m + 4);
        ws.scal.ensure(64);
        DevBuf lvd;
        lvd.ensure(8 * (size_t)nl);
        FOLTY_HIP(hipMemcpyAsync(lvd.p, lv.data(), 8 * (size_t)nl, hipMemcpyHostToDevice, s));
        int64_t hn = (int64_t)nl * ix.m;
        if (hn > 0) {
            k_fill<uint32_t><<<grid_for(hn, BLK, 1ll << 30), BLK, 0, s>>>(ws.hist.as<uint32_t>(), 0u, hn);
            FOLTY_LAUNCHED();
        }
        int64_t tests = 0;
        if (ix.T > 0) {
            bool enumerated = false;
            const uint32_t *tri = prepare_work(ix, variant, ws, s, have_tri, &enumerated);
            have_tri = have_tri || enumerated;
            PoolOp op{lvd.as<int64_t>(), nl, ix.m, ws.hist.as<uint32_t>()};
            launch_temporal(ix, variant, tri, ws.aux.as<int64_t>(), op, s);
            k_hist_prefix<<<grid_for(ix.m, BLK, 1ll << 30), BLK, 0, s>>>(ws.hist.as<uint32_t>(), nl, ix.m);
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipMemcpyAsync(&tests, ws.aux.as<int64_t>() + ix.T, 8, hipMemcpyDeviceToHost, s));
        }
        FOLTY_HIP(hipEventRecord(ws.ev[1], s));
        FOLTY_HIP(hipStreamSynchronize(s));
        double pass_ms = ev_ms(ws.ev[0], ws.ev[1]);
        for (int i : kv.second) {
            int j = (int)(std::lower_bound(lv.begin(), lv.end(), qs[i].delta) - lv.begin());
            const uint32_t *count = ws.hist.as<uint32_t>() + (int64_t)j * ix.m;
            FOLTY_HIP(hipEventRecord(ws.ev[2], s));
            finish_query(g, qs[i], count, ws, res[i].get(), s);
            FOLTY_HIP(hipEventRecord(ws.ev[3], s));
            if (!(qs[i].flags & FOLTY_QUERY_NO_COUNTS)) keep_counts(g, count, res[i].get(), s);
            FOLTY_HIP(hipStreamSynchronize(s));
            Result *r = res[i].get();
            fill_stats_from_index(ix, &r->stats);
            r->stats.tests = tests;
            r->stats.n_pairs = (int64_t)r->u.size();
            r->stats.n_certificates = r->n_certificates;
            r->stats.temporal_ms = pass_ms / (double)kv.second.size();
            r->stats.threshold_ms = ev_ms(ws.ev[2], ws.ev[3]);
            r->stats.query_ms = r->stats.temporal_ms + r->stats.threshold_ms;
        }
    }
    for (int i = 0; i < nq; i++) outs[i] = res[i].release();
}

void run_multi(Graph *const *gs, const folty_query *qs, int ng, Workspace &ws, Result **outs) {
    if (ng < 0) fail(FOLTY_EINVAL, "ng < 0");
    std::vector<std::unique_ptr<Result>> res(ng);
    for (int i = 0; i < ng; i++) {
        if (!gs[i]) fail(FOLTY_EINVAL, "graph %d is null", i);
        check_query(gs[i], qs[i]);
    }
    for (int i = 0; i < ng; i++) res[i].reset(run_query(gs[i], qs[i], ws));
    for (int i = 0; i < ng; i++) outs[i] = res[i].release();
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
    s->build_ms = ix.build_ms;
}

Workspace::~Workspace() {
    if (events)
        for (auto &e : ev) (void)hipEventDestroy(e);
}

void Workspace::ensure_events() {
    if (events) return;
    for (auto &e : ev) FOLTY_HIP(hipEventCreate(&e));
    events = true;
}

} // namespace folty
