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

#include "folty_internal.h"

namespace folty {

namespace {

constexpr int BLK = 256;
constexpr int WPB = BLK / 64;         // wavefronts per block
constexpr int CAP = 512;              // N+(u) staged in LDS up to this length
constexpr int IPT = 8;                // temporal tests per chunk
constexpr int PERSIST_BLOCKS = 4096;
constexpr int ENUM_BLOCKS = 4096;
constexpr int32_t CHUNK = 4096;       // closing probes per enumeration item

__device__ inline int lane_id() { return __lane_id(); }

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

template <class T> __global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// directed lists of a triangle
// ---------------------------------------------------------------------------
struct Span {
    int32_t s, n;    // start in ts, length
    int64_t lo, hi;  // first and last timestamp
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

__device__ inline void rec_spans(const EdgeRec *__restrict__ rec, int32_t p, Span &fwd, Span &bwd) {
    const int4 *q = reinterpret_cast<const int4 *>(rec + p);
    int4 a = q[0], b = q[1], c = q[2];
    fwd.s = a.x;
    fwd.n = a.y;
    bwd.s = a.z;
    bwd.n = a.w;
    fwd.lo = (int64_t)(((uint64_t)(uint32_t)b.y << 32) | (uint32_t)b.x);
    fwd.hi = (int64_t)(((uint64_t)(uint32_t)b.w << 32) | (uint32_t)b.z);
    bwd.lo = (int64_t)(((uint64_t)(uint32_t)c.y << 32) | (uint32_t)c.x);
    bwd.hi = (int64_t)(((uint64_t)(uint32_t)c.w << 32) | (uint32_t)c.z);
}

// the three oriented edges (x0,x1), (x0,x2), (x1,x2) of a triangle
__device__ inline TriLists load_lists(const EdgeRec *__restrict__ rec, int32_t p01, int32_t p02, int32_t p12) {
    TriLists L;
    rec_spans(rec, p01, L.d01, L.d10);
    rec_spans(rec, p02, L.d02, L.d20);
    rec_spans(rec, p12, L.d12, L.d21);
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
};

// A run can only count if all three lists are non-empty and some t <= t2 <= t3
// <= t + dmax is possible given each list's first and last timestamp.
template <int VAR, int I, int J>
__device__ inline bool run_lists(const TriLists &T, int64_t dmax, Span &l1, Span &l2, Span &l3) {
    using P = Pick<VAR, I, J>;
    l1 = T.template get<I, J>();
    l2 = T.template get<P::L2a, P::L2b>();
    l3 = T.template get<P::L3a, P::L3b>();
    if (l1.n == 0 || l2.n == 0 || l3.n == 0) return false;
    if (l2.hi < l1.lo || l3.hi < l2.lo) return false;
    if (l2.lo - l1.hi > dmax || l3.lo - l1.hi > dmax) return false;
    return true;
}

template <int VAR, int I, int J> __device__ inline int64_t run_work(const TriLists &T, int64_t dmax) {
    Span a, b, c;
    return run_lists<VAR, I, J>(T, dmax, a, b, c) ? a.n : 0;
}

template <int VAR> __device__ inline int64_t tri_work(const TriLists &T, int64_t dmax) {
    return run_work<VAR, 0, 1>(T, dmax) + run_work<VAR, 1, 0>(T, dmax) + run_work<VAR, 0, 2>(T, dmax) +
           run_work<VAR, 2, 0>(T, dmax) + run_work<VAR, 1, 2>(T, dmax) + run_work<VAR, 2, 1>(T, dmax);
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
struct DirectOp {
    int64_t delta;
    uint32_t *count;
    __device__ inline void operator()(const int64_t *__restrict__ ts, int32_t l1s, int32_t cnt, const Span &l2,
                                      const Span &l3) const {
        const int64_t *L2 = ts + l2.s, *L3 = ts + l3.s;
        int32_t c2 = 0, c3 = 0;
        for (int32_t q = 0; q < cnt; q++) {
            int32_t e = l1s + q;
            int64_t t = ts[e];
            c2 = lower_bound_from(L2, c2, l2.n, t);
            if (c2 == l2.n) break; // later edges are no earlier: no t2 for them either
            int64_t t2 = L2[c2];
            if (t2 - t > delta) continue;
            c3 = lower_bound_from(L3, c3, l3.n, t2);
            if (c3 == l3.n) break;
            if (L3[c3] - t <= delta) atomicAdd(&count[e], 1u);
        }
    }
};

// the smallest window per (e, w) into a histogram over sorted window levels:
// level j counts w whose smallest window lies in (lv[j-1], lv[j]]
struct PoolOp {
    const int64_t *lv;
    int nl;
    int64_t m;
    uint32_t *hist;
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
            atomicAdd(&hist[(int64_t)a * m + e], 1u);
        }
    }
};

// one run of a surviving triangle within the chunk [k, k1); r = tests of this
// triangle still to skip.  Returns false once the chunk is used up.
template <int VAR, int I, int J, class Op>
__device__ inline bool chunk_run(const TriLists &T, int64_t dmax, const int64_t *ts, int64_t &r, int64_t &k,
                                 int64_t k1, const Op &op) {
    Span l1, l2, l3;
    if (!run_lists<VAR, I, J>(T, dmax, l1, l2, l3)) return true;
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

// ---------------------------------------------------------------------------
// a.5: triangle enumeration, one wavefront per lowest vertex u
// ---------------------------------------------------------------------------
// Sinks receive every probe: hit(h, p_uv, p_uw, p_vw) is called by all lanes of
// the wave together (h = this lane found a triangle), so sinks may use ballots.
struct CountSink {
    int32_t *tri_u;
    int32_t c;
    __device__ void begin(int64_t) { c = 0; }
    __device__ void hit(bool h, int32_t, int32_t, int32_t) { c += (int32_t)__popcll(__ballot(h)); }
    __device__ void end(int64_t u) {
        if (lane_id() == 0) tri_u[u] = c;
    }
};

struct CacheSink {
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
};

struct TcntSink {
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
};

// first and last timestamp over both directed lists of an oriented edge
__device__ inline void edge_range(const EdgeRec *__restrict__ rec, int32_t p, int64_t &lo, int64_t &hi) {
    Span f, b;
    rec_spans(rec, p, f, b);
    lo = INT64_MAX;
    hi = INT64_MIN;
    if (f.n) { lo = f.lo; hi = f.hi; }
    if (b.n) { lo = b.lo < lo ? b.lo : lo; hi = b.hi > hi ? b.hi : hi; }
}

// Keeps triangles with at least one run that can count, in the slots of their
// item, with each survivor's test offset inside that item.  Every run uses one
// list of each of the three edges, and its three timestamps lie within dmax of
// each other, so the two edges at u must have time ranges within dmax of each
// other before the third edge is read at all.
template <int VAR> struct FilterSink {
    const int64_t *base;
    const EdgeRec *rec;
    int64_t dmax;
    int32_t *sv;
    int64_t *sw;
    int32_t *su;
    int64_t *wu;
    int64_t slot;
    int32_t ns;
    int64_t work;
    __device__ void begin(int64_t it) {
        slot = base[it];
        ns = 0;
        work = 0;
    }
    __device__ void hit(bool h, int32_t a, int32_t b, int32_t c) {
        int64_t wk = 0;
        if (h) {
            int64_t alo, ahi, blo, bhi;
            edge_range(rec, a, alo, ahi);
            edge_range(rec, b, blo, bhi);
            bool ranges = alo <= ahi && blo <= bhi; // every static edge has at least one temporal edge
            if (ranges && alo - bhi <= dmax && blo - ahi <= dmax) wk = tri_work<VAR>(load_lists(rec, a, b, c), dmax);
        }
        bool keep = wk > 0;
        unsigned long long mask = __ballot(keep);
        if (!mask) return;
        int64_t incl = wave_inclusive_sum(wk);
        if (keep) {
            int64_t pos = slot + ns + __popcll(mask & lanes_below());
            sv[3 * pos] = a;
            sv[3 * pos + 1] = b;
            sv[3 * pos + 2] = c;
            sw[pos] = work + incl - wk;
        }
        ns += (int32_t)__popcll(mask);
        work += __shfl(incl, 63);
    }
    __device__ void end(int64_t it) {
        if (lane_id() == 0) {
            su[it] = ns;
            wu[it] = work;
        }
    }
};

// One wavefront per item: the item's vertex u, and a range of the flattened
// wedge space of u (position q = sum of |N+(v_j)| over j < i, plus the position
// of x in N+(v_i)).
template <class Sink>
__global__ __launch_bounds__(BLK) void k_tri_enum(const int32_t *__restrict__ ooff, const int32_t *__restrict__ oadj,
                                                  const int32_t *__restrict__ item_u,
                                                  const int32_t *__restrict__ item_off, int32_t NI, Sink sink) {
    __shared__ int32_t s_nu[WPB][CAP];
    __shared__ int32_t s_vo[WPB][CAP];
    __shared__ int32_t s_pre[WPB][CAP + 1];
    const int w = threadIdx.x >> 6, lane = lane_id();
    int32_t *NU = s_nu[w], *VO = s_vo[w], *PRE = s_pre[w];
    for (int64_t it = (int64_t)blockIdx.x * WPB + w; it < NI; it += (int64_t)gridDim.x * WPB) {
        const int32_t u = item_u[it];
        const int32_t part = (int32_t)(it - item_off[u]);
        const int32_t b = ooff[u], d = ooff[u + 1] - b;
        sink.begin(it);
        if (d >= 2 && d <= CAP) {
            // stage N+(u), the row start of each v and a prefix of |N+(v)|
            int32_t carry = 0;
            for (int32_t i0 = 0; i0 < d; i0 += 64) {
                int32_t i = i0 + lane;
                int32_t dv = 0;
                if (i < d) {
                    int32_t v = oadj[b + i];
                    int32_t vo = ooff[v];
                    dv = ooff[v + 1] - vo;
                    NU[i] = v;
                    VO[i] = vo;
                }
                int32_t x = wave_inclusive_sum(dv);
                if (i < d) PRE[i + 1] = carry + x;
                carry += __shfl(x, 63);
            }
            if (lane == 0) PRE[0] = 0;
            wave_sync();
            const int32_t q_begin = part * CHUNK;
            const int32_t q_end = carry < q_begin + CHUNK ? carry : q_begin + CHUNK;
            int32_t i = 0; // this lane's segment; q only grows, so i only grows
            for (int32_t q0 = q_begin; q0 < q_end; q0 += 64) {
                int32_t q = q0 + lane;
                bool hit = false;
                int32_t pa = 0, pb = 0, pc = 0;
                if (q < q_end) {
                    int32_t lo = i, hi = d;
                    while (lo < hi) {
                        int32_t mid = (lo + hi) >> 1;
                        if (PRE[mid + 1] <= q) lo = mid + 1;
                        else hi = mid;
                    }
                    i = lo;
                    const int32_t p = VO[i] + (q - PRE[i]);
                    const int32_t x = oadj[p];
                    int32_t a = i + 1, c = d; // x > v_i, so it can only sit after i
                    while (a < c) {
                        int32_t mid = (a + c) >> 1;
                        if (NU[mid] < x) a = mid + 1;
                        else c = mid;
                    }
                    hit = a < d && NU[a] == x;
                    pa = b + i;
                    pb = b + a;
                    pc = p;
                }
                sink.hit(hit, pa, pb, pc);
            }
            wave_sync(); // the next item overwrites this wave's LDS
        } else if (d > CAP) {
            // long rows (only for orientations without the degeneracy bound): one
            // item per vertex, the same probes against N+(u) in global memory
            for (int32_t i = 0; i < d; i++) {
                const int32_t v = oadj[b + i];
                const int32_t vb = ooff[v], ve = ooff[v + 1];
                for (int32_t p0 = vb; p0 < ve; p0 += 64) {
                    const int32_t p = p0 + lane;
                    bool hit = false;
                    int32_t a = i + 1;
                    if (p < ve) {
                        const int32_t x = oadj[p];
                        int32_t c = d;
                        while (a < c) {
                            int32_t mid = (a + c) >> 1;
                            if (oadj[b + mid] < x) a = mid + 1;
                            else c = mid;
                        }
                        hit = a < d && oadj[b + a] == x;
                    }
                    sink.hit(hit, b + i, b + a, p);
                }
            }
        }
        sink.end(it);
    }
}

// cached triangle list: the same filter, one wavefront per item
template <int VAR>
__global__ __launch_bounds__(BLK) void k_filter_cached(const int64_t *__restrict__ base, const int32_t *__restrict__ tri,
                                                       int32_t NI, FilterSink<VAR> sink) {
    const int w = threadIdx.x >> 6, lane = lane_id();
    for (int64_t it = (int64_t)blockIdx.x * WPB + w; it < NI; it += (int64_t)gridDim.x * WPB) {
        const int64_t b = base[it], e = base[it + 1];
        sink.begin(it);
        for (int64_t p0 = b; p0 < e; p0 += 64) {
            int64_t p = p0 + lane;
            bool valid = p < e;
            sink.hit(valid, valid ? tri[3 * p] : 0, valid ? tri[3 * p + 1] : 0, valid ? tri[3 * p + 2] : 0);
        }
        sink.end(it);
    }
}

// ---------------------------------------------------------------------------
// a.6: temporal tests over the surviving runs, flat chunks of IPT tests
// ---------------------------------------------------------------------------
template <int VAR, class Op>
__global__ __launch_bounds__(BLK) void k_temporal(const int64_t *__restrict__ wbase, int32_t NI,
                                                  const int64_t *__restrict__ base, const int32_t *__restrict__ su,
                                                  const int32_t *__restrict__ sv, const int64_t *__restrict__ sw,
                                                  const EdgeRec *__restrict__ rec, const int64_t *__restrict__ ts,
                                                  int64_t dmax, Op op) {
    const int64_t total = wbase[NI];
    const int64_t nchunks = (total + IPT - 1) / IPT;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchunks; c += stride) {
        int64_t k = c * IPT;
        const int64_t k1 = k + IPT < total ? k + IPT : total;
        while (k < k1) {
            const int64_t k_start = k;
            // the item whose tests contain k, then the survivor inside it
            int64_t a = 0, b = NI;
            while (a < b) {
                int64_t mid = (a + b) >> 1;
                if (wbase[mid + 1] <= k) a = mid + 1;
                else b = mid;
            }
            const int64_t u = a;
            int64_t r = k - wbase[u];
            const int64_t s0 = base[u];
            const int32_t ns = su[u];
            if (ns <= 0) break; // cannot happen when the offsets are consistent
            int32_t lo = 0, hi = ns - 1;
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (sw[s0 + mid] <= r) lo = mid;
                else hi = mid - 1;
            }
            r -= sw[s0 + lo];
            for (int32_t s = lo; s < ns && k < k1; s++) {
                const int64_t p = s0 + s;
                TriLists L = load_lists(rec, sv[3 * p], sv[3 * p + 1], sv[3 * p + 2]);
                if (chunk_run<VAR, 0, 1>(L, dmax, ts, r, k, k1, op) && chunk_run<VAR, 1, 0>(L, dmax, ts, r, k, k1, op) &&
                    chunk_run<VAR, 0, 2>(L, dmax, ts, r, k, k1, op) && chunk_run<VAR, 2, 0>(L, dmax, ts, r, k, k1, op) &&
                    chunk_run<VAR, 1, 2>(L, dmax, ts, r, k, k1, op))
                    chunk_run<VAR, 2, 1>(L, dmax, ts, r, k, k1, op);
                r = 0;
            }
            if (k == k_start) break; // every survivor has tests, so this never triggers
        }
    }
}

// ---------------------------------------------------------------------------
// index helpers
// ---------------------------------------------------------------------------
__global__ void k_edge_recs(const uint32_t *__restrict__ oeid, const int32_t *__restrict__ soff,
                            const int32_t *__restrict__ smid, const int64_t *__restrict__ ts, int32_t S,
                            EdgeRec *__restrict__ rec) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S) return;
    uint32_t id = oeid[p];
    int32_t e = (int32_t)(id & 0x7fffffffu);
    int32_t a = soff[e], mid = smid[e], b = soff[e + 1];
    int32_t fs, fn, bs, bn;
    if (id >> 31) {
        fs = a; fn = mid - a; bs = mid; bn = b - mid;
    } else {
        fs = mid; fn = b - mid; bs = a; bn = mid - a;
    }
    EdgeRec r;
    r.fs = fs;
    r.fn = fn;
    r.bs = bs;
    r.bn = bn;
    r.ftmin = fn ? ts[fs] : 0;
    r.ftmax = fn ? ts[fs + fn - 1] : 0;
    r.btmin = bn ? ts[bs] : 0;
    r.btmax = bn ? ts[bs + bn - 1] : 0;
    r.sid = e;
    r.pad[0] = r.pad[1] = r.pad[2] = 0;
    rec[p] = r;
}

// closing probes of vertex u: sum over v in N+(u) of |N+(v)|; the vertex gets
// ceil(probes / CHUNK) enumeration items (one if its row is too long for LDS,
// none if it has fewer than two out-neighbours)
__global__ void k_probes(const int32_t *__restrict__ ooff, const int32_t *__restrict__ oadj, int32_t n,
                         int32_t *__restrict__ items, unsigned long long *total) {
    __shared__ unsigned long long s_sum[BLK / 64];
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long pr = 0;
    if (u < n) {
        int32_t b = ooff[u], d = ooff[u + 1] - b;
        for (int32_t i = 0; i < d; i++) {
            int32_t v = oadj[b + i];
            pr += (unsigned long long)(ooff[v + 1] - ooff[v]);
        }
        int32_t k = 0;
        if (d >= 2 && pr > 0) k = d > CAP ? 1 : (int32_t)((pr + CHUNK - 1) / CHUNK);
        items[u] = k;
    }
    for (int o = 32; o > 0; o >>= 1) pr += __shfl_xor(pr, o);
    if (lane_id() == 0) s_sum[threadIdx.x >> 6] = pr;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < BLK / 64; i++) pr += s_sum[i];
        if (pr) atomicAdd(total, pr);
    }
}

__global__ void k_item_owner(const int32_t *__restrict__ item_off, int32_t n, int32_t *__restrict__ item_u) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    for (int32_t it = item_off[u]; it < item_off[u + 1]; it++) item_u[it] = (int32_t)u;
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
    __shared__ unsigned long long s_tot[BLK / 64];
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

unsigned enum_grid(int32_t n) {
    int64_t g = ((int64_t)n + WPB - 1) / WPB;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, ENUM_BLOCKS));
}

// a.5 for one predicate code and window bound: surviving triangles per lowest
// vertex, then exclusive test offsets per vertex in ws.wbase (total at [n]).
void find_survivors(const Index &ix, int variant, int64_t dmax, Workspace &ws, hipStream_t s) {
    const int32_t NI = ix.NI;
    ws.sv.ensure(12 * (size_t)ix.T + 12);
    ws.sw.ensure(8 * (size_t)ix.T + 8);
    ws.su.ensure(4 * (size_t)NI + 4);
    ws.wu.ensure(8 * ((size_t)NI + 1));
    ws.wbase.ensure(8 * ((size_t)NI + 1));
    dispatch_variant(variant, [&](auto V) {
        FilterSink<decltype(V)::value> sink;
        sink.base = ix.tri_base.as<int64_t>();
        sink.rec = ix.rec.as<EdgeRec>();
        sink.dmax = dmax;
        sink.sv = ws.sv.as<int32_t>();
        sink.sw = ws.sw.as<int64_t>();
        sink.su = ws.su.as<int32_t>();
        sink.wu = ws.wu.as<int64_t>();
        if (ix.tri_cached)
            k_filter_cached<decltype(V)::value><<<enum_grid(NI), BLK, 0, s>>>(ix.tri_base.as<int64_t>(),
                                                                              ix.tri.as<int32_t>(), NI, sink);
        else
            k_tri_enum<<<enum_grid(NI), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.oadj.as<int32_t>(),
                                                     ix.item_u.as<int32_t>(), ix.item_off.as<int32_t>(), NI, sink);
    });
    FOLTY_LAUNCHED();
    // wu[NI] = 0 so that the exclusive scan leaves the total in wbase[NI]
    k_fill<int64_t><<<1, 1, 0, s>>>(ws.wu.as<int64_t>() + NI, (int64_t)0, 1);
    size_t need = exclusive_scan_i64(nullptr, 0, ws.wu.as<int64_t>(), ws.wbase.as<int64_t>(), (int64_t)NI + 1, s);
    ws.cub.ensure(need);
    exclusive_scan_i64(ws.cub.p, need, ws.wu.as<int64_t>(), ws.wbase.as<int64_t>(), (int64_t)NI + 1, s);
}

template <class Op>
void launch_temporal(const Index &ix, int variant, int64_t dmax, const Workspace &ws, const Op &op, hipStream_t s) {
    dispatch_variant(variant, [&](auto V) {
        k_temporal<decltype(V)::value, Op><<<PERSIST_BLOCKS, BLK, 0, s>>>(
            ws.wbase.as<int64_t>(), ix.NI, ix.tri_base.as<int64_t>(), ws.su.as<int32_t>(), ws.sv.as<int32_t>(),
            ws.sw.as<int64_t>(), ix.rec.as<EdgeRec>(), ix.ts.as<int64_t>(), dmax, op);
    });
    FOLTY_LAUNCHED();
}

void ensure_tcnt(Index &ix, hipStream_t s) {
    if (ix.tcnt_ready) return;
    ix.tcnt.ensure(4 * (size_t)ix.S + 4);
    if (ix.S > 0) {
        k_fill<int32_t><<<grid_for(ix.S, BLK, 1ll << 30), BLK, 0, s>>>(ix.tcnt.as<int32_t>(), 0, ix.S);
        FOLTY_LAUNCHED();
        TcntSink sink{ix.oeid.as<uint32_t>(), ix.tcnt.as<int32_t>()};
        k_tri_enum<<<enum_grid(ix.NI), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.oadj.as<int32_t>(),
                                                    ix.item_u.as<int32_t>(), ix.item_off.as<int32_t>(), ix.NI, sink);
        FOLTY_LAUNCHED();
    }
    ix.tcnt_ready = true;
}

// threshold + pairs for one query given device counts (sorted edge order)
void finish_query(const Graph *g, const folty_query &q, const uint32_t *count, Workspace &ws, Result *res,
                  hipStream_t s) {
    const Index &ix = g->ix;
    const int32_t S = ix.S, m = ix.m;
    ws.ncert.ensure(8 * (size_t)S + 8);
    ws.scal.ensure(64);
    k_fill<unsigned long long><<<1, 8, 0, s>>>(ws.scal.as<unsigned long long>(), 0ull, 8);
    if (S > 0) {
        k_fill<uint32_t><<<grid_for(2 * (int64_t)S, BLK, 1ll << 30), BLK, 0, s>>>(ws.ncert.as<uint32_t>(), 0u,
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

void index_triangles(Index &ix, bool cache, DevBuf &cub, hipStream_t s) {
    const int32_t n = ix.n, S = ix.S;
    ix.rec.ensure(sizeof(EdgeRec) * ((size_t)S + 1));
    ix.item_off.ensure(4 * ((size_t)n + 1));
    ix.tcnt_ready = false;
    DevBuf items, probes;
    items.ensure(4 * ((size_t)n + 1));
    probes.ensure(8);
    k_fill<unsigned long long><<<1, 1, 0, s>>>(probes.as<unsigned long long>(), 0ull, 1);
    k_fill<int32_t><<<1, 1, 0, s>>>(items.as<int32_t>() + n, 0, 1);
    FOLTY_LAUNCHED();
    if (S > 0) {
        k_edge_recs<<<grid_for(S, BLK, 1ll << 30), BLK, 0, s>>>(ix.oeid.as<uint32_t>(), ix.soff.as<int32_t>(),
                                                                ix.smid.as<int32_t>(), ix.ts.as<int64_t>(), S,
                                                                ix.rec.as<EdgeRec>());
        FOLTY_LAUNCHED();
    }
    k_probes<<<grid_for(n, BLK, 1ll << 30), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.oadj.as<int32_t>(), n,
                                                          items.as<int32_t>(), probes.as<unsigned long long>());
    FOLTY_LAUNCHED();
    {
        size_t need = exclusive_scan_i32(nullptr, 0, items.as<int32_t>(), ix.item_off.as<int32_t>(), (int64_t)n + 1, s);
        cub.ensure(need);
        exclusive_scan_i32(cub.p, need, items.as<int32_t>(), ix.item_off.as<int32_t>(), (int64_t)n + 1, s);
    }
    int64_t h[2] = {0, 0};
    int32_t ni = 0;
    FOLTY_HIP(hipMemcpyAsync(&ni, ix.item_off.as<int32_t>() + n, 4, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipMemcpyAsync(&h[1], probes.p, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    ix.NI = ni;
    ix.probes = h[1];
    ix.item_u.ensure(4 * (size_t)ni + 4);
    ix.tri_base.ensure(8 * ((size_t)ni + 1));
    k_item_owner<<<grid_for(n, BLK, 1ll << 30), BLK, 0, s>>>(ix.item_off.as<int32_t>(), n, ix.item_u.as<int32_t>());
    FOLTY_LAUNCHED();
    DevBuf tri_it;
    tri_it.ensure(4 * ((size_t)ni + 1));
    k_fill<int32_t><<<1, 1, 0, s>>>(tri_it.as<int32_t>() + ni, 0, 1);
    CountSink cs{tri_it.as<int32_t>(), 0};
    k_tri_enum<<<enum_grid(ni), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.oadj.as<int32_t>(), ix.item_u.as<int32_t>(),
                                             ix.item_off.as<int32_t>(), ni, cs);
    FOLTY_LAUNCHED();
    size_t need = exclusive_scan_i32_to_i64(nullptr, 0, tri_it.as<int32_t>(), ix.tri_base.as<int64_t>(), (int64_t)ni + 1, s);
    cub.ensure(need);
    exclusive_scan_i32_to_i64(cub.p, need, tri_it.as<int32_t>(), ix.tri_base.as<int64_t>(), (int64_t)ni + 1, s);
    FOLTY_HIP(hipMemcpyAsync(&h[0], ix.tri_base.as<int64_t>() + ni, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    ix.T = h[0];
    ix.tri_cached = false;
    ix.tri.release();
    if (cache && ix.T > 0) {
        ix.tri.ensure(12 * (size_t)ix.T);
        CacheSink sink{ix.tri_base.as<int64_t>(), ix.tri.as<int32_t>(), 0};
        k_tri_enum<<<enum_grid(ni), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.oadj.as<int32_t>(), ix.item_u.as<int32_t>(),
                                                 ix.item_off.as<int32_t>(), ni, sink);
        FOLTY_LAUNCHED();
        ix.tri_cached = true;
    }
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
    Index &ix = g->ix;
    hipStream_t s = g->stream;
    if (q.universe == FOLTY_UNIVERSE_COMMON) ensure_tcnt(ix, s);
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
        find_survivors(ix, q.variant, q.delta, ws, s);
        FOLTY_HIP(hipEventRecord(ws.ev[1], s));
        DirectOp op{q.delta, count};
        launch_temporal(ix, q.variant, q.delta, ws, op, s);
        FOLTY_HIP(hipMemcpyAsync(&tests, ws.wbase.as<int64_t>() + ix.NI, 8, hipMemcpyDeviceToHost, s));
    } else {
        FOLTY_HIP(hipEventRecord(ws.ev[1], s));
    }
    FOLTY_HIP(hipEventRecord(ws.ev[2], s));
    finish_query(g, q, count, ws, res.get(), s);
    FOLTY_HIP(hipEventRecord(ws.ev[3], s));
    if (!(q.flags & FOLTY_QUERY_NO_COUNTS)) keep_counts(g, count, res.get(), s);
    FOLTY_HIP(hipStreamSynchronize(s));
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
    Index &ix = g->ix;
    hipStream_t s = g->stream;
    std::map<int, std::vector<int>> by_var;
    bool need_tcnt = false;
    for (int i = 0; i < nq; i++) {
        by_var[qs[i].variant].push_back(i);
        need_tcnt = need_tcnt || qs[i].universe == FOLTY_UNIVERSE_COMMON;
    }
    if (need_tcnt) ensure_tcnt(ix, s);
    std::vector<std::unique_ptr<Result>> res(nq);
    for (int i = 0; i < nq; i++) res[i].reset(new Result());
    ws.ensure_events();
    for (auto &kv : by_var) {
        int variant = kv.first;
        std::vector<int64_t> lv;
        for (int i : kv.second) lv.push_back(qs[i].delta);
        std::sort(lv.begin(), lv.end());
        lv.erase(std::unique(lv.begin(), lv.end()), lv.end());
        const int nl = (int)lv.size();
        const int64_t dmax = lv.back();
        FOLTY_HIP(hipEventRecord(ws.ev[0], s));
        ws.hist.ensure(4 * (size_t)nl * (size_t)ix.m + 4);
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
            find_survivors(ix, variant, dmax, ws, s);
            PoolOp op{lvd.as<int64_t>(), nl, ix.m, ws.hist.as<uint32_t>()};
            launch_temporal(ix, variant, dmax, ws, op, s);
            k_hist_prefix<<<grid_for(ix.m, BLK, 1ll << 30), BLK, 0, s>>>(ws.hist.as<uint32_t>(), nl, ix.m);
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipMemcpyAsync(&tests, ws.wbase.as<int64_t>() + ix.NI, 8, hipMemcpyDeviceToHost, s));
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
    for (int i = 0; i < ng; i++) {
        StreamScope sc(gs[i]->stream);
        res[i].reset(run_query(gs[i], qs[i], ws));
    }
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
    s->closing_probes = ix.probes;
    s->enum_items = ix.NI;
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
