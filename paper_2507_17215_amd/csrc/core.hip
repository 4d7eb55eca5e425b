// Core numbers and the degeneracy rank (paper, Section "Main Ideas",
// Preliminaries: the degeneracy ordering by repeated removal of a vertex of
// minimum degree).
//
// The order built here is the one that level-synchronous min-degree peeling
// gives: at level k, rounds remove every remaining vertex with at most k
// remaining neighbours until none is left; a vertex's rank key is (core number,
// round within its level, id).  A vertex removed in a round of level k has at
// most k neighbours left at that point, and all of them rank after it, so every
// out-degree of the orientation is at most the vertex's core number, hence at
// most the degeneracy.
//
// Peeling the levels one after another is a chain of one dependent step per
// round of every level (thousands of rounds on power-law graphs).  Two facts
// break the chain:
//  1. Core numbers are the largest fixed point below the degrees of
//     c(v) = H({c(u) : u in N(v)}), with H the h-index (the largest h such that
//     at least h of the values are >= h).  Lowering values towards it in any
//     order converges, also when neighbours' values are read while they change:
//     each value stays an upper bound of the core number.  A sweep re-evaluates
//     only the vertices that a neighbour's drop may have affected.
//  2. Once core numbers are known, the rounds of level k involve only the
//     k-core: the vertices of core k, which it removes, and those of higher
//     core, which stay.  A vertex v of core k starts level k with
//     cnt(v) = |{u in N(v) : core(u) >= k}| remaining neighbours, loses one per
//     removed neighbour of core k, and goes in the first round at which
//     cnt(v) <= k.  Levels therefore do not interact, and all of them are
//     peeled at once: the dependent rounds are only as many as the most any one
//     level needs, and every vertex gets the same round within its level as in
//     the level-by-level peel.
#include <cmath>

#include "folty_internal.h"

namespace folty {

namespace {

constexpr int BLK = 256;
constexpr int WPB = BLK / 64;
constexpr int GRID = 2048;           // persistent grid of the sweep and round kernels
constexpr int FIN_GRID = 2048;       // grid of the kernels over long rows only (a block per row, latency-bound)
constexpr int32_t C0_MAX = 16;       // rows up to this length: one lane per vertex
constexpr int32_t C1_MAX = 1024;     // up to this length: one wavefront per vertex (16 entries per lane)
constexpr int32_t CH = 2048;         // row work on longer rows goes in chunks of this many entries
constexpr int32_t CPT = CH / BLK;    // chunk entries per thread
constexpr int32_t HX_BINS = 4096;    // LDS histogram of the h-index of a long row
constexpr int32_t HG_BINS = (1 << 16) + 1; // degree histogram for the global h-index: levels up to 2^16 - 1,
                                           // and one bin above
constexpr int32_t HG_LDS = 1024;     // degrees below this are counted in LDS first
// Buffered list entries per wavefront and class.  Every flush is an atomic on
// one of a few counters, and those serialise (about 10 ns each): listing all 4M
// vertices of the 70M-edge graph took 172 us with 256 entries, 79 us with 1024
// (the level counts' frontier 127 -> 42 us); 32 KB of LDS per block.
constexpr int PB_CAP = 1024;
// Sweeps that rescan long rows before their histograms are kept and the rows
// reordered (70M edges, build ms: 4 -> 19.8, 3 -> 19.9, 5 -> 20.0, 8 -> 20.3).
constexpr int RESCAN_SWEEPS = 4;
// Sweeps that evaluate every vertex, without marking: early on most vertices
// drop in each sweep, and a marking pass over their rows plus a sweep over the
// listed ones costs more than one sweep over all (70M edges, 32-bit values:
// sweep over all 0.74 ms; marking + listed sweep 1.58, 1.18, 0.89, 0.66 ms for
// sweeps 1-4; build ms with 4 rescanning sweeps: 2 dense 20.5, 3 20.1, 4 19.8).
constexpr int DENSE_SWEEPS = 4;
static_assert(DENSE_SWEEPS >= 1 && DENSE_SWEEPS <= RESCAN_SWEEPS, "kept histograms need every drop marked");

__device__ inline int lane_id() { return __lane_id(); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int32_t wave_sum(int32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// rows of up to C0_MAX entries (class 0), up to C1_MAX (class 1), longer ("long rows", class 2)
__device__ inline int row_class(int32_t d) { return d <= C0_MAX ? 0 : (d <= C1_MAX ? 1 : 2); }

// Counters (int32 words of one small device array).  A list set has four:
// vertex lists of classes 0, 1 and 2, then a list of (vertex, chunk) pairs that
// splits the row work of its class-2 vertices.
enum : int {
    CT_ALL = 0,     // [4]     every vertex (sweep 0 and the level counts)
    CT_H = 4,       // [2][4]  vertices to re-evaluate, by sweep parity
    CT_D = 12,      // [2][4]  vertices whose value dropped, by sweep parity
    CT_F = 20,      // [3][4]  round frontiers, by round mod 3
    CT_HG = 32,     // global h-index of the degrees
    CT_SWEEPS = 33, // sweeps with work
    CT_ROUNDS = 34, // rounds with work
    CT_LEFT = 35,   // vertices without a round (must stay 0)
    CT_WORDS = 40
};

// where class-2 appends go: the vertex list, the chunk list (row work), or both
enum : int { BIG_VERTEX = 1, BIG_CHUNKS = 2, BIG_BOTH = 3 };

struct ListSet {
    int32_t *l[3];
    int2 *ch;
    int32_t *cnt; // [4]
    int big;      // BIG_*
};

struct CoreBufs {
    const int64_t *uoff;
    const int32_t *uadj;
    const int32_t *deg;
    uint16_t *c;    // upper bound of the core number; the core number at the end (values
                    // are at most the h-index of the degrees, below 2^16 for fewer than
                    // 2^31 static edges; 16 bits halve the bytes every gather moves)
    int32_t *old;   // value before this sweep's drop
    int32_t *stamp; // 1 + the sweep that last listed the vertex
    int32_t *cnt;   // remaining neighbours in the vertex's level (rounds)
    int32_t *lr;    // round within the level
    int32_t *bigid; // slot of a class-2 vertex (its place in all[2] and in gh)
    int32_t *gh;    // per class-2 vertex: how many neighbours hold each value, capped at its own
    int32_t hbw;    // histogram levels per class-2 vertex (0: they do not fit; rows are rescanned)
    // Once the histograms are kept: each class-2 row reordered by its
    // neighbours' values at that point (capped at the row's own value x0),
    // highest first, in hadj at the row's place in uadj; pc[k] = how many of
    // its entries had value >= k then (k <= x0).  Values only fall, so a
    // neighbour whose value is >= k now lies in the first pc[k] entries.
    const int32_t *hadj; // null while rows are rescanned
    const int32_t *pc;
    int32_t *ctr;
    int32_t *all[3];
    int2 *allc;
    int32_t *pool[8]; // sweeps: [3 * parity + class] re-evaluation lists, [6 + class] dropped;
                      // rounds: [2 * (round mod 3) + class] frontiers
    int2 *poolc[3];   // sweeps: [0] dropped chunks, [1 + parity] re-evaluation chunks;
                      // rounds: frontier chunks by round mod 3
    int32_t n;
};

// entries of class-2 row v (reordered) whose value was >= k at the reorder; k <= x0
__device__ inline int32_t big_prefix(const CoreBufs &B, int32_t v, int32_t k) {
    return B.pc[(int64_t)B.bigid[v] * B.hbw + k];
}

__device__ inline ListSet list_set(int32_t *l0, int32_t *l1, int32_t *l2, int2 *ch, int32_t *cnt, int big) {
    ListSet L;
    L.l[0] = l0;
    L.l[1] = l1;
    L.l[2] = l2;
    L.ch = ch;
    L.cnt = cnt;
    L.big = big;
    return L;
}

__device__ inline void push_chunks(const ListSet &L, int32_t v, int32_t d) {
    const int32_t nch = (d + CH - 1) / CH;
    const int32_t base = atomicAdd(&L.cnt[3], nch);
    for (int32_t i = 0; i < nch; i++) L.ch[base + i] = make_int2(v, i);
}

// a class-2 vertex: one atomic each (they are few)
__device__ inline void push_big(const ListSet &L, int32_t v, int32_t d) {
    if (L.big & BIG_CHUNKS) push_chunks(L, v, d);
    if (L.big & BIG_VERTEX) L.l[2][atomicAdd(&L.cnt[2], 1)] = v;
}

// Class 0/1 appends go through per-wavefront LDS buffers (one atomic per PB_CAP
// entries, and at the end one atomic per block and class), so thousands of
// wavefronts do not serialise on two counters.
struct PushLds {
    int32_t buf[WPB][2][PB_CAP];
    int32_t wn[WPB][2];
    int32_t base[WPB][2];
};

struct Pusher {
    PushLds *P;
    ListSet L;
    int32_t n[2]; // entries in this wavefront's buffers (wavefront-uniform)
};

__device__ inline void push_flush_wave(Pusher &p, int j) {
    const int w = threadIdx.x >> 6, lane = lane_id();
    wave_sync();
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&p.L.cnt[j], p.n[j]);
    base = __shfl(base, 0);
    for (int32_t i = lane; i < p.n[j]; i += 64) p.L.l[j][base + i] = p.P->buf[w][j][i];
    p.n[j] = 0;
    wave_sync();
}

// every lane of the wavefront calls this; cls 0/1 appends val to that list,
// cls 2 appends it as a class-2 vertex (d = its row length), anything else nothing
__device__ inline void push(Pusher &p, int cls, int32_t val, int32_t d) {
    const int w = threadIdx.x >> 6, lane = lane_id();
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const unsigned long long mask = __ballot(cls == j);
        if (!mask) continue;
        const int32_t c = (int32_t)__popcll(mask);
        if (p.n[j] + c > PB_CAP) push_flush_wave(p, j);
        if (cls == j) p.P->buf[w][j][p.n[j] + (int32_t)__popcll(mask & ((1ull << lane) - 1ull))] = val;
        p.n[j] += c;
    }
    if (cls == 2) push_big(p.L, val, d);
    wave_sync();
}

// end of the kernel: every thread of the block calls this
__device__ inline void push_finish(Pusher &p) {
    const int w = threadIdx.x >> 6, lane = lane_id();
    if (lane == 0)
        for (int j = 0; j < 2; j++) p.P->wn[w][j] = p.n[j];
    __syncthreads();
    if (threadIdx.x < 2) {
        const int j = threadIdx.x;
        int32_t tot = 0;
        for (int k = 0; k < WPB; k++) tot += p.P->wn[k][j];
        int32_t b = tot ? atomicAdd(&p.L.cnt[j], tot) : 0;
        for (int k = 0; k < WPB; k++) {
            p.P->base[k][j] = b;
            b += p.P->wn[k][j];
        }
    }
    __syncthreads();
    for (int j = 0; j < 2; j++)
        for (int32_t i = lane; i < p.n[j]; i += 64) p.L.l[j][p.P->base[w][j] + i] = p.P->buf[w][j][i];
}

__device__ inline Pusher make_pusher(PushLds *P, const ListSet &L) {
    Pusher p;
    p.P = P;
    p.L = L;
    p.n[0] = p.n[1] = 0;
    return p;
}

// ---- global h-index of the degrees: an upper bound of every core number -----------
// degrees above `cap` are counted in bin cap
__global__ __launch_bounds__(BLK) void k_deg_hist(const int32_t *__restrict__ deg, int32_t n, int32_t cap,
                                                  int32_t *__restrict__ hist) {
    __shared__ int32_t s_h[HG_LDS];
    for (int i = threadIdx.x; i < HG_LDS; i += BLK) s_h[i] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * BLK + threadIdx.x; v < n; v += (int64_t)gridDim.x * BLK) {
        int32_t d = deg[v];
        d = d < cap ? d : cap;
        if (d < HG_LDS) atomicAdd(&s_h[d], 1);
        else atomicAdd(&hist[d], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HG_LDS; i += BLK)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// the largest h with at least h counts at or above h.  h vertices of degree >= h
// hold h^2 <= sum of degrees entries, so h <= top = floor(sqrt(sum)) (at most
// 2^16 - 1 for fewer than 2^31 static edges); bin top + 1 counts every degree
// above top, and thread t walks the levels top - t * per down to
// top - (t + 1) * per + 1.
__global__ __launch_bounds__(BLK) void k_global_h(const int32_t *__restrict__ hist, int32_t top, int32_t *ctr) {
    __shared__ int64_t s_tot[BLK];
    __shared__ int32_t s_best;
    const int t = threadIdx.x;
    const int32_t per = (top + 1 + BLK - 1) / BLK;
    const int32_t hi = top - t * per;
    int64_t mine = 0;
    for (int32_t i = 0; i < per && hi - i >= 0; i++) mine += hist[hi - i];
    s_tot[t] = mine;
    if (t == 0) s_best = 0;
    __syncthreads();
    int64_t above = hist[top + 1];
    for (int k = 0; k < t; k++) above += s_tot[k];
    for (int32_t i = 0; i < per && hi - i >= 0; i++) {
        const int32_t h = hi - i;
        above += hist[h];
        if (above >= h) {
            atomicMax(&s_best, h);
            break;
        }
    }
    __syncthreads();
    if (t == 0) ctr[CT_HG] = s_best;
}

// c = min(deg, global h-index); every vertex listed; class-2 vertices also get
// their slot and their rows' chunks
__global__ __launch_bounds__(BLK) void k_core_init(CoreBufs B) {
    __shared__ PushLds P;
    const int32_t hg = B.ctr[CT_HG];
    Pusher p = make_pusher(&P, list_set(B.all[0], B.all[1], B.all[2], B.allc, B.ctr + CT_ALL, BIG_VERTEX));
    const int64_t stride = (int64_t)gridDim.x * BLK;
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < B.n; base += stride) {
        const int64_t v = base + threadIdx.x;
        int cls = -1;
        int32_t d = 0;
        if (v < B.n) {
            d = B.deg[v];
            B.c[v] = (uint16_t)(d < hg ? d : hg);
            B.stamp[v] = 0;
            B.cnt[v] = 0;
            B.lr[v] = -1;
            cls = row_class(d);
        }
        // class-2 vertices: slots and chunk ranges, one atomic per wavefront on
        // each of the two counters
        const bool big = cls == 2;
        const unsigned long long bm = __ballot(big);
        if (bm) {
            const int32_t nch = big ? (d + CH - 1) / CH : 0;
            int32_t incl = nch;
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(incl, o);
                if (lane_id() >= o) incl += y;
            }
            int32_t id0 = 0, ch0 = 0;
            if (lane_id() == 63) {
                id0 = atomicAdd(&B.ctr[CT_ALL + 2], (int32_t)__popcll(bm));
                ch0 = atomicAdd(&B.ctr[CT_ALL + 3], incl);
            }
            id0 = __shfl(id0, 63);
            ch0 = __shfl(ch0, 63);
            if (big) {
                const int32_t id = id0 + (int32_t)__popcll(bm & ((1ull << lane_id()) - 1ull));
                B.bigid[v] = id;
                B.all[2][id] = (int32_t)v;
                for (int32_t i = 0; i < nch; i++) B.allc[ch0 + incl - nch + i] = make_int2((int32_t)v, i);
            }
        }
        push(p, cls < 2 ? cls : -1, (int32_t)v, 0);
    }
    push_finish(p);
}

// the chunk's entries: row positions lo + j * BLK + t, j < CPT, below hi
struct ChunkRow {
    int32_t u[CPT];
    bool ok[CPT];
};

__device__ inline ChunkRow load_chunk(const int32_t *__restrict__ adj, int64_t b, int32_t lo, int32_t hi) {
    ChunkRow r;
#pragma unroll
    for (int j = 0; j < CPT; j++) {
        const int32_t q = lo + j * BLK + (int32_t)threadIdx.x;
        r.ok[j] = q < hi;
        r.u[j] = r.ok[j] ? adj[b + q] : 0;
    }
    return r;
}

// Histogram of each long row's neighbour values, capped at the row's own value,
// from the current values (no kernel changes them while this runs); the marking
// kernels keep it up to date from then on.
__global__ __launch_bounds__(BLK) void k_big_hist(CoreBufs B) {
    __shared__ int32_t s_h[HX_BINS];
    const int32_t n2 = B.ctr[CT_ALL + 3];
    const int t = threadIdx.x;
    for (int32_t i = blockIdx.x; i < n2; i += gridDim.x) {
        const int2 ck = B.allc[i];
        const int32_t v = ck.x;
        const int64_t b = B.uoff[v];
        const int32_t d = (int32_t)(B.uoff[v + 1] - b);
        const int32_t x = B.c[v];
        const int32_t lo = ck.y * CH, hi = lo + CH < d ? lo + CH : d;
        for (int32_t k = t; k <= x; k += BLK) s_h[k] = 0;
        __syncthreads();
        const ChunkRow r = load_chunk(B.uadj, b, lo, hi);
        int32_t y[CPT];
#pragma unroll
        for (int j = 0; j < CPT; j++) y[j] = r.ok[j] ? B.c[r.u[j]] : -1;
#pragma unroll
        for (int j = 0; j < CPT; j++)
            if (y[j] >= 0) atomicAdd(&s_h[y[j] < x ? y[j] : x], 1);
        __syncthreads();
        int32_t *gh = B.gh + (int64_t)B.bigid[v] * B.hbw;
        for (int32_t k = t; k <= x; k += BLK)
            if (s_h[k]) atomicAdd(&gh[k], s_h[k]);
        __syncthreads();
    }
}

// Reorder of the class-2 rows when their histograms start being kept, from the
// same values as k_big_hist (nothing changes them in between).  k_big_prefix:
// per row, pc[k] = entries at level >= k (level = min(value, x0)) from the
// fresh histogram, and the write cursor of level k = entries above it.
__global__ __launch_bounds__(BLK) void k_big_prefix(CoreBufs B, int32_t *__restrict__ pc, int32_t *__restrict__ cur) {
    __shared__ int32_t s_h[HX_BINS];
    __shared__ int32_t s_sum[BLK];
    const int32_t n2 = B.ctr[CT_ALL + 2];
    const int t = threadIdx.x;
    for (int32_t i = blockIdx.x; i < n2; i += gridDim.x) {
        const int32_t v = B.all[2][i];
        const int32_t x = B.c[v];
        const int64_t row = (int64_t)B.bigid[v] * B.hbw;
        for (int32_t k = t; k <= x; k += BLK) s_h[k] = B.gh[row + k];
        __syncthreads();
        // thread t sums the levels [t * per, (t + 1) * per), then walks them top down
        const int32_t per = (x + 1 + BLK - 1) / BLK;
        const int32_t lo = t * per, hi = lo + per < x + 1 ? lo + per : x + 1;
        int32_t part = 0;
        for (int32_t k = lo; k < hi; k++) part += s_h[k];
        s_sum[t] = part;
        __syncthreads();
        int32_t above = 0;
        for (int k = t + 1; k < BLK; k++) above += s_sum[k];
        for (int32_t k = hi - 1; k >= lo; k--) {
            cur[row + k] = above;
            above += s_h[k];
            pc[row + k] = above;
        }
        for (int32_t k = x + 1 + t; k < B.hbw; k += BLK) pc[row + k] = 0;
        __syncthreads();
    }
}

// k_big_scatter: each chunk reserves, per level, a range of its row's level
// (one global atomic per level present), then places its entries in LDS order.
__global__ __launch_bounds__(BLK) void k_big_scatter(CoreBufs B, int32_t *__restrict__ cur,
                                                     int32_t *__restrict__ hadj) {
    __shared__ int32_t s_h[HX_BINS];
    const int32_t n2 = B.ctr[CT_ALL + 3];
    const int t = threadIdx.x;
    for (int32_t i = blockIdx.x; i < n2; i += gridDim.x) {
        const int2 ck = B.allc[i];
        const int32_t v = ck.x;
        const int64_t b = B.uoff[v];
        const int32_t d = (int32_t)(B.uoff[v + 1] - b);
        const int32_t x = B.c[v];
        const int32_t lo = ck.y * CH, hi = lo + CH < d ? lo + CH : d;
        for (int32_t k = t; k <= x; k += BLK) s_h[k] = 0;
        __syncthreads();
        const ChunkRow r = load_chunk(B.uadj, b, lo, hi);
        int32_t y[CPT];
#pragma unroll
        for (int j = 0; j < CPT; j++) {
            y[j] = r.ok[j] ? B.c[r.u[j]] : -1;
            y[j] = y[j] < x ? y[j] : x;
        }
#pragma unroll
        for (int j = 0; j < CPT; j++)
            if (y[j] >= 0) atomicAdd(&s_h[y[j]], 1);
        __syncthreads();
        int32_t *cr = cur + (int64_t)B.bigid[v] * B.hbw;
        for (int32_t k = t; k <= x; k += BLK)
            if (s_h[k]) s_h[k] = atomicAdd(&cr[k], s_h[k]);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPT; j++)
            if (y[j] >= 0) hadj[b + atomicAdd(&s_h[y[j]], 1)] = r.u[j];
        __syncthreads();
    }
}

// ---- h-index evaluations ---------------------------------------------------------------
// H capped at x (the current value): the largest h <= x with count(>= h) >= h.
// count(ge) >= ge for ge = count(>= x) < x, so the search runs over [ge, x - 1].

// Both also give ge_out = count(>= the answer) over the row, which is the
// vertex's count of neighbours at or above its own value.
__device__ inline int32_t h_lane(const uint16_t *c, const int32_t *__restrict__ adj, int64_t b, int32_t d,
                                 int32_t x, int32_t &ge_out) {
    int32_t u[C0_MAX], val[C0_MAX];
#pragma unroll
    for (int j = 0; j < C0_MAX; j++) u[j] = j < d ? adj[b + j] : 0;
#pragma unroll
    for (int j = 0; j < C0_MAX; j++) val[j] = j < d ? c[u[j]] : -1;
    auto count = [&](int32_t h) {
        int32_t k = 0;
#pragma unroll
        for (int j = 0; j < C0_MAX; j++) k += val[j] >= h ? 1 : 0;
        return k;
    };
    const int32_t ge = count(x);
    if (ge >= x) {
        ge_out = ge;
        return x;
    }
    int32_t lo = ge, hi = x - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (count(mid) >= mid) lo = mid;
        else hi = mid - 1;
    }
    ge_out = count(lo);
    return lo;
}

// one wavefront; x, b, d are wavefront-uniform
template <int NJ>
__device__ inline int32_t h_wave_n(const uint16_t *c, const int32_t *__restrict__ adj, int64_t b, int32_t d,
                                   int32_t x, int32_t &ge_out) {
    const int lane = lane_id();
    int32_t u[NJ], val[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int32_t i = lane + 64 * j;
        u[j] = i < d ? adj[b + i] : 0;
    }
#pragma unroll
    for (int j = 0; j < NJ; j++) val[j] = lane + 64 * j < d ? c[u[j]] : -1;
    auto count = [&](int32_t h) {
        int32_t k = 0;
#pragma unroll
        for (int j = 0; j < NJ; j++) k += val[j] >= h ? 1 : 0;
        return wave_sum(k);
    };
    const int32_t ge = count(x);
    if (ge >= x) {
        ge_out = ge;
        return x;
    }
    int32_t lo = ge, hi = x - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (count(mid) >= mid) lo = mid;
        else hi = mid - 1;
    }
    ge_out = count(lo);
    return lo;
}

// NJ = the row's 64-entry slots rounded up to a power of two (wavefront-uniform):
// most rows of this class fill one or two slots of the sixteen
__device__ inline int32_t h_wave(const uint16_t *c, const int32_t *__restrict__ adj, int64_t b, int32_t d,
                                 int32_t x, int32_t &ge_out) {
    static_assert(C1_MAX / 64 == 16, "slot classes");
    if (d <= 64) return h_wave_n<1>(c, adj, b, d, x, ge_out);
    if (d <= 128) return h_wave_n<2>(c, adj, b, d, x, ge_out);
    if (d <= 256) return h_wave_n<4>(c, adj, b, d, x, ge_out);
    if (d <= 512) return h_wave_n<8>(c, adj, b, d, x, ge_out);
    return h_wave_n<16>(c, adj, b, d, x, ge_out);
}

// A row of at most 64 entries over a group of 16 lanes (four entries each); b,
// d and x are uniform within the group, and sums stay inside it.
__device__ inline int32_t h_group16(const uint16_t *c, const int32_t *__restrict__ adj, int64_t b, int32_t d,
                                    int32_t x, int32_t &ge_out) {
    const int gl = lane_id() & 15;
    int32_t u[4], val[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int32_t i = gl + 16 * j;
        u[j] = i < d ? adj[b + i] : 0;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) val[j] = gl + 16 * j < d ? c[u[j]] : -1;
    auto count = [&](int32_t h) {
        int32_t k = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) k += val[j] >= h ? 1 : 0;
        for (int o = 8; o > 0; o >>= 1) k += __shfl_xor(k, o);
        return k;
    };
    const int32_t ge = count(x);
    if (ge >= x) {
        ge_out = ge;
        return x;
    }
    int32_t lo = ge, hi = x - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (count(mid) >= mid) lo = mid;
        else hi = mid - 1;
    }
    ge_out = count(lo);
    return lo;
}

// A block's histogram workspace in dynamic LDS: bins levels (the per-row
// histogram width, or HX_BINS for windowed evaluation), a sum per thread and the
// answer.  Sized to the graph, so kernels that carry it keep their occupancy
// (70M edges: 1,468 levels, 7 KB instead of 17 KB).
struct HxView {
    int32_t *hist;
    int32_t *tsum;
    int32_t *best;
};
__device__ inline HxView hx_view(int32_t *base, int32_t bins) {
    HxView v;
    v.hist = base;
    v.tsum = base + bins;
    v.best = base + bins + BLK;
    return v;
}
__host__ __device__ inline int32_t hx_bins(int32_t hbw) { return hbw > 0 ? hbw : HX_BINS; }
inline size_t hx_bytes(int32_t hbw) { return 4 * ((size_t)hx_bins(hbw) + BLK + 1); }

// With hist[i] = how many values equal bot + i (values above top counted in
// `above`): the largest h in [bot, top] with count(>= h) >= h, or -1.  Thread t
// walks the levels top - t * per down to top - (t + 1) * per + 1.
__device__ inline int32_t window_best(const HxView &L, int32_t bot, int32_t top, int32_t above) {
    const int t = threadIdx.x;
    const int32_t nb = top - bot + 1;
    const int32_t per = (nb + BLK - 1) / BLK;
    const int32_t hi_t = top - t * per;
    if (t == 0) *L.best = -1;
    int32_t s = 0;
    for (int32_t i = 0; i < per; i++) {
        const int32_t h = hi_t - i;
        if (h >= bot) s += L.hist[h - bot];
    }
    L.tsum[t] = s;
    __syncthreads();
    int32_t run = above;
    for (int k = 0; k < t; k++) run += L.tsum[k];
    for (int32_t i = 0; i < per; i++) {
        const int32_t h = hi_t - i;
        if (h < bot) break;
        run += L.hist[h - bot];
        if (run >= h) {
            atomicMax(L.best, h);
            break;
        }
    }
    __syncthreads();
    const int32_t best = *L.best;
    __syncthreads();
    return best;
}

// One block over a whole row: LDS histograms of windows of at most HX_BINS
// levels, from the top down until one holds the answer.  Used only when the
// per-row histograms would not fit (h-index of the degrees at or above HX_BINS).
__device__ inline int32_t h_block(const uint16_t *c, const int32_t *__restrict__ adj, int64_t b, int32_t d,
                                  int32_t x, const HxView &L) {
    const int t = threadIdx.x;
    int32_t top = x;
    int32_t above = 0;
    for (;;) {
        const int32_t bot = top - (HX_BINS - 1) > 0 ? top - (HX_BINS - 1) : 0;
        const int32_t nb = top - bot + 1;
        for (int32_t i = t; i < nb; i += BLK) L.hist[i] = 0;
        __syncthreads();
        // values are capped at x; those above top (below x) are already in `above`
        for (int64_t q = t; q < d; q += BLK) {
            int32_t y = c[adj[b + q]];
            y = y < x ? y : x;
            if (y >= bot && y <= top) atomicAdd(&L.hist[y - bot], 1);
        }
        __syncthreads();
        const int32_t best = window_best(L, bot, top, above);
        if (best >= 0 || bot == 0) return best >= 0 ? best : 0;
        for (int k = 0; k < BLK; k++) above += L.tsum[k];
        top = bot - 1;
        __syncthreads();
    }
}

// Sweep s, long rows: a listed row is re-evaluated from its histogram (or, if
// histograms do not fit, from its row).  With `rescan` the histogram was made
// by this sweep's k_core_sweep and is cleared after use; otherwise it is the
// kept one, and a drop to h folds its levels above h into level h.  Every
// thread of the block calls this.
__device__ inline void finish_rows(const CoreBufs &B, int32_t s, bool rescan, bool dense, bool list,
                                   const HxView &H) {
    int32_t *ctr = B.ctr;
    const int par = s & 1;
    const int32_t n2 = dense ? ctr[CT_ALL + 2] : ctr[CT_H + 4 * par + 2];
    const int32_t *L2 = dense ? B.all[2] : B.pool[3 * par + 2];
    const ListSet D = list_set(B.pool[6], B.pool[7], nullptr, B.poolc[0], ctr + CT_D + 4 * par, BIG_CHUNKS);
    const int t = threadIdx.x;
    for (int32_t i = blockIdx.x; i < n2; i += gridDim.x) {
        const int32_t v = L2[i];
        const int32_t x = B.c[v];
        const int64_t b = B.uoff[v];
        const int32_t d = (int32_t)(B.uoff[v + 1] - b);
        int32_t h = x;
        if (B.hbw > 0 && rescan) {
            int32_t *gh = B.gh + (int64_t)B.bigid[v] * B.hbw;
            for (int32_t k = t; k <= x; k += BLK) {
                H.hist[k] = gh[k];
                gh[k] = 0;
            }
            __syncthreads();
            h = window_best(H, 0, x, 0);
        } else if (B.hbw > 0) {
            int32_t *gh = B.gh + (int64_t)B.bigid[v] * B.hbw;
            if (gh[x] < x) { // block-uniform: only this block writes gh[v] during the sweep
                for (int32_t k = t; k <= x; k += BLK) H.hist[k] = gh[k];
                __syncthreads();
                h = window_best(H, 0, x, 0);
                // level h now holds every value at or above h
                int32_t part = 0;
                for (int32_t k = h + 1 + t; k <= x; k += BLK) {
                    part += H.hist[k];
                    gh[k] = 0;
                }
                part = wave_sum(part);
                if (lane_id() == 0 && part) atomicAdd(&gh[h], part);
            }
        } else {
            h = h_block(B.c, B.uadj, b, d, x, H);
        }
        if (t == 0 && h < x) {
            B.old[v] = x;
            B.c[v] = h;
            // a reordered row is marked only where values were above h
            if (list) push_chunks(D, v, B.pc && !rescan ? big_prefix(B, v, h + 1) : d);
        }
        __syncthreads();
    }
}

// A separate launch only when this sweep's k_core_sweep builds the histograms.
__global__ __launch_bounds__(BLK) void k_core_finish(CoreBufs B, int32_t s, bool rescan, bool dense, bool list) {
    extern __shared__ int32_t dyn[];
    finish_rows(B, s, rescan, dense, list, hx_view(dyn, hx_bins(B.hbw)));
}

// Sweep s, rows up to C1_MAX: re-evaluate the listed vertices (`dense`: every
// vertex) from their rows; the ones whose value drops are listed for the
// marking kernel.  With `rescan` (and histograms that fit), the listed long
// rows' chunks also add their histograms into the rows' global histograms
// (zero beforehand), which k_core_finish reads after this kernel; otherwise the
// long rows are evaluated here too (`fused`), from the kept histograms, which
// only the marking kernels change.  `list`: the drops are listed for a marking
// pass (not after the dense sweeps before the last one, whose drops no pass
// reads).
__global__ __launch_bounds__(BLK) void k_core_sweep(CoreBufs B, int32_t s, bool rescan, bool dense, bool fused,
                                                    bool list) {
    __shared__ PushLds P;
    extern __shared__ int32_t dyn[]; // hx_bytes(B.hbw): the long rows' histograms
    int32_t *s_h = dyn;
    int32_t *ctr = B.ctr;
    const int par = s & 1;
    const int32_t *in_cnt = dense ? ctr + CT_ALL : ctr + CT_H + 4 * par;
    const int32_t n0 = in_cnt[0], n1 = in_cnt[1], n2 = in_cnt[2];
    const int32_t *L0 = dense ? B.all[0] : B.pool[3 * par + 0];
    const int32_t *L1 = dense ? B.all[1] : B.pool[3 * par + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int j = 0; j < 4; j++) {
            ctr[CT_H + 4 * (par ^ 1) + j] = 0; // filled by this sweep's marking kernel
            ctr[CT_D + 4 * (par ^ 1) + j] = 0; // filled by the next sweep
        }
        if (n0 + n1 + n2 > 0) ctr[CT_SWEEPS] = s + 1;
    }
    Pusher p = make_pusher(&P, list_set(B.pool[6], B.pool[7], nullptr, B.poolc[0], ctr + CT_D + 4 * par, BIG_CHUNKS));
    const int lane = lane_id();
    const int t = threadIdx.x;
    if (fused) finish_rows(B, s, rescan, dense, list, hx_view(dyn, hx_bins(B.hbw)));
    if (rescan && B.hbw > 0) {
        const int32_t n3 = in_cnt[3];
        const int2 *L3 = dense ? B.allc : B.poolc[1 + par];
        for (int32_t i = blockIdx.x; i < n3; i += gridDim.x) {
            const int2 ck = L3[i];
            const int32_t v = ck.x;
            const int64_t b = B.uoff[v];
            const int32_t d = (int32_t)(B.uoff[v + 1] - b);
            const int32_t x = B.c[v]; // only k_core_finish writes c of a long row
            const int32_t lo = ck.y * CH, hi = lo + CH < d ? lo + CH : d;
            for (int32_t k = t; k <= x; k += BLK) s_h[k] = 0;
            __syncthreads();
            const ChunkRow r = load_chunk(B.uadj, b, lo, hi);
            int32_t y[CPT];
#pragma unroll
            for (int j = 0; j < CPT; j++) y[j] = r.ok[j] ? B.c[r.u[j]] : -1;
#pragma unroll
            for (int j = 0; j < CPT; j++)
                if (y[j] >= 0) atomicAdd(&s_h[y[j] < x ? y[j] : x], 1);
            __syncthreads();
            int32_t *gh = B.gh + (int64_t)B.bigid[v] * B.hbw;
            for (int32_t k = t; k <= x; k += BLK)
                if (s_h[k]) atomicAdd(&gh[k], s_h[k]);
            __syncthreads();
        }
    }
    const int64_t gwave = ((int64_t)blockIdx.x * BLK + t) >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * WPB;
    // four list entries per wavefront and step: rows of at most 64 entries take
    // a group of 16 lanes each, longer ones the whole wavefront in turn
    for (int64_t i0 = gwave * 4; i0 < n1; i0 += nwaves * 4) {
        const int grp = lane >> 4, gl = lane & 15;
        const int64_t i = i0 + grp;
        int32_t v = -1, d = 0, x = 0;
        int64_t b = 0;
        if (i < n1) {
            v = L1[i];
            b = B.uoff[v];
            d = (int32_t)(B.uoff[v + 1] - b);
            x = B.c[v];
        }
        const bool small = v >= 0 && d <= 64;
        bool drop = false;
        if (small) { // uniform within the group
            int32_t ge;
            const int32_t h = h_group16(B.c, B.uadj, b, d, x, ge);
            drop = gl == 0 && h < x;
            if (gl == 0) B.cnt[v] = ge;
            if (drop) {
                B.old[v] = x;
                B.c[v] = h;
            }
        }
        if (list) push(p, drop ? 1 : -1, v, d);
        unsigned long long big = __ballot(gl == 0 && v >= 0 && !small);
        while (big) {
            const int src = __ffsll((long long)big) - 1;
            big &= big - 1;
            const int32_t vv = __shfl(v, src), dd = __shfl(d, src), xx = __shfl(x, src);
            const int64_t bb = __shfl(b, src);
            int32_t ge;
            const int32_t h = h_wave(B.c, B.uadj, bb, dd, xx, ge);
            const bool dr = lane == 0 && h < xx;
            if (lane == 0) B.cnt[vv] = ge;
            if (dr) {
                B.old[vv] = xx;
                B.c[vv] = h;
            }
            if (list) push(p, dr ? 1 : -1, vv, dd);
        }
    }
    const int64_t stride = (int64_t)gridDim.x * BLK;
    for (int64_t base = (int64_t)blockIdx.x * BLK + (t & ~63); base < n0; base += stride) {
        const int64_t i = base + lane;
        int cls = -1;
        int32_t v = 0;
        if (i < n0) {
            v = L0[i];
            const int64_t b = B.uoff[v];
            const int32_t d = (int32_t)(B.uoff[v + 1] - b);
            const int32_t x = B.c[v];
            int32_t ge;
            const int32_t h = h_lane(B.c, B.uadj, b, d, x, ge);
            B.cnt[v] = ge;
            if (h < x) {
                B.old[v] = x;
                B.c[v] = h;
                cls = 0;
            }
        }
        if (list) push(p, cls, v, 0);
    }
    push_finish(p);
}

// Marking of sweep s, for a dropped vertex u (value xo -> h) and its neighbour w.
// A vertex w that is not listed holds a value with count(>= c(w)) >= c(w) over
// its neighbours' values; u's drop lowers that count only if xo >= c(w) > h,
// so exactly those w are listed (also when w read xo or h during the sweep:
// either way its value counted u only if c(w) <= xo).  Long rows with a kept
// histogram (not `rescan`) also move u from level min(xo, c(w)) to h whenever
// c(w) > h.  Each vertex is listed once per sweep.
// J entries of one lane at a time: every dependent load and atomic of the batch
// is issued before any result is used
template <int J>
__device__ inline void mark_batch(const CoreBufs &B, Pusher &p, const int32_t (&w)[J], const int32_t (&cw)[J],
                                  const bool (&ok)[J], int32_t xo, int32_t h, int32_t tag, bool rescan) {
    bool cand[J], want[J];
    int32_t dw[J], st[J];
    const bool keep = B.hbw > 0 && !rescan;
#pragma unroll
    for (int j = 0; j < J; j++) {
        cand[j] = ok[j] && cw[j] > h;
        dw[j] = cand[j] && (keep || cw[j] <= xo) ? B.deg[w[j]] : 0;
    }
    int32_t id[J];
#pragma unroll
    for (int j = 0; j < J; j++) id[j] = (keep && cand[j] && dw[j] > C1_MAX) ? B.bigid[w[j]] : -1;
#pragma unroll
    for (int j = 0; j < J; j++) {
        want[j] = cand[j] && cw[j] <= xo;
        if (id[j] >= 0) {
            const int32_t bo = xo < cw[j] ? xo : cw[j]; // h < cw here, so the new level is h
            int32_t *gh = B.gh + (int64_t)id[j] * B.hbw;
            atomicSub(&gh[bo], 1);
            atomicAdd(&gh[h], 1);
            want[j] = bo == cw[j];
        }
    }
#pragma unroll
    for (int j = 0; j < J; j++) st[j] = want[j] ? B.stamp[w[j]] : tag;
#pragma unroll
    for (int j = 0; j < J; j++) st[j] = (want[j] && st[j] != tag) ? atomicExch(&B.stamp[w[j]], tag) : tag;
    for (int j = 0; j < J; j++) push(p, st[j] != tag ? row_class(dw[j]) : -1, w[j], dw[j]);
}

// a row of at most 64 * NJ entries, one wavefront (NJ wavefront-uniform)
template <int NJ>
__device__ inline void mark_row(const CoreBufs &B, Pusher &p, int64_t b, int32_t d, int32_t xo, int32_t h,
                                int32_t tag, bool rescan) {
    const int lane = lane_id();
    int32_t u[NJ], cw[NJ];
    bool ok[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        ok[j] = lane + 64 * j < d;
        u[j] = ok[j] ? B.uadj[b + lane + 64 * j] : 0;
    }
#pragma unroll
    for (int j = 0; j < NJ; j++) cw[j] = ok[j] ? B.c[u[j]] : 0;
    mark_batch<NJ>(B, p, u, cw, ok, xo, h, tag, rescan);
}

__global__ __launch_bounds__(BLK) void k_core_mark(CoreBufs B, int32_t s, bool rescan) {
    __shared__ PushLds P;
    int32_t *ctr = B.ctr;
    const int par = s & 1;
    const int32_t *in_cnt = ctr + CT_D + 4 * par;
    const int32_t n0 = in_cnt[0], n1 = in_cnt[1], n3 = in_cnt[3];
    Pusher p = make_pusher(&P, list_set(B.pool[3 * (par ^ 1)], B.pool[3 * (par ^ 1) + 1], B.pool[3 * (par ^ 1) + 2],
                                        B.poolc[1 + (par ^ 1)], ctr + CT_H + 4 * (par ^ 1),
                                        rescan ? BIG_BOTH : BIG_VERTEX));
    const int32_t tag = s + 1;
    const int lane = lane_id();
    const int t = threadIdx.x;
    const bool sorted = B.pc && !rescan;
    const int32_t *big_adj = sorted ? B.hadj : B.uadj;
    for (int32_t i = blockIdx.x; i < n3; i += gridDim.x) {
        const int2 ck = B.poolc[0][i];
        const int32_t v = ck.x;
        const int64_t b = B.uoff[v];
        const int32_t h = B.c[v], xo = B.old[v];
        // reordered rows: only neighbours whose value was above h can have c(w) > h
        const int32_t d = sorted ? big_prefix(B, v, h + 1) : (int32_t)(B.uoff[v + 1] - b);
        const int32_t lo = ck.y * CH, hi = lo + CH < d ? lo + CH : d;
        const ChunkRow r = load_chunk(big_adj, b, lo, hi);
        int32_t cw[CPT];
#pragma unroll
        for (int j = 0; j < CPT; j++) cw[j] = r.ok[j] ? B.c[r.u[j]] : 0;
        mark_batch<CPT>(B, p, r.u, cw, r.ok, xo, h, tag, rescan);
    }
    const int64_t gwave = ((int64_t)blockIdx.x * BLK + t) >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * WPB;
    for (int64_t i = gwave; i < n1; i += nwaves) {
        const int32_t v = B.pool[7][i];
        const int64_t b = B.uoff[v];
        const int32_t d = (int32_t)(B.uoff[v + 1] - b);
        const int32_t h = B.c[v], xo = B.old[v];
        if (d <= 64) mark_row<1>(B, p, b, d, xo, h, tag, rescan);
        else if (d <= 128) mark_row<2>(B, p, b, d, xo, h, tag, rescan);
        else if (d <= 256) mark_row<4>(B, p, b, d, xo, h, tag, rescan);
        else if (d <= 512) mark_row<8>(B, p, b, d, xo, h, tag, rescan);
        else mark_row<16>(B, p, b, d, xo, h, tag, rescan);
    }
    const int64_t stride = (int64_t)gridDim.x * BLK;
    for (int64_t base = (int64_t)blockIdx.x * BLK + (t & ~63); base < n0; base += stride) {
        const int64_t i = base + lane;
        int64_t b = 0;
        int32_t d = 0, h = 0, xo = 0;
        if (i < n0) {
            const int32_t v = B.pool[6][i];
            b = B.uoff[v];
            d = (int32_t)(B.uoff[v + 1] - b);
            h = B.c[v];
            xo = B.old[v];
        }
        int32_t u[C0_MAX], cw[C0_MAX];
        bool ok[C0_MAX];
#pragma unroll
        for (int j = 0; j < C0_MAX; j++) {
            ok[j] = j < d;
            u[j] = ok[j] ? B.uadj[b + j] : 0;
        }
#pragma unroll
        for (int j = 0; j < C0_MAX; j++) cw[j] = ok[j] ? B.c[u[j]] : 0;
        mark_batch<C0_MAX>(B, p, u, cw, ok, xo, h, tag, rescan);
    }
    push_finish(p);
}

// ---- the levels' rounds, all levels at once ------------------------------------------------
// cnt(v) = |{u in N(v) : core(u) >= core(v)}|; a vertex with cnt(v) <= core(v)
// goes in round 0 of its level.  Rows up to C1_MAX hold the count their last
// h-index evaluation stored: it is exact once the values settle, since a later
// drop of a neighbour from at or above the vertex's value to below it lists the
// vertex for another evaluation.  Long rows read level core(v) of their kept
// histogram in k_level_big, or, when histograms do not fit, their chunks add
// partial counts here and k_level_big decides.
__global__ __launch_bounds__(BLK) void k_level_count(CoreBufs B) {
    __shared__ PushLds P;
    int32_t *ctr = B.ctr;
    const int32_t n0 = ctr[CT_ALL + 0], n1 = ctr[CT_ALL + 1], n3 = ctr[CT_ALL + 3];
    Pusher p = make_pusher(&P, list_set(B.pool[0], B.pool[1], nullptr, B.poolc[0], ctr + CT_F + 0, BIG_CHUNKS));
    const int lane = lane_id();
    const int t = threadIdx.x;
    if (B.hbw == 0) {
        for (int32_t i = blockIdx.x; i < n3; i += gridDim.x) {
            const int2 ck = B.allc[i];
            const int32_t v = ck.x;
            const int64_t b = B.uoff[v];
            const int32_t k = B.c[v];
            const int32_t d = (int32_t)(B.uoff[v + 1] - b);
            const int32_t lo = ck.y * CH, hi = lo + CH < d ? lo + CH : d;
            const ChunkRow r = load_chunk(B.uadj, b, lo, hi);
            int32_t part = 0;
#pragma unroll
            for (int j = 0; j < CPT; j++) part += (r.ok[j] && B.c[r.u[j]] >= k) ? 1 : 0;
            part = wave_sum(part);
            if (lane == 0 && part) atomicAdd(&B.cnt[v], part);
        }
    }
    // rows of classes 0 and 1, one lane per vertex
    const int64_t stride = (int64_t)gridDim.x * BLK;
    for (int64_t base = (int64_t)blockIdx.x * BLK + (t & ~63); base < (int64_t)n0 + n1; base += stride) {
        const int64_t i = base + lane;
        int cls = -1;
        int32_t v = 0;
        if (i < (int64_t)n0 + n1) {
            const int j = i < n0 ? 0 : 1;
            v = j == 0 ? B.all[0][i] : B.all[1][i - n0];
            if (B.cnt[v] <= B.c[v]) cls = j;
        }
        push(p, cls, v, 0);
    }
    push_finish(p);
}

// round 0 of the long rows, from their kept histograms or their chunks' counts
__global__ __launch_bounds__(BLK) void k_level_big(CoreBufs B) {
    const int32_t n2 = B.ctr[CT_ALL + 2];
    const ListSet F = list_set(B.pool[0], B.pool[1], nullptr, B.poolc[0], B.ctr + CT_F + 0, BIG_CHUNKS);
    for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n2; i += (int64_t)gridDim.x * BLK) {
        const int32_t v = B.all[2][i];
        const int32_t k = B.c[v];
        int32_t cnt = B.cnt[v];
        if (B.hbw > 0) {
            cnt = B.gh[(int64_t)B.bigid[v] * B.hbw + k]; // the level holds every value >= k
            B.cnt[v] = cnt;
        }
        if (cnt <= k) push_chunks(F, v, (int32_t)(B.uoff[v + 1] - B.uoff[v]));
    }
}

// removing v (core k) takes one from each same-core neighbour; the one step
// from k + 1 to k puts the neighbour in the next round.  Neighbours already
// removed, or removed in this round, are at k or below and never cross, so
// they are skipped after round 0: counts only fall during the rounds, so a
// plain read of k or less is final, and a stale read is larger and only costs
// the atomic.  (In round 0 few neighbours are settled and the read only adds
// latency: 70M edges, round 0 307 -> 360 us with it, later rounds 2x faster.)
template <int J>
__device__ inline void level_batch(const CoreBufs &B, Pusher &p, const int32_t (&u)[J], const int32_t (&cu)[J],
                                   const bool (&ok)[J], int32_t k, bool skip) {
    int32_t now[J], old[J], du[J];
#pragma unroll
    for (int j = 0; j < J; j++) now[j] = (ok[j] && cu[j] == k) ? (skip ? B.cnt[u[j]] : k + 1) : 0;
#pragma unroll
    for (int j = 0; j < J; j++) old[j] = now[j] > k ? atomicSub(&B.cnt[u[j]], 1) : 0;
#pragma unroll
    for (int j = 0; j < J; j++) du[j] = (ok[j] && cu[j] == k && old[j] == k + 1) ? B.deg[u[j]] : -1;
    for (int j = 0; j < J; j++) push(p, du[j] >= 0 ? row_class(du[j]) : -1, u[j], du[j]);
}

// a row of at most 64 * NJ entries, one wavefront (NJ wavefront-uniform)
template <int NJ>
__device__ inline void level_row(const CoreBufs &B, Pusher &p, int64_t b, int32_t d, int32_t k, bool skip) {
    const int lane = lane_id();
    int32_t u[NJ], cu[NJ];
    bool ok[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        ok[j] = lane + 64 * j < d;
        u[j] = ok[j] ? B.uadj[b + lane + 64 * j] : 0;
    }
#pragma unroll
    for (int j = 0; j < NJ; j++) cu[j] = ok[j] ? B.c[u[j]] : -1;
    level_batch<NJ>(B, p, u, cu, ok, k, skip);
}

__global__ __launch_bounds__(BLK) void k_level_round(CoreBufs B, int32_t r) {
    __shared__ PushLds P;
    int32_t *ctr = B.ctr;
    const int cur = r % 3, nxt = (r + 1) % 3, clr = (r + 2) % 3;
    const int32_t n0 = ctr[CT_F + 4 * cur], n1 = ctr[CT_F + 4 * cur + 1], n3 = ctr[CT_F + 4 * cur + 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int j = 0; j < 4; j++) ctr[CT_F + 4 * clr + j] = 0;
        if (n0 + n1 + n3 > 0) ctr[CT_ROUNDS] = r + 1;
    }
    const int32_t *in0 = B.pool[2 * cur], *in1 = B.pool[2 * cur + 1];
    const int2 *in3 = B.poolc[cur];
    Pusher p = make_pusher(&P, list_set(B.pool[2 * nxt], B.pool[2 * nxt + 1], nullptr, B.poolc[nxt],
                                        ctr + CT_F + 4 * nxt, BIG_CHUNKS));
    const int lane = lane_id();
    const int t = threadIdx.x;
    for (int32_t i = blockIdx.x; i < n3; i += gridDim.x) {
        const int2 ck = in3[i];
        const int32_t v = ck.x;
        if (ck.y == 0 && t == 0) B.lr[v] = r;
        const int64_t b = B.uoff[v];
        const int32_t k = B.c[v];
        // reordered rows: a neighbour of core k had a value >= k at the reorder
        const int32_t d = B.pc ? big_prefix(B, v, k) : (int32_t)(B.uoff[v + 1] - b);
        const int32_t lo = ck.y * CH, hi = lo + CH < d ? lo + CH : d;
        if (lo >= hi) continue; // block-uniform
        const ChunkRow rw = load_chunk(B.pc ? B.hadj : B.uadj, b, lo, hi);
        int32_t cu[CPT];
#pragma unroll
        for (int j = 0; j < CPT; j++) cu[j] = rw.ok[j] ? B.c[rw.u[j]] : -1;
        level_batch<CPT>(B, p, rw.u, cu, rw.ok, k, r > 0);
    }
    const int64_t gwave = ((int64_t)blockIdx.x * BLK + t) >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * WPB;
    for (int64_t i = gwave; i < n1; i += nwaves) {
        const int32_t v = in1[i];
        if (lane == 0) B.lr[v] = r;
        const int64_t b = B.uoff[v];
        const int32_t d = (int32_t)(B.uoff[v + 1] - b);
        const int32_t k = B.c[v];
        if (d <= 64) level_row<1>(B, p, b, d, k, r > 0);
        else if (d <= 128) level_row<2>(B, p, b, d, k, r > 0);
        else if (d <= 256) level_row<4>(B, p, b, d, k, r > 0);
        else if (d <= 512) level_row<8>(B, p, b, d, k, r > 0);
        else level_row<16>(B, p, b, d, k, r > 0);
    }
    const int64_t stride = (int64_t)gridDim.x * BLK;
    for (int64_t base = (int64_t)blockIdx.x * BLK + (t & ~63); base < n0; base += stride) {
        const int64_t i = base + lane;
        int64_t b = 0;
        int32_t d = 0, k = 0;
        if (i < n0) {
            const int32_t v = in0[i];
            B.lr[v] = r;
            b = B.uoff[v];
            d = (int32_t)(B.uoff[v + 1] - b);
            k = B.c[v];
        }
        int32_t u[C0_MAX], cu[C0_MAX];
        bool ok[C0_MAX];
#pragma unroll
        for (int j = 0; j < C0_MAX; j++) {
            ok[j] = j < d;
            u[j] = ok[j] ? B.uadj[b + j] : 0;
        }
#pragma unroll
        for (int j = 0; j < C0_MAX; j++) cu[j] = ok[j] ? B.c[u[j]] : -1;
        level_batch<C0_MAX>(B, p, u, cu, ok, k, r > 0);
    }
    push_finish(p);
}

// rank key core * R + round within the level (R = the rounds taken); the sort
// that follows breaks ties by id
__global__ void k_level_keys(const uint16_t *__restrict__ c, const int32_t *__restrict__ lr, int32_t n, uint32_t R,
                             uint32_t *__restrict__ key, int32_t *__restrict__ core, int32_t *ctr) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t r = lr[v];
    if (r < 0) atomicAdd(&ctr[CT_LEFT], 1);
    core[v] = c[v];
    key[v] = (uint32_t)c[v] * R + (uint32_t)(r < 0 ? 0 : r);
}

} // namespace

// Core numbers (into `core`, original ids) and the rank keys (into `key`); returns
// the number of key bits.  uoff/uadj: the undirected CSR (neighbour ids only).
int core_rank_keys(int32_t n, const int64_t *uoff, const int32_t *uadj, const int32_t *deg, int32_t *core,
                   uint32_t *key, hipStream_t s, CoreStats *out) {
    *out = CoreStats{};
    if (n <= 0) return 1;
    PinnedBuf hb;
    hb.ensure(4 * CT_WORDS);
    int32_t *h = hb.as<int32_t>();
    int64_t adj_n = 0;
    FOLTY_HIP(hipMemcpyAsync(&adj_n, uoff + n, 8, hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    // chunk lists: every class-2 row has more than C1_MAX entries
    const int64_t chunk_cap = adj_n / CH + adj_n / (C1_MAX + 1) + 1;
    DevBuf ctr, hist, val, old, stamp, cnt, lr, bigid, all, allc, pool, poolc;
    ctr.ensure(4 * CT_WORDS);
    val.ensure(2 * (size_t)n);
    hist.ensure(4 * (size_t)HG_BINS);
    old.ensure(4 * (size_t)n);
    stamp.ensure(4 * (size_t)n);
    cnt.ensure(4 * (size_t)n);
    lr.ensure(4 * (size_t)n);
    bigid.ensure(4 * (size_t)n);
    all.ensure(4 * 3 * (size_t)n);
    allc.ensure(sizeof(int2) * (size_t)chunk_cap);
    pool.ensure(4 * 8 * (size_t)n);
    poolc.ensure(sizeof(int2) * 3 * (size_t)chunk_cap);
    FOLTY_HIP(hipMemsetAsync(ctr.p, 0, 4 * CT_WORDS, s));
    FOLTY_HIP(hipMemsetAsync(hist.p, 0, 4 * (size_t)HG_BINS, s));
    CoreBufs B{};
    B.uoff = uoff;
    B.uadj = uadj;
    B.deg = deg;
    B.c = val.as<uint16_t>();
    B.old = old.as<int32_t>();
    B.stamp = stamp.as<int32_t>();
    B.cnt = cnt.as<int32_t>();
    B.lr = lr.as<int32_t>();
    B.bigid = bigid.as<int32_t>();
    B.ctr = ctr.as<int32_t>();
    for (int j = 0; j < 3; j++) B.all[j] = all.as<int32_t>() + (size_t)j * n;
    B.allc = allc.as<int2>();
    for (int j = 0; j < 8; j++) B.pool[j] = pool.as<int32_t>() + (size_t)j * n;
    for (int j = 0; j < 3; j++) B.poolc[j] = poolc.as<int2>() + (size_t)j * chunk_cap;
    B.n = n;
    const unsigned g_all = grid_for(n, BLK, GRID);
    int64_t top = (int64_t)std::sqrt((double)adj_n);
    while ((top + 1) * (top + 1) <= adj_n) top++;
    while (top > 0 && top * top > adj_n) top--;
    if (top > HG_BINS - 2) fail(FOLTY_EOVERFLOW, "%lld adjacency entries exceed the degree histogram", (long long)adj_n);
    // a few blocks: each merges its LDS bins into the same global counters
    k_deg_hist<<<grid_for(n, BLK, 256), BLK, 0, s>>>(deg, n, (int32_t)top + 1, hist.as<int32_t>());
    k_global_h<<<1, BLK, 0, s>>>(hist.as<int32_t>(), (int32_t)top, ctr.as<int32_t>());
    k_core_init<<<g_all, BLK, 0, s>>>(B);
    FOLTY_LAUNCHED();
    auto read_ctr = [&]() {
        FOLTY_HIP(hipMemcpyAsync(h, ctr.p, 4 * CT_WORDS, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
    };
    read_ctr();
    const int32_t hg = h[CT_HG], nbig = h[CT_ALL + 2];
    if (hg > UINT16_MAX) fail(FOLTY_EOVERFLOW, "degree h-index %d does not fit 16-bit core values", hg);
    // per class-2 vertex: a histogram over the levels 0..hg
    DevBuf gh, pc, cur, hadj;
    B.hbw = hg < HX_BINS ? hg + 1 : 0;
    if (B.hbw > 0 && nbig > 0) {
        gh.ensure(4 * (size_t)B.hbw * (size_t)nbig);
        FOLTY_HIP(hipMemsetAsync(gh.p, 0, 4 * (size_t)B.hbw * (size_t)nbig, s));
        B.gh = gh.as<int32_t>();
    }

    // sweeps until none lists a vertex: every sweep with work lowers some value,
    // and the values start at most at the degrees, so sum of degrees + 1 sweeps
    // bound them; the cap turns a logic error into an error code
    // The first sweeps drop many vertices at once; long rows are rescanned then,
    // since keeping their histograms would send every drop next to a hub to the
    // same few counters.  After them the histograms are made once and kept, and
    // the long rows reordered by their neighbours' values.
    int32_t sw = 0;
    int batch = RESCAN_SWEEPS;
    bool rescan = true;
    for (;;) {
        for (int i = 0; i < batch; i++, sw++) {
            // dense sweeps need no lists; the last one's drops are marked for
            // the first listed sweep
            const bool dense = sw < DENSE_SWEEPS;
            const bool fused = !(rescan && B.hbw > 0);
            const bool list = sw + 1 >= DENSE_SWEEPS; // a marking pass follows
            k_core_sweep<<<GRID, BLK, hx_bytes(B.hbw), s>>>(B, sw, rescan, dense, fused, list);
            if (!fused) k_core_finish<<<FIN_GRID, BLK, hx_bytes(B.hbw), s>>>(B, sw, rescan, dense, list);
            if (list) k_core_mark<<<GRID, BLK, 0, s>>>(B, sw, rescan);
        }
        FOLTY_LAUNCHED();
        if (rescan && B.hbw > 0 && nbig > 0) {
            // histograms and reordered rows from the current values
            const size_t hn = (size_t)B.hbw * (size_t)nbig;
            pc.ensure(4 * hn);
            cur.ensure(4 * hn);
            hadj.ensure(4 * (size_t)adj_n + 4);
            k_big_hist<<<GRID, BLK, 0, s>>>(B);
            k_big_prefix<<<FIN_GRID, BLK, 0, s>>>(B, pc.as<int32_t>(), cur.as<int32_t>());
            k_big_scatter<<<GRID, BLK, 0, s>>>(B, cur.as<int32_t>(), hadj.as<int32_t>());
            FOLTY_LAUNCHED();
            B.hadj = hadj.as<int32_t>();
            B.pc = pc.as<int32_t>();
        }
        rescan = false;
        read_ctr();
        const int par = sw & 1; // the lists the next sweep would read
        if (h[CT_H + 4 * par] + h[CT_H + 4 * par + 1] + h[CT_H + 4 * par + 2] == 0) break;
        if ((int64_t)sw > adj_n + 64) fail(FOLTY_EDEVICE, "core sweeps did not settle in %d sweeps", sw);
        // 16 sweeps, then 8 at a time: an empty sweep costs about 5 us of
        // launches, a counter read about as much as 3 of them
        batch = batch == RESCAN_SWEEPS ? 16 : 8;
    }
    const int32_t sweeps = h[CT_SWEEPS];

    k_level_count<<<GRID, BLK, 0, s>>>(B);
    k_level_big<<<FIN_GRID, BLK, 0, s>>>(B);
    FOLTY_LAUNCHED();
    int32_t r = 0;
    batch = 8;
    for (;;) {
        for (int i = 0; i < batch; i++, r++) k_level_round<<<GRID, BLK, 0, s>>>(B, r);
        FOLTY_LAUNCHED();
        read_ctr();
        const int cur = r % 3;
        if (h[CT_F + 4 * cur] + h[CT_F + 4 * cur + 1] + h[CT_F + 4 * cur + 3] == 0) break;
        if (r > n + 64) fail(FOLTY_EDEVICE, "level rounds did not finish in %d rounds", r);
        batch = batch < 16 ? 2 * batch : 16;
    }
    const int32_t rounds = h[CT_ROUNDS] > 0 ? h[CT_ROUNDS] : 1;
    // every core number is at most the global h-index
    const uint64_t max_key = (uint64_t)hg * (uint64_t)rounds + (uint64_t)(rounds - 1);
    if (max_key > UINT32_MAX)
        fail(FOLTY_EOVERFLOW, "rank keys need %d bits (h-index %d, %d rounds)", bit_length(max_key), hg, rounds);
    k_level_keys<<<grid_for(n, BLK), BLK, 0, s>>>(B.c, lr.as<int32_t>(), n, (uint32_t)rounds, key, core,
                                                  ctr.as<int32_t>());
    FOLTY_LAUNCHED();
    read_ctr();
    if (h[CT_LEFT] != 0) fail(FOLTY_EDEVICE, "%d vertices were not removed by the level rounds", h[CT_LEFT]);
    out->sweeps = sweeps;
    out->rounds = rounds;
    out->global_h = hg;
    return bit_length(max_key > 0 ? max_key : 1);
}

} // namespace folty
