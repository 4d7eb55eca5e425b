// Index build for the temporal graph (paper, Section "Main Ideas",
// Preliminaries, and the preamble of Section 3):
//   * group temporal edges into time-sorted lists E_{x,y} and static edges of G_S
//     (self-loops dropped; G_S has no directions or parallel edges);
//   * degrees |N(x)| and core numbers by min-degree peeling (the degeneracy
//     ordering the paper attributes to Matula and Beck), run level by level on
//     the GPU; the rank (core, peel round, id) bounds every out-degree by the
//     degeneracy;
//   * orient G_S from lower to higher rank (the graph G->_pi of the paper) as a
//     CSR sorted by head;
//   * count static triangles per oriented edge and per static edge (the latter
//     is |N(u) & N(v)|, the counter c_uv of Section 3's preamble).
#include <cstring>

#include "folty_internal.h"

namespace folty {

namespace {

constexpr int BLK = 256;

__device__ inline int lane_id() { return __lane_id(); }

// make this wavefront's LDS writes visible to all of its lanes
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// wave-aggregated append: one atomic per wave, slots in lane order
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

struct ValOut {
    unsigned long long first_bad;
    unsigned long long loops;
    unsigned long long tmax;
    unsigned long long descents;
};

__global__ void k_validate(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                           const int64_t *__restrict__ t, int64_t m, int32_t n, ValOut *out) {
    unsigned long long loops = 0, tmax = 0, desc = 0, bad = ~0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        int32_t a = src[i], b = dst[i];
        int64_t ti = t[i];
        bool ok = a >= 0 && a < n && b >= 0 && b < n && ti >= 0 && ti < (int64_t(1) << 62);
        if (!ok) bad = (unsigned long long)i < bad ? (unsigned long long)i : bad;
        loops += (a == b);
        if (ok && (unsigned long long)ti > tmax) tmax = (unsigned long long)ti;
        if (i > 0 && t[i - 1] > ti) desc++;
    }
    // one atomic per wavefront and quantity
    for (int o = 32; o > 0; o >>= 1) {
        loops += __shfl_xor(loops, o);
        desc += __shfl_xor(desc, o);
        const unsigned long long tm = __shfl_xor(tmax, o), bd = __shfl_xor(bad, o);
        tmax = tm > tmax ? tm : tmax;
        bad = bd < bad ? bd : bad;
    }
    if (lane_id() != 0) return;
    if (loops) atomicAdd(&out->loops, loops);
    if (desc) atomicAdd(&out->descents, desc);
    if (tmax) atomicMax(&out->tmax, tmax);
    if (bad != ~0ull) atomicMin(&out->first_bad, bad);
}

__global__ void k_init_val(ValOut *o) {
    o->first_bad = ~0ull;
    o->loops = 0;
    o->tmax = 0;
    o->descents = 0;
}

template <class T> __global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota_tkeys(const int64_t *__restrict__ t, uint64_t *__restrict__ keys,
                             int32_t *__restrict__ idx, int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        keys[i] = (uint64_t)t[i];
        idx[i] = (int32_t)i;
    }
}

// pair key of the edge at time-order position j: ((lo * n + hi) * 2 + dir);
// self-loops get 2 n^2, which sorts after every real key
__global__ void k_pair_keys(const int32_t *__restrict__ idx_t, const int32_t *__restrict__ src,
                            const int32_t *__restrict__ dst, int64_t n, uint64_t *__restrict__ key,
                            int32_t *__restrict__ pos, int64_t m) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    int64_t i = idx_t ? idx_t[j] : j;
    int64_t a = src[i], b = dst[i];
    uint64_t k;
    if (a == b) {
        k = 2ull * (uint64_t)n * (uint64_t)n;
    } else {
        uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        k = (lo * (uint64_t)n + hi) * 2ull + (a > b ? 1ull : 0ull);
    }
    key[j] = k;
    pos[j] = (int32_t)j;
}

__global__ void k_gather_sorted(const int32_t *__restrict__ pos, const int32_t *__restrict__ idx_t,
                                const int64_t *__restrict__ t, int32_t *__restrict__ perm,
                                int64_t *__restrict__ ts, int64_t m) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int32_t j = pos[k];
    int32_t i = idx_t ? idx_t[j] : j;
    perm[k] = i;
    ts[k] = t[i];
}

__global__ void k_static_flags(const uint64_t *__restrict__ key, int32_t m, int32_t *__restrict__ flag) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    flag[k] = (k == 0 || (key[k] >> 1) != (key[k - 1] >> 1)) ? 1 : 0;
}

__global__ void k_static_table(const uint64_t *__restrict__ key, int32_t *__restrict__ sid, int32_t m,
                               int64_t n, int32_t *__restrict__ soff, int32_t *__restrict__ smid,
                               int32_t *__restrict__ slo, int32_t *__restrict__ shi) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int32_t s = sid[k] - 1;
    sid[k] = s;
    uint64_t kk = key[k];
    uint64_t pk = kk >> 1;
    bool first = (k == 0) || ((key[k - 1] >> 1) != pk);
    if (first) {
        soff[s] = (int32_t)k;
        slo[s] = (int32_t)(pk / (uint64_t)n);
        shi[s] = (int32_t)(pk % (uint64_t)n);
    }
    if ((kk & 1ull) && (first || (key[k - 1] & 1ull) == 0)) smid[s] = (int32_t)k;
    if (k == m - 1) soff[s + 1] = m;
}

struct PairStats {
    unsigned long long pairs;
    unsigned long long sigma_max;
};

__global__ void k_fix_smid_stats(const int32_t *__restrict__ soff, int32_t *__restrict__ smid, int32_t S,
                                 PairStats *ps) {
    unsigned long long pairs = 0, smax = 0;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = soff[s], b = soff[s + 1];
        int32_t mid = smid[s];
        if (mid < 0) {
            mid = b;
            smid[s] = b;
        }
        unsigned long long l0 = (unsigned long long)(mid - a), l1 = (unsigned long long)(b - mid);
        pairs += (l0 > 0) + (l1 > 0);
        unsigned long long mx = l0 > l1 ? l0 : l1;
        smax = mx > smax ? mx : smax;
    }
    // wave, then block reduction: one atomic per block
    __shared__ unsigned long long s_p[BLK / 64], s_m[BLK / 64];
    for (int o = 32; o > 0; o >>= 1) {
        pairs += __shfl_xor(pairs, o);
        unsigned long long other = __shfl_xor(smax, o);
        smax = other > smax ? other : smax;
    }
    if (lane_id() == 0) {
        s_p[threadIdx.x >> 6] = pairs;
        s_m[threadIdx.x >> 6] = smax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLK / 64; w++) {
            pairs += s_p[w];
            smax = s_m[w] > smax ? s_m[w] : smax;
        }
        if (pairs) atomicAdd(&ps->pairs, pairs);
        if (smax) atomicMax(&ps->sigma_max, smax);
    }
}

// ---- min-degree peeling -------------------------------------------------------
// The peel runs as identical launches of one kernel over a fixed grid, one step
// per launch: either a level's collect (live vertices of degree <= k, taken from
// the compacted live list) or one peel round (remove the frontier, decrement its
// neighbours; neighbours crossing k+1 -> k form the next frontier).  Step i reads
// the state of step i-1 and the counters step i-1 produced, and every block
// derives step i's state from them identically, so no block waits for another.
// Block 0 publishes step i's state (double buffer by step parity) and clears
// the counters of step i+1 (triple buffer by step % 3).
constexpr int PEEL_BLOCKS_WIDE = 2048;  // while many vertices are live
constexpr int PEEL_BLOCKS_NARROW = 256; // late levels: small frontiers, launch cost dominates
constexpr int32_t PEEL_NARROW_BELOW = 1 << 20; // live vertices below which the narrow grid is used
constexpr int32_t TINY_DEG = 32;  // frontier vertices up to this degree get one lane each
constexpr int32_t BIG_DEG = 2048; // frontier vertices above this degree share the grid
constexpr int32_t BIG_LDS = 2048; // big frontier vertices whose chunk prefix fits in LDS
// Neighbours of degree above HUB_DEG ("hubs", at most HUB_SLOTS of them) are
// stored in the peeling adjacency as HUB_FLAG | slot.  A round counts its
// decrements of each hub in LDS and applies them with one atomic per block, so
// the thousands of leaves of a hub removed in one round do not serialise on the
// hub's degree counter.
constexpr int32_t HUB_DEG = 1024;
constexpr int32_t HUB_SLOTS = 4096;
constexpr uint32_t HUB_FLAG = 0x80000000u;
constexpr int32_t AGG_MIN_FRONTIER = 4096; // rounds above this frontier size aggregate in LDS

enum : int32_t { PEEL_BOOT = -1, PEEL_COLLECT = 0, PEEL_ROUND = 1, PEEL_DONE = 2 };

struct PeelState {   // what step i does
    int32_t mode;
    int32_t k;
    int32_t r;        // round number (the rank key) of the next round
    int32_t lp;       // current live list
    int32_t alive_n;  // entries in the current live list
    int32_t n_in;     // frontier size a round step consumes
    int32_t removed;  // vertices removed before this step
    int32_t pad;
};

struct PeelCount {    // what step i produced
    int32_t nT, nS, nB; // frontier written: degree <= TINY_DEG / <= BIG_DEG / above
    int32_t nA;         // live list written (collect)
    int32_t min_above;
};

// a frontier vertex with its adjacency row, so that a round reads the row
// without another lookup
struct alignas(16) FEntry {
    int32_t x, len;
    int64_t start;
};

struct PeelBufs {
    const int64_t *uoff;
    const int32_t *uadj;       // neighbour id, or HUB_FLAG | hub slot for a hub neighbour
    const int32_t *uadj_plain; // neighbour ids only (rounds that do not aggregate hubs)
    const int32_t *hub_vertex;
    int32_t n_hubs;
    const int32_t *deg;
    int32_t *dcur, *rnd, *core;
    FEntry *FT[3], *FS[3], *FB[3];
    int32_t *alive[2];
    PeelState *state;  // [2]
    PeelCount *count;  // [3]
    int32_t n;
};

__global__ void k_peel_init(const int32_t *__restrict__ deg, int32_t *__restrict__ dcur,
                            int32_t *__restrict__ rnd, int32_t *__restrict__ alive0, int32_t n) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    dcur[x] = deg[x];
    rnd[x] = -1;
    alive0[x] = (int32_t)x;
}

__device__ inline PeelState peel_next(const PeelState &p, const PeelCount &c, int32_t n) {
    PeelState s = p;
    if (p.mode == PEEL_BOOT) {
        s.mode = PEEL_COLLECT;
        s.k = 0;
        s.r = 0;
        s.lp = 0;
        s.alive_n = n;
        s.n_in = 0;
        s.removed = 0;
    } else if (p.mode == PEEL_COLLECT) {
        s.lp = p.lp ^ 1;
        s.alive_n = c.nA;
        if (c.nT + c.nS + c.nB > 0) {
            s.mode = PEEL_ROUND;
            s.n_in = c.nT + c.nS + c.nB;
        } else if (c.nA == 0) {
            s.mode = PEEL_DONE;
        } else {
            s.k = c.min_above; // nothing at degree <= k: jump to the smallest live degree
        }
    } else if (p.mode == PEEL_ROUND) {
        s.removed = p.removed + p.n_in;
        s.r = p.r + 1;
        if (c.nT + c.nS + c.nB > 0) {
            s.n_in = c.nT + c.nS + c.nB;
        } else {
            s.mode = PEEL_COLLECT;
            s.k = p.k + 1;
            s.n_in = 0;
        }
    }
    return s;
}

// Pushes of one round are buffered per wavefront in LDS and written out per
// block at the end of the step (one atomic per block and frontier class), so
// that thousands of waves do not serialise on the same three counters.
constexpr int PUSH_CAP = 256;

__device__ inline int push_class(int32_t d) { return d <= TINY_DEG ? 0 : (d <= BIG_DEG ? 1 : 2); }

struct PushBuf {
    int32_t *buf; // this wave's PUSH_CAP slots in LDS
    int32_t n;    // entries held (wave-uniform)
};

// move a wave's buffered pushes to the global lists with wave-level atomics
__device__ inline FEntry row_entry(const PeelBufs &B, int32_t y) {
    FEntry e;
    e.x = y;
    e.start = B.uoff[y];
    e.len = (int32_t)(B.uoff[y + 1] - e.start);
    return e;
}

__device__ inline void push_flush_wave(PushBuf &pb, const PeelBufs &B, PeelCount *out, FEntry *const L[3]) {
    int32_t *cnt[3] = {&out->nT, &out->nS, &out->nB};
    for (int32_t i0 = 0; i0 < pb.n; i0 += 64) {
        int32_t i = i0 + lane_id();
        bool v = i < pb.n;
        FEntry e{};
        if (v) e = row_entry(B, pb.buf[i]);
        int c = v ? push_class(e.len) : -1;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            int32_t slot = wave_append(cnt[j], c == j);
            if (slot >= 0) L[j][slot] = e;
        }
    }
    pb.n = 0;
}

// Decrement a neighbour's degree; the one decrement that takes it from k+1 to k
// puts it in the next frontier.  Removed vertices may be decremented too: their
// degree is already <= k, so they are never pushed again.
// agg = large round: hub decrements go to the block's LDS counters and pushes to
// the wave's LDS buffer; otherwise both go straight to global memory.
// AGG reads the hub-flagged adjacency, otherwise plain neighbour ids.
template <bool AGG>
__device__ inline void peel_neighbour(int32_t y, bool valid, int32_t k, const PeelBufs &B, PeelCount *out,
                                      PushBuf &pb, FEntry *const L[3], int32_t *hub_cnt) {
    bool push = false;
    FEntry e{};
    if (valid) {
        if (AGG && ((uint32_t)y & HUB_FLAG)) {
            const int32_t h = (int32_t)((uint32_t)y & ~HUB_FLAG);
            atomicAdd(&hub_cnt[h], 1);
            hub_cnt[HUB_SLOTS] = 1; // this block touched a hub
        } else {
            int32_t old = atomicSub(&B.dcur[y], 1);
            push = (old == k + 1);
        }
    }
    if (!AGG) {
        if (push) e = row_entry(B, y);
        int cls = push ? push_class(e.len) : -1;
        int32_t *cnt[3] = {&out->nT, &out->nS, &out->nB};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            int32_t slot = wave_append(cnt[j], cls == j);
            if (slot >= 0) L[j][slot] = e;
        }
        return;
    }
    unsigned long long mask = __ballot(push);
    if (!mask) return;
    int32_t c = (int32_t)__popcll(mask);
    if (pb.n + c > PUSH_CAP) {
        wave_sync();
        push_flush_wave(pb, B, out, L);
    }
    if (push) pb.buf[pb.n + (int32_t)__popcll(mask & ((1ull << lane_id()) - 1ull))] = y;
    pb.n += c;
    wave_sync();
}

// end of a round: every wave's buffered pushes go out with one atomic per block
// and class
__device__ inline void push_flush_block(PushBuf &pb, const PeelBufs &B, PeelCount *out, FEntry *const L[3]) {
    __shared__ int32_t s_cnt[BLK / 64][3];
    __shared__ int32_t s_off[BLK / 64][3];
    const int w = threadIdx.x >> 6, lane = lane_id();
    int32_t cc[3] = {0, 0, 0};
    for (int32_t i0 = 0; i0 < pb.n; i0 += 64) {
        int32_t i = i0 + lane;
        int c = i < pb.n ? push_class(B.deg[pb.buf[i]]) : -1; // deg[y] is the row length
#pragma unroll
        for (int j = 0; j < 3; j++) cc[j] += (int32_t)__popcll(__ballot(c == j));
    }
    if (lane == 0)
        for (int j = 0; j < 3; j++) s_cnt[w][j] = cc[j];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int j = threadIdx.x;
        int32_t *cnt = j == 0 ? &out->nT : (j == 1 ? &out->nS : &out->nB);
        int32_t tot = 0;
        for (int wv = 0; wv < BLK / 64; wv++) tot += s_cnt[wv][j];
        int32_t base = tot ? atomicAdd(cnt, tot) : 0;
        for (int wv = 0; wv < BLK / 64; wv++) {
            s_off[wv][j] = base;
            base += s_cnt[wv][j];
        }
    }
    __syncthreads();
    int32_t off[3] = {s_off[w][0], s_off[w][1], s_off[w][2]};
    for (int32_t i0 = 0; i0 < pb.n; i0 += 64) {
        int32_t i = i0 + lane;
        bool v = i < pb.n;
        FEntry e{};
        if (v) e = row_entry(B, pb.buf[i]);
        int c = v ? push_class(e.len) : -1;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            unsigned long long mask = __ballot(c == j);
            if (c == j) L[j][off[j] + (int32_t)__popcll(mask & ((1ull << lane) - 1ull))] = e;
            off[j] += (int32_t)__popcll(mask);
        }
    }
    pb.n = 0;
}

// block-aggregated append of four predicates: one global atomic per block and
// per predicate; slot[j] is this thread's index in list j or -1
__device__ inline void block_append4(const bool p[4], int32_t *const g[4], int32_t slot[4]) {
    __shared__ int32_t s_cnt[4], s_base[4];
    if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int lane = lane_id();
    int32_t local[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        unsigned long long mask = __ballot(p[j]);
        int32_t woff = 0;
        int leader = mask ? __ffsll((long long)mask) - 1 : 0;
        if (mask && lane == leader) woff = atomicAdd(&s_cnt[j], (int32_t)__popcll(mask));
        woff = __shfl(woff, leader);
        local[j] = p[j] ? woff + (int32_t)__popcll(mask & ((1ull << lane) - 1ull)) : -1;
    }
    __syncthreads();
    if (threadIdx.x < 4) s_base[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(g[threadIdx.x], s_cnt[threadIdx.x]) : 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; j++) slot[j] = local[j] >= 0 ? s_base[j] + local[j] : -1;
}

// one peel round: remove the frontier the previous step wrote, decrement the
// neighbours, collect the vertices that cross from k+1 to k
struct PeelLds {
    int32_t push[BLK / 64][PUSH_CAP];
    int32_t hub[HUB_SLOTS + 1];
    int32_t bpre[BIG_LDS + 1];
    int32_t wt[BLK / 64];
    int32_t carry;
};

template <bool AGG>
__device__ inline void peel_round(const PeelBufs &B, const PeelState &st, const PeelCount &s_prev, PeelCount *out,
                                  int cur, int prv, PeelLds &lds) {
    const int lane = lane_id();
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gwave = gtid >> 6, nwaves = stride >> 6;
    const int32_t n = B.n, k = st.k;
    // the frontier is what the previous step wrote
    int32_t nT = s_prev.nT < n ? s_prev.nT : n;
    int32_t nS = s_prev.nS < n ? s_prev.nS : n, nB = s_prev.nB < n ? s_prev.nB : n;
    const FEntry *FT = B.FT[prv], *FS = B.FS[prv], *FB = B.FB[prv];
    FEntry *const L[3] = {B.FT[cur], B.FS[cur], B.FB[cur]};
    const int32_t *adj = AGG ? B.uadj : B.uadj_plain;
    int32_t *s_hub = lds.hub;
    PushBuf pb{lds.push[threadIdx.x >> 6], 0};
    const int32_t r = st.r;
    const int32_t H = B.n_hubs;
    if (AGG) {
        for (int32_t h = threadIdx.x; h < H; h += BLK) s_hub[h] = 0;
        if (threadIdx.x == 0) s_hub[HUB_SLOTS] = 0;
        __syncthreads();
    }
    for (int64_t i = gtid; i < nT; i += stride) {
        int32_t x = FT[i].x;
        B.rnd[x] = r;
        B.core[x] = k;
    }
    for (int64_t i = gtid; i < nS; i += stride) {
        int32_t x = FS[i].x;
        B.rnd[x] = r;
        B.core[x] = k;
    }
    for (int64_t i = gtid; i < nB; i += stride) {
        int32_t x = FB[i].x;
        B.rnd[x] = r;
        B.core[x] = k;
    }
    // low-degree vertices: one lane each, the wave runs to its longest row
    for (int64_t base = gtid - lane; base < nT; base += stride) {
        int64_t i = base + lane;
        bool v = i < nT;
        FEntry fe{};
        if (v) fe = FT[i];
        int64_t b = fe.start;
        int32_t len = fe.len;
        int32_t mx = len;
        for (int o = 32; o > 0; o >>= 1) {
            int32_t other = __shfl_xor(mx, o);
            mx = other > mx ? other : mx;
        }
        for (int32_t j = 0; j < mx; j++) {
            bool valid = j < len;
            peel_neighbour<AGG>(valid ? adj[b + j] : 0, valid, k, B, out, pb, L, s_hub);
        }
    }
    // small frontiers get several waves per vertex (wave w works on vertex
    // w mod nS, every wpv-th chunk starting at chunk w / nS)
    const int64_t wpv = nS > 0 && nS < nwaves ? nwaves / nS : 1;
    for (int64_t w = gwave; w < nS * wpv; w += nwaves) {
        const FEntry fe = FS[w % nS];
        int64_t part = w / nS;
        int64_t b = fe.start, e = fe.start + fe.len;
        for (int64_t p0 = b + part * 64; p0 < e; p0 += wpv * 64) {
            int64_t p = p0 + lane;
            bool valid = p < e;
            peel_neighbour<AGG>(valid ? adj[p] : 0, valid, k, B, out, pb, L, s_hub);
        }
    }
    // high-degree vertices: the whole grid strides over the 64-entry chunks of
    // all their rows at once (chunk prefix per block in LDS)
    if (nB > 0 && nB <= BIG_LDS) {
        int32_t *s_bpre = lds.bpre;
        int32_t &s_carry = lds.carry;
        int32_t *s_wt = lds.wt;
        if (threadIdx.x == 0) s_carry = 0;
        __syncthreads();
        for (int32_t j0 = 0; j0 < nB; j0 += BLK) {
            int32_t j = j0 + threadIdx.x;
            int32_t c = 0;
            if (j < nB) c = (FB[j].len + 63) >> 6;
            // block inclusive scan of c (wave scans, then wave totals)
            int32_t v = c;
            for (int o = 1; o < 64; o <<= 1) {
                int32_t y = __shfl_up(v, o);
                if (lane >= o) v += y;
            }
            if (lane == 63) s_wt[threadIdx.x >> 6] = v;
            __syncthreads();
            int32_t before = s_carry;
            for (int wv = 0; wv < (int)(threadIdx.x >> 6); wv++) before += s_wt[wv];
            if (j < nB) s_bpre[j + 1] = before + v;
            __syncthreads();
            if (threadIdx.x == 0) {
                int32_t t = s_carry;
                for (int wv = 0; wv < BLK / 64; wv++) t += s_wt[wv];
                s_carry = t;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) s_bpre[0] = 0;
        __syncthreads();
        const int32_t total = s_bpre[nB];
        for (int64_t c = gwave; c < total; c += nwaves) {
            int32_t lo = 0, hi = nB;
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (s_bpre[mid + 1] <= c) lo = mid + 1;
                else hi = mid;
            }
            const FEntry fe = FB[lo];
            int64_t b = fe.start, e = fe.start + fe.len;
            int64_t p = b + (c - s_bpre[lo]) * 64 + lane;
            bool valid = p < e;
            peel_neighbour<AGG>(valid ? adj[p] : 0, valid, k, B, out, pb, L, s_hub);
        }
    } else {
        for (int32_t j = 0; j < nB; j++) {
            const FEntry fe = FB[j];
            int64_t b = fe.start, e = fe.start + fe.len;
            for (int64_t p0 = b + gwave * 64; p0 < e; p0 += nwaves * 64) {
                int64_t p = p0 + lane;
                bool valid = p < e;
                peel_neighbour<AGG>(valid ? adj[p] : 0, valid, k, B, out, pb, L, s_hub);
            }
        }
    }
    if (!AGG) return;
    // apply this block's hub decrements: one atomic per touched hub
    __syncthreads();
    const int32_t touched = s_hub[HUB_SLOTS];
    for (int32_t h0 = 0; touched && h0 < H; h0 += BLK) {
        int32_t h = h0 + threadIdx.x;
        int32_t c = h < H ? s_hub[h] : 0;
        bool push = false;
        FEntry fe{};
        if (c) {
            const int32_t y = B.hub_vertex[h];
            int32_t old = atomicSub(&B.dcur[y], c);
            push = old > k && old - c <= k;
            if (push) fe = row_entry(B, y);
        }
        int32_t slot = wave_append(&out->nB, push && fe.len > BIG_DEG);
        if (slot >= 0) L[2][slot] = fe;
        slot = wave_append(&out->nS, push && fe.len <= BIG_DEG);
        if (slot >= 0) L[1][slot] = fe;
    }
    push_flush_block(pb, B, out, L);
}

__global__ __launch_bounds__(BLK) void k_peel_step(PeelBufs B, int64_t step) {
    __shared__ PeelState s_st;
    __shared__ PeelCount s_prev;
    const int cur = (int)(step % 3), prv = (int)((step + 2) % 3), nxt = (int)((step + 1) % 3);
    if (threadIdx.x == 0) {
        PeelState p = B.state[(step + 1) & 1];
        PeelCount c = B.count[prv];
        s_prev = c;
        s_st = peel_next(p, c, B.n);
    }
    __syncthreads();
    const PeelState st = s_st;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        B.state[step & 1] = st;
        PeelCount z = {0, 0, 0, 0, 0x7fffffff};
        B.count[nxt] = z;
    }
    if (st.mode == PEEL_DONE) return;
    const int lane = lane_id();
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gwave = gtid >> 6, nwaves = stride >> 6;
    const int32_t n = B.n, k = st.k;
    PeelCount *out = &B.count[cur];

    if (st.mode == PEEL_COLLECT) {
        int32_t na = st.alive_n < n ? st.alive_n : n;
        const int32_t *A = B.alive[st.lp];
        int32_t *A2 = B.alive[st.lp ^ 1];
        FEntry *FT = B.FT[cur], *FS = B.FS[cur], *FB = B.FB[cur];
        int32_t *const g[4] = {&out->nT, &out->nS, &out->nB, &out->nA};
        int32_t local_min = 0x7fffffff;
        for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < na; base += stride) {
            int64_t i = base + threadIdx.x;
            bool valid = i < na;
            int32_t x = valid ? A[i] : 0;
            bool live = valid && B.rnd[x] < 0;
            int32_t d = live ? B.dcur[x] : 0;
            bool take = live && d <= k;
            FEntry fe{};
            if (take) fe = row_entry(B, x);
            const int32_t dx = fe.len;
            bool keep = live && d > k;
            if (keep && d < local_min) local_min = d;
            const bool p[4] = {take && dx <= TINY_DEG, take && dx > TINY_DEG && dx <= BIG_DEG, take && dx > BIG_DEG,
                               keep};
            int32_t slot[4];
            block_append4(p, g, slot);
            if (slot[0] >= 0) FT[slot[0]] = fe;
            if (slot[1] >= 0) FS[slot[1]] = fe;
            if (slot[2] >= 0) FB[slot[2]] = fe;
            if (slot[3] >= 0) A2[slot[3]] = x;
        }
        for (int o = 32; o > 0; o >>= 1) {
            int32_t other = __shfl_xor(local_min, o);
            local_min = other < local_min ? other : local_min;
        }
        __shared__ int32_t s_min[BLK / 64];
        if (lane == 0) s_min[threadIdx.x >> 6] = local_min;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t mm = s_min[0];
            for (int w = 1; w < BLK / 64; w++) mm = s_min[w] < mm ? s_min[w] : mm;
            if (mm != 0x7fffffff) atomicMin(&out->min_above, mm);
        }
    } else {
        const int32_t big_round = s_prev.nT + s_prev.nS + s_prev.nB > AGG_MIN_FRONTIER;
        __shared__ PeelLds lds;
        if (big_round) peel_round<true>(B, st, s_prev, out, cur, prv, lds);
        else peel_round<false>(B, st, s_prev, out, cur, prv, lds);
    }
}

// The undirected adjacency from the static edge table, whose edges are sorted
// by (lo, hi): vertex v's row is its lower neighbours (edges with hi = v, in lo
// order) followed by its higher ones (edges with lo = v, in hi order), so both
// halves are already ascending.  hkey/hval: the table's (hi, lo) pairs stably
// sorted by hi.  With loff[v] = #edges with lo < v and hoff[v] = #edges with
// hi < v, row v starts at loff[v] + hoff[v].
__device__ inline int64_t lower_bound_i32(const int32_t *__restrict__ a, int64_t len, int32_t x) {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_adj_rows(const int32_t *__restrict__ slo, const int32_t *__restrict__ hkey, int32_t S, int32_t n,
                           int32_t *__restrict__ loff, int32_t *__restrict__ hoff, int64_t *__restrict__ uoff) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > n) return;
    const int64_t a = lower_bound_i32(slo, S, (int32_t)x), b = lower_bound_i32(hkey, S, (int32_t)x);
    loff[x] = (int32_t)a;
    hoff[x] = (int32_t)b;
    uoff[x] = a + b;
}

// edge s = (lo, hi) in lo's row: after lo's hoff[lo + 1] - hoff[lo] lower
// neighbours, at uoff[lo] + that + (s - loff[lo]) = hoff[lo + 1] + s
// the neighbour id in the plain adjacency, and in the peel's copy for large
// rounds HUB_FLAG | slot for a hub (uadj_h null: no hubs)
__device__ inline void adj_put(int64_t pos, int32_t y, const int32_t *__restrict__ hub_of, int32_t *__restrict__ uadj,
                               int32_t *__restrict__ uadj_h) {
    uadj[pos] = y;
    if (uadj_h) {
        const int32_t h = hub_of[y];
        uadj_h[pos] = h >= 0 ? (int32_t)(HUB_FLAG | (uint32_t)h) : y;
    }
}

__global__ void k_adj_fill_up(const int32_t *__restrict__ slo, const int32_t *__restrict__ shi, int32_t S,
                              const int32_t *__restrict__ hoff, const int32_t *__restrict__ hub_of,
                              int32_t *__restrict__ uadj, int32_t *__restrict__ uadj_h) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < S) adj_put((int64_t)hoff[slo[e] + 1] + e, shi[e], hub_of, uadj, uadj_h);
}

// sorted position q (hi = hkey[q], lo = hval[q]) in hi's row: at
// uoff[hi] + (q - hoff[hi]) = loff[hi] + q
__global__ void k_adj_fill_down(const int32_t *__restrict__ hkey, const int32_t *__restrict__ hval, int32_t S,
                                const int32_t *__restrict__ loff, const int32_t *__restrict__ hub_of,
                                int32_t *__restrict__ uadj, int32_t *__restrict__ uadj_h) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < S) adj_put((int64_t)loff[hkey[q]] + q, hval[q], hub_of, uadj, uadj_h);
}

// hubs of the peeling adjacency: vertices of degree > HUB_DEG, first HUB_SLOTS found
__global__ void k_find_hubs(const int32_t *__restrict__ deg, int32_t n, int32_t *__restrict__ hub_of,
                            int32_t *__restrict__ hub_vertex, int32_t *__restrict__ n_hubs) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool hub = x < n && deg[x] > HUB_DEG;
    int32_t slot = wave_append(n_hubs, hub);
    if (x < n) hub_of[x] = -1;
    if (slot >= 0 && slot < HUB_SLOTS) {
        hub_of[x] = slot;
        hub_vertex[slot] = (int32_t)x;
    }
}

__global__ void k_adj_deg(const int64_t *__restrict__ uoff, int32_t n, int32_t *__restrict__ deg) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) deg[x] = (int32_t)(uoff[x + 1] - uoff[x]);
}

__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ void k_rank_keys(const int32_t *__restrict__ rnd, const int32_t *__restrict__ deg, int32_t n,
                            int mode, uint32_t seed, uint32_t *__restrict__ key, int32_t *__restrict__ val) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    uint32_t k;
    if (mode == FOLTY_RANK_DEGENERACY) k = (uint32_t)rnd[x];
    else if (mode == FOLTY_RANK_DEGREE) k = (uint32_t)deg[x];
    else k = mix32((uint32_t)x ^ mix32(seed));
    key[x] = k;
    val[x] = (int32_t)x;
}

__global__ void k_rank_scatter(const int32_t *__restrict__ order, int32_t n, int32_t *__restrict__ rank) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    rank[order[j]] = (int32_t)j;
}

__global__ void k_orient_keys(const int32_t *__restrict__ slo, const int32_t *__restrict__ shi,
                              const int32_t *__restrict__ rank, int32_t S, int64_t n,
                              uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int64_t a = rank[slo[s]], b = rank[shi[s]];
    uint64_t tail = a < b ? a : b, head = a < b ? b : a;
    key[s] = tail * (uint64_t)n + head;
    val[s] = (uint32_t)s | (a < b ? 0x80000000u : 0u);
}

__global__ void k_orient_unpack(const uint64_t *__restrict__ key, int32_t S, int64_t n,
                                int32_t *__restrict__ oadj, int32_t *__restrict__ otail) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    oadj[j] = (int32_t)(key[j] % (uint64_t)n);
    otail[j] = (int32_t)(key[j] / (uint64_t)n);
}

// oriented CSR rows: row x starts at the first key >= x * n
__global__ void k_orient_rows(const uint64_t *__restrict__ key, int32_t S, int64_t n, int32_t *__restrict__ ooff) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > n) return;
    uint64_t want = (uint64_t)x * (uint64_t)n;
    int32_t a = 0, b = S;
    while (a < b) {
        int32_t mid = (int32_t)(((int64_t)a + b) >> 1);
        if (key[mid] < want) a = mid + 1;
        else b = mid;
    }
    ooff[x] = a;
}

struct OrientStats {
    unsigned long long wedges;
    int32_t max_out;
    int32_t max_core;
};

__global__ void k_orient_stats(const int32_t *__restrict__ ooff, const int32_t *__restrict__ rank,
                               const int32_t *__restrict__ core, int32_t n,
                               int32_t *__restrict__ outdeg_orig, OrientStats *os) {
    unsigned long long w = 0;
    int32_t mo = 0, mc = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = rank[x];
        int32_t d = ooff[r + 1] - ooff[r];
        outdeg_orig[x] = d;
        w += (unsigned long long)d * (unsigned long long)(d > 0 ? d - 1 : 0) / 2ull;
        mo = d > mo ? d : mo;
        mc = core[x] > mc ? core[x] : mc;
    }
    __shared__ unsigned long long s_w[BLK / 64];
    __shared__ int32_t s_o[BLK / 64], s_c[BLK / 64];
    for (int o = 32; o > 0; o >>= 1) {
        w += __shfl_xor(w, o);
        int32_t a = __shfl_xor(mo, o), c = __shfl_xor(mc, o);
        mo = a > mo ? a : mo;
        mc = c > mc ? c : mc;
    }
    if (lane_id() == 0) {
        s_w[threadIdx.x >> 6] = w;
        s_o[threadIdx.x >> 6] = mo;
        s_c[threadIdx.x >> 6] = mc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < BLK / 64; i++) {
            w += s_w[i];
            mo = s_o[i] > mo ? s_o[i] : mo;
            mc = s_c[i] > mc ? s_c[i] : mc;
        }
        if (w) atomicAdd(&os->wedges, w);
        if (mo) atomicMax(&os->max_out, mo);
        if (mc) atomicMax(&os->max_core, mc);
    }
}

} // namespace


static double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    FOLTY_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
}

void load_graph(Graph *g, int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
                int32_t mem_kind, void *stream) {
    if (n < 1) fail(FOLTY_EINVAL, "n must be >= 1 (got %d)", n);
    if (m < 0) fail(FOLTY_EINVAL, "m must be >= 0");
    if (m >= (int64_t(1) << 31) - 1) fail(FOLTY_EOVERFLOW, "m = %lld needs 64-bit edge ids", (long long)m);
    if (m > 0 && (!src || !dst || !t)) fail(FOLTY_EINVAL, "null input array");
    if (mem_kind != FOLTY_MEM_HOST && mem_kind != FOLTY_MEM_DEVICE) fail(FOLTY_EINVAL, "bad mem_kind");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        fail(FOLTY_EDEVICE, "no HIP device available");
    }
    FOLTY_HIP(hipGetDevice(&g->device));
    if (stream) {
        g->stream = (hipStream_t)stream;
    } else {
        FOLTY_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
        g->own_stream = true;
    }
    hipStream_t s = g->stream;
    StreamScope sc(s);
    g->ix.n = n;
    g->ix.m_input = m;
    g->src.ensure(sizeof(int32_t) * m);
    g->dst.ensure(sizeof(int32_t) * m);
    g->t.ensure(sizeof(int64_t) * m);
    hipMemcpyKind kind = mem_kind == FOLTY_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (m > 0) {
        FOLTY_HIP(hipMemcpyAsync(g->src.p, src, sizeof(int32_t) * m, kind, s));
        FOLTY_HIP(hipMemcpyAsync(g->dst.p, dst, sizeof(int32_t) * m, kind, s));
        FOLTY_HIP(hipMemcpyAsync(g->t.p, t, sizeof(int64_t) * m, kind, s));
    }
    DevBuf vo;
    vo.ensure(sizeof(ValOut));
    k_init_val<<<1, 1, 0, s>>>(vo.as<ValOut>());
    FOLTY_LAUNCHED();
    if (m > 0) {
        k_validate<<<grid_for(m, BLK, 4096), BLK, 0, s>>>(g->src.as<int32_t>(), g->dst.as<int32_t>(),
                                                          g->t.as<int64_t>(), m, n, vo.as<ValOut>());
        FOLTY_LAUNCHED();
    }
    ValOut h{};
    FOLTY_HIP(hipMemcpyAsync(&h, vo.p, sizeof(ValOut), hipMemcpyDeviceToHost, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    if (h.first_bad != ~0ull)
        fail(FOLTY_EINVAL, "temporal edge %llu has a vertex id outside [0, %d) or a timestamp outside [0, 2^62)",
             h.first_bad, n);
    g->ix.self_loops = (int64_t)h.loops;
    g->tmax = (int64_t)h.tmax;
    g->sorted_by_time = h.descents == 0;
}

void build_index(Graph *g, const folty_build_opts *opts) {
    folty_build_opts o{};
    if (opts) o = *opts;
    if (o.rank_mode < 0 || o.rank_mode > 2) fail(FOLTY_EINVAL, "unknown rank_mode %d", o.rank_mode);
    if (g->ix.m_input > 0 && !g->src.p) fail(FOLTY_EINVAL, "graph inputs were released");
    Index &ix = g->ix;
    hipStream_t s = g->stream;
    const int32_t n = ix.n;
    const int64_t min = ix.m_input;
    ix.built = false;
    ix.tri_cached = false;
    ix.tri.release();

    hipEvent_t e0, e1;
    FOLTY_HIP(hipEventCreate(&e0));
    FOLTY_HIP(hipEventCreate(&e1));
    struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } evg{e0, e1};
    FOLTY_HIP(hipEventRecord(e0, s));

    PinnedBuf hb;
    hb.ensure(256);
    DevBuf cub;
    auto cub_ensure = [&](size_t b) { cub.ensure(b); return cub.p; };

    // ---- a.2: group by (lo, hi, dir, t, input position) ----------------------
    const int32_t m = (int32_t)(min - ix.self_loops);
    ix.m = m;
    DevBuf idx_t, tkeys, tkeys2, idx_t2, pkey, pkey2, pos, pos2;
    const int32_t *idx_time = nullptr; // nullptr = identity (input already in time order)
    if (min > 0 && !g->sorted_by_time) {
        tkeys.ensure(8 * min);
        tkeys2.ensure(8 * min);
        idx_t.ensure(4 * min);
        idx_t2.ensure(4 * min);
        k_iota_tkeys<<<grid_for(min, BLK), BLK, 0, s>>>(g->t.as<int64_t>(), tkeys.as<uint64_t>(),
                                                        idx_t.as<int32_t>(), min);
        FOLTY_LAUNCHED();
        int tb = bit_length((uint64_t)g->tmax);
        size_t need = sort_pairs_u64_i32(nullptr, 0, tkeys.as<uint64_t>(), tkeys2.as<uint64_t>(),
                                         idx_t.as<int32_t>(), idx_t2.as<int32_t>(), min, tb, s);
        sort_pairs_u64_i32(cub_ensure(need), need, tkeys.as<uint64_t>(), tkeys2.as<uint64_t>(),
                           idx_t.as<int32_t>(), idx_t2.as<int32_t>(), min, tb, s);
        tkeys.release();
        tkeys2.release();
        idx_time = idx_t2.as<int32_t>();
    }
    if (min > 0) {
        pkey.ensure(8 * min);
        pkey2.ensure(8 * min);
        pos.ensure(4 * min);
        pos2.ensure(4 * min);
        k_pair_keys<<<grid_for(min, BLK), BLK, 0, s>>>(idx_time, g->src.as<int32_t>(), g->dst.as<int32_t>(),
                                                       n, pkey.as<uint64_t>(), pos.as<int32_t>(), min);
        FOLTY_LAUNCHED();
        int kb = bit_length(2ull * (uint64_t)n * (uint64_t)n);
        size_t need = sort_pairs_u64_i32(nullptr, 0, pkey.as<uint64_t>(), pkey2.as<uint64_t>(),
                                         pos.as<int32_t>(), pos2.as<int32_t>(), min, kb, s);
        sort_pairs_u64_i32(cub_ensure(need), need, pkey.as<uint64_t>(), pkey2.as<uint64_t>(),
                           pos.as<int32_t>(), pos2.as<int32_t>(), min, kb, s);
        pkey.release();
        pos.release();
    }
    ix.ts.ensure(8 * (size_t)m);
    ix.perm.ensure(4 * (size_t)m);
    ix.sid.ensure(4 * (size_t)m);
    if (m > 0) {
        k_gather_sorted<<<grid_for(m, BLK), BLK, 0, s>>>(pos2.as<int32_t>(), idx_time, g->t.as<int64_t>(),
                                                         ix.perm.as<int32_t>(), ix.ts.as<int64_t>(), m);
        FOLTY_LAUNCHED();
    }
    idx_t.release();
    idx_t2.release();
    pos2.release();

    // ---- static edge table -----------------------------------------------------
    int32_t S = 0;
    if (m > 0) {
        DevBuf flag;
        flag.ensure(4 * (size_t)m);
        k_static_flags<<<grid_for(m, BLK), BLK, 0, s>>>(pkey2.as<uint64_t>(), m, flag.as<int32_t>());
        FOLTY_LAUNCHED();
        size_t need = inclusive_scan_i32(nullptr, 0, flag.as<int32_t>(), ix.sid.as<int32_t>(), m, s);
        inclusive_scan_i32(cub_ensure(need), need, flag.as<int32_t>(), ix.sid.as<int32_t>(), m, s);
        FOLTY_HIP(hipMemcpyAsync(hb.p, ix.sid.as<int32_t>() + (m - 1), 4, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
        S = *hb.as<int32_t>();
    }
    ix.S = S;
    ix.soff.ensure(4 * ((size_t)S + 1));
    ix.smid.ensure(4 * (size_t)S + 4);
    ix.slo.ensure(4 * (size_t)S + 4);
    ix.shi.ensure(4 * (size_t)S + 4);
    DevBuf pstat;
    pstat.ensure(sizeof(PairStats));
    FOLTY_HIP(hipMemsetAsync(pstat.p, 0, sizeof(PairStats), s));
    if (S == 0) {
        FOLTY_HIP(hipMemsetAsync(ix.soff.p, 0, 4, s));
    } else {
        k_fill<int32_t><<<grid_for(S, BLK), BLK, 0, s>>>(ix.smid.as<int32_t>(), -1, S);
        k_static_table<<<grid_for(m, BLK), BLK, 0, s>>>(pkey2.as<uint64_t>(), ix.sid.as<int32_t>(), m, n,
                                                        ix.soff.as<int32_t>(), ix.smid.as<int32_t>(),
                                                        ix.slo.as<int32_t>(), ix.shi.as<int32_t>());
        k_fix_smid_stats<<<grid_for(S, BLK, 2048), BLK, 0, s>>>(ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), S,
                                                                pstat.as<PairStats>());
        FOLTY_LAUNCHED();
    }
    pkey2.release();

    // ---- degrees and undirected adjacency (sorted (x, y) keys) -----------------------
    ix.deg.ensure(4 * ((size_t)n + 1));
    DevBuf uoff, uadj, uadj_h;
    uoff.ensure(8 * ((size_t)n + 1));
    uadj.ensure(8 * (size_t)S + 8);
    DevBuf hub_of, hub_vertex, hub_n;
    hub_of.ensure(4 * (size_t)n);
    hub_vertex.ensure(4 * (size_t)HUB_SLOTS);
    hub_n.ensure(4);
    int32_t n_hubs = 0;
    {
        DevBuf hkey, hval, loff, hoff;
        hkey.ensure(4 * (size_t)S + 4);
        hval.ensure(4 * (size_t)S + 4);
        loff.ensure(4 * ((size_t)n + 1));
        hoff.ensure(4 * ((size_t)n + 1));
        if (S > 0) {
            int kb = bit_length((uint64_t)n);
            size_t need = sort_pairs_u32_i32(nullptr, 0, reinterpret_cast<const uint32_t *>(ix.shi.as<int32_t>()),
                                             hkey.as<uint32_t>(), ix.slo.as<int32_t>(), hval.as<int32_t>(), S, kb, s);
            sort_pairs_u32_i32(cub_ensure(need), need, reinterpret_cast<const uint32_t *>(ix.shi.as<int32_t>()),
                               hkey.as<uint32_t>(), ix.slo.as<int32_t>(), hval.as<int32_t>(), S, kb, s);
        }
        k_adj_rows<<<grid_for((int64_t)n + 1, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), hkey.as<int32_t>(), S, n,
                                                                 loff.as<int32_t>(), hoff.as<int32_t>(),
                                                                 uoff.as<int64_t>());
        k_adj_deg<<<grid_for(n, BLK), BLK, 0, s>>>(uoff.as<int64_t>(), n, ix.deg.as<int32_t>());
        FOLTY_LAUNCHED();
        // the hubs first, so that each fill writes the plain row and the flagged copy together
        FOLTY_HIP(hipMemsetAsync(hub_n.p, 0, 4, s));
        k_find_hubs<<<grid_for(n, BLK), BLK, 0, s>>>(ix.deg.as<int32_t>(), n, hub_of.as<int32_t>(),
                                                    hub_vertex.as<int32_t>(), hub_n.as<int32_t>());
        FOLTY_LAUNCHED();
        FOLTY_HIP(hipMemcpyAsync(hb.p, hub_n.p, 4, hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
        n_hubs = *hb.as<int32_t>();
        if (n_hubs > HUB_SLOTS) n_hubs = HUB_SLOTS;
        if (n_hubs > 0 && S > 0) uadj_h.ensure(8 * (size_t)S + 8);
        int32_t *flagged = n_hubs > 0 && S > 0 ? uadj_h.as<int32_t>() : nullptr;
        if (S > 0) {
            k_adj_fill_up<<<grid_for(S, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), S,
                                                           hoff.as<int32_t>(), hub_of.as<int32_t>(),
                                                           uadj.as<int32_t>(), flagged);
            k_adj_fill_down<<<grid_for(S, BLK), BLK, 0, s>>>(hkey.as<int32_t>(), hval.as<int32_t>(), S,
                                                             loff.as<int32_t>(), hub_of.as<int32_t>(),
                                                             uadj.as<int32_t>(), flagged);
            FOLTY_LAUNCHED();
        }
    }

    // ---- a.3: core numbers by min-degree peeling ------------------------------------
    ix.core.ensure(4 * (size_t)n);
    DevBuf dcur, rnd, fr, alive, pst;
    dcur.ensure(4 * (size_t)n);
    rnd.ensure(4 * (size_t)n);
    fr.ensure(sizeof(FEntry) * 9 * (size_t)n);
    alive.ensure(4 * 2 * (size_t)n);
    pst.ensure(2 * sizeof(PeelState) + 3 * sizeof(PeelCount));
    k_peel_init<<<grid_for(n, BLK), BLK, 0, s>>>(ix.deg.as<int32_t>(), dcur.as<int32_t>(), rnd.as<int32_t>(),
                                                 alive.as<int32_t>(), n);
    FOLTY_LAUNCHED();
    {
        // step 0 reads state[1] (boot) and count[2] (empty)
        char init[2 * sizeof(PeelState) + 3 * sizeof(PeelCount)];
        PeelState boot{};
        boot.mode = PEEL_BOOT;
        PeelCount zero = {0, 0, 0, 0, 0x7fffffff};
        memcpy(init, &boot, sizeof boot);
        memcpy(init + sizeof(PeelState), &boot, sizeof boot);
        for (int i = 0; i < 3; i++) memcpy(init + 2 * sizeof(PeelState) + i * sizeof(PeelCount), &zero, sizeof zero);
        FOLTY_HIP(hipMemcpyAsync(pst.p, init, sizeof init, hipMemcpyHostToDevice, s));
        PeelBufs B;
        B.uoff = uoff.as<int64_t>();
        B.uadj = n_hubs > 0 ? uadj_h.as<int32_t>() : uadj.as<int32_t>();
        B.uadj_plain = uadj.as<int32_t>();
        B.hub_vertex = hub_vertex.as<int32_t>();
        B.n_hubs = n_hubs;
        B.deg = ix.deg.as<int32_t>();
        B.dcur = dcur.as<int32_t>();
        B.rnd = rnd.as<int32_t>();
        B.core = ix.core.as<int32_t>();
        for (int i = 0; i < 3; i++) {
            B.FT[i] = fr.as<FEntry>() + (size_t)i * n;
            B.FS[i] = fr.as<FEntry>() + (size_t)(3 + i) * n;
            B.FB[i] = fr.as<FEntry>() + (size_t)(6 + i) * n;
        }
        B.alive[0] = alive.as<int32_t>();
        B.alive[1] = alive.as<int32_t>() + (size_t)n;
        B.state = pst.as<PeelState>();
        B.count = reinterpret_cast<PeelCount *>(pst.as<char>() + 2 * sizeof(PeelState));
        B.n = n;
        // every step removes a vertex or raises k past a live degree, so the peel
        // ends within about 3n steps; the cap turns a logic error into an error code
        const int64_t cap = 3 * (int64_t)n + 4096;
        int64_t step = 0;
        int batch = 32;
        int blocks = PEEL_BLOCKS_WIDE;
        PeelState h{};
        for (;;) {
            for (int i = 0; i < batch; i++, step++) k_peel_step<<<blocks, BLK, 0, s>>>(B, step);
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipMemcpyAsync(hb.p, B.state + ((step - 1) & 1), sizeof(PeelState), hipMemcpyDeviceToHost, s));
            FOLTY_HIP(hipStreamSynchronize(s));
            memcpy(&h, hb.p, sizeof h);
            if (h.mode == PEEL_DONE) break;
            if (step > cap) fail(FOLTY_EDEVICE, "core peeling did not finish in %lld steps", (long long)step);
            batch = batch < 256 ? 2 * batch : 256;
            // every loop of the step is grid-stride, so any grid size is correct
            blocks = h.alive_n < PEEL_NARROW_BELOW ? PEEL_BLOCKS_NARROW : PEEL_BLOCKS_WIDE;
        }
        if (h.removed != n) fail(FOLTY_EDEVICE, "core peeling removed %d of %d vertices", h.removed, n);
        ix.peel_rounds = h.r;
    }
    dcur.release();
    fr.release();
    alive.release();

    // ---- orientation order and oriented CSR ---------------------------------------------
    ix.rank.ensure(4 * (size_t)n);
    {
        DevBuf key, key2, val, val2;
        key.ensure(4 * (size_t)n);
        key2.ensure(4 * (size_t)n);
        val.ensure(4 * (size_t)n);
        val2.ensure(4 * (size_t)n);
        k_rank_keys<<<grid_for(n, BLK), BLK, 0, s>>>(rnd.as<int32_t>(), ix.deg.as<int32_t>(), n, o.rank_mode,
                                                     (uint32_t)(o.rank_seed ^ (o.rank_seed >> 32)),
                                                     key.as<uint32_t>(), val.as<int32_t>());
        FOLTY_LAUNCHED();
        int kb = o.rank_mode == FOLTY_RANK_DEGENERACY ? bit_length((uint64_t)(ix.peel_rounds > 0 ? ix.peel_rounds : 1))
               : o.rank_mode == FOLTY_RANK_DEGREE ? 32 : 32;
        size_t need = sort_pairs_u32_i32(nullptr, 0, key.as<uint32_t>(), key2.as<uint32_t>(), val.as<int32_t>(),
                                         val2.as<int32_t>(), n, kb, s);
        sort_pairs_u32_i32(cub_ensure(need), need, key.as<uint32_t>(), key2.as<uint32_t>(), val.as<int32_t>(),
                           val2.as<int32_t>(), n, kb, s);
        k_rank_scatter<<<grid_for(n, BLK), BLK, 0, s>>>(val2.as<int32_t>(), n, ix.rank.as<int32_t>());
        FOLTY_LAUNCHED();
    }
    rnd.release();
    ix.rank_mode = o.rank_mode;

    ix.oadj.ensure(4 * (size_t)S + 4);
    ix.otail.ensure(4 * (size_t)S + 4);
    ix.oeid.ensure(4 * (size_t)S + 4);
    ix.ooff.ensure(4 * ((size_t)n + 1));
    ix.outdeg.ensure(4 * (size_t)n);
    {
        DevBuf key, key2, val;
        key.ensure(8 * (size_t)S + 8);
        key2.ensure(8 * (size_t)S + 8);
        val.ensure(4 * (size_t)S + 4);
        if (S > 0) {
            k_orient_keys<<<grid_for(S, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), ix.shi.as<int32_t>(),
                                                           ix.rank.as<int32_t>(), S, n, key.as<uint64_t>(),
                                                           val.as<uint32_t>());
            FOLTY_LAUNCHED();
            int kb = bit_length((uint64_t)n * (uint64_t)n);
            size_t need = sort_pairs_u64_u32(nullptr, 0, key.as<uint64_t>(), key2.as<uint64_t>(), val.as<uint32_t>(),
                                             ix.oeid.as<uint32_t>(), S, kb, s);
            sort_pairs_u64_u32(cub_ensure(need), need, key.as<uint64_t>(), key2.as<uint64_t>(), val.as<uint32_t>(),
                               ix.oeid.as<uint32_t>(), S, kb, s);
            k_orient_unpack<<<grid_for(S, BLK), BLK, 0, s>>>(key2.as<uint64_t>(), S, n, ix.oadj.as<int32_t>(),
                                                             ix.otail.as<int32_t>());
            FOLTY_LAUNCHED();
        }
        k_orient_rows<<<grid_for((int64_t)n + 1, BLK), BLK, 0, s>>>(key2.as<uint64_t>(), S, n, ix.ooff.as<int32_t>());
        FOLTY_LAUNCHED();
    }
    DevBuf ostat;
    ostat.ensure(sizeof(OrientStats));
    FOLTY_HIP(hipMemsetAsync(ostat.p, 0, sizeof(OrientStats), s));
    k_orient_stats<<<grid_for(n, BLK, 2048), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.rank.as<int32_t>(),
                                                          ix.core.as<int32_t>(), n, ix.outdeg.as<int32_t>(),
                                                          ostat.as<OrientStats>());
    FOLTY_LAUNCHED();

    // ---- read back sizes ------------------------------------------------------------
    {
        char *h = hb.as<char>();
        FOLTY_HIP(hipMemcpyAsync(h, pstat.p, sizeof(PairStats), hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(h + 32, ostat.p, sizeof(OrientStats), hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipStreamSynchronize(s));
        PairStats ps;
        OrientStats os;
        memcpy(&ps, h, sizeof ps);
        memcpy(&os, h + 32, sizeof os);
        ix.P = (int64_t)ps.pairs;
        ix.sigma_max = (int64_t)ps.sigma_max;
        ix.W = (int64_t)os.wedges;
        ix.max_out = os.max_out;
        ix.max_core = os.max_core;
    }
    // ---- oriented-edge records and triangles per lowest vertex ------------------------
    ix.tshift = std::max(0, bit_length((uint64_t)g->tmax) - 32);
    index_triangles(ix, o.cache_triangles != 0, cub, s);
    FOLTY_HIP(hipEventRecord(e1, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    ix.build_ms = elapsed_ms(e0, e1);
    ix.built = true;
}

size_t Index::device_bytes() const {
    const DevBuf *b[] = {&ts, &perm, &sid, &soff, &smid, &slo, &shi, &deg, &core, &rank,
                         &outdeg, &ooff, &oadj, &oeid, &rec, &erng, &item, &seg, &tri_base, &tcnt, &tri};
    size_t t = 0;
    for (auto *x : b) t += x->bytes;
    return t;
}

} // namespace folty
