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
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long pairs = 0, smax = 0;
    if (s < S) {
        int32_t a = soff[s], b = soff[s + 1];
        int32_t mid = smid[s];
        if (mid < 0) {
            mid = b;
            smid[s] = b;
        }
        unsigned long long l0 = (unsigned long long)(mid - a), l1 = (unsigned long long)(b - mid);
        pairs = (l0 > 0) + (l1 > 0);
        smax = l0 > l1 ? l0 : l1;
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
constexpr int PEEL_BLOCKS = 512;
constexpr int32_t BIG_DEG = 2048; // frontier vertices above this degree share the grid

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

struct PeelCount {   // what step i produced
    int32_t nS, nB;   // frontier written (degree <= BIG_DEG / above)
    int32_t nA;       // live list written (collect)
    int32_t min_above;
};

struct PeelBufs {
    const int64_t *uoff;
    const int32_t *uadj;
    const int32_t *deg;
    int32_t *dcur, *rnd, *core;
    int32_t *FS[3], *FB[3];
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
        if (c.nS + c.nB > 0) {
            s.mode = PEEL_ROUND;
            s.n_in = c.nS + c.nB;
        } else if (c.nA == 0) {
            s.mode = PEEL_DONE;
        } else {
            s.k = c.min_above; // nothing at degree <= k: jump to the smallest live degree
        }
    } else if (p.mode == PEEL_ROUND) {
        s.removed = p.removed + p.n_in;
        s.r = p.r + 1;
        if (c.nS + c.nB > 0) {
            s.n_in = c.nS + c.nB;
        } else {
            s.mode = PEEL_COLLECT;
            s.k = p.k + 1;
            s.n_in = 0;
        }
    }
    return s;
}

__device__ inline void peel_neighbour(int32_t y, bool valid, int32_t k, const PeelBufs &B, PeelCount *out,
                                      int32_t *FS, int32_t *FB) {
    bool push = false;
    if (valid && B.rnd[y] < 0) {
        int32_t old = atomicSub(&B.dcur[y], 1);
        push = (old == k + 1);
    }
    bool big = push && B.deg[y] > BIG_DEG;
    int32_t a = wave_append(&out->nS, push && !big);
    if (a >= 0) FS[a] = y;
    int32_t b = wave_append(&out->nB, big);
    if (b >= 0) FB[b] = y;
}

// block-aggregated append of up to three predicates: one global atomic per block
// and per predicate; slot[j] is this thread's index in list j or -1
__device__ inline void block_append3(bool p0, bool p1, bool p2, int32_t *g0, int32_t *g1, int32_t *g2,
                                     int32_t slot[3]) {
    __shared__ int32_t s_cnt[3], s_base[3];
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int lane = lane_id();
    bool p[3] = {p0, p1, p2};
    int32_t local[3];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        unsigned long long mask = __ballot(p[j]);
        int32_t woff = 0;
        int leader = mask ? __ffsll((long long)mask) - 1 : 0;
        if (mask && lane == leader) woff = atomicAdd(&s_cnt[j], (int32_t)__popcll(mask));
        woff = __shfl(woff, leader);
        local[j] = p[j] ? woff + (int32_t)__popcll(mask & ((1ull << lane) - 1ull)) : -1;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int32_t *g = threadIdx.x == 0 ? g0 : (threadIdx.x == 1 ? g1 : g2);
        s_base[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(g, s_cnt[threadIdx.x]) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; j++) slot[j] = local[j] >= 0 ? s_base[j] + local[j] : -1;
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
        PeelCount z = {0, 0, 0, 0x7fffffff};
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
        int32_t *FS = B.FS[cur], *FB = B.FB[cur];
        int32_t local_min = 0x7fffffff;
        for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < na; base += stride) {
            int64_t i = base + threadIdx.x;
            bool valid = i < na;
            int32_t x = valid ? A[i] : 0;
            bool live = valid && B.rnd[x] < 0;
            int32_t d = live ? B.dcur[x] : 0;
            bool take = live && d <= k;
            bool big = take && B.deg[x] > BIG_DEG;
            bool keep = live && d > k;
            if (keep && d < local_min) local_min = d;
            int32_t slot[3];
            block_append3(take && !big, big, keep, &out->nS, &out->nB, &out->nA, slot);
            if (slot[0] >= 0) FS[slot[0]] = x;
            if (slot[1] >= 0) FB[slot[1]] = x;
            if (slot[2] >= 0) A2[slot[2]] = x;
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
        // the frontier is what the previous step wrote
        int32_t nS = s_prev.nS < n ? s_prev.nS : n, nB = s_prev.nB < n ? s_prev.nB : n;
        const int32_t *FS = B.FS[prv], *FB = B.FB[prv];
        int32_t *NS = B.FS[cur], *NB = B.FB[cur];
        const int32_t r = st.r;
        for (int64_t i = gtid; i < nS; i += stride) {
            int32_t x = FS[i];
            B.rnd[x] = r;
            B.core[x] = k;
        }
        for (int64_t i = gtid; i < nB; i += stride) {
            int32_t x = FB[i];
            B.rnd[x] = r;
            B.core[x] = k;
        }
        // a frontier vertex seen as live here is only decremented, never pushed:
        // its degree is already <= k
        for (int64_t w = gwave; w < nS; w += nwaves) {
            int32_t x = FS[w];
            int64_t b = B.uoff[x], e = B.uoff[x + 1];
            for (int64_t p0 = b; p0 < e; p0 += 64) {
                int64_t p = p0 + lane;
                bool valid = p < e;
                peel_neighbour(valid ? B.uadj[p] : 0, valid, k, B, out, NS, NB);
            }
        }
        for (int32_t j = 0; j < nB; j++) {
            int32_t x = FB[j];
            int64_t b = B.uoff[x], e = B.uoff[x + 1];
            for (int64_t p0 = b + gwave * 64; p0 < e; p0 += nwaves * 64) {
                int64_t p = p0 + lane;
                bool valid = p < e;
                peel_neighbour(valid ? B.uadj[p] : 0, valid, k, B, out, NS, NB);
            }
        }
    }
}

// undirected adjacency from the static edge table: both (x, y) keys per edge
__global__ void k_adj_keys(const int32_t *__restrict__ slo, const int32_t *__restrict__ shi, int32_t S,
                           uint64_t *__restrict__ key) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint64_t a = (uint32_t)slo[s], b = (uint32_t)shi[s];
    key[2 * s] = (a << 32) | b;
    key[2 * s + 1] = (b << 32) | a;
}

__global__ void k_adj_unpack(const uint64_t *__restrict__ key, int64_t E, int32_t *__restrict__ uadj) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < E) uadj[i] = (int32_t)(key[i] & 0xffffffffu);
}

// row starts by binary search over the sorted keys; degrees from consecutive starts
__global__ void k_adj_rows(const uint64_t *__restrict__ key, int64_t E, int32_t n, int64_t *__restrict__ uoff) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > n) return;
    uint64_t want = (uint64_t)x << 32;
    int64_t a = 0, b = E;
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if (key[mid] < want) a = mid + 1;
        else b = mid;
    }
    uoff[x] = a;
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
                                int32_t *__restrict__ osrc, int32_t *__restrict__ oadj,
                                int32_t *__restrict__ outdeg_new) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    uint64_t k = key[j];
    int32_t tail = (int32_t)(k / (uint64_t)n), head = (int32_t)(k % (uint64_t)n);
    osrc[j] = tail;
    oadj[j] = head;
    atomicAdd(&outdeg_new[tail], 1);
}

struct OrientStats {
    unsigned long long wedges;
    int32_t max_out;
    int32_t max_core;
};

__global__ void k_orient_stats(const int32_t *__restrict__ outdeg_new, const int32_t *__restrict__ rank,
                               const int32_t *__restrict__ core, int32_t n,
                               int32_t *__restrict__ outdeg_orig, OrientStats *os) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long w = 0;
    int32_t mo = 0, mc = 0;
    if (x < n) {
        int32_t d = outdeg_new[rank[x]];
        outdeg_orig[x] = d;
        w = (unsigned long long)d * (unsigned long long)(d > 0 ? d - 1 : 0) / 2ull;
        mo = d;
        mc = core[x];
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

// triangles closed from each oriented edge (u -> v): heads w of u after v that
// are also heads of v.  Both rows ascend, so the search window in v's row only
// moves forward.
__global__ void k_tri_count(const int32_t *__restrict__ osrc, const int32_t *__restrict__ oadj,
                            const int32_t *__restrict__ ooff, const uint32_t *__restrict__ oeid,
                            int32_t S, int32_t *__restrict__ tri_cnt, int32_t *__restrict__ tcnt) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    int32_t u = osrc[j], v = oadj[j];
    int32_t end = ooff[u + 1];
    int32_t lo = ooff[v], hi = ooff[v + 1];
    int32_t c = 0;
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
            c++;
            atomicAdd(&tcnt[oeid[j2] & 0x7fffffffu], 1);
            atomicAdd(&tcnt[oeid[a] & 0x7fffffffu], 1);
            lo = a + 1;
        }
    }
    tri_cnt[j] = c;
    if (c) atomicAdd(&tcnt[oeid[j] & 0x7fffffffu], c);
}

} // namespace

// defined in query.hip: writes the triangle list of the index
void enumerate_triangles(const Index &ix, uint32_t *tri, hipStream_t s);

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
        k_fix_smid_stats<<<grid_for(S, BLK), BLK, 0, s>>>(ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), S,
                                                          pstat.as<PairStats>());
        FOLTY_LAUNCHED();
    }
    pkey2.release();

    // ---- degrees and undirected adjacency (sorted (x, y) keys) -----------------------
    ix.deg.ensure(4 * ((size_t)n + 1));
    DevBuf uoff, uadj;
    uoff.ensure(8 * ((size_t)n + 1));
    uadj.ensure(8 * (size_t)S + 8);
    {
        const int64_t E = 2 * (int64_t)S;
        DevBuf k1, k2;
        k1.ensure(8 * (size_t)E + 8);
        k2.ensure(8 * (size_t)E + 8);
        if (S > 0) {
            k_adj_keys<<<grid_for(S, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), S,
                                                        k1.as<uint64_t>());
            FOLTY_LAUNCHED();
            int kb = 32 + bit_length((uint64_t)n);
            size_t need = sort_keys_u64(nullptr, 0, k1.as<uint64_t>(), k2.as<uint64_t>(), E, kb, s);
            sort_keys_u64(cub_ensure(need), need, k1.as<uint64_t>(), k2.as<uint64_t>(), E, kb, s);
            k_adj_unpack<<<grid_for(E, BLK), BLK, 0, s>>>(k2.as<uint64_t>(), E, uadj.as<int32_t>());
            FOLTY_LAUNCHED();
        }
        k_adj_rows<<<grid_for((int64_t)n + 1, BLK), BLK, 0, s>>>(k2.as<uint64_t>(), E, n, uoff.as<int64_t>());
        k_adj_deg<<<grid_for(n, BLK), BLK, 0, s>>>(uoff.as<int64_t>(), n, ix.deg.as<int32_t>());
        FOLTY_LAUNCHED();
    }

    // ---- a.3: core numbers by min-degree peeling ------------------------------------
    ix.core.ensure(4 * (size_t)n);
    DevBuf dcur, rnd, fr, alive, pst;
    dcur.ensure(4 * (size_t)n);
    rnd.ensure(4 * (size_t)n);
    fr.ensure(4 * 6 * (size_t)n);
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
        PeelCount zero = {0, 0, 0, 0x7fffffff};
        memcpy(init, &boot, sizeof boot);
        memcpy(init + sizeof(PeelState), &boot, sizeof boot);
        for (int i = 0; i < 3; i++) memcpy(init + 2 * sizeof(PeelState) + i * sizeof(PeelCount), &zero, sizeof zero);
        FOLTY_HIP(hipMemcpyAsync(pst.p, init, sizeof init, hipMemcpyHostToDevice, s));
        PeelBufs B;
        B.uoff = uoff.as<int64_t>();
        B.uadj = uadj.as<int32_t>();
        B.deg = ix.deg.as<int32_t>();
        B.dcur = dcur.as<int32_t>();
        B.rnd = rnd.as<int32_t>();
        B.core = ix.core.as<int32_t>();
        for (int i = 0; i < 3; i++) {
            B.FS[i] = fr.as<int32_t>() + (size_t)i * n;
            B.FB[i] = fr.as<int32_t>() + (size_t)(3 + i) * n;
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
        int batch = 64;
        PeelState h{};
        for (;;) {
            for (int i = 0; i < batch; i++, step++) k_peel_step<<<PEEL_BLOCKS, BLK, 0, s>>>(B, step);
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipMemcpyAsync(hb.p, B.state + ((step - 1) & 1), sizeof(PeelState), hipMemcpyDeviceToHost, s));
            FOLTY_HIP(hipStreamSynchronize(s));
            memcpy(&h, hb.p, sizeof h);
            if (h.mode == PEEL_DONE) break;
            if (step > cap) fail(FOLTY_EDEVICE, "core peeling did not finish in %lld steps", (long long)step);
            batch = batch < 512 ? 2 * batch : 512;
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

    ix.osrc.ensure(4 * (size_t)S + 4);
    ix.oadj.ensure(4 * (size_t)S + 4);
    ix.oeid.ensure(4 * (size_t)S + 4);
    ix.ooff.ensure(4 * ((size_t)n + 1));
    ix.outdeg.ensure(4 * (size_t)n);
    DevBuf od_new;
    od_new.ensure(4 * ((size_t)n + 1));
    FOLTY_HIP(hipMemsetAsync(od_new.p, 0, 4 * ((size_t)n + 1), s));
    if (S > 0) {
        DevBuf key, key2, val;
        key.ensure(8 * (size_t)S);
        key2.ensure(8 * (size_t)S);
        val.ensure(4 * (size_t)S);
        k_orient_keys<<<grid_for(S, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), ix.shi.as<int32_t>(),
                                                       ix.rank.as<int32_t>(), S, n, key.as<uint64_t>(),
                                                       val.as<uint32_t>());
        FOLTY_LAUNCHED();
        int kb = bit_length((uint64_t)n * (uint64_t)n);
        size_t need = sort_pairs_u64_u32(nullptr, 0, key.as<uint64_t>(), key2.as<uint64_t>(), val.as<uint32_t>(),
                                         ix.oeid.as<uint32_t>(), S, kb, s);
        sort_pairs_u64_u32(cub_ensure(need), need, key.as<uint64_t>(), key2.as<uint64_t>(), val.as<uint32_t>(),
                           ix.oeid.as<uint32_t>(), S, kb, s);
        k_orient_unpack<<<grid_for(S, BLK), BLK, 0, s>>>(key2.as<uint64_t>(), S, n, ix.osrc.as<int32_t>(),
                                                         ix.oadj.as<int32_t>(), od_new.as<int32_t>());
        FOLTY_LAUNCHED();
    }
    {
        size_t need = exclusive_scan_i32(nullptr, 0, od_new.as<int32_t>(), ix.ooff.as<int32_t>(), n + 1, s);
        exclusive_scan_i32(cub_ensure(need), need, od_new.as<int32_t>(), ix.ooff.as<int32_t>(), n + 1, s);
    }
    DevBuf ostat;
    ostat.ensure(sizeof(OrientStats));
    FOLTY_HIP(hipMemsetAsync(ostat.p, 0, sizeof(OrientStats), s));
    k_orient_stats<<<grid_for(n, BLK), BLK, 0, s>>>(od_new.as<int32_t>(), ix.rank.as<int32_t>(), ix.core.as<int32_t>(),
                                                    n, ix.outdeg.as<int32_t>(), ostat.as<OrientStats>());
    FOLTY_LAUNCHED();
    od_new.release();

    // ---- triangles per oriented edge and per static edge ----------------------------------
    ix.tri_off.ensure(8 * ((size_t)S + 1));
    ix.tcnt.ensure(4 * (size_t)S + 4);
    {
        DevBuf tri_cnt;
        tri_cnt.ensure(4 * ((size_t)S + 1));
        FOLTY_HIP(hipMemsetAsync(tri_cnt.p, 0, 4 * ((size_t)S + 1), s));
        FOLTY_HIP(hipMemsetAsync(ix.tcnt.p, 0, 4 * (size_t)S + 4, s));
        if (S > 0) {
            k_tri_count<<<grid_for(S, BLK), BLK, 0, s>>>(ix.osrc.as<int32_t>(), ix.oadj.as<int32_t>(),
                                                         ix.ooff.as<int32_t>(), ix.oeid.as<uint32_t>(), S,
                                                         tri_cnt.as<int32_t>(), ix.tcnt.as<int32_t>());
            FOLTY_LAUNCHED();
        }
        size_t need = exclusive_scan_i32_to_i64(nullptr, 0, tri_cnt.as<int32_t>(), ix.tri_off.as<int64_t>(), S + 1, s);
        exclusive_scan_i32_to_i64(cub_ensure(need), need, tri_cnt.as<int32_t>(), ix.tri_off.as<int64_t>(), S + 1, s);
    }

    // ---- read back sizes ------------------------------------------------------------
    {
        char *h = hb.as<char>();
        FOLTY_HIP(hipMemcpyAsync(h, pstat.p, sizeof(PairStats), hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(h + 32, ostat.p, sizeof(OrientStats), hipMemcpyDeviceToHost, s));
        FOLTY_HIP(hipMemcpyAsync(h + 64, ix.tri_off.as<int64_t>() + S, 8, hipMemcpyDeviceToHost, s));
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
        memcpy(&ix.T, h + 64, 8);
    }
    if (o.cache_triangles && ix.T > 0) {
        ix.tri.ensure(12 * (size_t)ix.T);
        enumerate_triangles(ix, ix.tri.as<uint32_t>(), s);
        ix.tri_cached = true;
    }
    FOLTY_HIP(hipEventRecord(e1, s));
    FOLTY_HIP(hipStreamSynchronize(s));
    ix.build_ms = elapsed_ms(e0, e1);
    ix.built = true;
}

size_t Index::device_bytes() const {
    const DevBuf *b[] = {&ts, &perm, &sid, &soff, &smid, &slo, &shi, &deg, &core, &rank,
                         &outdeg, &ooff, &oadj, &oeid, &osrc, &tri_off, &tcnt, &tri};
    size_t t = 0;
    for (auto *x : b) t += x->bytes;
    return t;
}

} // namespace folty
