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
    // block reduction through one atomic per wave
    for (int o = 32; o > 0; o >>= 1) {
        pairs += __shfl_xor(pairs, o);
        unsigned long long other = __shfl_xor(smax, o);
        smax = other > smax ? other : smax;
    }
    if (lane_id() == 0) {
        if (pairs) atomicAdd(&ps->pairs, pairs);
        if (smax) atomicMax(&ps->sigma_max, smax);
    }
}

__global__ void k_degrees(const int32_t *__restrict__ slo, const int32_t *__restrict__ shi, int32_t S,
                          int32_t *__restrict__ deg) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    atomicAdd(&deg[slo[s]], 1);
    atomicAdd(&deg[shi[s]], 1);
}

__global__ void k_fill_uadj(const int32_t *__restrict__ slo, const int32_t *__restrict__ shi, int32_t S,
                            unsigned long long *__restrict__ cursor, int32_t *__restrict__ uadj) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int32_t a = slo[s], b = shi[s];
    unsigned long long p = atomicAdd(&cursor[a], 1ull);
    uadj[p] = b;
    p = atomicAdd(&cursor[b], 1ull);
    uadj[p] = a;
}

// ---- min-degree peeling -------------------------------------------------------
__global__ void k_peel_init(const int32_t *__restrict__ deg, int32_t *__restrict__ dcur,
                            int32_t *__restrict__ rnd, int32_t n) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    dcur[x] = deg[x];
    rnd[x] = -1;
}

// all live vertices with current degree <= k, plus the smallest live degree above k
__global__ void k_collect(const int32_t *__restrict__ dcur, const int32_t *__restrict__ rnd, int32_t n,
                          int32_t k, int32_t *__restrict__ F, int32_t *__restrict__ counters) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool live = x < n && rnd[x] < 0;
    int32_t d = live ? dcur[x] : 0x7fffffff;
    int32_t slot = wave_append(&counters[0], live && d <= k);
    if (slot >= 0) F[slot] = (int32_t)x;
    int32_t above = (live && d > k) ? d : 0x7fffffff;
    for (int o = 32; o > 0; o >>= 1) {
        int32_t other = __shfl_xor(above, o);
        above = other < above ? other : above;
    }
    if (lane_id() == 0 && above != 0x7fffffff) atomicMin(&counters[1], above);
}

__global__ void k_mark(const int32_t *__restrict__ F, int32_t nF, int32_t r, int32_t k,
                       int32_t *__restrict__ rnd, int32_t *__restrict__ core) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nF) return;
    int32_t x = F[i];
    rnd[x] = r;
    core[x] = k;
}

// one wave per removed vertex; a neighbour whose degree crosses from k+1 to k
// joins the next round
__global__ void k_peel(const int32_t *__restrict__ F, int32_t nF, const int64_t *__restrict__ uoff,
                       const int32_t *__restrict__ uadj, int32_t k, int32_t *__restrict__ dcur,
                       const int32_t *__restrict__ rnd, int32_t *__restrict__ next,
                       int32_t *__restrict__ counters) {
    int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wave >= nF) return;
    int lane = lane_id();
    int32_t x = F[wave];
    int64_t b = uoff[x], e = uoff[x + 1];
    for (int64_t base = b; base < e; base += 64) {
        int64_t p = base + lane;
        bool push = false;
        int32_t y = -1;
        if (p < e) {
            y = uadj[p];
            if (rnd[y] < 0) {
                int32_t old = atomicSub(&dcur[y], 1);
                push = (old == k + 1);
            }
        }
        int32_t slot = wave_append(&counters[2], push);
        if (slot >= 0) next[slot] = y;
    }
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
    for (int o = 32; o > 0; o >>= 1) {
        w += __shfl_xor(w, o);
        int32_t a = __shfl_xor(mo, o), c = __shfl_xor(mc, o);
        mo = a > mo ? a : mo;
        mc = c > mc ? c : mc;
    }
    if (lane_id() == 0) {
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

    // ---- degrees and undirected adjacency ----------------------------------------
    ix.deg.ensure(4 * ((size_t)n + 1));
    FOLTY_HIP(hipMemsetAsync(ix.deg.p, 0, 4 * ((size_t)n + 1), s));
    DevBuf uoff, uadj, cursor;
    uoff.ensure(8 * ((size_t)n + 1));
    uadj.ensure(8 * (size_t)S + 8);
    if (S > 0) {
        k_degrees<<<grid_for(S, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), S,
                                                   ix.deg.as<int32_t>());
        FOLTY_LAUNCHED();
    }
    {
        size_t need = exclusive_scan_i32_to_i64(nullptr, 0, ix.deg.as<int32_t>(), uoff.as<int64_t>(), n + 1, s);
        exclusive_scan_i32_to_i64(cub_ensure(need), need, ix.deg.as<int32_t>(), uoff.as<int64_t>(), n + 1, s);
    }
    if (S > 0) {
        cursor.ensure(8 * ((size_t)n + 1));
        FOLTY_HIP(hipMemcpyAsync(cursor.p, uoff.p, 8 * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
        k_fill_uadj<<<grid_for(S, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), S,
                                                     cursor.as<unsigned long long>(), uadj.as<int32_t>());
        FOLTY_LAUNCHED();
        cursor.release();
    }

    // ---- a.3: core numbers by min-degree peeling ------------------------------------
    ix.core.ensure(4 * (size_t)n);
    DevBuf dcur, rnd, F0, F1, ctr;
    dcur.ensure(4 * (size_t)n);
    rnd.ensure(4 * (size_t)n);
    F0.ensure(4 * (size_t)n);
    F1.ensure(4 * (size_t)n);
    ctr.ensure(16);
    k_peel_init<<<grid_for(n, BLK), BLK, 0, s>>>(ix.deg.as<int32_t>(), dcur.as<int32_t>(), rnd.as<int32_t>(), n);
    FOLTY_LAUNCHED();
    {
        int64_t remaining = n;
        int32_t k = 0, r = 0;
        int32_t *hc = hb.as<int32_t>();
        int32_t *F = F0.as<int32_t>(), *Nx = F1.as<int32_t>();
        while (remaining > 0) {
            int32_t init[4] = {0, 0x7fffffff, 0, 0};
            FOLTY_HIP(hipMemcpyAsync(ctr.p, init, 16, hipMemcpyHostToDevice, s));
            k_collect<<<grid_for(n, BLK), BLK, 0, s>>>(dcur.as<int32_t>(), rnd.as<int32_t>(), n, k, F,
                                                      ctr.as<int32_t>());
            FOLTY_LAUNCHED();
            FOLTY_HIP(hipMemcpyAsync(hc, ctr.p, 16, hipMemcpyDeviceToHost, s));
            FOLTY_HIP(hipStreamSynchronize(s));
            int32_t nF = hc[0];
            if (nF == 0) {
                // every live vertex has degree > k: the next level is the smallest live degree
                if (hc[1] == 0x7fffffff || hc[1] <= k)
                    fail(FOLTY_EDEVICE, "peeling lost track of %lld vertices", (long long)remaining);
                k = hc[1];
                continue;
            }
            while (nF > 0) {
                k_mark<<<grid_for(nF, BLK), BLK, 0, s>>>(F, nF, r, k, rnd.as<int32_t>(), ix.core.as<int32_t>());
                FOLTY_HIP(hipMemsetAsync(ctr.as<int32_t>() + 2, 0, 4, s));
                k_peel<<<grid_for((int64_t)nF * 64, BLK), BLK, 0, s>>>(F, nF, uoff.as<int64_t>(), uadj.as<int32_t>(),
                                                                       k, dcur.as<int32_t>(), rnd.as<int32_t>(),
                                                                       Nx, ctr.as<int32_t>());
                FOLTY_LAUNCHED();
                remaining -= nF;
                r++;
                std::swap(F, Nx);
                FOLTY_HIP(hipMemcpyAsync(hc + 2, ctr.as<int32_t>() + 2, 4, hipMemcpyDeviceToHost, s));
                FOLTY_HIP(hipStreamSynchronize(s));
                nF = hc[2];
            }
        }
        ix.peel_rounds = r;
    }
    dcur.release();
    F0.release();
    F1.release();

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
