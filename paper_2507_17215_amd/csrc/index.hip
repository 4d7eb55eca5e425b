// Index build for the temporal graph (paper, Section "Main Ideas",
// Preliminaries, and the preamble of Section 3):
//   * group temporal edges into time-sorted lists E_{x,y} and static edges of G_S
//     (self-loops dropped; G_S has no directions or parallel edges);
//   * degrees |N(x)| and core numbers, and the rank (core, peel round within
//     the level, id) of level-synchronous min-degree peeling (the degeneracy
//     ordering the paper attributes to Matula and Beck; core.hip), which bounds
//     every out-degree by the degeneracy;
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

// VU edges per thread and step, each a coalesced load of its own, all in flight
// before any is used; the previous timestamp comes from the lane below.
constexpr int VU = 4;
__global__ void k_validate(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                           const int64_t *__restrict__ t, int64_t m, int32_t n, ValOut *out) {
    unsigned long long loops = 0, tmax = 0, desc = 0, bad = ~0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = lane_id();
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < m; i0 += VU * stride) {
        int32_t a[VU], b[VU];
        int64_t ti[VU], tp[VU];
#pragma unroll
        for (int u = 0; u < VU; u++) {
            const int64_t i = i0 + u * stride + lane;
            const bool in = i < m;
            a[u] = in ? src[i] : 0;
            b[u] = in ? dst[i] : 0;
            ti[u] = in ? t[i] : 0;
            tp[u] = (lane == 0 && in && i > 0) ? t[i - 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < VU; u++) {
            const int64_t i = i0 + u * stride + lane;
            const int64_t below = __shfl_up(ti[u], 1);
            if (i >= m) continue;
            const int64_t prev = lane == 0 ? tp[u] : below;
            const bool ok = a[u] >= 0 && a[u] < n && b[u] >= 0 && b[u] < n && ti[u] >= 0 &&
                            ti[u] < (int64_t(1) << 62);
            if (!ok) bad = (unsigned long long)i < bad ? (unsigned long long)i : bad;
            loops += (a[u] == b[u]);
            if (ok && (unsigned long long)ti[u] > tmax) tmax = (unsigned long long)ti[u];
            if (i > 0 && prev > ti[u]) desc++;
        }
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

// x / n and x % n for x < n^2 and 1 <= n < 2^31 (keys lo * n + hi), from a
// double-precision product with 1/n (inv_n, rounded once on the host) and one
// correction step: the estimate is within one of the quotient (below 2^31), in
// place of a software 64-bit division of about a hundred instructions.
__device__ inline void divmod_n(uint64_t x, uint64_t n, double inv_n, int32_t &q, int32_t &r) {
    int64_t qq = (int64_t)((double)x * inv_n);
    int64_t rr = (int64_t)(x - (uint64_t)qq * n);
    if (rr < 0) {
        qq--;
        rr += (int64_t)n;
    } else if (rr >= (int64_t)n) {
        qq++;
        rr -= (int64_t)n;
    }
    q = (int32_t)qq;
    r = (int32_t)rr;
}

__global__ void k_static_table(const uint64_t *__restrict__ key, int32_t *__restrict__ sid, int32_t m,
                               int64_t n, double inv_n, int32_t *__restrict__ soff, int32_t *__restrict__ smid,
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
        int32_t lo, hi;
        divmod_n(pk, (uint64_t)n, inv_n, lo, hi);
        slo[s] = lo;
        shi[s] = hi;
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

// The undirected adjacency from the static edge table, whose edges are sorted
// by (lo, hi): vertex v's row is its lower neighbours (edges with hi = v, in lo
// order) followed by its higher ones (edges with lo = v, in hi order), so both
// halves are already ascending.  hkey/hval: the table's (hi, lo) pairs stably
// sorted by hi.  With loff[v] = #edges with lo < v and hoff[v] = #edges with
// hi < v, row v starts at loff[v] + hoff[v].
// first position in a[lo, hi) holding a value >= x (hi if none)
__device__ inline int64_t lower_bound_i32(const int32_t *__restrict__ a, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One block per 256 consecutive vertices: four threads bound the block's
// positions in both key arrays, then each vertex searches only that range (the
// rows of 256 neighbouring vertices, a few cache lines shared by the block)
// instead of all S keys.
__global__ __launch_bounds__(BLK) void k_adj_rows(const int32_t *__restrict__ slo, const int32_t *__restrict__ hkey,
                                                  int32_t S, int32_t n, int32_t *__restrict__ loff,
                                                  int32_t *__restrict__ hoff, int64_t *__restrict__ uoff) {
    __shared__ int64_t s_b[4];
    const int64_t x0 = (int64_t)blockIdx.x * BLK;
    const int64_t x1 = x0 + BLK - 1 < n ? x0 + BLK - 1 : n; // last vertex of the block (n: the end)
    const int t = threadIdx.x;
    if (t < 4) {
        const int32_t *a = t < 2 ? slo : hkey;
        const int64_t xx = (t & 1) ? x1 + 1 : x0;
        s_b[t] = lower_bound_i32(a, 0, S, xx > n ? n : (int32_t)xx);
        if ((t & 1) && x1 + 1 > n) s_b[t] = S;
    }
    __syncthreads();
    const int64_t x = x0 + t;
    if (x > n) return;
    const int64_t a = lower_bound_i32(slo, s_b[0], s_b[1], (int32_t)x);
    const int64_t b = lower_bound_i32(hkey, s_b[2], s_b[3], (int32_t)x);
    loff[x] = (int32_t)a;
    hoff[x] = (int32_t)b;
    uoff[x] = a + b;
}

// edge s = (lo, hi) in lo's row: after lo's hoff[lo + 1] - hoff[lo] lower
// neighbours, at uoff[lo] + that + (s - loff[lo]) = hoff[lo + 1] + s
__global__ void k_adj_fill_up(const int32_t *__restrict__ slo, const int32_t *__restrict__ shi, int32_t S,
                              const int32_t *__restrict__ hoff, int32_t *__restrict__ uadj) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < S) uadj[(int64_t)hoff[slo[e] + 1] + e] = shi[e];
}

// sorted position q (hi = hkey[q], lo = hval[q]) in hi's row: at
// uoff[hi] + (q - hoff[hi]) = loff[hi] + q
__global__ void k_adj_fill_down(const int32_t *__restrict__ hkey, const int32_t *__restrict__ hval, int32_t S,
                                const int32_t *__restrict__ loff, int32_t *__restrict__ uadj) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < S) uadj[(int64_t)loff[hkey[q]] + q] = hval[q];
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

__global__ void k_orient_unpack(const uint64_t *__restrict__ key, int32_t S, int64_t n, double inv_n,
                                int32_t *__restrict__ oadj, int32_t *__restrict__ otail) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    int32_t tail, head;
    divmod_n(key[j], (uint64_t)n, inv_n, tail, head);
    oadj[j] = head;
    otail[j] = tail;
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
    if (mem_kind != FOLTY_MEM_HOST && mem_kind != FOLTY_MEM_DEVICE && mem_kind != FOLTY_MEM_DEVICE_BORROWED)
        fail(FOLTY_EINVAL, "bad mem_kind %d", mem_kind);
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
    if (mem_kind == FOLTY_MEM_DEVICE_BORROWED) {
        g->in_src = src;
        g->in_dst = dst;
        g->in_t = t;
    } else {
        g->src.ensure(sizeof(int32_t) * m);
        g->dst.ensure(sizeof(int32_t) * m);
        g->t.ensure(sizeof(int64_t) * m);
        hipMemcpyKind kind = mem_kind == FOLTY_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        if (m > 0) {
            FOLTY_HIP(hipMemcpyAsync(g->src.p, src, sizeof(int32_t) * m, kind, s));
            FOLTY_HIP(hipMemcpyAsync(g->dst.p, dst, sizeof(int32_t) * m, kind, s));
            FOLTY_HIP(hipMemcpyAsync(g->t.p, t, sizeof(int64_t) * m, kind, s));
        }
        g->in_src = g->src.as<int32_t>();
        g->in_dst = g->dst.as<int32_t>();
        g->in_t = g->t.as<int64_t>();
    }
    DevBuf vo;
    vo.ensure(sizeof(ValOut));
    k_init_val<<<1, 1, 0, s>>>(vo.as<ValOut>());
    FOLTY_LAUNCHED();
    if (m > 0) {
        // 1,024 blocks: the wavefronts' closing atomics on one cache line are
        // serialised (a few ns each), so a larger grid loses more there than it
        // gains in loads in flight (70M edges: 0.21 ms; 4,096 blocks 0.28 ms)
        k_validate<<<grid_for(m, BLK, 1024), BLK, 0, s>>>(g->in_src, g->in_dst, g->in_t, m, n, vo.as<ValOut>());
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
    if (g->ix.m_input > 0 && !g->in_src) fail(FOLTY_EINVAL, "graph inputs were released");
    if ((o.alloc == nullptr) != (o.free == nullptr)) fail(FOLTY_EINVAL, "alloc and free must both be set or both be null");
    Index &ix = g->ix;
    hipStream_t s = g->stream;
    // index memory from the caller's allocator when given (buffers of an earlier
    // build go back to wherever they came from)
    g->hook = AllocHook{o.alloc, o.free, o.alloc_ctx, s};
    HookScope hs(&g->hook);
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
        k_iota_tkeys<<<grid_for(min, BLK), BLK, 0, s>>>(g->in_t, tkeys.as<uint64_t>(),
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
        k_pair_keys<<<grid_for(min, BLK), BLK, 0, s>>>(idx_time, g->in_src, g->in_dst,
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
        k_gather_sorted<<<grid_for(m, BLK), BLK, 0, s>>>(pos2.as<int32_t>(), idx_time, g->in_t,
                                                         ix.perm.as<int32_t>(), ix.ts.as<int64_t>(), m);
        FOLTY_LAUNCHED();
    }
    idx_t.release();
    idx_t2.release();
    pos2.release();

    // ---- static edge table -----------------------------------------------------
    int32_t S = 0;
    if (m > 0) {
        // sid[k] = 1 + the static pair of sorted edge k (k_static_table makes it 0-based)
        size_t need = inclusive_scan_pair_starts(nullptr, 0, pkey2.as<uint64_t>(), ix.sid.as<int32_t>(), m, s);
        inclusive_scan_pair_starts(cub_ensure(need), need, pkey2.as<uint64_t>(), ix.sid.as<int32_t>(), m, s);
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
                                                        1.0 / (double)n, ix.soff.as<int32_t>(), ix.smid.as<int32_t>(),
                                                        ix.slo.as<int32_t>(), ix.shi.as<int32_t>());
        k_fix_smid_stats<<<grid_for(S, BLK, 2048), BLK, 0, s>>>(ix.soff.as<int32_t>(), ix.smid.as<int32_t>(), S,
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
        if (S > 0) {
            k_adj_fill_up<<<grid_for(S, BLK), BLK, 0, s>>>(ix.slo.as<int32_t>(), ix.shi.as<int32_t>(), S,
                                                           hoff.as<int32_t>(), uadj.as<int32_t>());
            k_adj_fill_down<<<grid_for(S, BLK), BLK, 0, s>>>(hkey.as<int32_t>(), hval.as<int32_t>(), S,
                                                             loff.as<int32_t>(), uadj.as<int32_t>());
            FOLTY_LAUNCHED();
        }
    }

    // ---- a.3: core numbers and the (core, round within the level) rank keys -------------
    ix.core.ensure(4 * (size_t)n);
    DevBuf rnd;
    rnd.ensure(4 * (size_t)n);
    CoreStats cst{};
    const int key_bits = core_rank_keys(n, uoff.as<int64_t>(), uadj.as<int32_t>(), ix.deg.as<int32_t>(),
                                        ix.core.as<int32_t>(), rnd.as<uint32_t>(), s, &cst);
    ix.peel_rounds = cst.rounds;
    ix.core_sweeps = cst.sweeps;
    uoff.release();
    uadj.release();

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
        int kb = o.rank_mode == FOLTY_RANK_DEGENERACY ? key_bits : 32;
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
            k_orient_unpack<<<grid_for(S, BLK), BLK, 0, s>>>(key2.as<uint64_t>(), S, n, 1.0 / (double)n,
                                                             ix.oadj.as<int32_t>(), ix.otail.as<int32_t>());
            FOLTY_LAUNCHED();
        }
        k_orient_rows<<<grid_for((int64_t)n + 1, BLK), BLK, 0, s>>>(key2.as<uint64_t>(), S, n, ix.ooff.as<int32_t>());
        FOLTY_LAUNCHED();
    }
    DevBuf ostat;
    ostat.ensure(sizeof(OrientStats));
    FOLTY_HIP(hipMemsetAsync(ostat.p, 0, sizeof(OrientStats), s));
    // 512 blocks: few per-vertex reads, and each block's closing atomics share
    // one cache line (4M vertices: 52 us; 2,048 blocks 86 us)
    k_orient_stats<<<grid_for(n, BLK, 512), BLK, 0, s>>>(ix.ooff.as<int32_t>(), ix.rank.as<int32_t>(),
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
