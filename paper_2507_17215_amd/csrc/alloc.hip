// Caching device allocator for the library's own buffers.
//
// hipMalloc and hipFree are slow and hipFree waits for the whole device, which
// leaves the GPU idle between the many buffers of an index build.  Freed blocks
// are kept per device and handed out again.  A block freed while a stream may
// still use it carries an event recorded on that stream; a reuse on another
// stream waits for that event first, a reuse on the same stream is ordered by
// the stream itself.  Every public call synchronises its stream before it
// returns, so blocks freed outside any call are idle.
#include <map>
#include <mutex>

#include "folty_internal.h"

namespace folty {

namespace {

struct Block {
    void *p;
    size_t bytes;
    hipStream_t stream; // stream that last used it (nullptr: idle)
    hipEvent_t ev;      // recorded on `stream` when freed (nullptr: idle)
};

struct Pool {
    std::mutex mu;
    std::multimap<size_t, Block> free_blocks;
    size_t cached = 0;
};

std::mutex g_pools_mu;
std::map<int, Pool *> g_pools;

thread_local hipStream_t t_stream = nullptr;
thread_local ArenaScope *t_arena = nullptr;
thread_local const AllocHook *t_hook = nullptr;

Pool &pool_for(int dev) {
    std::lock_guard<std::mutex> lk(g_pools_mu);
    Pool *&p = g_pools[dev];
    if (!p) p = new Pool(); // kept until the process ends
    return *p;
}

size_t round_size(size_t b) {
    if (b < 256) return 256;
    if (b < (1u << 20)) return (b + 255) & ~size_t(255);
    const size_t g = size_t(2) << 20;
    return (b + g - 1) / g * g;
}

void drop_block(Block &b) {
    if (b.ev) (void)hipEventDestroy(b.ev);
    (void)hipFree(b.p);
}

} // namespace

StreamScope::StreamScope(hipStream_t s) : prev(t_stream) { t_stream = s; }
StreamScope::~StreamScope() { t_stream = prev; }

HookScope::HookScope(const AllocHook *h) : prev(t_hook) { t_hook = h && h->set() ? h : nullptr; }
HookScope::~HookScope() { t_hook = prev; }
// an arena on the thread takes precedence over any caller's allocator
const AllocHook *current_hook() { return t_arena ? nullptr : t_hook; }

ArenaScope::ArenaScope(void *b, size_t c) : base(static_cast<char *>(b)), cap(c), prev(t_arena) { t_arena = this; }
ArenaScope::~ArenaScope() { t_arena = prev; }

void *dev_alloc(size_t bytes, size_t *got) {
    if (ArenaScope *a = t_arena) {
        const size_t want = (bytes + 255) & ~size_t(255);
        if (a->off + want > a->cap)
            fail(FOLTY_ENOMEM, "this call needs more than the %zu bytes of its fixed device scratch (%zu in use, "
                 "%zu more asked for)", a->cap, a->off, want);
        void *p = a->base + a->off;
        a->off += want;
        *got = want;
        return p;
    }
    int dev = 0;
    FOLTY_HIP(hipGetDevice(&dev));
    Pool &P = pool_for(dev);
    const size_t want = round_size(bytes);
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.free_blocks.lower_bound(want);
        if (it != P.free_blocks.end() && it->first <= 2 * want) {
            Block b = it->second;
            P.free_blocks.erase(it);
            P.cached -= b.bytes;
            if (b.ev) {
                // the block's last use must be done before the new owner's work
                // (the same stream orders it by itself)
                hipError_t e = hipSuccess;
                if (!t_stream) e = hipEventSynchronize(b.ev);
                else if (b.stream != t_stream) e = hipStreamWaitEvent(t_stream, b.ev, 0);
                if (e != hipSuccess) {
                    // no wait could be set up: wait for the whole device, and keep
                    // the failed call's error from being reported by a later check
                    (void)hipGetLastError();
                    (void)hipDeviceSynchronize();
                    (void)hipGetLastError();
                }
                (void)hipEventDestroy(b.ev);
            }
            *got = b.bytes;
            return b.p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        // give the cached blocks back and try once more
        (void)hipDeviceSynchronize();
        std::lock_guard<std::mutex> lk(P.mu);
        for (auto &kv : P.free_blocks) drop_block(kv.second);
        P.free_blocks.clear();
        P.cached = 0;
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(FOLTY_ENOMEM, "hipMalloc of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    *got = want;
    return p;
}

void dev_free(void *p, size_t bytes) {
    if (!p) return;
    for (ArenaScope *a = t_arena; a; a = a->prev)
        if (static_cast<char *>(p) >= a->base && static_cast<char *>(p) < a->base + a->cap) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipFree(p);
        return;
    }
    Block b{p, bytes, t_stream, nullptr};
    if (t_stream) {
        if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(b.ev, t_stream) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(t_stream);
            if (b.ev) (void)hipEventDestroy(b.ev);
            b.ev = nullptr;
        }
    }
    Pool &P = pool_for(dev);
    std::lock_guard<std::mutex> lk(P.mu);
    P.free_blocks.emplace(bytes, b);
    P.cached += bytes;
}

// A stream is about to be destroyed: the cached blocks whose last use was on it
// wait for that use now and drop its event, so no later owner waits on an event
// of a destroyed stream.
void dev_forget_stream(hipStream_t s) {
    if (!s) return;
    std::lock_guard<std::mutex> lk(g_pools_mu);
    for (auto &kv : g_pools) {
        Pool &P = *kv.second;
        std::lock_guard<std::mutex> lp(P.mu);
        for (auto &fb : P.free_blocks) {
            Block &b = fb.second;
            if (b.stream != s || !b.ev) continue;
            (void)hipEventSynchronize(b.ev);
            (void)hipEventDestroy(b.ev);
            b.ev = nullptr;
            b.stream = nullptr;
        }
    }
    (void)hipGetLastError();
}

size_t dev_trim() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Pool &P = pool_for(dev);
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lk(P.mu);
    size_t n = P.cached;
    for (auto &kv : P.free_blocks) drop_block(kv.second);
    P.free_blocks.clear();
    P.cached = 0;
    return n;
}

size_t dev_trim_to(size_t keep) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Pool &P = pool_for(dev);
    std::lock_guard<std::mutex> lk(P.mu);
    size_t n = 0;
    while (P.cached > keep && !P.free_blocks.empty()) {
        auto it = std::prev(P.free_blocks.end());
        Block b = it->second;
        P.free_blocks.erase(it);
        P.cached -= b.bytes;
        n += b.bytes;
        if (b.ev) (void)hipEventSynchronize(b.ev); // the last stream that used it is done with it
        drop_block(b);
    }
    return n;
}

// ---------------------------------------------------------------------------
// Pinned host blocks for large result arrays.  Results are filled by device
// copies: into pinned memory they run as a DMA at full speed, and a block taken
// from the cache has its pages mapped already (a fresh pageable array is copied
// through a staging buffer and faults on every page).  Released blocks are kept,
// up to HOST_CACHE_CAP bytes, for the next result.
// ---------------------------------------------------------------------------
namespace {

struct HostPool {
    std::mutex mu;
    std::multimap<size_t, void *> free_blocks;
    std::map<void *, size_t> live; // block -> its size, for every block handed out
    size_t cached = 0;
};

HostPool &host_pool() {
    static HostPool *p = new HostPool(); // kept until the process ends
    return *p;
}

constexpr size_t HOST_CACHE_CAP = size_t(4) << 30;

size_t host_round(size_t b) {
    const size_t g = size_t(2) << 20;
    return (b + g - 1) / g * g;
}

} // namespace

void *host_alloc(size_t bytes) {
    HostPool &P = host_pool();
    const size_t want = host_round(bytes);
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.free_blocks.lower_bound(want);
    if (it != P.free_blocks.end() && it->first <= 2 * want) {
        void *p = it->second;
        P.live[p] = it->first;
        P.cached -= it->first;
        P.free_blocks.erase(it);
        return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocPortable) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr; // the caller falls back to pageable memory
    }
    P.live[p] = want;
    return p;
}

bool host_free(void *p) {
    HostPool &P = host_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return false;
    const size_t b = it->second;
    P.live.erase(it);
    if (P.cached + b > HOST_CACHE_CAP) {
        (void)hipHostFree(p);
    } else {
        P.free_blocks.emplace(b, p);
        P.cached += b;
    }
    return true;
}

size_t host_trim() {
    HostPool &P = host_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    size_t n = P.cached;
    for (auto &kv : P.free_blocks) (void)hipHostFree(kv.second);
    P.free_blocks.clear();
    P.cached = 0;
    return n;
}

size_t dev_cached() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    Pool &P = pool_for(dev);
    std::lock_guard<std::mutex> lk(P.mu);
    return P.cached;
}

} // namespace folty
