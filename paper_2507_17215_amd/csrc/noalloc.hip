// The single query for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// Every scratch buffer of the query (per-edge counts, survivors and their
// offsets, per-pair certificate counts, pair keys, sort and scan scratch) is
// carved from `scratch`, a fixed device array of FOLTY_NOALLOC_SCRATCH_BYTES
// that each device the library runs on holds until the process ends.  Its
// device address comes from hipGetSymbolAddress, once per device, with that
// device current; host code uses only that address, never the array's name.
// The outputs go to the caller's device memory.  Every call on a device
// shares that device's array and leaves its contents behind; each buffer is
// cleared by the call that uses it.  Calls on one device are serialised here,
// since two of them would use the same scratch at once.
#include <map>

#include "folty_internal.h"

namespace folty {

namespace {

static __device__ __align__(256) unsigned char scratch[FOLTY_NOALLOC_SCRATCH_BYTES];

// per device: the scratch's address, a workspace whose buffers are lent from
// it during a call, events and a small host buffer made at set-up
struct NoAllocDevice {
    void *ptr = nullptr;
    std::mutex mu;
    Workspace ws;
    alignas(64) char host[256];
};

std::mutex g_mu;
std::map<int, NoAllocDevice *> g_dev; // kept until the process ends

NoAllocDevice &device_state(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    NoAllocDevice *&d = g_dev[dev];
    if (!d) {
        std::unique_ptr<NoAllocDevice> n(new NoAllocDevice());
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(FOLTY_EDEVICE, "hipGetSymbolAddress of the fixed scratch failed on device %d: %s", dev,
                 hipGetErrorString(e));
        }
        n->ptr = p;
        n->ws.ensure_events();
        n->ws.host.lend(n->host, sizeof n->host);
        d = n.release();
    }
    return *d;
}

} // namespace

void run_query_noalloc(Graph *g, const folty_query &q, int32_t *pair_u, int32_t *pair_v, uint32_t *n_cert,
                       int64_t pair_cap, uint32_t *edge_count, int64_t *n_pairs, int64_t *n_certificates) {
    FOLTY_HIP(hipSetDevice(g->device));
    NoAllocDevice &d = device_state(g->device);
    std::lock_guard<std::mutex> lk(d.mu);
    // the workspace's buffers point into the scratch only while this call runs
    struct Forget {
        Workspace &ws;
        hipStream_t s;
        ~Forget() {
            (void)hipStreamSynchronize(s); // a failed call may still have work on the stream
            ws.forget_buffers();
        }
    } forget{d.ws, g->stream};
    d.ws.forget_buffers();
    StreamScope sc(g->stream);
    ArenaScope arena(d.ptr, FOLTY_NOALLOC_SCRATCH_BYTES);
    run_query_into(g, q, d.ws, pair_u, pair_v, n_cert, pair_cap, edge_count, n_pairs, n_certificates);
}

} // namespace folty
