// Library primitives (radix sort, prefix scan) from rocPRIM through hipCUB.
// Each wrapper returns the temporary storage it needs when tmp is null, and
// otherwise runs on `stream`.  Used for grouping edges, orienting the static
// graph and sorting the output pairs; the query's own kernels are in query.hip.
#include <hipcub/hipcub.hpp>

#include "folty_internal.h"

namespace folty {

#define FOLTY_CUB(call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            fail(FOLTY_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));                 \
    } while (0)

template <class K, class V>
static size_t sort_pairs(void *tmp, size_t tmp_bytes, const K *kin, K *kout, const V *vin,
                         V *vout, int64_t n, int end_bit, hipStream_t s) {
    size_t need = 0;
    if (end_bit < 1) end_bit = 1;
    if (end_bit > (int)(8 * sizeof(K))) end_bit = 8 * sizeof(K);
    FOLTY_CUB(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kin, kout, vin, vout, (int)n, 0,
                                                 end_bit, s));
    if (!tmp) return need;
    if (tmp_bytes < need) fail(FOLTY_EDEVICE, "sort scratch too small");
    FOLTY_CUB(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, (int)n, 0,
                                                 end_bit, s));
    return need;
}

size_t sort_pairs_u64_i32(void *tmp, size_t tb, const uint64_t *kin, uint64_t *kout,
                          const int32_t *vin, int32_t *vout, int64_t n, int end_bit,
                          hipStream_t s) {
    return sort_pairs(tmp, tb, kin, kout, vin, vout, n, end_bit, s);
}
size_t sort_pairs_u64_u32(void *tmp, size_t tb, const uint64_t *kin, uint64_t *kout,
                          const uint32_t *vin, uint32_t *vout, int64_t n, int end_bit,
                          hipStream_t s) {
    return sort_pairs(tmp, tb, kin, kout, vin, vout, n, end_bit, s);
}
size_t sort_pairs_u32_i32(void *tmp, size_t tb, const uint32_t *kin, uint32_t *kout,
                          const int32_t *vin, int32_t *vout, int64_t n, int end_bit,
                          hipStream_t s) {
    return sort_pairs(tmp, tb, kin, kout, vin, vout, n, end_bit, s);
}

size_t exclusive_scan_i64(void *tmp, size_t tb, const int64_t *in, int64_t *out, int64_t n,
                          hipStream_t s) {
    size_t need = 0;
    FOLTY_CUB(hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, n, s));
    if (!tmp) return need;
    FOLTY_CUB(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, n, s));
    return need;
}

size_t exclusive_scan_i32_to_i64(void *tmp, size_t tb, const int32_t *in, int64_t *out, int64_t n,
                                 hipStream_t s) {
    size_t need = 0;
    FOLTY_CUB(hipcub::DeviceScan::ExclusiveScan(nullptr, need, in, out, hipcub::Sum(),
                                                (int64_t)0, n, s));
    if (!tmp) return need;
    FOLTY_CUB(hipcub::DeviceScan::ExclusiveScan(tmp, tb, in, out, hipcub::Sum(), (int64_t)0, n, s));
    return need;
}

size_t inclusive_scan_i32(void *tmp, size_t tb, const int32_t *in, int32_t *out, int64_t n,
                          hipStream_t s) {
    size_t need = 0;
    FOLTY_CUB(hipcub::DeviceScan::InclusiveSum(nullptr, need, in, out, n, s));
    if (!tmp) return need;
    FOLTY_CUB(hipcub::DeviceScan::InclusiveSum(tmp, tb, in, out, n, s));
    return need;
}

size_t exclusive_scan_i32(void *tmp, size_t tb, const int32_t *in, int32_t *out, int64_t n,
                          hipStream_t s) {
    size_t need = 0;
    FOLTY_CUB(hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, n, s));
    if (!tmp) return need;
    FOLTY_CUB(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, n, s));
    return need;
}

} // namespace folty
