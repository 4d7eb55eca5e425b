// Library primitives (radix sort, prefix scan), called from rocPRIM directly.
// Each wrapper returns the temporary storage it needs when tmp is null, and
// otherwise runs on `stream`.  Used for grouping edges, orienting the static
// graph and sorting the output pairs; the query's own kernels are in query.hip.
//
// Radix sorts use 9-bit digits with 1024-thread tiles of 8 keys each, and a
// digit-histogram pass of 512 threads x 32 keys per block (with 256 x 12 keys
// per block that pass takes as long as a whole scatter pass, about as many
// global atomics as keys / 1.2 landing on a few thousand counters).  Measured on gfx950,
// keys with 32-bit values, rocPRIM default -> this configuration:
//   70M keys of 45 bits 3.65 -> 3.04 ms;  26M keys of 44 bits 1.48 -> 1.22 ms;
//   26M keys of 22 bits 0.69 -> 0.55 ms;  4M keys of 32 bits 0.18 -> 0.17 ms.
// Histogram blocks of 256 x 12 keys: 3.36 / 1.32 / 0.69 / 0.19 ms.  8-bit
// digits were slower at every size, 10-bit digits much slower (4.90 ms for the
// 70M keys), and 11 or 12 bits exceed the LDS of one workgroup.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "folty_internal.h"

namespace folty {

#define FOLTY_PRIM(call)                                                                 \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            fail(FOLTY_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));                 \
    } while (0)

namespace {

using Onesweep = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<512, 32>, rocprim::kernel_config<1024, 8>, 9,
                                        rocprim::block_radix_rank_algorithm::match>>;

template <class Cfg, class K, class V>
size_t sort_with(void *tmp, size_t tmp_bytes, const K *kin, K *kout, const V *vin, V *vout, int64_t n, int end_bit,
                 hipStream_t s) {
    size_t need = 0;
    FOLTY_PRIM((rocprim::radix_sort_pairs<Cfg>(nullptr, need, kin, kout, vin, vout, (size_t)n, 0u,
                                               (unsigned)end_bit, s)));
    if (!tmp) return need;
    if (tmp_bytes < need) fail(FOLTY_EDEVICE, "sort scratch too small");
    FOLTY_PRIM((rocprim::radix_sort_pairs<Cfg>(tmp, need, kin, kout, vin, vout, (size_t)n, 0u, (unsigned)end_bit,
                                               s)));
    return need;
}

// stable ascending sort of (key, value) pairs on bits [0, end_bit) of the keys
template <class K, class V>
size_t sort_pairs(void *tmp, size_t tmp_bytes, const K *kin, K *kout, const V *vin, V *vout, int64_t n, int end_bit,
                  hipStream_t s) {
    if (end_bit < 1) end_bit = 1;
    if (end_bit > (int)(8 * sizeof(K))) end_bit = 8 * sizeof(K);
    return sort_with<Onesweep>(tmp, tmp_bytes, kin, kout, vin, vout, n, end_bit, s);
}

// Scans: 256-thread blocks with more items per thread than rocPRIM's default
// for this target.  Measured on gfx950 (default -> this): 70M int32 inclusive
// 0.236 -> 0.148 ms (64 items), 26M int32 inclusive 0.106 -> 0.061 ms (64),
// 26M int32 -> int64 exclusive 0.174 -> 0.098 ms (32; 64 items: 0.114 ms).
// The scan over pair starts read through a transform keeps the default.
template <unsigned ITEMS>
using ScanCfg = rocprim::scan_config<256, ITEMS, rocprim::block_load_method::block_load_transpose,
                                     rocprim::block_store_method::block_store_transpose,
                                     rocprim::block_scan_algorithm::reduce_then_scan>;
template <class Out> using ScanFor = ScanCfg<sizeof(Out) <= 4 ? 64 : 32>;

template <class In, class Out>
size_t scan_exclusive(void *tmp, size_t tb, const In *in, Out *out, int64_t n, hipStream_t s) {
    size_t need = 0;
    FOLTY_PRIM(rocprim::exclusive_scan<ScanFor<Out>>(nullptr, need, in, out, (Out)0, (size_t)n,
                                                     rocprim::plus<Out>(), s));
    if (!tmp) return need;
    FOLTY_PRIM(rocprim::exclusive_scan<ScanFor<Out>>(tmp, tb, in, out, (Out)0, (size_t)n, rocprim::plus<Out>(), s));
    return need;
}

} // namespace

size_t sort_pairs_u64_i32(void *tmp, size_t tb, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                          int32_t *vout, int64_t n, int end_bit, hipStream_t s) {
    return sort_pairs(tmp, tb, kin, kout, vin, vout, n, end_bit, s);
}
size_t sort_pairs_u64_u32(void *tmp, size_t tb, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                          uint32_t *vout, int64_t n, int end_bit, hipStream_t s) {
    return sort_pairs(tmp, tb, kin, kout, vin, vout, n, end_bit, s);
}
size_t sort_pairs_u32_i32(void *tmp, size_t tb, const uint32_t *kin, uint32_t *kout, const int32_t *vin,
                          int32_t *vout, int64_t n, int end_bit, hipStream_t s) {
    return sort_pairs(tmp, tb, kin, kout, vin, vout, n, end_bit, s);
}

size_t exclusive_scan_i64(void *tmp, size_t tb, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    return scan_exclusive(tmp, tb, in, out, n, s);
}

size_t exclusive_scan_i32_to_i64(void *tmp, size_t tb, const int32_t *in, int64_t *out, int64_t n,
                                 hipStream_t s) {
    return scan_exclusive(tmp, tb, in, out, n, s);
}

size_t exclusive_scan_i32(void *tmp, size_t tb, const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
    return scan_exclusive(tmp, tb, in, out, n, s);
}

namespace {
// 1 where a new (lo, hi) pair starts in the sorted grouping keys (key >> 1)
struct PairStart {
    const uint64_t *key;
    __device__ int32_t operator()(int64_t k) const { return k == 0 || (key[k] >> 1) != (key[k - 1] >> 1); }
};
} // namespace

// out[k] = 1 + the index of the static pair of sorted key k: an inclusive scan
// of pair starts computed from the keys as the scan reads them
size_t inclusive_scan_pair_starts(void *tmp, size_t tb, const uint64_t *key, int32_t *out, int64_t n,
                                  hipStream_t s) {
    // rocPRIM's default configuration: with 64 items per thread the key reads of
    // the transform slow it down (70M keys: 0.32 ms default, 0.40 ms with 64)
    auto in = rocprim::make_transform_iterator(rocprim::counting_iterator<int64_t>(0), PairStart{key});
    size_t need = 0;
    FOLTY_PRIM(rocprim::inclusive_scan(nullptr, need, in, out, (size_t)n, rocprim::plus<int32_t>(), s));
    if (!tmp) return need;
    FOLTY_PRIM(rocprim::inclusive_scan(tmp, tb, in, out, (size_t)n, rocprim::plus<int32_t>(), s));
    return need;
}

size_t inclusive_scan_i32(void *tmp, size_t tb, const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
    size_t need = 0;
    FOLTY_PRIM(rocprim::inclusive_scan<ScanFor<int32_t>>(nullptr, need, in, out, (size_t)n, rocprim::plus<int32_t>(),
                                                         s));
    if (!tmp) return need;
    FOLTY_PRIM(rocprim::inclusive_scan<ScanFor<int32_t>>(tmp, tb, in, out, (size_t)n, rocprim::plus<int32_t>(), s));
    return need;
}

} // namespace folty
