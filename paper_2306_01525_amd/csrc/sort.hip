// Library sort and scan used by the weight build (stable radix sort of the
// Hilbert keys, exclusive scan for CSR offsets). Kept in its own translation
// unit because the hipcub headers are slow to compile.
#include <hipcub/hipcub.hpp>

#include "common.h"

namespace mlbm {

// Temporary storage of the library calls (a failed size query gives 0: the
// call itself then reports the error).
size_t sort_pairs_temp_bytes(int n) {
    size_t bytes = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr,
                                           (uint32_t *)nullptr, (const int32_t *)nullptr,
                                           (int32_t *)nullptr, n, 0, 32,
                                           (hipStream_t)0) != hipSuccess)
        return 0;
    return bytes;
}

hipError_t sort_pairs(void *tmp, size_t tmp_bytes, const uint32_t *kin, uint32_t *kout,
                      const int32_t *vin, int32_t *vout, int n, int end_bit, hipStream_t s) {
    size_t bytes = tmp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, n, 0,
                                              end_bit, s);
}

size_t scan_temp_bytes(int n) {
    size_t bytes = 0;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int32_t *)nullptr,
                                         (int32_t *)nullptr, n, (hipStream_t)0) != hipSuccess)
        return 0;
    return bytes;
}

hipError_t exclusive_scan(void *tmp, size_t tmp_bytes, const int32_t *in, int32_t *out,
                          int n, hipStream_t s) {
    size_t bytes = tmp_bytes;
    return hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, n, s);
}

}  // namespace mlbm
