// Stable radix sorts (hipCUB / rocPRIM) used for the SMAD order (stable
// ascending (SMAD, index)) and for the final ranking of evaluated poses.
#include <hipcub/hipcub.hpp>

#include "reloc_internal.h"

namespace reloc {

hipError_t sort_pairs_u64_i32(void* tmp, size_t* tmp_bytes, const uint64_t* kin,
                              uint64_t* kout, const int32_t* vin, int32_t* vout, int n,
                              hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, kin, kout, vin, vout, n, 0, 64,
                                            s);
}

hipError_t sort_keys_u64(void* tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout,
                         int n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortKeys(tmp, *tmp_bytes, kin, kout, n, 0, 64, s);
}

hipError_t seg_sort_pairs_u64_i32(void* tmp, size_t* tmp_bytes, const uint64_t* kin,
                                  uint64_t* kout, const int32_t* vin, int32_t* vout, int64_t n,
                                  int nseg, const int64_t* offsets, hipStream_t s) {
  return hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, *tmp_bytes, kin, kout, vin, vout,
                                                     (int)n, nseg, offsets, offsets + 1, 0, 64,
                                                     s);
}

hipError_t seg_sort_keys_u64(void* tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout,
                             int64_t n, int nseg, const int64_t* offsets, hipStream_t s) {
  return hipcub::DeviceSegmentedRadixSort::SortKeys(tmp, *tmp_bytes, kin, kout, (int)n, nseg,
                                                    offsets, offsets + 1, 0, 64, s);
}

}  // namespace reloc
