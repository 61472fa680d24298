// Device radix sort of the scheduler (epi_sort.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace epi {

constexpr int kSortChunk = 2048;  // keys per workgroup of one pass

// uint32 words of the digit-count buffer a sort of n keys needs.
int64_t radix_hist_words(int64_t n);

// Stable sort of n (< 2^32) pairs (k0[i], v0[i]) by the 8-bit key digits at
// bit offsets shifts[0..npass) (least significant digit first), ping-ponging
// with (k1, v1).  On return *in_second says whether the sorted pairs are in
// (k1, v1) (an odd number of passes) or back in (k0, v0).  Only launches on
// st: capturable.
hipError_t radix_sort(uint64_t *k0, int32_t *v0, uint64_t *k1, int32_t *v1, int64_t n, const int *shifts, int npass,
                      uint32_t *hist, hipStream_t st, bool *in_second);

}  // namespace epi
