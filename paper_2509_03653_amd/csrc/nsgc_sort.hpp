// Device-wide radix sort and scan (nsgc_sort.hip), host-side launchers.
#ifndef NSGC_SORT_HPP_
#define NSGC_SORT_HPP_

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstddef>

namespace nsgc {

typedef unsigned long long u64;

// u32 words of scratch an exclusive scan of n elements needs.
size_t scan_scratch_words(u64 n);
// u32 words of scratch radix_sort_u64 needs for n keys.
size_t radix_sort_scratch_words(u64 n);

// In-place exclusive prefix sum of a[0..n) (the total must fit 32 bits);
// bsum holds scan_scratch_words(n) words, and afterwards the total at
// scan_total(bsum, n) (for n > 0).
hipError_t exclusive_scan_u32(uint32_t* a, u64 n, uint32_t* bsum, hipStream_t s);
uint32_t* scan_total(uint32_t* bsum, u64 n);

// Stable sort of keys[0..n) by bits [lo, hi), ping-ponging with tmp (n keys);
// *sorted is set to the buffer that holds the result (keys or tmp).  scratch
// holds radix_sort_scratch_words(n) words; grid caps the workgroups of the
// tile kernels.  Asynchronous on s.
hipError_t radix_sort_u64(u64* keys, u64* tmp, u64 n, uint32_t lo, uint32_t hi, uint32_t* scratch,
                          uint32_t grid, hipStream_t s, u64** sorted);

}  // namespace nsgc

#endif  // NSGC_SORT_HPP_
