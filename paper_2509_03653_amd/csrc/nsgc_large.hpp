// Large-window tier (nsgc_large.hip): the statistics of one window by
// sorting, for windows too large for one level of LDS hash partitioning.
#ifndef NSGC_LARGE_HPP_
#define NSGC_LARGE_HPP_

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace nsgc {

// Workspace bytes large_window_stats needs for a window of n packets
// (about 32 bytes per packet).
size_t large_window_bytes(unsigned long long n);

// The nine statistics of the window src[0..n), dst[0..n) into out[0..9)
// (device), using the device workspace ws of large_window_bytes(n) bytes.
// grid caps the workgroups of each pass.  Enqueued on s, with one wait for s
// part-way (the window's link count is read back to size the column sort).
hipError_t large_window_stats(const uint32_t* src, const uint32_t* dst, unsigned long long n,
                              void* ws, unsigned long long* out, uint32_t grid, hipStream_t s);

}  // namespace nsgc

#endif  // NSGC_LARGE_HPP_
