// Address anonymization (nsgc_anon.hip), host-side launcher.
#ifndef NSGC_ANON_HPP_
#define NSGC_ANON_HPP_

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace nsgc {

// Workspace bytes anonymize needs for n packets (about 48 bytes per packet).
size_t anonymize_bytes(unsigned long long n);

// Anonymized columns of n packets (n < 2^31) into asrc / adst (device; may be
// src / dst themselves) and the number of unique addresses into *num
// (device).  ws holds anonymize_bytes(n) bytes; grid caps the workgroups of
// each pass.  Asynchronous on s.
hipError_t anonymize(const uint32_t* src, const uint32_t* dst, unsigned long long n,
                     unsigned long long seed, uint32_t* asrc, uint32_t* adst,
                     unsigned long long* num, void* ws, uint32_t grid, hipStream_t s);

}  // namespace nsgc

#endif  // NSGC_ANON_HPP_
