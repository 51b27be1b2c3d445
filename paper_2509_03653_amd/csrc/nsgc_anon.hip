// Address anonymization on the device (Section IV, "IP Address
// Anonymization"): every address of the source and destination columns is
// replaced by a distinct integer in [0, N), N the number of unique addresses,
// through a seeded permutation of 0..N-1.
//
// The unique addresses are listed in ascending order and the i-th one maps to
// pi(i), where pi is a keyed pseudo-random permutation of [0, N): a
// four-round Feistel network on the smallest even bit count b with 2^b >=
// max(N, 4), round function F_r(R) = mix(seed ^ (r + 1) * 0x9E3779B97F4A7C15
// ^ R) on the low b/2 bits (mix = the SplitMix64 output function), restricted
// to [0, N) by cycle walking (Black and Rogaway, 2002).  A Feistel network is
// a bijection for any round function, so pi is one too.
//
// On the device, the paper's unique / shuffle / gather becomes one sort:
//   1. every column entry is packed as (address << 32 | position), positions
//      0..n-1 for sources and n..2n-1 for destinations;
//   2. a stable radix sort by the address half brings equal addresses
//      together, in ascending order;
//   3. run starts, scanned, number the unique addresses (the rank i);
//   4. each entry writes pi(rank) to its own position of the output columns.
#include <hip/hip_runtime.h>

#include "nsgc_anon.hpp"
#include "nsgc_device.hpp"
#include "nsgc_sort.hpp"

namespace nsgc {

namespace {

constexpr uint32_t AT = 256;

__global__ __launch_bounds__(AT) void k_an_pack(const uint32_t* __restrict__ src,
                                                const uint32_t* __restrict__ dst, u64 n,
                                                u64* __restrict__ v) {
  for (u64 i = u64(blockIdx.x) * AT + threadIdx.x; i < n; i += u64(gridDim.x) * AT) {
    v[i] = (u64(src[i]) << 32) | i;
    v[n + i] = (u64(dst[i]) << 32) | (n + i);
  }
}

// 1 where a new address starts in the sorted entries.
__global__ __launch_bounds__(AT) void k_an_flags(const u64* __restrict__ s, u64 m,
                                                 uint32_t* __restrict__ f) {
  for (u64 i = u64(blockIdx.x) * AT + threadIdx.x; i < m; i += u64(gridDim.x) * AT)
    f[i] = i == 0 || (s[i] >> 32) != (s[i - 1] >> 32);
}

__device__ __forceinline__ u64 sm_out(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The Feistel permutation of [0, 2^(2h)) for `seed`.
__device__ __forceinline__ u64 feistel_e(u64 x, uint32_t h, u64 seed) {
  const u64 mask = (u64(1) << h) - 1;
  u64 lo = x & mask, hi = x >> h;
#pragma unroll
  for (u64 r = 1; r <= 4; ++r) {
    const u64 t = hi ^ (sm_out(seed ^ (r * 0x9E3779B97F4A7C15ull) ^ lo) & mask);
    hi = lo;
    lo = t;
  }
  return (hi << h) | lo;
}

// Each entry: its address's rank among the unique ones (exclusive scan of the
// run starts, plus its own start flag, minus one), through the permutation,
// to its position in the output columns.
__global__ __launch_bounds__(AT) void k_an_map(const u64* __restrict__ s, u64 m, u64 n,
                                               const uint32_t* __restrict__ e,
                                               const uint32_t* __restrict__ total, u64 seed,
                                               uint32_t* __restrict__ asrc,
                                               uint32_t* __restrict__ adst,
                                               unsigned long long* __restrict__ num) {
  const u64 N = *total;
  uint32_t h = 1;                       // b = 2h: the smallest even b with 2^b >= max(N, 4)
  while ((u64(1) << (2 * h)) < N) ++h;
  for (u64 i = u64(blockIdx.x) * AT + threadIdx.x; i < m; i += u64(gridDim.x) * AT) {
    const u64 x = s[i];
    const bool start = i == 0 || (x >> 32) != (s[i - 1] >> 32);
    const u64 rank = u64(e[i]) + (start ? 1u : 0u) - 1u;
    u64 y = rank;
    if (N > 1) {
      y = feistel_e(rank, h, seed);
      while (y >= N) y = feistel_e(y, h, seed);
    }
    const u64 pos = x & 0xFFFFFFFFull;
    if (pos < n) asrc[pos] = uint32_t(y);
    else adst[pos - n] = uint32_t(y);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *num = N;
}

__global__ void k_an_zero(unsigned long long* num) {
  if (threadIdx.x == 0) *num = 0;
}

}  // namespace

size_t anonymize_bytes(u64 n) {
  const u64 m = 2 * n;
  const size_t words = size_t(m) + std::max(radix_sort_scratch_words(m), scan_scratch_words(m)) + 64;
  return size_t(m) * 16 + words * 4 + 1024;
}

hipError_t anonymize(const uint32_t* src, const uint32_t* dst, u64 n, u64 seed, uint32_t* asrc,
                     uint32_t* adst, unsigned long long* num, void* ws, uint32_t grid,
                     hipStream_t s) {
  if (n == 0) {
    hipLaunchKernelGGL(k_an_zero, dim3(1), dim3(64), 0, s, num);
    return hipGetLastError();
  }
  const u64 m = 2 * n;
  u64* V = static_cast<u64*>(ws);
  u64* T = V + m;
  uint32_t* E = reinterpret_cast<uint32_t*>(T + m);
  uint32_t* scratch = E + m;
  const uint32_t g = uint32_t(std::min<u64>((m + AT - 1) / AT, grid));
  hipLaunchKernelGGL(k_an_pack, dim3(g), dim3(AT), 0, s, src, dst, n, V);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  u64* S = nullptr;
  if ((e = radix_sort_u64(V, T, m, 32, 64, scratch, grid, s, &S)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_an_flags, dim3(g), dim3(AT), 0, s, S, m, E);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = exclusive_scan_u32(E, m, scratch, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_an_map, dim3(g), dim3(AT), 0, s, S, m, n, E, scan_total(scratch, m), seed,
                     asrc, adst, num);
  return hipGetLastError();
}

}  // namespace nsgc
