// Device-wide stable LSD radix sort of 64-bit keys, and the exclusive scan it
// is built on.  Used where a window or a whole batch is too large for LDS
// hashing to aggregate in one partitioning level (the large-window tier and
// the address anonymization).
//
// One pass sorts by an 8-bit digit (the last may be narrower) in three
// steps over tiles of 4096 keys:
//   1. per-tile digit histograms, stored digit-major ([digit][tile]);
//   2. one exclusive scan of that array: the output position of each
//      (digit, tile) group, stable across tiles;
//   3. a scatter in which every wavefront ranks its 512 consecutive keys
//      (eight rounds of 64, in order) among equal digits with ballots, so the
//      order within a tile is kept too.
// Passes ping-pong between the key buffer and a second buffer of equal size.
#include <hip/hip_runtime.h>

#include "nsgc_device.hpp"
#include "nsgc_sort.hpp"

namespace nsgc {

namespace {

constexpr uint32_t RS_THREADS = 512;
constexpr uint32_t RS_PER = 8;                       // keys per thread
constexpr uint32_t RS_TILE = RS_THREADS * RS_PER;    // keys per tile
constexpr uint32_t RS_WAVES = RS_THREADS / 64;
constexpr uint32_t SCAN_TILE = RS_THREADS * RS_PER;  // elements per scan block

__device__ __forceinline__ uint32_t digit_of(u64 k, uint32_t shift, uint32_t mask) {
  return uint32_t(k >> shift) & mask;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const u64* __restrict__ keys, u64 n,
                                                        uint32_t shift, uint32_t bits,
                                                        uint32_t* __restrict__ counts, u64 ntiles) {
  __shared__ uint32_t hist[256];
  const uint32_t mask = (1u << bits) - 1u, nd = 1u << bits;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (uint32_t i = threadIdx.x; i < nd; i += RS_THREADS) hist[i] = 0;
    __syncthreads();
    const u64 base = tile * RS_TILE;
#pragma unroll
    for (uint32_t k = 0; k < RS_PER; ++k) {
      const u64 i = base + u64(k) * RS_THREADS + threadIdx.x;
      if (i < n) lds_add(&hist[digit_of(keys[i], shift, mask)], 1);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nd; d += RS_THREADS) counts[u64(d) * ntiles + tile] = hist[d];
    __syncthreads();
  }
}

// Scan, first level: the sum of every block of SCAN_TILE elements.
__global__ __launch_bounds__(RS_THREADS) void k_scan_reduce(const uint32_t* __restrict__ a, u64 n,
                                                            uint32_t* __restrict__ bsum) {
  __shared__ uint32_t red[RS_WAVES];
  const u64 base = u64(blockIdx.x) * SCAN_TILE;
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < RS_PER; ++k) {
    const u64 i = base + u64(k) * RS_THREADS + threadIdx.x;
    if (i < n) s += a[i];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

// Scan, second level: exclusive scan of the block sums in one workgroup.
__global__ __launch_bounds__(RS_THREADS) void k_scan_top(uint32_t* __restrict__ bsum, uint32_t nb) {
  __shared__ uint32_t red[RS_WAVES];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < nb; c0 += RS_THREADS) {
    const uint32_t i = c0 + threadIdx.x;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    const uint32_t incl = wave_inclusive_scan(v);
    const uint32_t w = threadIdx.x >> 6;
    if (lane_id() == 63) red[w] = incl;
    __syncthreads();
    uint32_t before = carry, total = 0;
    for (uint32_t k = 0; k < RS_WAVES; ++k) {
      if (k < w) before += red[k];
      total += red[k];
    }
    if (i < nb) bsum[i] = before + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;   // the grand total, after the block prefixes
}

// Scan, third level: each block's elements in place, offset by its block's
// exclusive prefix.  Thread t takes RS_PER consecutive elements.
__global__ __launch_bounds__(RS_THREADS) void k_scan_down(uint32_t* __restrict__ a, u64 n,
                                                          const uint32_t* __restrict__ bsum) {
  __shared__ uint32_t red[RS_WAVES];
  const u64 base = u64(blockIdx.x) * SCAN_TILE + u64(threadIdx.x) * RS_PER;
  uint32_t v[RS_PER];
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < RS_PER; ++k) {
    v[k] = base + k < n ? a[base + k] : 0u;
    s += v[k];
  }
  const uint32_t incl = wave_inclusive_scan(s);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 63) red[w] = incl;
  __syncthreads();
  uint32_t run = bsum[blockIdx.x] + incl - s;
  for (uint32_t k = 0; k < w; ++k) run += red[k];
#pragma unroll
  for (uint32_t k = 0; k < RS_PER; ++k) {
    if (base + k < n) a[base + k] = run;
    run += v[k];
  }
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const u64* __restrict__ in,
                                                           u64* __restrict__ out, u64 n,
                                                           uint32_t shift, uint32_t bits,
                                                           const uint32_t* __restrict__ offs,
                                                           u64 ntiles) {
  __shared__ uint32_t cnt[RS_WAVES][256];
  const uint32_t mask = (1u << bits) - 1u, nd = 1u << bits;
  const uint32_t w = threadIdx.x >> 6, lane = lane_id();
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (uint32_t i = lane; i < nd; i += 64) cnt[w][i] = 0;
    // wavefront w ranks keys [w * 512, w * 512 + 512) of the tile, 64 per round
    const u64 base = tile * RS_TILE + u64(w) * (RS_PER * 64);
    u64 key[RS_PER];
    uint32_t dg[RS_PER], rk[RS_PER];
#pragma unroll
    for (uint32_t r = 0; r < RS_PER; ++r) {
      const u64 i = base + u64(r) * 64 + lane;
      const bool ok = i < n;
      key[r] = ok ? in[i] : 0ull;
      dg[r] = digit_of(key[r], shift, mask);
      // lanes with the same digit: intersect the ballots of its bits
      u64 m = __ballot(ok);
      for (uint32_t b = 0; b < bits; ++b) {
        const u64 mb = __ballot((dg[r] >> b) & 1u);
        m &= ((dg[r] >> b) & 1u) ? mb : ~mb;
      }
      const uint32_t leader = ok ? uint32_t(__ffsll(static_cast<unsigned long long>(m)) - 1) : 0u;
      uint32_t old = 0;
      if (ok && lane == leader) old = lds_add(&cnt[w][dg[r]], uint32_t(__popcll(m)));
      old = lane_take(old, leader);
      rk[r] = old + rank_below(m);
    }
    __syncthreads();
    // digit totals of the waves before this one
    for (uint32_t d = threadIdx.x; d < nd; d += RS_THREADS) {
      uint32_t run = 0;
      for (uint32_t k = 0; k < RS_WAVES; ++k) {
        const uint32_t c = cnt[k][d];
        cnt[k][d] = run;
        run += c;
      }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < RS_PER; ++r) {
      const u64 i = base + u64(r) * 64 + lane;
      if (i < n) out[u64(offs[u64(dg[r]) * ntiles + tile]) + cnt[w][dg[r]] + rk[r]] = key[r];
    }
    __syncthreads();
  }
}

}  // namespace

size_t scan_scratch_words(u64 n) { return size_t((n + SCAN_TILE - 1) / SCAN_TILE) + 64; }

size_t radix_sort_scratch_words(u64 n) {
  const u64 ntiles = (n + RS_TILE - 1) / RS_TILE;
  const u64 m = 256 * ntiles;
  return size_t(m) + scan_scratch_words(m) + 64;
}

uint32_t* scan_total(uint32_t* bsum, u64 n) { return bsum + (n + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t exclusive_scan_u32(uint32_t* a, u64 n, uint32_t* bsum, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const u64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb > 0xFFFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_reduce, dim3(uint32_t(nb)), dim3(RS_THREADS), 0, s, a, n, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(RS_THREADS), 0, s, bsum, uint32_t(nb));
  hipLaunchKernelGGL(k_scan_down, dim3(uint32_t(nb)), dim3(RS_THREADS), 0, s, a, n, bsum);
  return hipGetLastError();
}

hipError_t radix_sort_u64(u64* keys, u64* tmp, u64 n, uint32_t lo, uint32_t hi, uint32_t* scratch,
                          uint32_t grid, hipStream_t s, u64** sorted) {
  *sorted = keys;
  if (n <= 1 || hi <= lo) return hipSuccess;
  const u64 ntiles = (n + RS_TILE - 1) / RS_TILE;
  uint32_t* counts = scratch;
  uint32_t* bsum = scratch + 256 * ntiles;
  const uint32_t g = uint32_t(std::min<u64>(ntiles, grid));
  u64* a = keys;
  u64* b = tmp;
  for (uint32_t shift = lo; shift < hi; shift += 8) {
    const uint32_t bits = std::min(8u, hi - shift);
    hipLaunchKernelGGL(k_rs_hist, dim3(g), dim3(RS_THREADS), 0, s, a, n, shift, bits, counts,
                       ntiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // only the first (1 << bits) digit rows are used
    if ((e = exclusive_scan_u32(counts, u64(1u << bits) * ntiles, bsum, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3(g), dim3(RS_THREADS), 0, s, a, b, n, shift, bits, counts,
                       ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    u64* t = a;
    a = b;
    b = t;
  }
  *sorted = a;
  return hipSuccess;
}

}  // namespace nsgc
