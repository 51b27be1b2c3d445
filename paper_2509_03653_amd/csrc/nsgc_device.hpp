// Device primitives for gfx950: hashing, wavefront reductions, block scans and
// LDS open-addressing tables.  Header-only, included by the kernel file.
#ifndef NSGC_DEVICE_HPP_
#define NSGC_DEVICE_HPP_

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsgc_plan.h"

namespace nsgc {

typedef unsigned long long u64;

// Empty-slot markers.  Every 64-bit key and every 32-bit address is a legal
// value, so the one key equal to a marker is counted outside the table.
constexpr u64 EMPTY64 = ~0ull;
constexpr uint32_t EMPTY32 = 0xFFFFFFFFu;
constexpr int WAVES = NSGC_BLOCK / 64;

// ---- hashing: invertible xorshift / odd-multiply mixers ------------------
// Bijections, so the bucket, sweep and slot bits taken from one mix of a key
// can always be refined until a group holds a single key.

__device__ __forceinline__ u64 link_hash(u64 x) {
  x ^= x >> 32;
  x *= 0x22781625FEAE7023ull;
  x ^= x >> 29;
  x *= 0xFDEAD8A9C227D53Dull;
  x ^= x >> 32;
  return x;
}

__device__ __forceinline__ uint32_t row_hash(uint32_t x) {
  x ^= 0x421E9A93u;
  x ^= x >> 16;
  x *= 0x897EA68Du;
  x ^= x >> 15;
  x *= 0x3EA9E261u;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint32_t col_hash(uint32_t x) {
  x ^= 0x3F4760C9u;
  x ^= x >> 16;
  x *= 0xE8F25BB3u;
  x ^= x >> 15;
  x *= 0xA84F7BAFu;
  x ^= x >> 16;
  return x;
}

// top k bits (k may be 0)
__device__ __forceinline__ uint32_t top64(u64 h, uint32_t k) {
  return k ? uint32_t(h >> (64 - k)) : 0u;
}
__device__ __forceinline__ uint32_t top32(uint32_t h, uint32_t k) {
  return k ? (h >> (32 - k)) : 0u;
}
// the `s` bits that follow the top `k` bits (s may be 0)
__device__ __forceinline__ uint32_t next64(u64 h, uint32_t k, uint32_t s) {
  return s ? uint32_t((h << k) >> (64 - s)) : 0u;
}
__device__ __forceinline__ uint32_t next32(uint32_t h, uint32_t k, uint32_t s) {
  return s ? ((h << k) >> (32 - s)) : 0u;
}

// ---- wavefront primitives -------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// DPP row shift right by N lanes within each row of 16; lanes shifted in from
// outside the row read 0 (bound_ctrl), the identity of sum and unsigned max.
template <int N>
__device__ __forceinline__ uint32_t dpp_row_shr(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x110 + N, 0xF, 0xF, true));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), lane));
}

// Sum over all 64 lanes (call with the whole wavefront active).  Row-local
// inclusive scan by DPP row shifts, then the four row totals by readlane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  v += dpp_row_shr<1>(v);
  v += dpp_row_shr<2>(v);
  v += dpp_row_shr<4>(v);
  v += dpp_row_shr<8>(v);
  return readlane(v, 15) + readlane(v, 31) + readlane(v, 47) + readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  v = max(v, dpp_row_shr<1>(v));
  v = max(v, dpp_row_shr<2>(v));
  v = max(v, dpp_row_shr<4>(v));
  v = max(v, dpp_row_shr<8>(v));
  return max(max(readlane(v, 15), readlane(v, 31)), max(readlane(v, 47), readlane(v, 63)));
}

// Inclusive prefix sum across the wavefront (lane-shuffle form; used for the
// small scans of bucket counters, not in per-packet loops).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const uint32_t t = __shfl_up(v, k, 64);
    if (lane >= uint32_t(k)) v += t;
  }
  return v;
}

// ---- block primitives -----------------------------------------------------

// Block-wide sum and max of per-thread values; every thread gets the result.
// `red` is LDS scratch of 2*WAVES words.
__device__ __forceinline__ void block_sum_max(uint32_t& sum, uint32_t& mx, uint32_t* red) {
  const uint32_t s = wave_sum(sum);
  const uint32_t m = wave_max(mx);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[w] = s;
    red[WAVES + w] = m;
  }
  __syncthreads();
  uint32_t ts = 0, tm = 0;
#pragma unroll
  for (int k = 0; k < WAVES; ++k) {
    ts += red[k];
    tm = max(tm, red[WAVES + k]);
  }
  __syncthreads();
  sum = ts;
  mx = tm;
}

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* red) {
  const uint32_t s = wave_sum(v);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 0) red[w] = s;
  __syncthreads();
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < WAVES; ++k) t += red[k];
  __syncthreads();
  return t;
}

// In-place exclusive scan of a[0..n) in LDS; a[n] receives the total, which is
// also returned to every thread.  `red` is LDS scratch of WAVES words.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t* a, uint32_t n, uint32_t* red) {
  const uint32_t per = (n + NSGC_BLOCK - 1) / NSGC_BLOCK;
  const uint32_t beg = min(n, threadIdx.x * per);
  const uint32_t end = min(n, beg + per);
  uint32_t s = 0;
  for (uint32_t i = beg; i < end; ++i) s += a[i];
  const uint32_t incl = wave_inclusive_scan(s);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 63) red[w] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < WAVES; ++k) {
    const uint32_t t = red[k];
    if (uint32_t(k) < w) before += t;
    total += t;
  }
  uint32_t run = before + incl - s;
  for (uint32_t i = beg; i < end; ++i) {
    const uint32_t x = a[i];
    a[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) a[n] = total;
  __syncthreads();
  return total;
}

// Largest i in [0, count) with pref[i] <= x (pref non-decreasing, pref[0] <= x).
__device__ __forceinline__ uint32_t owner_of(const uint32_t* pref, uint32_t count, uint32_t x) {
  uint32_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (pref[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---- LDS open-addressing tables (linear probing) --------------------------

// Find or insert key (!= EMPTY64).  Returns the slot, or -1 when the table is
// full.  `fresh` tells whether this call inserted the key.
__device__ __forceinline__ int lds_insert64(u64* tk, uint32_t mask, u64 key, uint32_t h,
                                            bool& fresh) {
  uint32_t slot = h & mask;
  for (uint32_t p = 0; p <= mask; ++p) {
    u64 cur = __hip_atomic_load(&tk[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == key) { fresh = false; return int(slot); }
    if (cur == EMPTY64) {
      u64 expected = EMPTY64;
      if (__hip_atomic_compare_exchange_strong(&tk[slot], &expected, key, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
        fresh = true;
        return int(slot);
      }
      if (expected == key) { fresh = false; return int(slot); }
    }
    slot = (slot + 1) & mask;
  }
  fresh = false;
  return -1;
}

__device__ __forceinline__ int lds_insert32(uint32_t* tk, uint32_t mask, uint32_t key,
                                            uint32_t h, bool& fresh) {
  uint32_t slot = h & mask;
  for (uint32_t p = 0; p <= mask; ++p) {
    uint32_t cur = __hip_atomic_load(&tk[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == key) { fresh = false; return int(slot); }
    if (cur == EMPTY32) {
      uint32_t expected = EMPTY32;
      if (__hip_atomic_compare_exchange_strong(&tk[slot], &expected, key, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
        fresh = true;
        return int(slot);
      }
      if (expected == key) { fresh = false; return int(slot); }
    }
    slot = (slot + 1) & mask;
  }
  fresh = false;
  return -1;
}

__device__ __forceinline__ uint32_t lds_add(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---- global combine of partial statistics ---------------------------------

__device__ __forceinline__ void stat_add(u64* out, u64 v) {
  if (v) atomicAdd(out, v);
}
__device__ __forceinline__ void stat_max(u64* out, u64 v) {
  if (v) atomicMax(out, v);
}

}  // namespace nsgc

#endif  // NSGC_DEVICE_HPP_
