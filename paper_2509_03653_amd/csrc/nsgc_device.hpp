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

// ---- global-memory pointers ------------------------------------------------
// Pointers read out of the plan are generic to the compiler; generic (flat)
// loads count against the LDS wait counter too, so an LDS wait would also
// wait for every global load in flight.  Casting them to the global address
// space keeps global loads and LDS operations on separate counters.
#define NSGC_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ NSGC_GLOBAL T* gptr(T* p) {
  return (NSGC_GLOBAL T*)(p);
}

// Load a descriptor struct (size a multiple of 8) from global memory.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  static_assert(sizeof(T) % 8 == 0, "descriptor size must be a multiple of 8");
  const NSGC_GLOBAL u64* q = (const NSGC_GLOBAL u64*)(p);
  u64 tmp[sizeof(T) / 8];
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 8; ++i) tmp[i] = q[i];
  T out;
  __builtin_memcpy(&out, tmp, sizeof(T));
  return out;
}

typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

// Load through the scalar data cache: for plan data that no kernel writes
// while it runs, read at a wave-uniform address.  These loads count against
// the LDS/scalar wait counter, not the vector memory one, so they do not wait
// for the wave's outstanding global stores.
template <class T>
__device__ __forceinline__ T sload(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

// A window descriptor read as sixteen 32-bit words through sload (the scalar
// cache has no byte loads).
template <class T>
__device__ __forceinline__ T sload_words(const T* p) {
  static_assert(sizeof(T) % 16 == 0, "descriptor size must be a multiple of 16");
  constexpr int N = int(sizeof(T) / 16);
  const __attribute__((address_space(4))) v4u32* q = (const __attribute__((address_space(4))) v4u32*)(p);
  v4u32 raw[N];
#pragma unroll
  for (int i = 0; i < N; ++i) raw[i] = q[i];
  T out;
  __builtin_memcpy(&out, raw, sizeof(T));
  return out;
}

// ---- hashing: invertible xorshift / odd-multiply mixers ------------------
// row_hash and col_hash are bijections on 32 bits.  Every kernel works on
// addresses in this hashed form: a source s is represented by row_hash(s), a
// destination d by col_hash(d), and a link (s, d) by the 64-bit key
// row_hash(s) << 32 | col_hash(d).  Equality is preserved both ways, so
// counting distinct hashed values counts distinct addresses or links, and the
// values are already mixed: bucket, sweep and slot bits are read off them
// without hashing again in the later phases.

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

// Inverse of an odd multiplier modulo 2^32 (Newton's iteration doubles the
// correct low bits each step: 3 -> 6 -> 12 -> 24 -> 48).
constexpr uint32_t odd_inverse(uint32_t m) {
  uint32_t x = m;   // correct to 3 bits for odd m
  for (int i = 0; i < 4; ++i) x *= 2u - m * x;
  return x;
}
static_assert(0x897EA68Du * odd_inverse(0x897EA68Du) == 1u, "multiplier inverse");
static_assert(0x3EA9E261u * odd_inverse(0x3EA9E261u) == 1u, "multiplier inverse");

// row_hash^-1: the steps of row_hash undone in reverse order (x ^= x >> 16
// is its own inverse on 32 bits; x ^= x >> 15 is undone by x ^= x >> 15 ^ x >> 30).
__device__ __forceinline__ uint32_t row_unhash(uint32_t x) {
  x ^= x >> 16;
  x *= odd_inverse(0x3EA9E261u);
  x ^= (x >> 15) ^ (x >> 30);
  x *= odd_inverse(0x897EA68Du);
  x ^= x >> 16;
  x ^= 0x421E9A93u;
  return x;
}

__device__ __forceinline__ uint32_t rotl32(uint32_t x, uint32_t r) {
  return (x << r) | (x >> (32u - r));
}

// The hashed link key of packet (s, d).  With `same` (the entity outputs,
// which need sources and destinations in one hashed space to count their
// union) the destination is hashed like a source.
__device__ __forceinline__ u64 link_key(uint32_t s, uint32_t d, bool same = false) {
  return (u64(row_hash(s)) << 32) | (same ? row_hash(d) : col_hash(d));
}

// Position bits of a hashed link key (r, c): the link bucket is the top bits,
// the overflow sweeps take the bits that follow, and the low bits pick the
// LDS table slot.  hi = r ^ rotl(c, 13), lo = c ^ hi, a bijection of (r, c).
// Both halves of the key are already mixed, so the rotation is enough to make
// every bit depend on source and destination, and the bits are placed so that
// the slot stays uniform inside one bucket for the links of one source and for
// those of one destination: with the top j bits of hi fixed, a fixed c fixes
// r's top j bits while slot bit i < 13 still gets r's bit i (j <= 19), and a
// fixed r fixes c's bits 19 - j .. 18 while slot bit i still gets c's bit
// i + 19.  (A slot taken from bits of r that the bucket fixes would put all
// the links of a popular destination in a few probe chains.)
__device__ __forceinline__ u64 link_pos(u64 k) {
  const uint32_t r = uint32_t(k >> 32), c = uint32_t(k);
  const uint32_t hi = r ^ rotl32(c, 13);
  return (u64(hi) << 32) | (c ^ hi);
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

// The value of `v` held by lane `src` (a per-lane index 0..63), by ds_bpermute.
__device__ __forceinline__ uint32_t lane_take(uint32_t v, uint32_t src) {
  return static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(static_cast<int>(src << 2),
                                                            static_cast<int>(v)));
}

// Set bits of `m` below the calling lane.
__device__ __forceinline__ uint32_t rank_below(u64 m) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

// Append the lanes with `want` to a list whose length is the LDS word *len:
// one atomic per wavefront instead of one per lane (LDS atomics on a single
// address are processed one lane at a time), each lane gets base + rank.
// Call with the whole wavefront active; the result is defined where `want`.
__device__ __forceinline__ uint32_t wave_append(uint32_t* len, bool want) {
  const u64 m = __ballot(want);
  if (m == 0) return 0;
  const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
  uint32_t base = 0;
  if (int(lane_id()) == leader)
    base = __hip_atomic_fetch_add(len, uint32_t(__popcll(m)), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
  return readlane(base, leader) + rank_below(m);
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

// Inclusive prefix sum across the wavefront (call with the whole wavefront
// active): the row-local inclusive scan by DPP row shifts, plus the totals of
// the rows below, read with readlane.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  v += dpp_row_shr<1>(v);
  v += dpp_row_shr<2>(v);
  v += dpp_row_shr<4>(v);
  v += dpp_row_shr<8>(v);
  const uint32_t r0 = readlane(v, 15), r1 = readlane(v, 31), r2 = readlane(v, 47);
  const uint32_t row = lane_id() >> 4;
  return v + (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
}

// The same by lane shuffles (LDS permutes): in the partition's 1024-thread
// bucket scan this form measured 4 us per launch faster than the DPP form.
__device__ __forceinline__ uint32_t wave_inclusive_scan_shfl(uint32_t v) {
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

// Sums of a and b and the max of m over the block, valid in thread 0 only
// (one barrier).  `red` (3*WAVES words) must not be reused before the block
// has passed another barrier.
__device__ __forceinline__ void block_sum2_max_to0(uint32_t& a, uint32_t& b, uint32_t& m,
                                                   uint32_t* red) {
  const uint32_t sa = wave_sum(a), sb = wave_sum(b), sm = wave_max(m);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[w] = sa;
    red[WAVES + w] = sb;
    red[2 * WAVES + w] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ta = 0, tb = 0, tm = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
      ta += red[k];
      tb += red[WAVES + k];
      tm = max(tm, red[2 * WAVES + k]);
    }
    a = ta;
    b = tb;
    m = tm;
  }
}

// The sum of s and the maxima of m1 and m2 over the block, valid in thread 0
// only (one barrier; same reuse rule for `red` as above).
__device__ __forceinline__ void block_sum_max2_to0(uint32_t& s, uint32_t& m1, uint32_t& m2,
                                                   uint32_t* red) {
  const uint32_t ss = wave_sum(s), s1 = wave_max(m1), s2 = wave_max(m2);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[w] = ss;
    red[WAVES + w] = s1;
    red[2 * WAVES + w] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ts = 0, t1 = 0, t2 = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
      ts += red[k];
      t1 = max(t1, red[WAVES + k]);
      t2 = max(t2, red[2 * WAVES + k]);
    }
    s = ts;
    m1 = t1;
    m2 = t2;
  }
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

// Two independent in-place exclusive scans, of a[0..na) and b[0..nb), with
// one pair of barriers (one barrier when both fit one wavefront); a[na] and
// b[nb] receive the totals.  `red` is LDS
// scratch of 2*WAVES words.
__device__ __forceinline__ void block_exclusive_scan2(uint32_t* a, uint32_t na, uint32_t* b,
                                                      uint32_t nb, uint32_t* red) {
  if (na <= 64 && nb <= 64) {   // one wavefront, one barrier
    if (threadIdx.x < 64) {
      const uint32_t l = threadIdx.x;
      const uint32_t x = l < na ? a[l] : 0u, y = l < nb ? b[l] : 0u;
      const uint32_t ix = wave_inclusive_scan(x), iy = wave_inclusive_scan(y);
      if (l < na) a[l] = ix - x;
      if (l < nb) b[l] = iy - y;
      if (l == 63) {   // lanes at and above na (nb) add nothing: the totals
        a[na] = ix;
        b[nb] = iy;
      }
    }
    __syncthreads();
    return;
  }
  const uint32_t pa = (na + NSGC_BLOCK - 1) / NSGC_BLOCK, pb = (nb + NSGC_BLOCK - 1) / NSGC_BLOCK;
  const uint32_t a0 = min(na, threadIdx.x * pa), a1 = min(na, a0 + pa);
  const uint32_t b0 = min(nb, threadIdx.x * pb), b1 = min(nb, b0 + pb);
  uint32_t sa = 0, sb = 0;
  for (uint32_t i = a0; i < a1; ++i) sa += a[i];
  for (uint32_t i = b0; i < b1; ++i) sb += b[i];
  const uint32_t ia = wave_inclusive_scan(sa), ib = wave_inclusive_scan(sb);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 63) {
    red[w] = ia;
    red[WAVES + w] = ib;
  }
  __syncthreads();
  uint32_t ba = 0, ta = 0, bb = 0, tb = 0;
#pragma unroll
  for (int k = 0; k < WAVES; ++k) {
    const uint32_t x = red[k], y = red[WAVES + k];
    if (uint32_t(k) < w) {
      ba += x;
      bb += y;
    }
    ta += x;
    tb += y;
  }
  uint32_t run = ba + ia - sa;
  for (uint32_t i = a0; i < a1; ++i) {
    const uint32_t x = a[i];
    a[i] = run;
    run += x;
  }
  run = bb + ib - sb;
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t x = b[i];
    b[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) {
    a[na] = ta;
    b[nb] = tb;
  }
  __syncthreads();
}

// In-place exclusive scan of a[0..n) in LDS; a[n] receives the total, which is
// also returned to every thread (of an NT-thread block).  `red` is LDS
// scratch of NT / 64 words.
template <uint32_t NT = NSGC_BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t* a, uint32_t n, uint32_t* red) {
  constexpr int NW = int(NT / 64);
  const uint32_t per = (n + NT - 1) / NT;
  const uint32_t beg = min(n, threadIdx.x * per);
  const uint32_t end = min(n, beg + per);
  uint32_t s = 0;
  for (uint32_t i = beg; i < end; ++i) s += a[i];
  const uint32_t incl = wave_inclusive_scan_shfl(s);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 63) red[w] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
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

// Largest i in [0, count) with pref[i] <= x, for a non-decreasing array in
// global memory with pref[0] <= x: a 64-ary search in which every lane of the
// wavefront tests one probe per round (one memory round trip per 64x
// narrowing).  Every wavefront computes the same result.
__device__ __forceinline__ uint32_t owner_of_wave(const NSGC_GLOBAL uint32_t* pref, uint32_t count,
                                                  uint32_t x) {
  uint32_t lo = 0, n = count;
  const uint32_t lane = lane_id();
  while (n > 1) {
    const uint32_t step = (n + 63) >> 6;
    const uint32_t at = lane * step;
    const bool ok = at < n && pref[lo + at] <= x;
    const u64 m = __ballot(ok);
    const uint32_t k = 63u - uint32_t(__clzll(static_cast<long long>(m)));
    lo += k * step;
    n = min(step, n - k * step);
  }
  return lo;
}

// End marker of the work queues (no item has this index).
constexpr uint32_t NO_ITEM = 0xFFFFFFFFu;

// Dynamic work queue, so that uneven items (heavy buckets, windows of very
// different sizes) spread over the grid.  Device-scope atomics on one
// address are serialised (tens of ns each), which a queue of thousands of
// items per launch would pay on every item, so: workgroup b takes item b
// first without any atomic, and the remaining items are dealt round-robin
// over K = min(classes, grid) classes (classes <= NSGC_QCLASSES), each with
// its own counter on its own cache line; workgroup b takes the items of
// class b mod K (every class has workgroups).  The next item is requested while the current one
// is processed.
//
// Queue positions map to items through `map` (a permutation of the items;
// null for the identity).  A kernel that maps may call resolve() part-way
// through an item, so that the next item's map entry is loaded while the
// current item finishes instead of when the next one starts.
//
// Loop shape (one barrier per item for the queue, shared with the item's
// last one; the item body must contain a barrier before stage_next):
//   for (item = q.first(items); item != NO_ITEM; item = q.read()) {
//     ...;  q.stage_next(items);  __syncthreads();
//   }
struct ItemQueue {
  NSGC_GLOBAL uint32_t* counter;  // this workgroup's class counter
  uint32_t* slot;                 // LDS word that broadcasts the item to the workgroup
  const NSGC_GLOBAL uint32_t* map;
  uint32_t base, step;            // dynamic positions of the class: base + step * ticket
  uint32_t pending;               // thread 0: prefetched next position
  uint32_t pending_item;          // thread 0: its item, once resolved
  bool resolved;

  __device__ ItemQueue(NSGC_GLOBAL uint32_t* counters, uint32_t* lds_slot, uint32_t classes,
                       const NSGC_GLOBAL uint32_t* item_map = nullptr)
      : slot(lds_slot), map(item_map), pending(0), pending_item(0), resolved(false) {
    step = min(min(classes, uint32_t(NSGC_QCLASSES)), gridDim.x);
    const uint32_t c = blockIdx.x % step;
    counter = counters + c * NSGC_QSTRIDE;
    base = gridDim.x + c;          // after the grid's static first positions
  }

  __device__ __forceinline__ uint32_t take() {
    const uint32_t t =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return base + step * t;
  }
  // The item at queue position pos, or NO_ITEM past the end (a mapped item
  // index may exceed the number of positions, so `items` cannot be the end).
  __device__ __forceinline__ uint32_t item_at(uint32_t pos, uint32_t items) const {
    return pos < items ? (map ? map[pos] : pos) : NO_ITEM;
  }
  __device__ __forceinline__ uint32_t first(uint32_t items) {
    if (threadIdx.x == 0) {
      const uint32_t v = blockIdx.x;
      slot[0] = item_at(v, items);
      pending = v < items ? take() : items;
      resolved = false;
    }
    __syncthreads();
    return slot[0];
  }
  __device__ __forceinline__ void resolve(uint32_t items) {
    if (threadIdx.x == 0 && !resolved) {
      pending_item = item_at(pending, items);
      resolved = true;
    }
  }
  // Thread 0 writes the next item (or NO_ITEM when there is none) to the LDS
  // word *at; visible after the caller's next barrier.
  __device__ __forceinline__ void announce(uint32_t* at, uint32_t items) {
    if (threadIdx.x == 0) {
      resolve(items);
      *at = pending_item;
    }
  }
  // Thread 0 publishes the next item; visible after the caller's barrier.
  __device__ __forceinline__ void stage_next(uint32_t items) {
    if (threadIdx.x == 0) {
      const uint32_t v = pending;
      slot[0] = resolved ? pending_item : item_at(v, items);
      resolved = false;
      pending = v < items ? take() : items;
    }
  }
  __device__ __forceinline__ uint32_t read() const { return slot[0]; }
};

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

// Compare-and-swap on LDS returning the previous value.
__device__ __forceinline__ u64 lds_cas64(u64* p, u64 expect, u64 val) {
  u64 e = expect;
  __hip_atomic_compare_exchange_strong(p, &e, val, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
  return e;
}
__device__ __forceinline__ uint32_t lds_cas32(uint32_t* p, uint32_t expect, uint32_t val) {
  uint32_t e = expect;
  __hip_atomic_compare_exchange_strong(p, &e, val, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
  return e;
}

// Find-or-insert of U keys per thread in an open-addressing LDS table with
// linear probing.  Stage 1 tries every key's home slot with one
// compare-and-swap, all U issued together; at the low load factors used here
// most keys settle there (the slot was empty, or already holds the key).
// Stage 2 walks the remaining keys of each lane one probe at a time, so the
// wavefront pays only for the probes that are actually left instead of
// U-wide rounds.  Slots only go from empty to a key, so a key is never placed
// twice.  slot[u] = the key's slot (-1 if not ok or out of probes), fresh[u]
// = whether this call inserted it.  Returns false if a key ran out of probes.
template <int U, class K>
__device__ __forceinline__ bool cas_insert(K* tk, uint32_t mask, const K (&key)[U],
                                           const uint32_t (&h)[U], const bool (&ok)[U],
                                           int (&slot)[U], bool (&fresh)[U],
                                           uint32_t max_probes) {
  constexpr K EMPTY = K(~K(0));
  K old[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    slot[u] = -1;
    fresh[u] = false;
    old[u] = EMPTY;
    if (ok[u]) {
      K* at = tk + (h[u] & mask);
      if constexpr (sizeof(K) == 8)
        old[u] = lds_cas64(reinterpret_cast<u64*>(at), EMPTY64, key[u]);
      else
        old[u] = lds_cas32(reinterpret_cast<uint32_t*>(at), EMPTY32, key[u]);
    }
  }
  uint32_t pending = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (ok[u]) {
      if (old[u] == EMPTY || old[u] == key[u]) {
        slot[u] = int(h[u] & mask);
        fresh[u] = old[u] == EMPTY;
      } else {
        pending |= 1u << u;
      }
    }
  }
  bool gave_up = false;
  while (pending) {
    const int cu = __builtin_ctz(pending);
    K ck = 0;
    uint32_t cp = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u == cu) { ck = key[u]; cp = h[u]; }
    int got = -1;
    bool fr = false;
    for (uint32_t probe = 1; probe < max_probes; ++probe) {
      const uint32_t s = (cp + probe) & mask;
      K o;
      if constexpr (sizeof(K) == 8)
        o = lds_cas64(reinterpret_cast<u64*>(tk + s), EMPTY64, ck);
      else
        o = lds_cas32(reinterpret_cast<uint32_t*>(tk + s), EMPTY32, ck);
      if (o == EMPTY || o == ck) {
        got = int(s);
        fr = o == EMPTY;
        break;
      }
    }
    if (got < 0) gave_up = true;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u == cu) { slot[u] = got; fresh[u] = fr; }
    pending &= pending - 1;
  }
  return !gave_up;
}

__device__ __forceinline__ uint32_t lds_add(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add64(u64* p, u64 v) {
  (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_sub(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---- global combine of partial statistics ---------------------------------

__device__ __forceinline__ void stat_add(NSGC_GLOBAL u64* out, u64 v) {
  if (v) __hip_atomic_fetch_add(out, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stat_max(NSGC_GLOBAL u64* out, u64 v) {
  if (v) __hip_atomic_fetch_max(out, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace nsgc

#endif  // NSGC_DEVICE_HPP_
