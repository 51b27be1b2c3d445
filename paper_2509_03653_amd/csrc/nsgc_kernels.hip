// Window-statistics kernels for gfx950 (tiers and phases: see nsgc_plan.h).
//
// All statistics are exact integer counts (Table III of arXiv 2509.03653 and
// its src/dst reverse).  Packets are packed into 64-bit keys src << 32 | dst;
// A(s,d) is the multiplicity of a key.  No contraction is involved, so no
// matrix cores are used: the work is hashing, LDS aggregation and
// order-independent integer reductions, bound by memory and LDS latency.
//
// Latency is the enemy here, so every per-element loop works on up to
// NSGC_UNROLL elements per thread in lockstep: segment searches, global loads
// and LDS compare-and-swap probes of those elements are issued together and
// their round trips overlap.  Each round takes the smallest unroll that
// covers the elements left, so short items do not pay for idle slots.
//
// The kernels that take uneven items (small windows, phases B and C) draw them
// from a work queue (ItemQueue: a static first item per workgroup, then
// per-class atomic counters); the partition kernel strides over its uniform
// tiles.  Phase C may take its items in the order k_order writes.  Grids are
// persistent, so a captured graph replays any batch that fits its workspace.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "nsgc_device.hpp"
#include "nsgc_plan.h"

namespace nsgc {

namespace {

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

constexpr int U = NSGC_UNROLL;
static_assert(U == 8, "for_rounds dispatches U = 8, 4, 2, 1");

template <class A>
__host__ __device__ constexpr int array_len() {
  return int(std::extent<std::remove_reference_t<A>>::value);
}

// Visits element indices [0, total) in rounds of UU * NSGC_BLOCK, calling
// body(j0, integral_constant<int, UU>) with the smallest UU of 8, 4, 2, 1 that
// covers what is left (UU = MAXU while more remains), so a short item does not
// pay for idle slots.  MAXU bounds the registers a round holds.  `total` must
// be uniform across the workgroup.
template <int MAXU = U, class Body>
__device__ __forceinline__ void for_rounds(uint32_t total, Body&& body) {
  static_assert(MAXU == 8 || MAXU == 4 || MAXU == 2 || MAXU == 1, "unroll");
  for (uint32_t j0 = 0; j0 < total;) {
    const uint32_t rem = total - j0;
    if (MAXU == 1 || (MAXU == 2 && rem > NSGC_BLOCK)) {
      body(j0, std::integral_constant<int, MAXU>());
      j0 += MAXU * NSGC_BLOCK;
    } else if (MAXU == 8 && rem > 4 * NSGC_BLOCK) {
      body(j0, std::integral_constant<int, 8>());
      j0 += 8 * NSGC_BLOCK;
    } else if (MAXU >= 4 && rem > 2 * NSGC_BLOCK) {
      body(j0, std::integral_constant<int, (MAXU >= 4 ? 4 : 1)>());
      j0 += 4 * NSGC_BLOCK;
    } else if (rem > NSGC_BLOCK) {
      body(j0, std::integral_constant<int, 2>());
      j0 += 2 * NSGC_BLOCK;
    } else {
      body(j0, std::integral_constant<int, 1>());
      j0 += NSGC_BLOCK;
    }
  }
}
// Probes before an insert of phases B and C gives up; the caller then splits
// the keys into sweeps, so giving up never changes a result.
constexpr uint32_t NSGC_MAX_PROBES = 64;
// A bucket whose table overflows even with 2^max_sweeps_log2 sweeps (plan
// header) is abandoned: every doubling halves the keys per sweep, so real
// data never gets near the default limit; it turns a broken invariant into a
// reported error instead of an endless loop.  The window's valid-packet count
// then carries bit 63 (no real count reaches it).
constexpr u64 NSGC_INVALID_BIT = 1ull << 63;
// Phase B holds 64-bit keys; four elements per thread keep it within 128
// VGPRs, i.e. two 512-thread workgroups per compute unit.
constexpr int LINK_MAXU = 4;
// Tile 2^14 of phase A runs with NSGC_BLOCK * PART14_SCALE threads.
constexpr int PART14_SCALE = 2;
// Work-queue classes of phase B (at most NSGC_QCLASSES): one measured best;
// its prefetched atomic hides behind the item.
constexpr uint32_t LINK_QCLASSES = 1;
// Phase C: four as well; eight spilled registers under its 80-VGPR budget
// (six waves per SIMD) and measured slower.
constexpr int RC_MAXU = 4;
// Links a thread holds while phase B combines them per source and
// destination: the link table has at most LK * NSGC_BLOCK slots.
constexpr int LK = 8;

constexpr uint32_t ENT_PMAX = (1u << NSGC_ENT_PACKET_BITS) - 1;
constexpr uint32_t ENT_LMAX = (1u << NSGC_ENT_LINK_BITS) - 1;
static_assert(NSGC_ENT_PACKET_BITS + NSGC_ENT_LINK_BITS == 32, "entry fields");
static_assert(LK * NSGC_BLOCK <= ENT_LMAX, "a bucket's links fit the link field");

// Entries needed for an (id, links, packets) triple (1 <= links <= packets).
__device__ __forceinline__ uint32_t entry_parts(uint32_t packets, uint32_t links) {
  if (packets <= ENT_PMAX && links <= ENT_LMAX) return 1u;
  const uint32_t a = packets / ENT_PMAX + (packets % ENT_PMAX != 0);
  const uint32_t b = links / ENT_LMAX + (links % ENT_LMAX != 0);
  return max(max(a, b), 1u);
}

// Write the `parts` entries of a triple at e[at], e[at + 1], ...
__device__ __forceinline__ void write_entry(NSGC_GLOBAL u64* e, uint32_t at, uint32_t id,
                                            uint32_t packets, uint32_t links, uint32_t parts) {
  if (parts == 1) {
    e[at] = (u64(id) << 32) | (u64(links) << NSGC_ENT_PACKET_BITS) | packets;
    return;
  }
  const uint32_t pq = packets / parts, pr = packets % parts;
  const uint32_t lq = links / parts, lr = links % parts;
  for (uint32_t i = 0; i < parts; ++i) {
    const uint32_t p = pq + (i < pr), l = lq + (i < lr);
    e[at + i] = (u64(id) << 32) | (u64(l) << NSGC_ENT_PACKET_BITS) | p;
  }
}

// ---- entity outputs ------------------------------------------------------
// Rows of the caller's lists: the lanes with `want` reserve consecutive rows
// of list `which` (0 links, 1 sources, 2 destinations) of window w with one
// 64-bit atomic per wavefront; a row at or past the window's end is not
// written (the window's count still reports every entity).
__device__ __forceinline__ u64 ent_reserve(const nsgc_dev_plan* P, uint32_t w, int which,
                                           bool want) {
  const u64 m = __ballot(want);
  if (m == 0) return ~0ull;
  const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
  u64 base = 0;
  if (int(lane_id()) == leader)
    base = __hip_atomic_fetch_add(P->ent_cur + u64(w) * 3 + which, u64(__popcll(m)),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const u64 b = (u64(readlane(uint32_t(base >> 32), leader)) << 32) | readlane(uint32_t(base), leader);
  return b + rank_below(m);
}

__device__ __forceinline__ void ent_row(const nsgc_dev_plan* P, long long* list, uint32_t w,
                                        int which, u64 row, u64 a, u64 b, u64 c) {
  if (row < P->ent_end[u64(w) * 3 + which]) {
    NSGC_GLOBAL long long* r = gptr(list) + row * 3;
    r[0] = (long long)a;
    r[1] = (long long)b;
    r[2] = (long long)c;
  }
}

// Find a 32-bit id in an open-addressing LDS table filled by cas_insert
// (probing from id & mask): true if present.
__device__ __forceinline__ bool lds_find32(const uint32_t* tk, uint32_t mask, uint32_t id) {
  uint32_t s = id & mask;
  for (uint32_t p = 0; p <= mask; ++p) {
    const uint32_t cur = tk[s];
    if (cur == id) return true;
    if (cur == EMPTY32) return false;
    s = (s + 1) & mask;
  }
  return false;
}

}  // namespace

// ---------------------------------------------------------------------------
// Tier "small": one workgroup per window, everything in LDS.
//
// Per packet, in hashed identities (link_key): find-or-insert the link key
// (the inserting lane learns that the link is new) and add one packet to it;
// add one packet to the source's row
// and, if the link is new, one link to its fan-out; the same for the
// destination's column.  Tables hold 2^k >= 2 n slots.
// ---------------------------------------------------------------------------

size_t lds_small_bytes(uint32_t slots_log2) {
  const size_t S = size_t(1) << slots_log2;
  return align16(S * 8) + align16(S * 4) * 7 + 256;
}

__global__ __launch_bounds__(NSGC_BLOCK) void k_small(nsgc_dev_plan* P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t S = 1u << P->small_slots_log2;
  u64* lk = reinterpret_cast<u64*>(smem);
  uint32_t* lc = reinterpret_cast<uint32_t*>(smem + align16(S * 8));
  uint32_t* rk = lc + S;
  uint32_t* rp = rk + S;
  uint32_t* rf = rp + S;
  uint32_t* ck = rf + S;
  uint32_t* cp = ck + S;
  uint32_t* cf = cp + S;
  uint32_t* misc = cf + S;  // [0] special link count, [1] special link seen,
                            // [2,3] special row (packets, links), [4,5] special
                            // column, [6] failure flag, [7] queue slot
  uint32_t* red = misc + 8;

  const uint32_t items = P->num_small;
  ItemQueue q(gptr(&P->queue[0][0]), misc + 7, NSGC_QCLASSES);
  for (uint32_t item = q.first(items); item != NO_ITEM; item = q.read()) {
    const nsgc_small_desc D = gload(P->small + item);
    for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
      lk[i] = EMPTY64;
      lc[i] = 0;
      rk[i] = EMPTY32;
      rp[i] = 0;
      rf[i] = 0;
      ck[i] = EMPTY32;
      cp[i] = 0;
      cf[i] = 0;
    }
    if (threadIdx.x < 7) misc[threadIdx.x] = 0;
    __syncthreads();

    const NSGC_GLOBAL uint32_t* src = gptr(P->src) + D.in_begin;
    const NSGC_GLOBAL uint32_t* dst = gptr(P->dst) + D.in_begin;
    for_rounds(D.n, [&](uint32_t j0, auto uc) {
      constexpr int U = decltype(uc)::value;
      uint32_t s[U], d[U], h[U];
      u64 key[U];
      bool ok[U], fresh[U], tab[U], rt[U];
      int slot[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t j = j0 + u * NSGC_BLOCK + threadIdx.x;
        ok[u] = j < D.n;
        s[u] = ok[u] ? src[j] : 0u;
        d[u] = ok[u] ? dst[j] : 0u;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {   // hashed identities (see link_key)
        s[u] = row_hash(s[u]);
        d[u] = P->entity ? row_hash(d[u]) : col_hash(d[u]);
        key[u] = (u64(s[u]) << 32) | d[u];
        h[u] = uint32_t(link_pos(key[u]));
        // the key equal to the empty marker is counted outside the table
        tab[u] = ok[u] && key[u] != EMPTY64;
      }
      if (!cas_insert<U>(lk, S - 1, key, h, tab, slot, fresh, S + 1)) lds_store(&misc[6], 1);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ok[u] && !tab[u]) {
          fresh[u] = lds_add(&misc[1], 1) == 0;
          lds_add(&misc[0], 1);
        }
        if (slot[u] >= 0) lds_add(&lc[slot[u]], 1);
      }
      // rows
#pragma unroll
      for (int u = 0; u < U; ++u) {
        rt[u] = ok[u] && s[u] != EMPTY32;
        h[u] = s[u];
      }
      if (!cas_insert<U>(rk, S - 1, s, h, rt, slot, tab, S + 1)) lds_store(&misc[6], 1);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ok[u] && !rt[u]) {
          lds_add(&misc[2], 1);
          if (fresh[u]) lds_add(&misc[3], 1);
        }
        if (slot[u] >= 0) {
          lds_add(&rp[slot[u]], 1);
          if (fresh[u]) lds_add(&rf[slot[u]], 1);
        }
      }
      // columns
#pragma unroll
      for (int u = 0; u < U; ++u) {
        rt[u] = ok[u] && d[u] != EMPTY32;
        h[u] = d[u];
      }
      if (!cas_insert<U>(ck, S - 1, d, h, rt, slot, tab, S + 1)) lds_store(&misc[6], 1);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ok[u] && !rt[u]) {
          lds_add(&misc[4], 1);
          if (fresh[u]) lds_add(&misc[5], 1);
        }
        if (slot[u] >= 0) {
          lds_add(&cp[slot[u]], 1);
          if (fresh[u]) lds_add(&cf[slot[u]], 1);
        }
      }
    });
    __syncthreads();

    uint32_t nl = 0, sl = 0, ml = 0, nr = 0, mr = 0, mf = 0, nc = 0, mc = 0, mg = 0;
    for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
      if (lk[i] != EMPTY64) { ++nl; sl += lc[i]; ml = max(ml, lc[i]); }
      if (rk[i] != EMPTY32) { ++nr; mr = max(mr, rp[i]); mf = max(mf, rf[i]); }
      if (ck[i] != EMPTY32) { ++nc; mc = max(mc, cp[i]); mg = max(mg, cf[i]); }
    }
    if (threadIdx.x == 0) {
      if (misc[0]) { ++nl; sl += misc[0]; ml = max(ml, misc[0]); }
      if (misc[2]) { ++nr; mr = max(mr, misc[2]); mf = max(mf, misc[3]); }
      if (misc[4]) { ++nc; mc = max(mc, misc[4]); mg = max(mg, misc[5]); }
    }
    block_sum_max(sl, ml, red);
    block_sum_max(nl, mr, red);
    block_sum_max(nr, mf, red);
    block_sum_max(nc, mc, red);
    uint32_t zero = 0;
    block_sum_max(zero, mg, red);
    if (threadIdx.x == 0) {
      // tables of >= 2n slots cannot fill; a failure would be a library bug,
      // reported as all-ones statistics rather than silently wrong numbers
      const bool bad = misc[6] != 0;
      NSGC_GLOBAL u64* o = gptr(P->out) + u64(D.out_index) * 9;
      o[0] = bad ? ~0ull : sl; o[1] = bad ? ~0ull : nl; o[2] = bad ? ~0ull : ml;
      o[3] = bad ? ~0ull : nr; o[4] = bad ? ~0ull : mr; o[5] = bad ? ~0ull : mf;
      o[6] = bad ? ~0ull : nc; o[7] = bad ? ~0ull : mc; o[8] = bad ? ~0ull : mg;
    }
    if (P->entity) {
      // the lists, and the sources and destinations counted once in their union
      // (destinations are hashed like sources in entity mode)
      const uint32_t w = D.out_index;
      uint32_t uni = 0;
      for (uint32_t i0 = 0; i0 < S; i0 += NSGC_BLOCK) {
        const uint32_t i = i0 + threadIdx.x;
        const bool l = i < S && lk[i] != EMPTY64;
        const bool r = i < S && rk[i] != EMPTY32;
        const bool c = i < S && ck[i] != EMPTY32;
        if (c && !lds_find32(rk, S - 1, ck[i])) ++uni;
        if (P->ent_links) {
          const u64 row = ent_reserve(P, w, 0, l);
          if (l) ent_row(P, P->ent_links, w, 0, row, row_unhash(uint32_t(lk[i] >> 32)),
                         row_unhash(uint32_t(lk[i])), lc[i]);
        }
        if (P->ent_src) {
          const u64 row = ent_reserve(P, w, 1, r);
          if (r) ent_row(P, P->ent_src, w, 1, row, row_unhash(rk[i]), rp[i], rf[i]);
        }
        if (P->ent_dst) {
          const u64 row = ent_reserve(P, w, 2, c);
          if (c) ent_row(P, P->ent_dst, w, 2, row, row_unhash(ck[i]), cp[i], cf[i]);
        }
      }
      if (threadIdx.x == 0) {   // the hashed id EMPTY32 lives outside the tables
        const uint32_t xe = row_unhash(EMPTY32);
        if (misc[0] && P->ent_links) {
          const u64 row = __hip_atomic_fetch_add(P->ent_cur + u64(w) * 3, 1ull, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          ent_row(P, P->ent_links, w, 0, row, xe, xe, misc[0]);
        }
        if (misc[2] && P->ent_src) {
          const u64 row = __hip_atomic_fetch_add(P->ent_cur + u64(w) * 3 + 1, 1ull,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ent_row(P, P->ent_src, w, 1, row, xe, misc[2], misc[3]);
        }
        if (misc[4] && P->ent_dst) {
          const u64 row = __hip_atomic_fetch_add(P->ent_cur + u64(w) * 3 + 2, 1ull,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ent_row(P, P->ent_dst, w, 2, row, xe, misc[4], misc[5]);
        }
        if (misc[4] && !misc[2]) ++uni;
      }
      uni = block_sum(uni, red);
      if (threadIdx.x == 0) {
        NSGC_GLOBAL long long* cnt = gptr(P->ent_counts) + u64(w) * 4;
        cnt[0] = (long long)nl;
        cnt[1] = (long long)nr;
        cnt[2] = (long long)nc;
        cnt[3] = (long long)(nr + uni);
      }
    }
    q.stage_next(items);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Heavy sources of the row-complete windows.
//
// One workgroup per window counts the hashed sources of a sample of
// NSGC_HEAVY_SAMPLE packets: sixteen runs of 256 consecutive packets spread
// evenly from the window's first packet to its last (all packets of a smaller
// window).  A source is heavy when its sample count puts it above half a link
// bucket's share of the packets.  The window's table holds them in sets of
// four, the set chosen by the id's low bits; a set keeps its four most
// frequent candidates (a dropped one would fill its home bucket alone), and
// an unused slot holds a value whose low bits name another set, so it matches
// no id.  Which sources the table names decides only how evenly the buckets
// fill: the partition and phase B read the same table, and every result is
// exact for any table.
// ---------------------------------------------------------------------------

constexpr uint32_t HEAVY_SETS = NSGC_HEAVY_SLOTS / 4;
constexpr uint32_t HEAVY_TABLE = 2 * NSGC_HEAVY_SAMPLE;   // sample counting table
constexpr uint32_t HEAVY_CAND = NSGC_HEAVY_SAMPLE / 2;    // counts >= 2: at most m / 2 candidates
static_assert(NSGC_HEAVY_SAMPLE == 16 * 256, "sixteen runs of 256 packets");
static_assert(HEAVY_SETS <= NSGC_BLOCK, "one thread per set");

size_t lds_heavy_bytes() { return size_t(HEAVY_TABLE) * 8 + size_t(HEAVY_CAND) * 8 + 16; }

__global__ __launch_bounds__(NSGC_BLOCK) void k_heavy(const nsgc_dev_plan* __restrict__ P) {
  extern __shared__ __align__(16) unsigned char smem[];
  u64* cand = reinterpret_cast<u64*>(smem);               // [HEAVY_CAND] count << 32 | id
  uint32_t* key = reinterpret_cast<uint32_t*>(cand + HEAVY_CAND);   // [HEAVY_TABLE]
  uint32_t* cnt = key + HEAVY_TABLE;                      // [HEAVY_TABLE]
  uint32_t* ncand = cnt + HEAVY_TABLE;
  const uint32_t tid = threadIdx.x;
  for (uint32_t wi = blockIdx.x; wi < P->num_part; wi += gridDim.x) {
    const nsgc_win_desc W = gload(P->win + wi);
    if (!W.rows) continue;   // the same for the whole workgroup
    for (uint32_t i = tid; i < HEAVY_TABLE; i += NSGC_BLOCK) {
      key[i] = EMPTY32;
      cnt[i] = 0;
    }
    if (tid == 0) *ncand = 0;
    __syncthreads();
    const uint32_t m = min(W.n, NSGC_HEAVY_SAMPLE);
    const NSGC_GLOBAL uint32_t* src = gptr(P->src) + W.in_begin;
    for (uint32_t i = tid; i < m; i += NSGC_BLOCK) {
      const uint32_t at = W.n <= NSGC_HEAVY_SAMPLE
                              ? i
                              : uint32_t(u64(W.n - 256u) * (i >> 8) / 15u) + (i & 255u);
      const uint32_t r = row_hash(src[at]);
      if (r == EMPTY32) continue;   // this id keeps per-link entries anyway
      bool fresh;
      const int sl = lds_insert32(key, HEAVY_TABLE - 1, r, r, fresh);   // never full: 2x the sample
      if (sl >= 0) lds_add(&cnt[sl], 1);
    }
    __syncthreads();
    // estimated packets cnt * n / m above n / (2 B): cnt > m / (2 B)
    const uint32_t thr = max(2u, (m >> (W.logB + 1)) + 1u);
    for (uint32_t i = tid; i < HEAVY_TABLE; i += NSGC_BLOCK) {
      const uint32_t c = cnt[i];
      if (c >= thr) cand[lds_add(ncand, 1)] = (u64(c) << 32) | key[i];
    }
    __syncthreads();
    // thread j keeps set j's four largest (count, id) candidates
    const uint32_t nc = *ncand;
    NSGC_GLOBAL uint32_t* out = gptr(P->heavy) + u64(W.counter) * NSGC_HEAVY_SLOTS;
    if (tid < HEAVY_SETS) {
      u64 top[4] = {0, 0, 0, 0};
      for (uint32_t i = 0; i < nc; ++i) {
        u64 v = cand[i];
        if ((uint32_t(v) & (HEAVY_SETS - 1)) != tid) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (v > top[k]) {
            const u64 t = top[k];
            top[k] = v;
            v = t;
          }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) out[tid * 4 + k] = top[k] ? uint32_t(top[k]) : ~tid;
    }
    __syncthreads();
  }
}

// Whether hashed source r is in a window's heavy table (LDS, 16-byte aligned).
__device__ __forceinline__ bool heavy_source(const uint32_t* hv, uint32_t r) {
  const v4u32 q = *reinterpret_cast<const v4u32*>(hv + (r & (HEAVY_SETS - 1)) * 4);
  return q.x == r || q.y == r || q.z == r || q.w == r;
}

// Link bucket of key k in a row-complete window of 2^logB >= 2 buckets: a
// light source's links all go to its home bucket, the top bits of its hashed
// id; a heavy source's links go to the other 2^logB - 1 buckets, home ^ x with
// x in 1 .. 2^logB - 1 from the destination hash, so they never meet the home.
__device__ __forceinline__ uint32_t row_bucket(u64 k, uint32_t logB, bool heavy) {
  const uint32_t r = uint32_t(k >> 32), c = uint32_t(k);
  const uint32_t home = top32(r, logB);
  const uint32_t x = 1u + uint32_t((u64(c) * ((1u << logB) - 1u)) >> 32);
  return heavy ? home ^ x : home;
}

// ---------------------------------------------------------------------------
// Phase A: partition a tile of packets by link bucket.
//
// Each thread holds PER packets in registers (16-byte loads when the tile is
// aligned).  An LDS histogram gives every packet its rank in its bucket, a
// block scan gives the bucket starts, the keys are placed in LDS in bucket
// order and leave in full coalesced lines.  The tile's bucket starts go to
// the bucket-major tile table.  When the plan orders phase C, a window's
// first tile also writes the window's phase-C item sizes (packets per row and
// column bucket in that tile), the only input of the ordering.
// ---------------------------------------------------------------------------

size_t lds_part_bytes(uint32_t max_link_buckets, uint32_t tile_log2, uint32_t max_rc_buckets) {
  (void)max_rc_buckets;   // the row/column sample shares the staging area
  return align16((max_link_buckets + 1) * 4) + align16((size_t(1) << tile_log2) * 8) + 256 +
         NSGC_HEAVY_SLOTS * 4;
}

// ROWS: the launch's batch has row-complete windows (the other instances
// carry none of their code).
template <int PER, int NT = NSGC_BLOCK, bool ROWS = false>
__global__ __launch_bounds__(NT) void k_partition(const nsgc_dev_plan* __restrict__ P,
                                                  uint32_t max_link_buckets) {
  static_assert(PER % 4 == 0, "PER must be a multiple of 4");
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr uint32_t T = NT * PER;
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem);
  u64* stage = reinterpret_cast<u64*>(smem + align16((max_link_buckets + 1) * 4));
  uint32_t* red = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(stage) + T * 8);
  uint32_t* hv = red + 64;   // the window's heavy sources (row-complete windows)
  // packets per row and column bucket of a window's first tile; in the staging
  // area, which is free until the bucket scan's barriers
  uint32_t* rch = reinterpret_cast<uint32_t*>(stage);
  const bool same = P->entity != 0;   // entity outputs: destinations hashed like sources
  const uint32_t items = P->itemsA;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t wi = owner_of_wave(gptr(P->prefA), P->num_part, item);
    const nsgc_win_desc W = gload(P->win + wi);
    const uint32_t t = item - gptr(P->prefA)[wi];
    const uint32_t B = 1u << W.logB, R = 1u << W.logR, C = 1u << W.logC;
    const uint32_t tbeg = t * T;
    const uint32_t len = min(T, W.n - tbeg);
    // The first tile of a window also counts its packets per row and column
    // bucket: the phase-C item sizes by which k_order starts large items first
    // (a sample, so only the order depends on it).
    const bool sample = t == 0 && P->order_items && R + C <= 2 * T;
    if (t == 0 && P->order_items && !sample) {   // too many buckets to sample: equal sizes
      NSGC_GLOBAL uint32_t* sz = gptr(P->rcsize) + gptr(P->prefC)[wi];
      for (uint32_t i = threadIdx.x; i < R + C; i += NT) sz[i] = 1;
    }
    for (uint32_t i = threadIdx.x; i < B; i += NT) hist[i] = 0;
    if (sample)
      for (uint32_t i = threadIdx.x; i < R + C; i += NT) rch[i] = 0;
    const bool rows = ROWS && W.rows != 0;
    if (rows)
      for (uint32_t i = threadIdx.x; i < NSGC_HEAVY_SLOTS; i += NT)
        hv[i] = gptr(P->heavy)[u64(W.counter) * NSGC_HEAVY_SLOTS + i];
    __syncthreads();

    const uint64_t gbeg = uint64_t(W.in_begin) + tbeg;
    const NSGC_GLOBAL uint32_t* src = gptr(P->src) + gbeg;
    const NSGC_GLOBAL uint32_t* dst = gptr(P->dst) + gbeg;
    u64 key[PER];
    uint32_t br[PER];   // rank in bucket << 12 | bucket (buckets <= 4096, ranks < 2^14)
    bool ok[PER];
    const bool aligned = ((reinterpret_cast<uintptr_t>(P->src + gbeg) |
                           reinterpret_cast<uintptr_t>(P->dst + gbeg)) & 15) == 0;
    if (aligned && len == T) {
      // full aligned tile: each thread loads 4 consecutive packets per step
#pragma unroll
      for (int k = 0; k < PER / 4; ++k) {
        const uint32_t idx = (k * NT + threadIdx.x) * 4;
        const v4u32 s4 = *(const NSGC_GLOBAL v4u32*)(src + idx);
        const v4u32 d4 = *(const NSGC_GLOBAL v4u32*)(dst + idx);
        key[4 * k + 0] = link_key(s4.x, d4.x, same);
        key[4 * k + 1] = link_key(s4.y, d4.y, same);
        key[4 * k + 2] = link_key(s4.z, d4.z, same);
        key[4 * k + 3] = link_key(s4.w, d4.w, same);
        ok[4 * k + 0] = ok[4 * k + 1] = ok[4 * k + 2] = ok[4 * k + 3] = true;
      }
    } else {
      // unaligned or partial tile: element loads, all issued before any is
      // used (a lane past the end loads the tile's first packet and is masked)
      uint32_t sv[PER], dv[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const uint32_t idx = k * NT + threadIdx.x;
        ok[k] = idx < len;
        const uint32_t at = ok[k] ? idx : 0u;
        sv[k] = src[at];
        dv[k] = dst[at];
      }
#pragma unroll
      for (int k = 0; k < PER; ++k) key[k] = link_key(sv[k], dv[k], same);
    }
    bool hvy[PER];   // row-complete windows: the packet's source is heavy
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      hvy[k] = rows && heavy_source(hv, uint32_t(key[k] >> 32));
      if (ok[k]) {
        const uint32_t bk =
            rows ? row_bucket(key[k], W.logB, hvy[k]) : top64(link_pos(key[k]), W.logB);
        br[k] = (lds_add(&hist[bk], 1) << 12) | bk;
      }
    }
    if (sample) {
      // a light source of a row-complete window sends nothing to phase C
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        if (ok[k]) {
          const uint32_t r = uint32_t(key[k] >> 32);
          if (!rows || hvy[k] || r == EMPTY32) lds_add(&rch[top32(r, W.logR)], 1);
          lds_add(&rch[R + top32(uint32_t(key[k]), W.logC)], 1);
        }
      }
    }
    __syncthreads();
    if (sample) {
      NSGC_GLOBAL uint32_t* sz = gptr(P->rcsize) + gptr(P->prefC)[wi];
      for (uint32_t i = threadIdx.x; i < R + C; i += NT) sz[i] = rch[i];
    }
    block_exclusive_scan<NT>(hist, B, red);
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (ok[k]) stage[hist[br[k] & 0xFFFu] + (br[k] >> 12)] = key[k];
    NSGC_GLOBAL uint32_t* tm = gptr(P->tilemeta) + W.tilemeta + t;
    for (uint32_t i = threadIdx.x; i <= B; i += NT) tm[u64(i) * W.ntiles] = hist[i];
    __syncthreads();
    NSGC_GLOBAL u64* out = gptr(P->keys) + W.ws + tbeg;
    for (uint32_t i = threadIdx.x; i < len; i += NT) out[i] = stage[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Shared machinery of phases B and C: visit the elements of `nseg` segments
// (`seg(i, base, len)` describes segment i) wavefront by wavefront.
//
// Wavefront w takes segments w, w + WAVES, w + 2 WAVES, ... of each group of
// 64 * WAVES segments; its lanes load the descriptions of the wave's (up to
// 64) segments at once, and the wave walks them in chunks of 64 consecutive
// elements, up to MAXU chunks per round.  Long segments are walked one at a
// time (lane = offset in the chunk; a segment's last chunk may be partly
// idle).  When the segments are short (large windows cut into many buckets
// and tiles) that would leave most lanes idle, so the wave instead walks the
// concatenation of its segments: lane l of a chunk at position v takes
// element v + l, whose segment a 6-step binary search over the lanes'
// inclusive length prefix finds.  There is no LDS staging and no barrier
// until the one at the end, so waves proceed independently.  `fn(pos, ok)`
// receives the round's positions (pos[u] valid when ok[u]; the array length
// is the round's unroll) with the whole wavefront active; it must not use
// workgroup barriers.
// ---------------------------------------------------------------------------

__device__ __forceinline__ u64 readlane64(u64 v, uint32_t k) {
  return (u64(readlane(uint32_t(v >> 32), int(k))) << 32) | readlane(uint32_t(v), int(k));
}

// Rounds over `total` chunks (uniform across the wavefront, not the block):
// body(integral_constant<int, UU>) with the smallest UU of 8, 4, 2, 1 (at
// most MAXU) that covers what is left.
template <int MAXU, class Body>
__device__ __forceinline__ void for_chunk_rounds(uint32_t total, Body&& body) {
  static_assert(MAXU == 8 || MAXU == 4 || MAXU == 2 || MAXU == 1, "unroll");
  for (uint32_t c = 0; c < total;) {
    const uint32_t rem = total - c;
    if (MAXU >= 8 && rem > 4) {
      body(std::integral_constant<int, (MAXU >= 8 ? 8 : 1)>());
      c += 8;
    } else if (MAXU >= 4 && rem > 2) {
      body(std::integral_constant<int, (MAXU >= 4 ? 4 : 1)>());
      c += 4;
    } else if (MAXU >= 2 && rem > 1) {
      body(std::integral_constant<int, (MAXU >= 2 ? 2 : 1)>());
      c += 2;
    } else {
      body(std::integral_constant<int, 1>());
      c += 1;
    }
  }
}

// Keeps a wave-uniform value in a scalar register (the compiler cannot always
// prove uniformity of values derived from threadIdx.x / 64).
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return uint32_t(__builtin_amdgcn_readfirstlane(int(v)));
}

// The packed walk is taken when it needs fewer than PACK_NUM / PACK_DEN of
// the segment-by-segment walk's chunks (its search costs part of a chunk).
constexpr uint32_t PACK_NUM = 7, PACK_DEN = 8;

// This lane's segment of the first group (segments w + WAVES * lane), when
// the caller loaded it beforehand (zero length where there is none).
struct SegPre {
  u64 base;
  uint32_t len;
};

struct NoTail {
  __device__ void operator()() const {}
};

// `tail()` runs in every thread just before the final barrier.
template <int MAXU, class SegFn, class BatchFn, class Tail = NoTail>
__device__ __forceinline__ void gather_by_wave(uint32_t nseg, SegFn seg, BatchFn fn,
                                               const SegPre* pre = nullptr, Tail tail = Tail()) {
  const uint32_t w = uniform(threadIdx.x >> 6), lane = lane_id();
  constexpr uint32_t GROUP = 64u * uint32_t(WAVES);
  constexpr int PACKU = MAXU < 4 ? MAXU : 4;
  for (uint32_t g0 = 0; g0 < nseg; g0 += GROUP) {
    const uint32_t si = g0 + w + uint32_t(WAVES) * lane;   // this lane's segment
    u64 mybase = 0;
    uint32_t mylen = 0;
    if (g0 == 0 && pre) {
      mybase = pre->base;
      mylen = pre->len;
    } else if (si < nseg) {
      seg(si, mybase, mylen);
    }
    const uint32_t nk = uniform(g0 + w < nseg ? min(64u, (nseg - g0 - w + WAVES - 1) / WAVES) : 0u);
    const uint32_t chunks = uniform(wave_sum((mylen + 63u) >> 6));   // segment by segment
    const uint32_t elems = uniform(wave_sum(mylen));
    const uint32_t packed_chunks = (elems + 63u) >> 6;               // concatenated
    if (PACK_DEN * packed_chunks < PACK_NUM * chunks) {
      // Packed walk, in rounds of at most 4 chunks (the search's registers
      // stay out of the widest round).  Lane l of the chunk at v takes
      // element v + l of the concatenation; its segment j is the number of
      // lanes whose inclusive prefix is <= v + l (empty segments skipped).
      const uint32_t incl = wave_inclusive_scan(mylen);
      const u64 mb = mybase - (incl - mylen);   // base - exclusive prefix
      uint32_t v0 = 0;
      for_chunk_rounds<PACKU>(packed_chunks, [&](auto uc) {
        constexpr int U = decltype(uc)::value;
        u64 pos[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t v = v0 + lane;
          uint32_t j = 0;
#pragma unroll
          for (uint32_t st = 32; st > 0; st >>= 1)
            if (lane_take(incl, j + st - 1) <= v) j += st;
          pos[u] = ((u64(lane_take(uint32_t(mb >> 32), j)) << 32) | lane_take(uint32_t(mb), j)) + v;
          ok[u] = v < elems;
          v0 = uniform(v0 + 64);
        }
        fn(pos, ok);
      });
      continue;
    }
    uint32_t k = 0, off = 0;                                          // uniform cursor
    while (k < nk && readlane(mylen, int(k)) == 0) k = uniform(k + 1);
    for_chunk_rounds<MAXU>(chunks, [&](auto uc) {
      constexpr int U = decltype(uc)::value;
      u64 pos[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k < nk) {
          const uint32_t len = readlane(mylen, int(k));
          pos[u] = readlane64(mybase, k) + off + lane;
          ok[u] = off + lane < len;
          off = uniform(off + 64);
          if (off >= len) {
            off = 0;
            k = uniform(k + 1);
            while (k < nk && readlane(mylen, int(k)) == 0) k = uniform(k + 1);
          }
        } else {
          pos[u] = 0;
          ok[u] = false;
        }
      }
      fn(pos, ok);
    });
  }
  tail();
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Phase B: link aggregation of one link bucket.
//
// The bucket's keys are gathered from every tile of the window into an LDS
// table key -> packet count (duplicates of the first valid lane's key are
// combined with one ballot first, which keeps heavy links from serialising on
// one LDS address).  Every newly inserted slot is also appended to a list of
// occupied slots, so everything after the inserts (statistics, emission and
// resetting the table for the next item) costs per link, not per slot.  The
// table gives the bucket's share of stats 0-2.  Each link is then emitted as
// a row entry (src, packets, links = 1) grouped by row bucket and a column
// entry (dst, packets, 1) grouped by column bucket into the bucket's
// emission region: the entries are counted per row and column bucket, the
// counts scanned into starts (also published for phase C), and the entries
// written at the starts; the emission pass also empties the table.
//
// With per-id combining (the COMBINE instantiation, tuning combine_probes >
// 0) the links are first combined per source and per destination in the
// same LDS region, so phase C receives one entry per (link bucket, id)
// instead of one per link; it costs phase B more than it saves phase C on
// the measured workloads, so it is off by default.
//
// If an insert gives up (more distinct keys than the table holds), the bucket
// is split into 2^s sweeps by further hash bits and redone; the sweeps
// partition the keys, so the result is unchanged.  With sweeps, every sweep
// emits its own links uncombined (links = 1) right after its build, into
// row and column segments sized by the bucket's packets (see the sweep loop).
// ---------------------------------------------------------------------------

size_t lds_link_bytes(uint32_t slots_log2, uint32_t max_rc_buckets) {
  const size_t S = size_t(1) << slots_log2;
  return align16(S * 8) + align16(S * 4) + align16(S * 4) + 2 * align16((max_rc_buckets + 1) * 4) +
         256;
}

// COMBINE selects the single-sweep emission: per link (false) or combined per
// source and destination (true, plan field combine_probes > 0); they are
// separate instantiations so the per-link kernel carries none of the
// combining code's registers.
template <bool COMBINE>
__global__ __launch_bounds__(NSGC_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_links(
    nsgc_dev_plan* P, uint32_t max_rc_buckets) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t S = 1u << P->link_slots_log2;
  unsigned char* p = smem;
  u64* tk = reinterpret_cast<u64*>(p);                 p += align16(S * 8);
  uint32_t* tc = reinterpret_cast<uint32_t*>(p);       p += align16(S * 4);
  uint32_t* occ = reinterpret_cast<uint32_t*>(p);      p += align16(S * 4);
  struct { uint32_t* red; } st;                        // reduction scratch (in misc)
  uint32_t* histR = reinterpret_cast<uint32_t*>(p);    p += align16((max_rc_buckets + 1) * 4);
  uint32_t* histC = reinterpret_cast<uint32_t*>(p);    p += align16((max_rc_buckets + 1) * 4);
  uint32_t* misc = reinterpret_cast<uint32_t*>(p);
  // misc: [0] fail flag, [1] special link count, [4] emission base,
  // [5] occupied slots, [7] queue slot, [8..24) reduction scratch
  st.red = misc + 8;

  // the table starts empty; every item leaves it empty again
  for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
    tk[i] = EMPTY64;
    tc[i] = 0;
  }
  if (threadIdx.x == 0) misc[5] = 0;

  const uint32_t T = 1u << P->tile_log2;
  const uint32_t items = P->itemsBb;
  const NSGC_GLOBAL uint32_t* map = P->mapBb ? gptr(P->mapBb) : nullptr;
  const uint32_t wave = uniform(threadIdx.x >> 6), lane = lane_id();
  // The first group of an item's segments: lane l of wave w holds tile
  // w + WAVES * l (its start s0 in the bucket and the segment).  Loaded for
  // the next item while the current one finishes, so that an item's gather
  // starts with its key loads instead of a chain of metadata loads.
  auto load_first = [&](uint32_t it, SegPre& pre, uint32_t& s0) {
    const uint32_t wi = sload(P->itemwinB + it);
    const nsgc_win_desc W = sload_words(P->win + wi);
    const uint32_t b = it - sload(P->prefB + wi);
    const NSGC_GLOBAL uint32_t* t0 = gptr(P->tilemeta) + W.tilemeta + u64(b) * W.ntiles;
    const uint32_t t = wave + uint32_t(WAVES) * lane;
    pre.base = 0;
    pre.len = 0;
    s0 = 0;
    if (t < W.ntiles) {
      const uint32_t a = t0[t], c = t0[t + W.ntiles];
      s0 = a;
      pre.base = u64(t) * T + a;
      pre.len = c - a;
    }
  };
  SegPre next_pre = {0, 0};
  uint32_t next_s0 = 0;
  bool have_next = false;

  ItemQueue q(gptr(&P->queue[1][0]), misc + 7, LINK_QCLASSES, map);
  for (uint32_t item = q.first(items); item != NO_ITEM; item = q.read()) {
    const uint32_t it = uniform(item);
    const uint32_t wi = sload(P->itemwinB + it);
    const nsgc_win_desc W = sload_words(P->win + wi);
    const uint32_t b = it - sload(P->prefB + wi);
    const uint32_t B = 1u << W.logB, R = 1u << W.logR, C = 1u << W.logC;
    const uint32_t nt = W.ntiles;
    const NSGC_GLOBAL u64* keys = gptr(P->keys) + W.ws;
    const NSGC_GLOBAL uint32_t* tm0 = gptr(P->tilemeta) + W.tilemeta + u64(b) * nt;  // bucket b
    const NSGC_GLOBAL uint32_t* tm1 = tm0 + nt;                                      // bucket b+1
    NSGC_GLOBAL uint32_t* rec = gptr(P->lbmeta) + W.lbmeta;

    SegPre pre;
    uint32_t pre_s0;
    if (have_next) {
      pre = next_pre;
      pre_s0 = next_s0;
    } else {
      load_first(it, pre, pre_s0);
    }
    have_next = false;
    // thread 0 names the next item (read by all after the gather's barrier)
    q.announce(&misc[6], items);
    bool fetched = false;

    // The emission base of bucket b (packets of the window in link buckets
    // below b) is the sum of b's starts over the tiles: summed while the
    // first gather loads them.
    if (threadIdx.x == 0) misc[4] = 0;
    uint32_t below = pre_s0;
    bool base_pending = true;

    auto seg = [&](uint32_t t, u64& sbase, uint32_t& len) {
      const uint32_t s0 = tm0[t], s1 = tm1[t];
      if (base_pending) below += s0;
      sbase = u64(t) * T + s0;
      len = s1 - s0;
    };

    // Empty the table through the occupied-slot list.
    auto reset = [&]() {
      const uint32_t n = misc[5];
      for (uint32_t i = threadIdx.x; i < n; i += NSGC_BLOCK) {
        const uint32_t s = occ[i];
        tk[s] = EMPTY64;
        tc[s] = 0;
      }
      __syncthreads();
      if (threadIdx.x == 0) misc[5] = 0;
      __syncthreads();
    };

    // Link table of sweep `sw` of 2^logS.  With `cap`, every packet of the
    // bucket (of any sweep) is also counted in histR / histC by its row and
    // column bucket.  An insert gives up after `probes` probes.
    auto build = [&](uint32_t logS, uint32_t sw, bool cap, uint32_t probes) {
      if (threadIdx.x < 2) misc[threadIdx.x] = 0;
      __syncthreads();
      gather_by_wave<LINK_MAXU>(nt, seg, [&](const auto& pos, const auto& okin) {
        constexpr int U = array_len<decltype(pos)>();
        u64 key[U];
        uint32_t h[U], add[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {   // unconditional load (position 0 exists), then mask
          const u64 kk = keys[okin[u] ? pos[u] : 0ull];
          key[u] = okin[u] ? kk : 0ull;
        }
        if (cap) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (okin[u]) {
              lds_add(&histR[top32(uint32_t(key[u] >> 32), W.logR)], 1);
              lds_add(&histC[top32(uint32_t(key[u]), W.logC)], 1);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const u64 hh = link_pos(key[u]);
          h[u] = uint32_t(hh);
          ok[u] = okin[u] && !(logS && next64(hh, W.logB, logS) != sw);
          add[u] = 1;
          if (ok[u] && key[u] == EMPTY64) {
            lds_add(&misc[1], 1);
            ok[u] = false;
          }
          // combine the lanes holding the first valid lane's key
          const u64 vm = __ballot(ok[u]);
          if (vm) {
            const int first = __ffsll(static_cast<unsigned long long>(vm)) - 1;
            const u64 k0 = (u64(readlane(uint32_t(key[u] >> 32), first)) << 32) |
                           readlane(uint32_t(key[u]), first);
            const bool same = ok[u] && key[u] == k0;
            const uint32_t nsame = __popcll(__ballot(same));
            if (nsame > 1 && same) {
              if (int(lane_id()) == first) add[u] = nsame;
              else ok[u] = false;
            }
          }
        }
        int slot[U];
        bool fresh[U];
        if (!cas_insert<U>(tk, S - 1, key, h, ok, slot, fresh, probes))
          lds_store(&misc[0], 1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (slot[u] >= 0) lds_add(&tc[slot[u]], add[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t at = wave_append(&misc[5], fresh[u]);
          if (fresh[u]) occ[at] = uint32_t(slot[u]);
        }
      }, &pre);
      if (!fetched) {   // the next item's first segments, loaded behind this item
        fetched = true;
        const uint32_t nx = uniform(misc[6]);
        if (nx != NO_ITEM) {
          load_first(nx, next_pre, next_s0);
          have_next = true;
        }
      }
      if (base_pending) {   // visible after the barriers before any emission
        base_pending = false;
        below = wave_sum(below);
        if (lane_id() == 0 && below) lds_add(&misc[4], below);
      }
    };

    // Count (or, with cursors, write) the links per row and column bucket.
    auto count = [&]() {
      const uint32_t n = misc[5];
      for (uint32_t i = threadIdx.x; i < n; i += NSGC_BLOCK) {
        const uint32_t s = occ[i];
        const u64 key = tk[s];
        const uint32_t parts = entry_parts(tc[s], 1);
        lds_add(&histR[top32(uint32_t(key >> 32), W.logR)], parts);
        lds_add(&histC[top32(uint32_t(key), W.logC)], parts);
      }
      if (threadIdx.x == 0 && misc[1]) {
        const uint32_t parts = entry_parts(misc[1], 1);
        lds_add(&histR[top32(EMPTY32, W.logR)], parts);
        lds_add(&histC[top32(EMPTY32, W.logC)], parts);
      }
    };
    // Emission also empties the table (each listed slot once); the list
    // length is cleared after its final barrier.
    auto emit = [&]() {
      const uint32_t base = misc[4];
      NSGC_GLOBAL u64* er = gptr(P->emit_row) + W.ws + base;
      NSGC_GLOBAL u64* ec = gptr(P->emit_col) + W.ws + base;
      const uint32_t n = misc[5];
      for_rounds<LINK_MAXU>(n, [&](uint32_t i0, auto uc) {
        constexpr int U = decltype(uc)::value;
        u64 key[U];
        uint32_t cnt[U], ar[U], ac[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t i = i0 + u * NSGC_BLOCK + threadIdx.x;
          ok[u] = i < n;
          const uint32_t s = ok[u] ? occ[i] : 0u;
          key[u] = ok[u] ? tk[s] : 0ull;
          cnt[u] = ok[u] ? tc[s] : 0u;
          if (ok[u]) {   // last use of the slot: empty it on the way
            tk[s] = EMPTY64;
            tc[s] = 0;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (ok[u]) {
            const uint32_t parts = entry_parts(cnt[u], 1);
            ar[u] = lds_add(&histR[top32(uint32_t(key[u] >> 32), W.logR)], parts);
            ac[u] = lds_add(&histC[top32(uint32_t(key[u]), W.logC)], parts);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (ok[u]) {
            const uint32_t parts = entry_parts(cnt[u], 1);
            write_entry(er, ar[u], uint32_t(key[u] >> 32), cnt[u], 1, parts);
            write_entry(ec, ac[u], uint32_t(key[u]), cnt[u], 1, parts);
          }
        }
        if (P->ent_links) {   // entity outputs: the links themselves
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const u64 row = ent_reserve(P, W.out_index, 0, ok[u]);
            if (ok[u])
              ent_row(P, P->ent_links, W.out_index, 0, row, row_unhash(uint32_t(key[u] >> 32)),
                      row_unhash(uint32_t(key[u])), cnt[u]);
          }
        }
      });
      if (threadIdx.x == 0 && misc[1]) {
        const uint32_t c = misc[1];
        if (P->ent_links) {
          const uint32_t xe = row_unhash(EMPTY32);
          const u64 row = __hip_atomic_fetch_add(P->ent_cur + u64(W.out_index) * 3, 1ull,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ent_row(P, P->ent_links, W.out_index, 0, row, xe, xe, c);
        }
        const uint32_t parts = entry_parts(c, 1);
        write_entry(er, lds_add(&histR[top32(EMPTY32, W.logR)], parts), EMPTY32, c, 1,
                    parts);
        write_entry(ec, lds_add(&histC[top32(EMPTY32, W.logC)], parts), EMPTY32, c, 1,
                    parts);
      }
      __syncthreads();
    };

    // Single-sweep emission with combining.  The bucket's links move to
    // registers (at most LK per thread), the table is emptied, and its region
    // is reused as an id table: ik = id (EMPTY32 when free), ip = complement
    // of the packets (all-ones is 0, so the emptied link table is already an
    // empty id table), il = links.  Each distinct id of the bucket is emitted
    // once with its packets and links; the id EMPTY32 (the table's empty
    // marker) is emitted per link.  If an insert gives up, the pass falls back
    // to emitting every link on its own (links = 1), which phase C sums the
    // same way; nothing has been emitted by then.  The touched slots are reset
    // afterwards, which leaves the region an empty link table again.
    auto combine_emit = [&](bool rows, const u64 (&lkey)[LK], const uint32_t (&lcnt)[LK],
                            uint32_t nl, uint32_t spc) {
      uint32_t* ik = reinterpret_cast<uint32_t*>(tk);
      uint32_t* ip = ik + S;
      uint32_t* il = tc;
      uint32_t* io = occ;
      uint32_t* hist = rows ? histR : histC;
      const uint32_t K = rows ? R : C;
      const uint32_t logK = rows ? W.logR : W.logC;
      auto ident = [&](u64 key) { return rows ? uint32_t(key >> 32) : uint32_t(key); };
      auto bucket = [&](uint32_t x) { return top32(x, logK); };
      for (uint32_t i = threadIdx.x; i <= K; i += NSGC_BLOCK) hist[i] = 0;
      if (threadIdx.x < 2) misc[2 + threadIdx.x] = 0;   // [2] distinct ids, [3] gave up
      __syncthreads();
#pragma unroll
      for (int c = 0; c < LK; c += 4) {
        uint32_t id[4], h[4], pk[4], ln[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          id[k] = ident(lkey[c + k]);
          h[k] = id[k];
          pk[k] = lcnt[c + k];
          ln[k] = 1;
          ok[k] = threadIdx.x + (c + k) * NSGC_BLOCK < nl && id[k] != EMPTY32;
          // combine the lanes holding the first valid lane's id (heavy ids)
          const u64 vm = __ballot(ok[k]);
          if (vm) {
            const int first = __ffsll(static_cast<unsigned long long>(vm)) - 1;
            const uint32_t id0 = readlane(id[k], first);
            const bool same = ok[k] && id[k] == id0;
            const uint32_t nsame = __popcll(__ballot(same));
            if (nsame > 1) {
              const uint32_t tot = wave_sum(same ? pk[k] : 0u);
              if (same) {
                if (int(lane_id()) == first) { pk[k] = tot; ln[k] = nsame; }
                else ok[k] = false;
              }
            }
          }
        }
        int slot[4];
        bool fresh[4];
        if (!cas_insert<4>(ik, S - 1, id, h, ok, slot, fresh, P->combine_probes))
          lds_store(&misc[3], 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (slot[k] >= 0) {
            lds_sub(&ip[slot[k]], pk[k]);
            lds_add(&il[slot[k]], ln[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t at = wave_append(&misc[2], fresh[k]);
          if (fresh[k]) io[at] = uint32_t(slot[k]);
        }
      }
      __syncthreads();
      const uint32_t nd = misc[2];
      const bool combined = misc[3] == 0;
      // entries emitted per link: every link (fallback) or those of id EMPTY32
      auto per_link = [&](int k) {
        return threadIdx.x + k * NSGC_BLOCK < nl && (!combined || ident(lkey[k]) == EMPTY32);
      };
      if (combined) {
        for (uint32_t i = threadIdx.x; i < nd; i += NSGC_BLOCK) {
          const uint32_t s = io[i];
          lds_add(&hist[bucket(ik[s])], entry_parts(~ip[s], il[s]));
        }
      }
#pragma unroll
      for (int k = 0; k < LK; ++k)
        if (per_link(k)) lds_add(&hist[bucket(ident(lkey[k]))], entry_parts(lcnt[k], 1));
      if (threadIdx.x == 0 && spc) lds_add(&hist[bucket(EMPTY32)], entry_parts(spc, 1));
      __syncthreads();
      block_exclusive_scan(hist, K, st.red);
      const u64 rbase = rows ? B : B + u64(R + 1) * B;
      for (uint32_t i = threadIdx.x; i <= K; i += NSGC_BLOCK) rec[rbase + u64(i) * B + b] = hist[i];
      __syncthreads();
      const uint32_t base = misc[4];
      NSGC_GLOBAL u64* e = gptr(rows ? P->emit_row : P->emit_col) + W.ws + base;
      if (combined) {
        for (uint32_t i = threadIdx.x; i < nd; i += NSGC_BLOCK) {
          const uint32_t s = io[i];
          const uint32_t x = ik[s], pk = ~ip[s], ln = il[s];
          const uint32_t parts = entry_parts(pk, ln);
          write_entry(e, lds_add(&hist[bucket(x)], parts), x, pk, ln, parts);
        }
      }
#pragma unroll
      for (int k = 0; k < LK; ++k) {
        if (per_link(k)) {
          const uint32_t x = ident(lkey[k]);
          const uint32_t parts = entry_parts(lcnt[k], 1);
          write_entry(e, lds_add(&hist[bucket(x)], parts), x, lcnt[k], 1, parts);
        }
      }
      if (threadIdx.x == 0 && spc) {
        const uint32_t parts = entry_parts(spc, 1);
        write_entry(e, lds_add(&hist[bucket(EMPTY32)], parts), EMPTY32, spc, 1, parts);
      }
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < nd; i += NSGC_BLOCK) {
        const uint32_t s = io[i];
        ik[s] = EMPTY32;
        ip[s] = EMPTY32;
        il[s] = 0;
      }
      __syncthreads();
    };
    // Counts -> starts (the caller's barrier must follow before emission,
    // whose atomics advance the starts).
    auto publish = [&]() {
      block_exclusive_scan2(histR, R, histC, C, st.red);
      for (uint32_t i = threadIdx.x; i <= R; i += NSGC_BLOCK) rec[B + u64(i) * B + b] = histR[i];
      for (uint32_t i = threadIdx.x; i <= C; i += NSGC_BLOCK)
        rec[B + u64(R + 1) * B + u64(i) * B + b] = histC[i];
    };

    // Attempt with 2^logS sweeps; any insert that gives up restarts the whole
    // bucket with twice the sweeps (the emission is rewritten from scratch).
    // A single sweep counts its links per row and column bucket and emits
    // them packed.  With sweeps, the first sweep's gather counts the bucket's
    // packets per row and column bucket instead: each row (column) bucket's
    // segment gets one slot per packet, the most entries it can receive, so
    // every sweep emits right after its build, and the slots left over hold
    // empty entries (packet count 0), which phase C skips.  The entity
    // outputs list each link once, so there the sweeps first all build and
    // count (pass 0) and then build again to emit (pass 1): a restart never
    // follows a partial emission.
    uint32_t links = 0, sum = 0, mx = 0;
    bool abandoned = false;
    for (uint32_t logS = 0;; ++logS) {
      if (logS > P->max_sweeps_log2) { abandoned = true; break; }
      links = sum = mx = 0;
      for (uint32_t i = threadIdx.x; i < R; i += NSGC_BLOCK) histR[i] = 0;
      for (uint32_t i = threadIdx.x; i < C; i += NSGC_BLOCK) histC[i] = 0;
      bool failed = false;
      const uint32_t passes = logS && P->ent_links ? 2u : 1u;
#pragma nounroll
      for (uint32_t pass = 0; pass < passes && !failed; ++pass) {
        if (pass == 1) {
          publish();
          __syncthreads();
        }
#pragma nounroll
        for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
          // pass 1 rebuilds sweeps that pass 0 showed to fit: it may probe the
          // whole table (chains depend on the order of concurrent inserts)
          build(logS, sw, logS > 0 && sw == 0 && passes == 1, pass ? S : NSGC_MAX_PROBES);
          if (misc[0]) { failed = true; reset(); break; }
          if (pass == 1) {
            emit();
            if (threadIdx.x == 0) misc[5] = 0;   // ordered by the next build's barrier
            continue;
          }
          const uint32_t n = misc[5];
          for (uint32_t i = threadIdx.x; i < n; i += NSGC_BLOCK) {
            const uint32_t c = tc[occ[i]];
            sum += c;
            mx = max(mx, c);
          }
          if (threadIdx.x == 0) {
            links += n;
            if (misc[1]) {
              ++links;
              sum += misc[1];
              mx = max(mx, misc[1]);
            }
          }
          if (logS == 0 && !COMBINE) {
            // the only sweep, emitted per link
            count();
            __syncthreads();
            publish();
            __syncthreads();
            emit();
            if (threadIdx.x == 0) misc[5] = 0;   // ordered by the reduction's barriers
          } else if (COMBINE && logS == 0) {
            // the only sweep: combine per source and per destination, emit
            u64 lkey[LK];
            uint32_t lcnt[LK];
#pragma unroll
            for (int k = 0; k < LK; ++k) {
              const uint32_t i = threadIdx.x + k * NSGC_BLOCK;
              const uint32_t s = i < n ? occ[i] : 0u;
              lkey[k] = i < n ? tk[s] : 0ull;
              lcnt[k] = i < n ? tc[s] : 0u;
            }
            const uint32_t spc = misc[1];
            __syncthreads();
            reset();
            combine_emit(true, lkey, lcnt, n, spc);
            combine_emit(false, lkey, lcnt, n, spc);
          } else if (passes == 2) {
            count();
            __syncthreads();
            reset();
          } else {
            if (sw == 0) {   // the slot counts become the segment starts and cursors
              publish();
              __syncthreads();
              const uint32_t nb = histR[R];   // the bucket's packets: its whole region
              NSGC_GLOBAL u64* er = gptr(P->emit_row) + W.ws + misc[4];
              NSGC_GLOBAL u64* ec = gptr(P->emit_col) + W.ws + misc[4];
              for (uint32_t i = threadIdx.x; i < nb; i += NSGC_BLOCK) {
                er[i] = 0ull;
                ec[i] = 0ull;
              }
              __threadfence_block();   // the empty entries land before any emission
              __syncthreads();
            }
            emit();
            if (threadIdx.x == 0) misc[5] = 0;   // ordered by the next build's barrier
          }
        }
      }
      if (!failed) break;
    }
    if (abandoned) {  // publish empty row/column segments so phase C reads nothing here
      for (uint32_t i = threadIdx.x; i <= R; i += NSGC_BLOCK) rec[B + u64(i) * B + b] = 0;
      for (uint32_t i = threadIdx.x; i <= C; i += NSGC_BLOCK)
        rec[B + u64(R + 1) * B + u64(i) * B + b] = 0;
    }
    if (threadIdx.x == 0) rec[b] = misc[4];

    // the bucket's totals (thread 0 holds them), combined per window by k_finish
    uint32_t nlinks = links;
    block_sum2_max_to0(sum, nlinks, mx, st.red);
    if (threadIdx.x == 0) {
      const v4u32 part = {sum, nlinks, mx, abandoned ? 1u : 0u};
      gptr(reinterpret_cast<v4u32*>(P->partB))[it] = part;
    }
    q.stage_next(items);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Phase B, one wavefront per link bucket (windows whose size class has a
// wave target, see nsgc_tune_class): every wavefront of the grid takes link
// buckets of about wave_target packets from its own work queue and
// aggregates each in a private LDS table.  No wavefront waits for another, so
// the latency of one wavefront's metadata loads, key gathers and LDS round
// trips hides behind the work of the others (up to 24 per compute unit);
// the workgroup-wide barriers of k_links are gone.  Lanes holding the same
// key insert it side by side (the compare-and-swap hands them one slot, and
// the counts add up in LDS): merging them first with ballots measured slower
// on 256-packet buckets.  The emission layout, the overflow sweeps and the
// statistics are the same as k_links' per-link form.
// ---------------------------------------------------------------------------

constexpr int WAVE_NT = 256;                 // threads per workgroup
constexpr int WAVE_WPB = WAVE_NT / 64;       // wavefronts per workgroup
constexpr uint32_t WAVE_SLOTS = 1u << NSGC_WAVE_SLOTS_LOG2;

static_assert(WAVE_SLOTS <= 65536, "slots are listed as 16-bit indices");

constexpr uint32_t WAVE_ROWS = NSGC_WAVE_ROW_SLOTS;

// LDS of one wavefront: keys, counts, the row and column bucket counters
// (`hist` per view: one more than the launch's largest row or column bucket
// count, so that batches of small windows fit more wavefronts per CU), the
// occupied-slot list and, in launches with row-complete windows, the row
// table (hashed source id, links << 20 | packets).  The counts take 2 bytes
// per slot, two slots to a word: a bucket of fewer than 2^16 packets cannot
// carry into its neighbour.  A larger bucket uses half the slots with a full
// word each (same bytes).  The 6.5 KB per wavefront fit 24 wavefronts in a
// compute unit's LDS, against 20 with 4-byte counts.
__host__ __device__ constexpr size_t wave_lds_stride(uint32_t hist, uint32_t rows) {
  return (size_t(WAVE_SLOTS) * 8 + size_t(WAVE_SLOTS) * 2 + 2 * size_t(hist) * 4 +
          size_t(WAVE_SLOTS) * 2 + (rows ? size_t(WAVE_ROWS) * 8 : 0) + 15) &
         ~size_t(15);
}

size_t lds_links_wave_bytes(uint32_t hist, uint32_t rows) {
  return size_t(WAVE_WPB) * wave_lds_stride(hist, rows);
}

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Exclusive scan of a[0..n) in LDS by one wavefront (n <= 64 * 8); a[n]
// receives the total.
__device__ __forceinline__ void wave_exclusive_scan_lds(uint32_t* a, uint32_t n) {
  const uint32_t lane = lane_id();
  const uint32_t per = (n + 63u) >> 6;
  const uint32_t beg = min(n, lane * per), end = min(n, beg + per);
  uint32_t sum = 0;
  for (uint32_t i = beg; i < end; ++i) sum += a[i];
  const uint32_t incl = wave_inclusive_scan(sum);
  uint32_t run = incl - sum;
  for (uint32_t i = beg; i < end; ++i) {
    const uint32_t x = a[i];
    a[i] = run;
    run += x;
  }
  if (lane == 63) a[n] = incl;
  wave_fence();
}

// Work queue of single wavefronts: wavefront g of the grid takes item g
// first, then items of its class (g mod K, K <= NSGC_QCLASSES) from a
// per-class counter; lane 0 requests the next position while the current
// item runs.
struct WaveQueue {
  NSGC_GLOBAL uint32_t* counter;
  const NSGC_GLOBAL uint32_t* map;
  uint32_t base, step, pending;
  __device__ WaveQueue(NSGC_GLOBAL uint32_t* counters, uint32_t gwave, uint32_t gwaves,
                       const NSGC_GLOBAL uint32_t* item_map)
      : map(item_map), pending(0) {
    step = min(uint32_t(NSGC_QCLASSES), gwaves);
    const uint32_t c = gwave % step;
    counter = counters + c * NSGC_QSTRIDE;
    base = gwaves + c;
  }
  __device__ __forceinline__ uint32_t take() {
    return base + step * __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ uint32_t item_at(uint32_t pos, uint32_t items) const {
    return pos < items ? (map ? map[pos] : pos) : NO_ITEM;
  }
  // The first item (position gwave); lane 0 requests the next position.
  __device__ __forceinline__ uint32_t first(uint32_t gwave, uint32_t items) {
    if (lane_id() == 0) pending = gwave < items ? take() : items;
    return uniform(item_at(gwave, items));
  }
  __device__ __forceinline__ uint32_t next(uint32_t items) {
    uint32_t pos = 0;
    if (lane_id() == 0) {
      pos = pending;
      pending = pos < items ? take() : items;
    }
    return uniform(item_at(uniform(pos), items));
  }
};

template <uint32_t NT>
__device__ __forceinline__ void order_items_by_size(const nsgc_dev_plan* P, uint32_t* cursor);

// `order_block`: workgroup 0 orders the phase-C items (see k_order) and the
// others aggregate the link buckets.  ROWS: the batch has row-complete
// windows (row tables in LDS; the other instance carries none of their code).
template <bool ROWS>
__global__ __launch_bounds__(WAVE_NT) void k_links_wave(nsgc_dev_plan* P, uint32_t hist,
                                                        uint32_t order_block) {
  constexpr uint32_t rows = ROWS ? 1u : 0u;
  extern __shared__ __align__(16) unsigned char smem[];
  if (order_block && blockIdx.x == 0) {
    order_items_by_size<WAVE_NT>(P, reinterpret_cast<uint32_t*>(smem));
    return;
  }
  const uint32_t w = uniform(threadIdx.x >> 6), lane = lane_id();
  unsigned char* p = smem + size_t(w) * wave_lds_stride(hist, rows);
  u64* tk = reinterpret_cast<u64*>(p);             p += size_t(WAVE_SLOTS) * 8;
  uint32_t* tc = reinterpret_cast<uint32_t*>(p);   p += size_t(WAVE_SLOTS) * 2;   // see above
  uint32_t* histR = reinterpret_cast<uint32_t*>(p);  p += size_t(hist) * 4;
  uint32_t* histC = reinterpret_cast<uint32_t*>(p);  p += size_t(hist) * 4;
  uint16_t* occ = reinterpret_cast<uint16_t*>(p);    p += size_t(WAVE_SLOTS) * 2;
  uint32_t* rk = reinterpret_cast<uint32_t*>(p);     p += size_t(WAVE_ROWS) * 4;   // if rows
  uint32_t* rv = reinterpret_cast<uint32_t*>(p);
  constexpr uint32_t S = WAVE_SLOTS;
  constexpr uint32_t TCW = WAVE_SLOTS / 2;   // count words

  // Count of slot s, and the empty count words.  A bucket of >= 2^16
  // packets uses slots 0 .. S/2-1 with a word each: cw = 0 (else 1) and
  // cmask = ~0 (else 0xFFFF), uniform, so no path branches on it.
  uint32_t cw = 1, cmask = 0xFFFFu;
  auto tcount = [&](uint32_t s) -> uint32_t {
    return (tc[s >> cw] >> ((s & cw) << 4)) & cmask;
  };
  auto tcount_add = [&](uint32_t s) { lds_add(&tc[s >> cw], 1u << ((s & cw) << 4)); };
  auto tclear = [&]() {
    for (uint32_t i = lane; i < TCW; i += 64) tc[i] = 0;
  };

  for (uint32_t i = lane; i < S; i += 64) tk[i] = EMPTY64;
  tclear();
  if (rows)
    for (uint32_t i = lane; i < WAVE_ROWS; i += 64) {
      rk[i] = EMPTY32;
      rv[i] = 0;
    }
  wave_fence();

  const uint32_t T = 1u << P->tile_log2;
  const uint32_t items = P->itemsBw;
  const uint32_t gwaves = (gridDim.x - order_block) * WAVE_WPB;
  const uint32_t gwave = (blockIdx.x - order_block) * WAVE_WPB + w;
  WaveQueue q(gptr(&P->queue[3][0]), gwave, gwaves, P->mapBw ? gptr(P->mapBw) : nullptr);
  for (uint32_t it = q.first(gwave, items); it != NO_ITEM; it = q.next(items)) {
    const uint32_t wi = sload(P->itemwinB + it);
    const nsgc_win_desc W = sload_words(P->win + wi);
    const uint32_t b = it - sload(P->prefB + wi);
    const uint32_t B = 1u << W.logB, R = 1u << W.logR, C = 1u << W.logC;
    const uint32_t nt = W.ntiles;
    const NSGC_GLOBAL u64* keys = gptr(P->keys) + W.ws;
    const NSGC_GLOBAL uint32_t* tm0 = gptr(P->tilemeta) + W.tilemeta + u64(b) * nt;
    NSGC_GLOBAL uint32_t* rec = gptr(P->lbmeta) + W.lbmeta;

    // The bucket's starts and ends in the first 64 tiles (lane = tile), loaded
    // once for every build of the item; the emission base of bucket b is the
    // sum of its starts over all tiles.
    uint32_t a0 = 0, c0 = 0;
    if (lane < nt) {
      a0 = tm0[lane];
      c0 = tm0[lane + nt];
    }
    uint32_t below = a0;
    for (uint32_t t = 64 + lane; t < nt; t += 64) below += tm0[t];
    below = uniform(wave_sum(below));
    uint32_t smask = S - 1;   // the table's slots - 1 (set by each build)

    uint32_t n = 0;        // occupied slots (uniform)
    uint32_t special = 0;  // packets of the key equal to the empty marker (uniform)
    uint32_t links = 0, sum = 0, mx = 0;   // the bucket's statistics
    uint32_t pk = 0;       // the bucket's packets (uniform)
    // Row-complete window, single table: the bucket's links are combined per
    // source in the row table; sources at home here are complete (their
    // totals go to partR), the others leave one entry each.  Per-link row
    // entries otherwise, and always for the id EMPTY32 (the table's marker).
    const bool rowc = rows && W.rows;
    bool local = false;
    uint32_t nrows = 0, rmaxp = 0, rmaxl = 0;   // complete sources: count and maxima

    // Link table of sweep `sw` of 2^logS; false if an insert gave up (after
    // `probes` probes).
    auto build = [&](uint32_t logS, uint32_t sw, uint32_t probes) -> bool {
      n = 0;
      special = 0;
      pk = 0;
      bool gave_up = false;
      bool first = true;
      for (uint32_t g0 = 0; g0 < nt; g0 += 64) {
        const uint32_t t = g0 + lane;
        u64 mb = 0;
        uint32_t len = 0;
        if (t < nt) {
          const uint32_t a = g0 == 0 ? a0 : tm0[t], c = g0 == 0 ? c0 : tm0[t + nt];
          mb = u64(t) * T + a;
          len = c - a;
        }
        // walk the concatenation of the group's segments, 64 keys per chunk
        const uint32_t incl = wave_inclusive_scan(len);
        const uint32_t elems = uniform(readlane(incl, 63));
        pk += elems;
        if (first) {   // 16-bit counts unless the bucket may reach 2^16 packets
          first = false;
          const bool wide = nt > 64 || elems >= 65536u;
          cw = wide ? 0u : 1u;
          cmask = wide ? ~0u : 0xFFFFu;
          smask = wide ? S / 2 - 1 : S - 1;
          probes = min(probes, smask + 1);
        }
        const uint32_t start = incl - len;      // exclusive prefix: the segment's first element
        const u64 nonempty = __ballot(len > 0);
        mb -= start;                            // base minus exclusive prefix
        for (uint32_t v0 = 0; v0 < elems; v0 += 64 * LINK_MAXU) {
          u64 key[LINK_MAXU];
          uint32_t h[LINK_MAXU];
          bool ok[LINK_MAXU];
#pragma unroll
          for (int u = 0; u < LINK_MAXU; ++u) {
            const uint32_t vc = v0 + uint32_t(u) * 64u;   // the chunk's first element
            const uint32_t v = vc + lane;
            ok[u] = v < elems;
            u64 pos = 0;
            if (vc < elems) {
              // the non-empty segments holding the chunk's first and last elements
              const uint32_t last = min(vc + 63u, elems - 1u);
              const int jlo = 63 - __clzll(__ballot(start <= vc) & nonempty);
              const int jhi = 63 - __clzll(__ballot(start <= last) & nonempty);
              if (jhi - jlo <= 8) {
                // few segments: walk them with uniform lane reads (no LDS)
                u64 base = (u64(readlane(uint32_t(mb >> 32), jlo)) << 32) |
                           readlane(uint32_t(mb), jlo);
                for (int k = jlo + 1; k <= jhi; ++k) {
                  const uint32_t sk = readlane(start, k);
                  const u64 bk = (u64(readlane(uint32_t(mb >> 32), k)) << 32) |
                                 readlane(uint32_t(mb), k);
                  if (v >= sk) base = bk;
                }
                pos = base + v;
              } else {
                // many short segments: each lane finds its own by a binary search
                uint32_t j = 0;
#pragma unroll
                for (uint32_t st = 32; st > 0; st >>= 1)
                  if (lane_take(incl, j + st - 1) <= v) j += st;
                pos = ((u64(lane_take(uint32_t(mb >> 32), j)) << 32) |
                       lane_take(uint32_t(mb), j)) + v;
              }
            }
            const u64 kk = keys[ok[u] ? pos : 0ull];   // position 0 exists; masked below
            key[u] = ok[u] ? kk : 0ull;
          }
#pragma unroll
          for (int u = 0; u < LINK_MAXU; ++u) {
            const u64 hh = link_pos(key[u]);
            h[u] = uint32_t(hh);
            ok[u] = ok[u] && !(logS && next64(hh, W.logB, logS) != sw);
            const bool spc = ok[u] && key[u] == EMPTY64;
            special += __popcll(__ballot(spc));
            if (spc) ok[u] = false;
          }
          int slot[LINK_MAXU];
          bool fresh[LINK_MAXU];
          if (!cas_insert<LINK_MAXU>(tk, smask, key, h, ok, slot, fresh, probes))
            gave_up = true;
#pragma unroll
          for (int u = 0; u < LINK_MAXU; ++u)
            if (slot[u] >= 0) tcount_add(uint32_t(slot[u]));
#pragma unroll
          for (int u = 0; u < LINK_MAXU; ++u) {
            const u64 m = __ballot(fresh[u]);
            if (fresh[u]) occ[n + rank_below(m)] = uint16_t(slot[u]);
            n += __popcll(m);
          }
        }
      }
      wave_fence();
      return !__ballot(gave_up);
    };

    auto reset = [&]() {
      for (uint32_t i = lane; i < n; i += 64) tk[occ[i]] = EMPTY64;
      tclear();
      n = 0;
      wave_fence();
    };

    // the statistics of the table's links and their entries per row and
    // column bucket
    auto count = [&]() {
      for (uint32_t i = lane; i < n; i += 64) {
        const uint32_t s = occ[i];
        const uint32_t c = tcount(s);
        sum += c;
        mx = max(mx, c);
        const u64 key = tk[s];
        const uint32_t parts = entry_parts(c, 1);
        const uint32_t r = uint32_t(key >> 32);
        if (!local || r == EMPTY32) lds_add(&histR[top32(r, W.logR)], parts);
        lds_add(&histC[top32(uint32_t(key), W.logC)], parts);
      }
      links += n + (special ? 1u : 0u);
      if (lane == 0 && special) {
        sum += special;
        mx = max(mx, special);
        const uint32_t parts = entry_parts(special, 1);
        lds_add(&histR[top32(EMPTY32, W.logR)], parts);
        lds_add(&histC[top32(EMPTY32, W.logC)], parts);
      }
      if (local) {
        // sources at home in bucket b are complete; the others leave an entry
        for (uint32_t i = lane; i < WAVE_ROWS; i += 64) {
          const uint32_t r = rk[i];
          if (r == EMPTY32) continue;
          const uint32_t v = rv[i], np = v & 0xFFFFFu, nl = v >> 20;
          if (top32(r, W.logB) == b) {
            ++nrows;
            rmaxp = max(rmaxp, np);
            rmaxl = max(rmaxl, nl);
          } else {
            lds_add(&histR[top32(r, W.logR)], entry_parts(np, nl));
          }
        }
      }
      wave_fence();
    };

    // The table's links per source into the row table (packets < 2^20 per
    // bucket, so links << 20 | packets cannot carry).  False, with the row
    // table emptied, if a source finds no slot within NSGC_MAX_PROBES probes.
    auto rows_build = [&]() -> bool {
      bool failed = false;
      for (uint32_t i0 = 0; i0 < n; i0 += 64) {
        const uint32_t i = i0 + lane;
        if (i < n) {
          const uint32_t s = occ[i];
          const uint32_t r = uint32_t(tk[s] >> 32);
          if (r != EMPTY32) {
            uint32_t at = r & (WAVE_ROWS - 1);
            int got = -1;
            for (uint32_t q = 0; q < NSGC_MAX_PROBES; ++q) {
              const uint32_t o = lds_cas32(&rk[at], EMPTY32, r);
              if (o == EMPTY32 || o == r) {
                got = int(at);
                break;
              }
              at = (at + 1) & (WAVE_ROWS - 1);
            }
            if (got >= 0) lds_add(&rv[got], (1u << 20) | tcount(s));
            else failed = true;
          }
        }
        if (__ballot(failed)) break;
      }
      const bool bad = __ballot(failed) != 0;
      if (bad)
        for (uint32_t i = lane; i < WAVE_ROWS; i += 64) {
          rk[i] = EMPTY32;
          rv[i] = 0;
        }
      wave_fence();
      return !bad;
    };

    // counts -> starts, published for phase C (and the phase-C sizes)
    auto publish = [&]() {
      wave_exclusive_scan_lds(histR, R);
      wave_exclusive_scan_lds(histC, C);
      for (uint32_t i = lane; i <= R; i += 64) rec[B + u64(i) * B + b] = histR[i];
      for (uint32_t i = lane; i <= C; i += 64) rec[B + u64(R + 1) * B + u64(i) * B + b] = histC[i];
    };

    // entries at the counted positions; empties the table
    auto emit = [&]() {
      NSGC_GLOBAL u64* er = gptr(P->emit_row) + W.ws + below;
      NSGC_GLOBAL u64* ec = gptr(P->emit_col) + W.ws + below;
      for (uint32_t i = lane; i < n; i += 64) {
        const uint32_t s = occ[i];
        const u64 key = tk[s];
        const uint32_t cnt = tcount(s);
        tk[s] = EMPTY64;
        const uint32_t parts = entry_parts(cnt, 1);
        const uint32_t r = uint32_t(key >> 32);
        if (!local || r == EMPTY32) {
          const uint32_t ar = lds_add(&histR[top32(r, W.logR)], parts);
          write_entry(er, ar, r, cnt, 1, parts);
        }
        const uint32_t ac = lds_add(&histC[top32(uint32_t(key), W.logC)], parts);
        write_entry(ec, ac, uint32_t(key), cnt, 1, parts);
        if (P->ent_links) {   // entity outputs: the links themselves
          const u64 row = ent_reserve(P, W.out_index, 0, true);
          ent_row(P, P->ent_links, W.out_index, 0, row, row_unhash(uint32_t(key >> 32)),
                  row_unhash(uint32_t(key)), cnt);
        }
      }
      if (lane == 0 && special) {
        if (P->ent_links) {
          const uint32_t xe = row_unhash(EMPTY32);
          const u64 row = __hip_atomic_fetch_add(P->ent_cur + u64(W.out_index) * 3, 1ull,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ent_row(P, P->ent_links, W.out_index, 0, row, xe, xe, special);
        }
        const uint32_t parts = entry_parts(special, 1);
        write_entry(er, lds_add(&histR[top32(EMPTY32, W.logR)], parts), EMPTY32, special, 1, parts);
        write_entry(ec, lds_add(&histC[top32(EMPTY32, W.logC)], parts), EMPTY32, special, 1, parts);
      }
      if (local) {   // one entry per source away from home; empties the row table
        for (uint32_t i = lane; i < WAVE_ROWS; i += 64) {
          const uint32_t r = rk[i];
          if (r == EMPTY32) continue;
          const uint32_t v = rv[i];
          rk[i] = EMPTY32;
          rv[i] = 0;
          if (top32(r, W.logB) != b) {
            const uint32_t np = v & 0xFFFFFu, nl = v >> 20, parts = entry_parts(np, nl);
            write_entry(er, lds_add(&histR[top32(r, W.logR)], parts), r, np, nl, parts);
          }
        }
      }
      tclear();   // after every read of the counts above (one wavefront, in order)
      n = 0;
      wave_fence();
    };

    bool abandoned = false;
    for (uint32_t logS = 0;; ++logS) {
      if (logS > P->max_sweeps_log2) { abandoned = true; break; }
      links = sum = mx = 0;
      nrows = rmaxp = rmaxl = 0;
      local = false;
      for (uint32_t i = lane; i <= R; i += 64) histR[i] = 0;
      for (uint32_t i = lane; i <= C; i += 64) histC[i] = 0;
      wave_fence();
      bool failed = false;
      const uint32_t passes = logS ? 2u : 1u;
      for (uint32_t pass = 0; pass < passes && !failed; ++pass) {
        if (pass == 1) publish();
        for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
          // pass 1 rebuilds sweeps that pass 0 showed to fit: it may probe the
          // whole table (chains depend on the order of concurrent inserts)
          if (!build(logS, sw, pass ? S : NSGC_MAX_PROBES)) { failed = true; reset(); break; }
          if (pass == 1) { emit(); continue; }
          if (logS == 0) local = rowc && pk < (1u << 20) && rows_build();
          count();
          if (logS == 0) {
            publish();
            emit();
          } else {
            reset();
          }
        }
      }
      if (!failed) break;
    }
    if (abandoned) {   // empty row/column segments, so phase C reads nothing here
      for (uint32_t i = lane; i <= R; i += 64) rec[B + u64(i) * B + b] = 0;
      for (uint32_t i = lane; i <= C; i += 64) rec[B + u64(R + 1) * B + u64(i) * B + b] = 0;
    }
    if (lane == 0) rec[b] = below;
    sum = wave_sum(sum);
    mx = wave_max(mx);
    if (lane == 0) {   // the bucket's totals, combined per window by k_finish
      const v4u32 part = {sum, links, mx, abandoned ? 1u : 0u};
      gptr(reinterpret_cast<v4u32*>(P->partB))[it] = part;
    }
    if (rowc) {   // the bucket's complete sources
      nrows = wave_sum(nrows);
      rmaxp = wave_max(rmaxp);
      rmaxl = wave_max(rmaxl);
      if (lane == 0) {
        const v4u32 part = {nrows, rmaxp, rmaxl, 0u};
        gptr(reinterpret_cast<v4u32*>(P->partR))[it] = part;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Order of the phase-C items, largest first (approximately: by half-octave
// classes of the entry count, a counting sort over 65 classes).
// A row bucket that holds a dominant source takes several times longer than
// the others; the work queue hands positions out in order, so large items
// start at once instead of possibly last, where they would set the kernel's
// end.  This matters when the grid gets a few items per workgroup, so the
// plan asks for it only for batches of at most NSGC_ORDER_MAX items (else
// the kernel returns and phase C takes the items in their own order).  One
// workgroup counts and then places the items, each thread a contiguous run
// of them.  The sizes come from the partition alone, so when the batch has
// wavefront phase-B items the first workgroup of k_links_wave does this
// beside phase B; otherwise k_order runs after phase B.  The result is a
// permutation of the items, which is all that the correctness of phase C
// depends on.
// ---------------------------------------------------------------------------

// 0 for empty items, else 1 + 2 floor(log2(size)) + the bit below the leading one
constexpr uint32_t ORDER_CLASSES = 65;

__device__ __forceinline__ uint32_t order_class(uint32_t v) {
  if (!v) return 0u;
  const uint32_t lg = 31u - uint32_t(__builtin_clz(v));
  return 1u + 2u * lg + (lg ? (v >> (lg - 1u)) & 1u : 0u);
}

// The ordering by one workgroup of NT threads, `cursor` in LDS
// (ORDER_CLASSES words): a count pass and a placement pass over the sizes,
// each thread taking a contiguous run of items (read twice, from L2).
template <uint32_t NT>
__device__ __forceinline__ void order_items_by_size(const nsgc_dev_plan* P, uint32_t* cursor) {
  const uint32_t n = P->itemsC;
  if (!P->order_items || n == 0) return;
  const NSGC_GLOBAL uint32_t* sz = gptr(P->rcsize);
  NSGC_GLOBAL uint32_t* order = gptr(P->order);
  for (uint32_t c = threadIdx.x; c < ORDER_CLASSES; c += NT) cursor[c] = 0;
  __syncthreads();
  const uint32_t per = (n + NT - 1) / NT;
  const uint32_t beg = min(n, threadIdx.x * per), end = min(n, beg + per);
  for (uint32_t i = beg; i < end; ++i) lds_add(&cursor[order_class(sz[i])], 1);
  __syncthreads();
  if (threadIdx.x == 0) {   // class starts, largest class first
    uint32_t run = 0;
    for (int c = int(ORDER_CLASSES) - 1; c >= 0; --c) {
      const uint32_t k = cursor[c];
      cursor[c] = run;
      run += k;
    }
  }
  __syncthreads();
  for (uint32_t i = beg; i < end; ++i) order[lds_add(&cursor[order_class(sz[i])], 1)] = i;
}

__global__ __launch_bounds__(NSGC_BLOCK) void k_order(nsgc_dev_plan* P) {
  __shared__ uint32_t cursor[ORDER_CLASSES];
  order_items_by_size<NSGC_BLOCK>(P, cursor);
}

// ---------------------------------------------------------------------------
// Phase C: aggregation of one row bucket (or column bucket).
//
// Gathers the bucket's (id, packets, links) entries -- one per link, or one
// per id and link bucket with combining -- from every link bucket into an LDS
// table id -> (packets, links): summing them yields r(s) and f(s) (or c(d)
// and g(d)) for every id of the bucket, hence its share of stats 3-5 (or
// 6-8).  Entries that repeat the first valid lane's id are pre-combined with
// one ballot and DPP sums.  One pass over the table folds the occupied slots
// into the statistics and empties it, and overflow splits the bucket into
// sweeps by id-hash bits.  Items are taken largest first when phase B's
// sizes were ordered (see k_order).
// ---------------------------------------------------------------------------

size_t lds_rc_bytes(uint32_t slots_log2) {
  const size_t S = size_t(1) << slots_log2;
  return align16(S * 4) + align16(S * 8) + 256;
}

__global__ __launch_bounds__(NSGC_BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_rowcol(nsgc_dev_plan* P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t S = 1u << P->rc_slots_log2;
  unsigned char* p = smem;
  uint32_t* tk = reinterpret_cast<uint32_t*>(p);       p += align16(S * 4);
  // per slot: links << 32 | packets, one 64-bit add per entry (neither half
  // carries: a bucket's packets and links stay below 2^32)
  u64* tv = reinterpret_cast<u64*>(p);                 p += align16(S * 8);
  struct { uint32_t* red; } st;                        // reduction scratch (in misc)
  uint32_t* misc = reinterpret_cast<uint32_t*>(p);     // [0] fail flag, [2,3] special id,
                                                       // [7] queue slot
  st.red = misc + 8;

  for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
    tk[i] = EMPTY32;
    tv[i] = 0;
  }

  const uint32_t items = P->itemsC;
  const uint32_t wave = uniform(threadIdx.x >> 6), lane = lane_id();
  // The first group of an item's segments (lane l of wave w: link bucket
  // w + WAVES * l), loaded for the next item while the current one finishes.
  auto load_first = [&](uint32_t it, SegPre& pre) {
    const uint32_t wi = sload(P->itemwinC + it);
    const nsgc_win_desc W = sload_words(P->win + wi);
    const uint32_t k = it - sload(P->prefC + wi);
    const uint32_t B = 1u << W.logB, R = 1u << W.logR;
    const bool is_row = k < R;
    const NSGC_GLOBAL uint32_t* rec = gptr(P->lbmeta) + W.lbmeta;
    const NSGC_GLOBAL uint32_t* st0 =
        rec + B + (is_row ? u64(k) * B : u64(R + 1) * B + u64(k - R) * B);
    const uint32_t lb = wave + uint32_t(WAVES) * lane;
    pre.base = 0;
    pre.len = 0;
    if (lb < B) {
      const uint32_t s0 = st0[lb], s1 = st0[lb + B];
      pre.base = u64(rec[lb]) + s0;
      pre.len = s1 - s0;
    }
  };
  SegPre next_pre = {0, 0};
  bool have_next = false;

  ItemQueue q(gptr(&P->queue[2][0]), misc + 7, NSGC_QCLASSES,
              P->order_items ? gptr(P->order) : nullptr);
  for (uint32_t item = q.first(items); item != NO_ITEM; item = q.read()) {
    const uint32_t it = uniform(item);
    const uint32_t wi = sload(P->itemwinC + it);
    const nsgc_win_desc W = sload_words(P->win + wi);
    const uint32_t k = it - sload(P->prefC + wi);
    const uint32_t B = 1u << W.logB, R = 1u << W.logR;
    const bool is_row = k < R;
    const uint32_t bucket = is_row ? k : k - R;
    const uint32_t logK = is_row ? W.logR : W.logC;
    const NSGC_GLOBAL uint32_t* rec = gptr(P->lbmeta) + W.lbmeta;
    const NSGC_GLOBAL uint32_t* st0 =
        rec + B + (is_row ? u64(bucket) * B : u64(R + 1) * B + u64(bucket) * B);
    const NSGC_GLOBAL uint32_t* st1 = st0 + B;
    const NSGC_GLOBAL u64* em = gptr(is_row ? P->emit_row : P->emit_col) + W.ws;

    SegPre pre;
    if (have_next) pre = next_pre;
    else load_first(it, pre);
    have_next = false;
    // thread 0 starts looking up the next item (its order entry) now and
    // names it to the workgroup at the end of the gather
    q.resolve(items);
    bool fetched = false;

    auto seg = [&](uint32_t lb, u64& base, uint32_t& len) {
      const uint32_t s0 = st0[lb], s1 = st1[lb];
      base = u64(rec[lb]) + s0;
      len = s1 - s0;
    };

    // One pass over every slot (16-byte LDS accesses): fold the occupied
    // slots into the statistics when `take`, and empty the table.  Tables of
    // <= 8192 slots make this a few accesses per thread, cheaper than keeping
    // a list of occupied slots in the inserts.
    uint32_t n = 0, mp = 0, ml = 0;
    auto harvest = [&](bool take) {
      const v4u32 empty4 = {EMPTY32, EMPTY32, EMPTY32, EMPTY32};
      const v4u32 zero4 = {0u, 0u, 0u, 0u};
      for (uint32_t i = threadIdx.x * 4; i < S; i += NSGC_BLOCK * 4) {
        const v4u32 k4 = *reinterpret_cast<const v4u32*>(tk + i);
        if (take) {
          const v4u32 v01 = *reinterpret_cast<const v4u32*>(tv + i);       // slots i, i + 1
          const v4u32 v23 = *reinterpret_cast<const v4u32*>(tv + i + 2);   // slots i + 2, i + 3
          const uint32_t ks[4] = {k4.x, k4.y, k4.z, k4.w};
          const uint32_t as[4] = {v01.x, v01.z, v23.x, v23.z};   // packets
          const uint32_t bs[4] = {v01.y, v01.w, v23.y, v23.w};   // links
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (ks[j] != EMPTY32) {
              ++n;
              mp = max(mp, as[j]);
              ml = max(ml, bs[j]);
            }
          }
        }
        *reinterpret_cast<v4u32*>(tk + i) = empty4;
        *reinterpret_cast<v4u32*>(tv + i) = zero4;
        *reinterpret_cast<v4u32*>(tv + i + 2) = zero4;
      }
      __syncthreads();
    };

    auto build = [&](uint32_t logS, uint32_t sw) {
      if (threadIdx.x < 4) misc[threadIdx.x] = 0;
      __syncthreads();
      gather_by_wave<RC_MAXU>(B, seg, [&](const auto& pos, const auto& okin) {
        constexpr int U = array_len<decltype(pos)>();
        uint32_t id[U], h[U], pk[U], ln[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const u64 ee = em[okin[u] ? pos[u] : 0ull];   // position 0 exists; masked below
          const u64 e = okin[u] ? ee : 0ull;
          id[u] = uint32_t(e >> 32);
          pk[u] = uint32_t(e) & ENT_PMAX;
          ln[u] = uint32_t(e) >> NSGC_ENT_PACKET_BITS;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          h[u] = id[u];
          // (an entry with no packets is an unused slot of a swept link bucket)
          ok[u] = okin[u] && pk[u] != 0 && !(logS && next32(h[u], logK, logS) != sw);
          if (ok[u] && id[u] == EMPTY32) {
            lds_add(&misc[2], pk[u]);
            lds_add(&misc[3], ln[u]);
            ok[u] = false;
          }
          // combine the lanes holding the first valid lane's id
          const u64 vm = __ballot(ok[u]);
          if (vm) {
            const int first = __ffsll(static_cast<unsigned long long>(vm)) - 1;
            const uint32_t id0 = readlane(id[u], first);
            const bool same = ok[u] && id[u] == id0;
            const uint32_t nsame = __popcll(__ballot(same));
            if (nsame > 1) {
              const uint32_t tot = wave_sum(same ? pk[u] : 0u);
              const uint32_t lns = wave_sum(same ? ln[u] : 0u);
              if (same) {
                if (int(lane_id()) == first) { pk[u] = tot; ln[u] = lns; }
                else ok[u] = false;
              }
            }
          }
        }
        int slot[U];
        bool fresh[U];
        if (!cas_insert<U>(tk, S - 1, id, h, ok, slot, fresh, NSGC_MAX_PROBES))
          lds_store(&misc[0], 1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (slot[u] >= 0) {
            lds_add64(&tv[slot[u]], (u64(ln[u]) << 32) | pk[u]);
          }
        }
        (void)fresh;
      }, &pre, [&]() {
        if (threadIdx.x == 0 && !fetched) misc[6] = q.pending_item;
      });
      if (!fetched) {   // the next item's first segments, loaded behind this item
        fetched = true;
        const uint32_t nx = uniform(misc[6]);
        if (nx != NO_ITEM) {
          load_first(nx, next_pre);
          have_next = true;
        }
      }
    };

    bool abandoned = false;
    for (uint32_t logS = 0;; ++logS) {
      if (logS > P->max_sweeps_log2) { abandoned = true; break; }
      n = mp = ml = 0;
      bool failed = false;
      for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
        build(logS, sw);
        if (misc[0]) { failed = true; harvest(false); break; }
        harvest(true);
        if (threadIdx.x == 0) {
          if (misc[3]) {
            ++n;
            mp = max(mp, misc[2]);
            ml = max(ml, misc[3]);
          }
        }
      }
      if (!failed) break;
    }
    block_sum_max2_to0(n, mp, ml, st.red);   // thread 0 holds the bucket's totals
    if (threadIdx.x == 0) {   // combined per window by k_finish
      const v4u32 part = {n, mp, ml, abandoned ? 1u : 0u};
      gptr(reinterpret_cast<v4u32*>(P->partC))[it] = part;
    }
    q.stage_next(items);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Phase C for the entity outputs: item b of a window aggregates row bucket b
// and column bucket b together (in entity mode destinations are hashed like
// sources and R = C, so both buckets cover the same hashed addresses).  Two
// LDS tables, one per view, give the bucket totals as in k_rowcol, the rows
// of the source and destination lists, and the bucket's share of the union
// |sources U destinations|: its sources plus its destinations that are not
// also sources.  Overflow sweeps split both views by the same id bits.  The
// lists are written only by a pass whose sweeps all fit: a single sweep
// writes as it goes; with more sweeps, a second pass over the final sweeps
// writes after a first one has found how many are needed.  The column
// positions of the queue have no work of their own.
// ---------------------------------------------------------------------------

size_t lds_rc_ent_bytes(uint32_t slots_log2) {
  const size_t S = size_t(1) << slots_log2;
  return align16(S * 4) * 6 + 256;
}

__global__ __launch_bounds__(NSGC_BLOCK) void k_rowcol_ent(nsgc_dev_plan* P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t S = 1u << P->rc_slots_log2;
  unsigned char* p = smem;
  uint32_t* tkv[2];
  uint32_t* tav[2];
  uint32_t* tbv[2];
  for (int v = 0; v < 2; ++v) {
    tkv[v] = reinterpret_cast<uint32_t*>(p);  p += align16(S * 4);
    tav[v] = reinterpret_cast<uint32_t*>(p);  p += align16(S * 4);
    tbv[v] = reinterpret_cast<uint32_t*>(p);  p += align16(S * 4);
  }
  uint32_t* misc = reinterpret_cast<uint32_t*>(p);   // [0] fail flag, [2,3] special row,
                                                     // [4,5] special column, [7] queue slot
  uint32_t* red = misc + 8;

  for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
    for (int v = 0; v < 2; ++v) {
      tkv[v][i] = EMPTY32;
      tav[v][i] = 0;
      tbv[v][i] = 0;
    }
  }

  const uint32_t items = P->itemsC;
  ItemQueue q(gptr(&P->queue[2][0]), misc + 7, NSGC_QCLASSES);
  for (uint32_t item = q.first(items); item != NO_ITEM; item = q.read()) {
    const uint32_t it = uniform(item);
    const uint32_t wi = sload(P->itemwinC + it);
    const nsgc_win_desc W = sload_words(P->win + wi);
    const uint32_t k = it - sload(P->prefC + wi);
    const uint32_t B = 1u << W.logB, R = 1u << W.logR;
    if (k >= R) {   // a column position: handled with row item k - R
      q.stage_next(items);
      __syncthreads();
      continue;
    }
    const uint32_t w = W.out_index;
    const uint32_t logK = W.logR;
    const NSGC_GLOBAL uint32_t* rec = gptr(P->lbmeta) + W.lbmeta;

    // Table of view v (0 rows, 1 columns) for sweep sw of 2^logS; an insert
    // gives up after `probes` probes.
    auto build = [&](int v, uint32_t logS, uint32_t sw, uint32_t probes) {
      const NSGC_GLOBAL uint32_t* st0 = rec + B + (v == 0 ? u64(k) * B : u64(R + 1) * B + u64(k) * B);
      const NSGC_GLOBAL uint32_t* st1 = st0 + B;
      const NSGC_GLOBAL u64* em = gptr(v == 0 ? P->emit_row : P->emit_col) + W.ws;
      uint32_t* tk = tkv[v];
      uint32_t* ta = tav[v];
      uint32_t* tb = tbv[v];
      uint32_t* spc = misc + 2 + 2 * v;
      auto seg = [&](uint32_t lb, u64& base, uint32_t& len) {
        const uint32_t s0 = st0[lb], s1 = st1[lb];
        base = u64(rec[lb]) + s0;
        len = s1 - s0;
      };
      gather_by_wave<RC_MAXU>(B, seg, [&](const auto& pos, const auto& okin) {
        constexpr int U = array_len<decltype(pos)>();
        uint32_t id[U], h[U], pk[U], ln[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const u64 ee = em[okin[u] ? pos[u] : 0ull];   // position 0 exists; masked below
          const u64 e = okin[u] ? ee : 0ull;
          id[u] = uint32_t(e >> 32);
          pk[u] = uint32_t(e) & ENT_PMAX;
          ln[u] = uint32_t(e) >> NSGC_ENT_PACKET_BITS;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          h[u] = id[u];
          // (an entry with no packets is an unused slot of a swept link bucket)
          ok[u] = okin[u] && pk[u] != 0 && !(logS && next32(h[u], logK, logS) != sw);
          if (ok[u] && id[u] == EMPTY32) {
            lds_add(&spc[0], pk[u]);
            lds_add(&spc[1], ln[u]);
            ok[u] = false;
          }
        }
        int slot[U];
        bool fresh[U];
        if (!cas_insert<U>(tk, S - 1, id, h, ok, slot, fresh, probes))
          lds_store(&misc[0], 1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (slot[u] >= 0) {
            lds_add(&ta[slot[u]], pk[u]);
            lds_add(&tb[slot[u]], ln[u]);
          }
        }
        (void)fresh;
      });
    };

    // One pass over both tables: the totals (when `stats`), the list rows
    // and the union share (when `write`), and emptying the tables.
    uint32_t nr = 0, mr = 0, mf = 0, nc = 0, mc = 0, mg = 0, uni = 0;
    auto harvest = [&](bool stats, bool write) {
      for (uint32_t i0 = 0; i0 < S; i0 += NSGC_BLOCK) {
        const uint32_t i = i0 + threadIdx.x;
        const uint32_t rid = tkv[0][i], cid = tkv[1][i];
        const bool r = rid != EMPTY32, c = cid != EMPTY32;
        if (stats) {
          if (r) { ++nr; mr = max(mr, tav[0][i]); mf = max(mf, tbv[0][i]); }
          if (c) { ++nc; mc = max(mc, tav[1][i]); mg = max(mg, tbv[1][i]); }
        }
        if (write) {
          if (r) ++uni;
          if (c && !lds_find32(tkv[0], S - 1, cid)) ++uni;
          if (P->ent_src) {
            const u64 row = ent_reserve(P, w, 1, r);
            if (r) ent_row(P, P->ent_src, w, 1, row, row_unhash(rid), tav[0][i], tbv[0][i]);
          }
          if (P->ent_dst) {
            const u64 row = ent_reserve(P, w, 2, c);
            if (c) ent_row(P, P->ent_dst, w, 2, row, row_unhash(cid), tav[1][i], tbv[1][i]);
          }
        }
      }
      if (threadIdx.x == 0) {   // the hashed id EMPTY32 lives outside the tables
        if (stats) {
          if (misc[3]) { ++nr; mr = max(mr, misc[2]); mf = max(mf, misc[3]); }
          if (misc[5]) { ++nc; mc = max(mc, misc[4]); mg = max(mg, misc[5]); }
        }
        if (write) {
          const uint32_t xe = row_unhash(EMPTY32);
          if (misc[3] || misc[5]) ++uni;
          if (misc[3] && P->ent_src) {
            const u64 row = __hip_atomic_fetch_add(P->ent_cur + u64(w) * 3 + 1, 1ull,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ent_row(P, P->ent_src, w, 1, row, xe, misc[2], misc[3]);
          }
          if (misc[5] && P->ent_dst) {
            const u64 row = __hip_atomic_fetch_add(P->ent_cur + u64(w) * 3 + 2, 1ull,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ent_row(P, P->ent_dst, w, 2, row, xe, misc[4], misc[5]);
          }
        }
      }
      __syncthreads();   // lookups done before the tables are emptied
      for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
        for (int v = 0; v < 2; ++v) {
          tkv[v][i] = EMPTY32;
          tav[v][i] = 0;
          tbv[v][i] = 0;
        }
      }
      __syncthreads();
    };

    auto sweep = [&](uint32_t logS, uint32_t sw, uint32_t probes) -> bool {
      if (threadIdx.x < 6) misc[threadIdx.x] = 0;
      __syncthreads();
      build(0, logS, sw, probes);
      build(1, logS, sw, probes);   // ends with a barrier
      return misc[0] == 0;
    };

    bool abandoned = false;
    uint32_t logS = 0;
    for (;; ++logS) {   // the totals, and the lists when a single sweep fits
      if (logS > P->max_sweeps_log2) { abandoned = true; break; }
      nr = mr = mf = nc = mc = mg = uni = 0;
      bool failed = false;
      for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
        if (!sweep(logS, sw, NSGC_MAX_PROBES)) { failed = true; harvest(false, false); break; }
        harvest(true, logS == 0);
      }
      if (!failed) break;
    }
    // The lists over the sweeps now known to fit.  Probe chains depend on the
    // order of concurrent inserts, so a rebuild may probe the whole table: it
    // then always succeeds, as each sweep holds at most S ids.
    if (!abandoned && logS > 0)
      for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
        sweep(logS, sw, S);
        harvest(false, true);
      }
    uint32_t zero = 0;
    block_sum_max2_to0(nr, mr, mf, red);
    __syncthreads();
    block_sum_max2_to0(nc, mc, mg, red);
    __syncthreads();
    block_sum_max2_to0(uni, zero, zero, red);
    if (threadIdx.x == 0) {
      const v4u32 pr = {nr, mr, mf, abandoned ? 1u : 0u};
      const v4u32 pc = {nc, mc, mg, abandoned ? 1u : 0u};
      gptr(reinterpret_cast<v4u32*>(P->partC))[it] = pr;
      gptr(reinterpret_cast<v4u32*>(P->partC))[it + R] = pc;
      gptr(P->partU)[it] = uni;
    }
    q.stage_next(items);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-window statistics of the partitioned windows from the bucket totals of
// phases B and C: stats 0-2 sum / sum / max over the link buckets, 3-5 and
// 6-8 count / max / max over the row and the column buckets.  Buckets
// partition the window's links and its sources (destinations), so the sums
// are exact.  Plain stores of partial totals in the earlier phases keep
// device-scope atomics off their per-item paths.  One workgroup per window.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_finish(nsgc_dev_plan* P) {
  // per wavefront: link sum, link count, row count, column count; maxima of
  // link packets, row packets, fan-out, column packets, fan-in; invalid flag
  __shared__ uint32_t red[4][11];   // [0][10]: the window's union count (entity mode)
  const uint32_t tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
  for (uint32_t wi = blockIdx.x; wi < P->num_part; wi += gridDim.x) {
    const nsgc_win_desc W = gload(P->win + wi);
    const uint32_t B = 1u << W.logB, R = 1u << W.logR, C = 1u << W.logC;
    const NSGC_GLOBAL v4u32* pb = gptr(reinterpret_cast<const v4u32*>(P->partB)) + gptr(P->prefB)[wi];
    const NSGC_GLOBAL v4u32* pc = gptr(reinterpret_cast<const v4u32*>(P->partC)) + gptr(P->prefC)[wi];
    // every sum is at most the window's packet count, below 2^32
    uint32_t v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t i = tid; i < B; i += 256) {
      const v4u32 x = pb[i];
      v[0] += x.x;
      v[1] += x.y;
      v[4] = max(v[4], x.z);
      v[9] |= x.w;
    }
    if (W.rows) {   // sources complete in their home link bucket
      const NSGC_GLOBAL v4u32* pr =
          gptr(reinterpret_cast<const v4u32*>(P->partR)) + gptr(P->prefB)[wi];
      for (uint32_t i = tid; i < B; i += 256) {
        const v4u32 x = pr[i];
        v[2] += x.x;
        v[5] = max(v[5], x.y);
        v[6] = max(v[6], x.z);
      }
    }
    for (uint32_t i = tid; i < R + C; i += 256) {
      const v4u32 x = pc[i];
      const bool row = i < R;
      v[row ? 2 : 3] += x.x;
      v[row ? 5 : 7] = max(v[row ? 5 : 7], x.y);
      v[row ? 6 : 8] = max(v[row ? 6 : 8], x.z);
      v[9] |= x.w;
    }
    uint32_t uni = 0;
    if (P->entity) {
      const NSGC_GLOBAL uint32_t* pu = gptr(P->partU) + gptr(P->prefC)[wi];
      for (uint32_t i = tid; i < R; i += 256) uni += pu[i];
      uni = wave_sum(uni);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
    for (int k = 4; k < 10; ++k) v[k] = wave_max(v[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 10; ++k) red[wv][k] = v[k];
      red[wv][10] = uni;
    }
    __syncthreads();
    if (tid == 0) red[0][10] += red[1][10] + red[2][10] + red[3][10];
    if (tid == 0) {
      uint32_t t[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        t[k] = red[0][k];
        for (int q = 1; q < 4; ++q) t[k] = k < 4 ? t[k] + red[q][k] : max(t[k], red[q][k]);
      }
      if (P->entity) {
        NSGC_GLOBAL long long* cnt = gptr(P->ent_counts) + u64(W.out_index) * 4;
        cnt[0] = (long long)t[1];
        cnt[1] = (long long)t[2];
        cnt[2] = (long long)t[3];
        cnt[3] = (long long)red[0][10];
      }
      NSGC_GLOBAL u64* o = gptr(P->out) + u64(W.out_index) * 9;
      o[0] = u64(t[0]) | (t[9] ? NSGC_INVALID_BIT : 0ull);
      o[1] = t[1];
      o[2] = t[4];
      o[3] = t[2];
      o[4] = t[5];
      o[5] = t[6];
      o[6] = t[3];
      o[7] = t[7];
      o[8] = t[8];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

hipError_t launch_small(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_small, dim3(grid), dim3(NSGC_BLOCK), lds, s, const_cast<nsgc_dev_plan*>(P));
  return hipGetLastError();
}

template <bool ROWS>
hipError_t launch_partition_t(const nsgc_dev_plan* P, uint32_t tile_log2,
                              uint32_t max_link_buckets, uint32_t grid, size_t lds, hipStream_t s) {
  switch (tile_log2) {
    case 11: hipLaunchKernelGGL((k_partition<4, NSGC_BLOCK, ROWS>), dim3(grid), dim3(NSGC_BLOCK), lds, s, P, max_link_buckets); break;
    case 12: hipLaunchKernelGGL((k_partition<8, NSGC_BLOCK, ROWS>), dim3(grid), dim3(NSGC_BLOCK), lds, s, P, max_link_buckets); break;
    case 13: hipLaunchKernelGGL((k_partition<16, NSGC_BLOCK, ROWS>), dim3(grid), dim3(NSGC_BLOCK), lds, s, P, max_link_buckets); break;
    case 14: hipLaunchKernelGGL((k_partition<32 / PART14_SCALE, NSGC_BLOCK * PART14_SCALE, ROWS>), dim3(grid), dim3(NSGC_BLOCK * PART14_SCALE), lds, s, P, max_link_buckets); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_partition(const nsgc_dev_plan* P, uint32_t tile_log2, uint32_t max_link_buckets,
                            bool rows, uint32_t grid, size_t lds, hipStream_t s) {
  return rows ? launch_partition_t<true>(P, tile_log2, max_link_buckets, grid, lds, s)
              : launch_partition_t<false>(P, tile_log2, max_link_buckets, grid, lds, s);
}

hipError_t launch_links(const nsgc_dev_plan* P, bool combine, uint32_t max_rc_buckets, uint32_t grid,
                        size_t lds, hipStream_t s) {
  if (combine)
    hipLaunchKernelGGL(k_links<true>, dim3(grid), dim3(NSGC_BLOCK), lds, s,
                       const_cast<nsgc_dev_plan*>(P), max_rc_buckets);
  else
    hipLaunchKernelGGL(k_links<false>, dim3(grid), dim3(NSGC_BLOCK), lds, s,
                       const_cast<nsgc_dev_plan*>(P), max_rc_buckets);
  return hipGetLastError();
}

hipError_t launch_links_wave(const nsgc_dev_plan* P, uint32_t hist, uint32_t rows,
                             uint32_t order_block, uint32_t grid, size_t lds, hipStream_t s) {
  if (rows)
    hipLaunchKernelGGL(k_links_wave<true>, dim3(grid + order_block), dim3(WAVE_NT), lds, s,
                       const_cast<nsgc_dev_plan*>(P), hist, order_block);
  else
    hipLaunchKernelGGL(k_links_wave<false>, dim3(grid + order_block), dim3(WAVE_NT), lds, s,
                       const_cast<nsgc_dev_plan*>(P), hist, order_block);
  return hipGetLastError();
}

hipError_t launch_heavy(const nsgc_dev_plan* P, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_heavy, dim3(grid), dim3(NSGC_BLOCK), lds_heavy_bytes(), s, P);
  return hipGetLastError();
}

hipError_t launch_rowcol_ent(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_rowcol_ent, dim3(grid), dim3(NSGC_BLOCK), lds, s, const_cast<nsgc_dev_plan*>(P));
  return hipGetLastError();
}

hipError_t launch_finish(const nsgc_dev_plan* P, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(grid), dim3(256), 0, s, const_cast<nsgc_dev_plan*>(P));
  return hipGetLastError();
}

hipError_t launch_order(const nsgc_dev_plan* P, hipStream_t s) {
  hipLaunchKernelGGL(k_order, dim3(1), dim3(NSGC_BLOCK), 0, s, const_cast<nsgc_dev_plan*>(P));
  return hipGetLastError();
}

hipError_t launch_rowcol(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_rowcol, dim3(grid), dim3(NSGC_BLOCK), lds, s, const_cast<nsgc_dev_plan*>(P));
  return hipGetLastError();
}

hipError_t resident_blocks(int which, uint32_t tile_log2, size_t lds, int* blocks) {
  const void* f = nullptr;
  switch (which) {
    case 0: f = reinterpret_cast<const void*>(&k_small); break;
    case 1:
      switch (tile_log2) {
        case 11: f = reinterpret_cast<const void*>(&k_partition<4>); break;
        case 12: f = reinterpret_cast<const void*>(&k_partition<8>); break;
        case 13: f = reinterpret_cast<const void*>(&k_partition<16>); break;
        case 14: f = reinterpret_cast<const void*>(&k_partition<32 / PART14_SCALE, NSGC_BLOCK * PART14_SCALE>); break;
        default: return hipErrorInvalidValue;
      }
      break;
    case 2: f = reinterpret_cast<const void*>(&k_links<false>); break;
    case 4: f = reinterpret_cast<const void*>(&k_links<true>); break;
    case 3: f = reinterpret_cast<const void*>(&k_rowcol); break;
    case 5: f = reinterpret_cast<const void*>(&k_links_wave<false>); break;
    case 7: f = reinterpret_cast<const void*>(&k_links_wave<true>); break;
    case 6: f = reinterpret_cast<const void*>(&k_rowcol_ent); break;
    default: return hipErrorInvalidValue;
  }
  const int threads = which == 1 && tile_log2 == 14 ? NSGC_BLOCK * PART14_SCALE
                      : which == 5 || which == 7    ? WAVE_NT
                                                    : NSGC_BLOCK;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, threads, lds);
}

hipError_t allow_large_lds(size_t bytes) {
  const int b = int(bytes);
  const void* fns[] = {
      reinterpret_cast<const void*>(&k_small),         reinterpret_cast<const void*>(&k_links<false>),
      reinterpret_cast<const void*>(&k_links<true>),   reinterpret_cast<const void*>(&k_links_wave<false>),
      reinterpret_cast<const void*>(&k_links_wave<true>),
      reinterpret_cast<const void*>(&k_rowcol_ent),    reinterpret_cast<const void*>(&k_heavy),
      reinterpret_cast<const void*>(&k_rowcol),        reinterpret_cast<const void*>(&k_partition<4>),
      reinterpret_cast<const void*>(&k_partition<8>),  reinterpret_cast<const void*>(&k_partition<16>),
      reinterpret_cast<const void*>(&k_partition<32 / PART14_SCALE, NSGC_BLOCK * PART14_SCALE>),
      reinterpret_cast<const void*>(&k_partition<4, NSGC_BLOCK, true>),
      reinterpret_cast<const void*>(&k_partition<8, NSGC_BLOCK, true>),
      reinterpret_cast<const void*>(&k_partition<16, NSGC_BLOCK, true>),
      reinterpret_cast<const void*>(&k_partition<32 / PART14_SCALE, NSGC_BLOCK * PART14_SCALE, true>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace nsgc
