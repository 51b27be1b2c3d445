// Window-statistics kernels for gfx950 (tiers and phases: see nsgc_plan.h).
//
// All statistics are exact integer counts (Table III of arXiv 2509.03653 and
// its src/dst reverse).  Packets are packed into 64-bit keys src << 32 | dst;
// A(s,d) is the multiplicity of a key.  No contraction is involved, so no
// matrix cores are used: the work is hashing, LDS aggregation and
// order-independent integer reductions.
//
// Every kernel is persistent: a fixed grid of workgroups strides over the work
// items whose count is read from the device plan, so a captured graph can
// replay any batch that fits its workspace.
#include <hip/hip_runtime.h>

#include "nsgc_device.hpp"
#include "nsgc_plan.h"

namespace nsgc {

namespace {

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

}  // namespace

// ---------------------------------------------------------------------------
// Tier "small": one workgroup per window, everything in LDS.
//
// Per packet: find-or-insert the link key (the inserting lane learns that the
// link is new), add one packet to the link; add one packet to the source's row
// and, if the link is new, one link to its fan-out; the same for the
// destination's column.  Tables hold 2^k >= 2 n slots, so they never fill.
// ---------------------------------------------------------------------------

size_t lds_small_bytes(uint32_t slots_log2) {
  const size_t S = size_t(1) << slots_log2;
  return align16(S * 8) + align16(S * 4) * 7 + 256;
}

__global__ __launch_bounds__(NSGC_BLOCK) void k_small(const nsgc_dev_plan* __restrict__ P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t S = 1u << P->small_slots_log2;
  const uint32_t mask = S - 1;
  u64* lk = reinterpret_cast<u64*>(smem);
  uint32_t* lc = reinterpret_cast<uint32_t*>(smem + align16(S * 8));
  uint32_t* rk = lc + S;
  uint32_t* rp = rk + S;
  uint32_t* rf = rp + S;
  uint32_t* ck = rf + S;
  uint32_t* cp = ck + S;
  uint32_t* cf = cp + S;
  uint32_t* misc = cf + S;  // [0] special link count, [1] special link seen,
                            // [2,3] special row (packets, links), [4,5] special column
  uint32_t* red = misc + 8;

  const uint32_t items = P->num_small;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    const nsgc_small_desc D = P->small[item];
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
    if (threadIdx.x < 8) misc[threadIdx.x] = 0;
    __syncthreads();

    const uint32_t* src = P->src + D.in_begin;
    const uint32_t* dst = P->dst + D.in_begin;
    for (uint32_t j = threadIdx.x; j < D.n; j += NSGC_BLOCK) {
      const uint32_t s = src[j];
      const uint32_t d = dst[j];
      const u64 key = (u64(s) << 32) | d;
      bool fresh;
      if (key == EMPTY64) {
        fresh = lds_add(&misc[1], 1) == 0;
        lds_add(&misc[0], 1);
      } else {
        const int slot = lds_insert64(lk, mask, key, uint32_t(link_hash(key)), fresh);
        lds_add(&lc[slot], 1);
      }
      if (s == EMPTY32) {
        lds_add(&misc[2], 1);
        if (fresh) lds_add(&misc[3], 1);
      } else {
        bool f2;
        const int slot = lds_insert32(rk, mask, s, row_hash(s), f2);
        lds_add(&rp[slot], 1);
        if (fresh) lds_add(&rf[slot], 1);
      }
      if (d == EMPTY32) {
        lds_add(&misc[4], 1);
        if (fresh) lds_add(&misc[5], 1);
      } else {
        bool f2;
        const int slot = lds_insert32(ck, mask, d, col_hash(d), f2);
        lds_add(&cp[slot], 1);
        if (fresh) lds_add(&cf[slot], 1);
      }
    }
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
      u64* o = P->out + u64(D.out_index) * 9;
      o[0] = sl; o[1] = nl; o[2] = ml;
      o[3] = nr; o[4] = mr; o[5] = mf;
      o[6] = nc; o[7] = mc; o[8] = mg;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Phase A: partition a tile of packets by link bucket.
// Each thread holds PER packets in registers; an LDS histogram gives every
// packet its rank inside its bucket, a block scan gives the bucket starts, and
// the keys are written to the tile's region in bucket order.
// ---------------------------------------------------------------------------

size_t lds_part_bytes(uint32_t max_buckets) { return align16((max_buckets + 1) * 4) + 256; }

template <int PER>
__global__ __launch_bounds__(NSGC_BLOCK) void k_partition(const nsgc_dev_plan* __restrict__ P) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem);
  const uint32_t items = P->itemsA;
  const uint32_t T = NSGC_BLOCK * PER;
  uint32_t* red = nullptr;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t wi = owner_of(P->prefA, P->num_part, item);
    const nsgc_win_desc W = P->win[wi];
    const uint32_t t = item - P->prefA[wi];
    const uint32_t B = 1u << W.logB;
    red = hist + ((B + 1 + 3) & ~3u);
    const uint32_t tbeg = t * T;
    const uint32_t len = min(T, W.n - tbeg);
    for (uint32_t i = threadIdx.x; i < B; i += NSGC_BLOCK) hist[i] = 0;
    if (t == 0) {
      if (threadIdx.x < 9) P->out[u64(W.out_index) * 9 + threadIdx.x] = 0;
      if (threadIdx.x == 0) P->counters[W.counter] = 0;
    }
    __syncthreads();

    const uint32_t* src = P->src + W.in_begin + tbeg;
    const uint32_t* dst = P->dst + W.in_begin + tbeg;
    u64 key[PER];
    uint32_t bk[PER], rk[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t idx = k * NSGC_BLOCK + threadIdx.x;
      if (idx < len) {
        key[k] = (u64(src[idx]) << 32) | dst[idx];
      }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t idx = k * NSGC_BLOCK + threadIdx.x;
      if (idx < len) {
        bk[k] = top64(link_hash(key[k]), W.logB);
        rk[k] = lds_add(&hist[bk[k]], 1);
      }
    }
    __syncthreads();
    block_exclusive_scan(hist, B, red);
    uint32_t* tm = P->tilemeta + W.tilemeta + u64(t) * (B + 1);
    for (uint32_t i = threadIdx.x; i <= B; i += NSGC_BLOCK) tm[i] = hist[i];
    u64* out = P->keys + W.ws + tbeg;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t idx = k * NSGC_BLOCK + threadIdx.x;
      if (idx < len) out[hist[bk[k]] + rk[k]] = key[k];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Shared machinery of phases B and C: stream the elements of up to
// NSGC_MAX_SEG segments at a time.  Segment i holds `seg_len` elements
// starting at element `seg_base` of some array; the callback gets the flat
// element position (and a validity flag) with the whole wavefront active,
// so it may use wavefront-wide operations.
// ---------------------------------------------------------------------------

struct SegStage {
  u64* base;       // [NSGC_MAX_SEG]
  uint32_t* off;   // [NSGC_MAX_SEG + 1]
  uint32_t* red;   // [2 * WAVES]
};

template <class SegFn, class ElemFn>
__device__ __forceinline__ void for_each_segment_element(uint32_t nseg, const SegStage& st,
                                                         SegFn seg, ElemFn fn) {
  for (uint32_t c0 = 0; c0 < nseg; c0 += NSGC_MAX_SEG) {
    const uint32_t cn = min(uint32_t(NSGC_MAX_SEG), nseg - c0);
    for (uint32_t i = threadIdx.x; i < cn; i += NSGC_BLOCK) {
      u64 b;
      uint32_t l;
      seg(c0 + i, b, l);
      st.base[i] = b;
      st.off[i] = l;
    }
    __syncthreads();
    const uint32_t total = block_exclusive_scan(st.off, cn, st.red);
    for (uint32_t j0 = 0; j0 < total; j0 += NSGC_BLOCK) {
      const uint32_t j = j0 + threadIdx.x;
      const bool valid = j < total;
      u64 pos = 0;
      if (valid) {
        const uint32_t i = owner_of(st.off, cn, j);
        pos = st.base[i] + (j - st.off[i]);
      }
      fn(pos, valid);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Phase B: link aggregation of one link bucket.
//
// The bucket's keys are gathered from every tile of the window into an LDS
// table key -> packet count (duplicates of the first active lane's key are
// combined with one ballot first, which keeps heavy links from serialising on
// one LDS address).  If the bucket holds more distinct keys than the table's
// load limit, it is split into 2^s sweeps by further hash bits and redone;
// the split is a partition of the keys, so the result is unchanged.  The
// table gives the bucket's share of stats 0-2; its links are then emitted as
// (src, count) grouped by row bucket and (dst, count) grouped by column
// bucket.
// ---------------------------------------------------------------------------

size_t lds_link_bytes(uint32_t slots_log2, uint32_t max_buckets) {
  const size_t S = size_t(1) << slots_log2;
  return align16(S * 8) + align16(S * 4) + align16(NSGC_MAX_SEG * 8) +
         align16((NSGC_MAX_SEG + 1) * 4) + 2 * align16((max_buckets + 1) * 4) + 256;
}

__global__ __launch_bounds__(NSGC_BLOCK) void k_links(const nsgc_dev_plan* __restrict__ P,
                                                      uint32_t max_buckets) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t S = 1u << P->link_slots_log2;
  const uint32_t mask = S - 1;
  const uint32_t limit = S - (S >> 2);
  unsigned char* p = smem;
  u64* tk = reinterpret_cast<u64*>(p);                 p += align16(S * 8);
  uint32_t* tc = reinterpret_cast<uint32_t*>(p);       p += align16(S * 4);
  SegStage st;
  st.base = reinterpret_cast<u64*>(p);                 p += align16(NSGC_MAX_SEG * 8);
  st.off = reinterpret_cast<uint32_t*>(p);             p += align16((NSGC_MAX_SEG + 1) * 4);
  uint32_t* histR = reinterpret_cast<uint32_t*>(p);    p += align16((max_buckets + 1) * 4);
  uint32_t* histC = reinterpret_cast<uint32_t*>(p);    p += align16((max_buckets + 1) * 4);
  uint32_t* misc = reinterpret_cast<uint32_t*>(p);     // [0] occupancy [1] overflow
                                                       // [2] special count [3] emission base
  st.red = misc + 8;

  const uint32_t T = 1u << P->tile_log2;
  const uint32_t items = P->itemsB;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t wi = owner_of(P->prefB, P->num_part, item);
    const nsgc_win_desc W = P->win[wi];
    const uint32_t b = item - P->prefB[wi];
    const uint32_t B = 1u << W.logB, R = 1u << W.logR, C = 1u << W.logC;
    const u64* keys = P->keys + W.ws;
    const uint32_t* tm = P->tilemeta + W.tilemeta;

    auto seg = [&](uint32_t t, u64& base, uint32_t& len) {
      const uint32_t* row = tm + u64(t) * (B + 1);
      const uint32_t s0 = row[b], s1 = row[b + 1];
      base = u64(t) * T + s0;
      len = s1 - s0;
    };

    // Build the table for sweep `sw` of 2^logS.
    auto build = [&](uint32_t logS, uint32_t sw) {
      for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
        tk[i] = EMPTY64;
        tc[i] = 0;
      }
      if (threadIdx.x < 4) misc[threadIdx.x] = 0;
      __syncthreads();
      for_each_segment_element(W.ntiles, st, seg, [&](u64 pos, bool valid) {
        u64 key = 0;
        u64 h = 0;
        if (valid) {
          key = keys[pos];
          h = link_hash(key);
          if (logS && next64(h, W.logB, logS) != sw) valid = false;
        }
        if (valid && key == EMPTY64) {
          lds_add(&misc[2], 1);
          valid = false;
        }
        if (valid && lds_load(&misc[1])) valid = false;
        const u64 vm = __ballot(valid);
        if (!vm) return;
        const int first = __ffsll(static_cast<unsigned long long>(vm)) - 1;
        const u64 k0 = (u64(readlane(uint32_t(key >> 32), first)) << 32) |
                       readlane(uint32_t(key), first);
        const bool same = valid && key == k0;
        const u64 sm = __ballot(same);
        const uint32_t nsame = __popcll(sm);
        uint32_t add = 1;
        if (same) {
          if (int(lane_id()) != first) valid = false;
          else add = nsame;
        }
        if (valid) {
          bool fresh;
          const int slot = lds_insert64(tk, mask, key, uint32_t(h), fresh);
          if (slot < 0) {
            lds_store(&misc[1], 1);
          } else {
            if (fresh && lds_add(&misc[0], 1) >= limit) lds_store(&misc[1], 1);
            lds_add(&tc[slot], add);
          }
        }
      });
    };

    uint32_t logS = 0;
    uint32_t links = 0, sum = 0, mx = 0;
    for (;;) {
      links = sum = mx = 0;
      for (uint32_t i = threadIdx.x; i < R; i += NSGC_BLOCK) histR[i] = 0;
      for (uint32_t i = threadIdx.x; i < C; i += NSGC_BLOCK) histC[i] = 0;
      bool failed = false;
      for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
        build(logS, sw);
        if (misc[1]) { failed = true; break; }
        for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
          const u64 key = tk[i];
          if (key != EMPTY64) {
            const uint32_t c = tc[i];
            ++links;
            sum += c;
            mx = max(mx, c);
            lds_add(&histR[top32(row_hash(uint32_t(key >> 32)), W.logR)], 1);
            lds_add(&histC[top32(col_hash(uint32_t(key)), W.logC)], 1);
          }
        }
        if (threadIdx.x == 0 && misc[2]) {
          const uint32_t c = misc[2];
          ++links;
          sum += c;
          mx = max(mx, c);
          lds_add(&histR[top32(row_hash(EMPTY32), W.logR)], 1);
          lds_add(&histC[top32(col_hash(EMPTY32), W.logC)], 1);
        }
        __syncthreads();
      }
      if (!failed) break;
      ++logS;
      __syncthreads();
    }

    // bucket totals -> window statistics 0..2
    block_sum_max(sum, mx, st.red);
    const uint32_t nlinks = block_sum(links, st.red);
    if (threadIdx.x == 0) {
      u64* o = P->out + u64(W.out_index) * 9;
      stat_add(o + 0, sum);
      stat_add(o + 1, nlinks);
      stat_max(o + 2, mx);
      misc[3] = nlinks ? atomicAdd(&P->counters[W.counter], nlinks) : 0u;
    }
    __syncthreads();
    const uint32_t base = misc[3];
    block_exclusive_scan(histR, R, st.red);
    block_exclusive_scan(histC, C, st.red);
    uint32_t* rec = P->lbmeta + W.lbmeta + u64(b) * (R + C + 3);
    if (threadIdx.x == 0) rec[0] = base;
    for (uint32_t i = threadIdx.x; i <= R; i += NSGC_BLOCK) rec[1 + i] = histR[i];
    for (uint32_t i = threadIdx.x; i <= C; i += NSGC_BLOCK) rec[R + 2 + i] = histC[i];
    __syncthreads();

    // emission: histR / histC now serve as per-bucket cursors
    u64* erow = P->emit_row + W.ws + base;
    u64* ecol = P->emit_col + W.ws + base;
    for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
      if (logS) build(logS, sw);  // a sweep that fit once fits again
      for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
        const u64 key = tk[i];
        if (key != EMPTY64) {
          const uint32_t c = tc[i];
          const uint32_t s = uint32_t(key >> 32), d = uint32_t(key);
          const uint32_t pr = lds_add(&histR[top32(row_hash(s), W.logR)], 1);
          const uint32_t pc = lds_add(&histC[top32(col_hash(d), W.logC)], 1);
          erow[pr] = (u64(s) << 32) | c;
          ecol[pc] = (u64(d) << 32) | c;
        }
      }
      if (threadIdx.x == 0 && misc[2]) {
        const uint32_t c = misc[2];
        const uint32_t pr = lds_add(&histR[top32(row_hash(EMPTY32), W.logR)], 1);
        const uint32_t pc = lds_add(&histC[top32(col_hash(EMPTY32), W.logC)], 1);
        erow[pr] = (u64(EMPTY32) << 32) | c;
        ecol[pc] = (u64(EMPTY32) << 32) | c;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Phase C: aggregation of one row bucket (or column bucket).
//
// Gathers the bucket's run from every link bucket's emission into an LDS table
// id -> (packets, links); each entry is one link with its packet count, so the
// table yields r(s) and f(s) (or c(d) and g(d)) for every id of the bucket.
// Entries that repeat the first active lane's id are pre-combined with one
// ballot and one DPP sum.  Overflow splits the bucket into sweeps as in B.
// ---------------------------------------------------------------------------

size_t lds_rc_bytes(uint32_t slots_log2) {
  const size_t S = size_t(1) << slots_log2;
  return align16(S * 4) * 3 + align16(NSGC_MAX_SEG * 8) + align16((NSGC_MAX_SEG + 1) * 4) +
         256;
}

__global__ __launch_bounds__(NSGC_BLOCK) void k_rowcol(const nsgc_dev_plan* __restrict__ P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t S = 1u << P->rc_slots_log2;
  const uint32_t mask = S - 1;
  const uint32_t limit = S - (S >> 2);
  unsigned char* p = smem;
  uint32_t* tk = reinterpret_cast<uint32_t*>(p);       p += align16(S * 4);
  uint32_t* tp = reinterpret_cast<uint32_t*>(p);       p += align16(S * 4);
  uint32_t* tl = reinterpret_cast<uint32_t*>(p);       p += align16(S * 4);
  SegStage st;
  st.base = reinterpret_cast<u64*>(p);                 p += align16(NSGC_MAX_SEG * 8);
  st.off = reinterpret_cast<uint32_t*>(p);             p += align16((NSGC_MAX_SEG + 1) * 4);
  uint32_t* misc = reinterpret_cast<uint32_t*>(p);     // [0] occupancy [1] overflow
                                                       // [2,3] special id (packets, links)
  st.red = misc + 8;

  const uint32_t items = P->itemsC;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t wi = owner_of(P->prefC, P->num_part, item);
    const nsgc_win_desc W = P->win[wi];
    const uint32_t k = item - P->prefC[wi];
    const uint32_t B = 1u << W.logB, R = 1u << W.logR, C = 1u << W.logC;
    const bool is_row = k < R;
    const uint32_t bucket = is_row ? k : k - R;
    const uint32_t logK = is_row ? W.logR : W.logC;
    const uint32_t stride = R + C + 3;
    const uint32_t first_word = is_row ? 1 + bucket : R + 2 + bucket;
    const uint32_t* recs = P->lbmeta + W.lbmeta;
    const u64* em = (is_row ? P->emit_row : P->emit_col) + W.ws;

    auto seg = [&](uint32_t lb, u64& base, uint32_t& len) {
      const uint32_t* rec = recs + u64(lb) * stride;
      const uint32_t s0 = rec[first_word], s1 = rec[first_word + 1];
      base = u64(rec[0]) + s0;
      len = s1 - s0;
    };

    auto build = [&](uint32_t logS, uint32_t sw) {
      for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
        tk[i] = EMPTY32;
        tp[i] = 0;
        tl[i] = 0;
      }
      if (threadIdx.x < 4) misc[threadIdx.x] = 0;
      __syncthreads();
      for_each_segment_element(B, st, seg, [&](u64 pos, bool valid) {
        uint32_t id = 0, cnt = 0, h = 0;
        if (valid) {
          const u64 e = em[pos];
          id = uint32_t(e >> 32);
          cnt = uint32_t(e);
          h = is_row ? row_hash(id) : col_hash(id);
          if (logS && next32(h, logK, logS) != sw) valid = false;
        }
        if (valid && id == EMPTY32) {
          lds_add(&misc[2], cnt);
          lds_add(&misc[3], 1);
          valid = false;
        }
        if (valid && lds_load(&misc[1])) valid = false;
        const u64 vm = __ballot(valid);
        if (!vm) return;
        const int first = __ffsll(static_cast<unsigned long long>(vm)) - 1;
        const uint32_t id0 = readlane(id, first);
        const bool same = valid && id == id0;
        const u64 sm = __ballot(same);
        const uint32_t nsame = __popcll(sm);
        uint32_t addp = cnt, addl = 1;
        if (nsame > 1) {
          const uint32_t tot = wave_sum(same ? cnt : 0u);
          if (same) {
            if (int(lane_id()) != first) valid = false;
            else { addp = tot; addl = nsame; }
          }
        }
        if (valid) {
          bool fresh;
          const int slot = lds_insert32(tk, mask, id, h, fresh);
          if (slot < 0) {
            lds_store(&misc[1], 1);
          } else {
            if (fresh && lds_add(&misc[0], 1) >= limit) lds_store(&misc[1], 1);
            lds_add(&tp[slot], addp);
            lds_add(&tl[slot], addl);
          }
        }
      });
    };

    uint32_t logS = 0;
    uint32_t n = 0, mp = 0, ml = 0;
    for (;;) {
      n = mp = ml = 0;
      bool failed = false;
      for (uint32_t sw = 0; sw < (1u << logS); ++sw) {
        build(logS, sw);
        if (misc[1]) { failed = true; break; }
        for (uint32_t i = threadIdx.x; i < S; i += NSGC_BLOCK) {
          if (tk[i] != EMPTY32) {
            ++n;
            mp = max(mp, tp[i]);
            ml = max(ml, tl[i]);
          }
        }
        if (threadIdx.x == 0 && misc[3]) {
          ++n;
          mp = max(mp, misc[2]);
          ml = max(ml, misc[3]);
        }
        __syncthreads();
      }
      if (!failed) break;
      ++logS;
      __syncthreads();
    }
    block_sum_max(n, mp, st.red);
    uint32_t zero = 0;
    block_sum_max(zero, ml, st.red);
    if (threadIdx.x == 0) {
      u64* o = P->out + u64(W.out_index) * 9 + (is_row ? 3 : 6);
      stat_add(o + 0, n);
      stat_max(o + 1, mp);
      stat_max(o + 2, ml);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

hipError_t launch_small(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_small, dim3(grid), dim3(NSGC_BLOCK), lds, s, P);
  return hipGetLastError();
}

hipError_t launch_partition(const nsgc_dev_plan* P, uint32_t tile_log2, uint32_t grid, size_t lds,
                            hipStream_t s) {
  switch (tile_log2) {
    case 11: hipLaunchKernelGGL(k_partition<4>, dim3(grid), dim3(NSGC_BLOCK), lds, s, P); break;
    case 12: hipLaunchKernelGGL(k_partition<8>, dim3(grid), dim3(NSGC_BLOCK), lds, s, P); break;
    case 13: hipLaunchKernelGGL(k_partition<16>, dim3(grid), dim3(NSGC_BLOCK), lds, s, P); break;
    case 14: hipLaunchKernelGGL(k_partition<32>, dim3(grid), dim3(NSGC_BLOCK), lds, s, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_links(const nsgc_dev_plan* P, uint32_t max_buckets, uint32_t grid, size_t lds,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_links, dim3(grid), dim3(NSGC_BLOCK), lds, s, P, max_buckets);
  return hipGetLastError();
}

hipError_t launch_rowcol(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_rowcol, dim3(grid), dim3(NSGC_BLOCK), lds, s, P);
  return hipGetLastError();
}

hipError_t allow_large_lds(size_t bytes) {
  hipError_t e;
  const int b = int(bytes);
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small),
                               hipFuncAttributeMaxDynamicSharedMemorySize, b)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_links),
                               hipFuncAttributeMaxDynamicSharedMemorySize, b)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rowcol),
                               hipFuncAttributeMaxDynamicSharedMemorySize, b)) != hipSuccess)
    return e;
  return hipSuccess;
}

}  // namespace nsgc
