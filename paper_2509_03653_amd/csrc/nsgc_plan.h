// Plan layout shared by the host planner and the device kernels.
//
// A batch is planned on the host from the window offsets alone (sizes are
// known without a device round-trip) and uploaded as one contiguous plan
// buffer: a header, then the window descriptors and the item-prefix arrays the
// persistent kernels use to map a work item to its window.
//
// Tiers:
//   small : n <= small_max (including empty windows).  One workgroup computes
//           the window entirely in LDS (link, row and column tables at once).
//   part  : everything else, in three phases over the window's packets:
//     A  partition: tiles of 2^tile_log2 packets; each tile is reordered by
//        link bucket (top bits of a 64-bit mix of the packed (src,dst) key)
//        and written to the window's key region, with per-tile bucket starts.
//     B  link aggregation: one item per link bucket gathers its segments from
//        every tile into an LDS hash table (key -> packet count).  This gives
//        A's non-zeros: sum, count and max per bucket (stats 0-2).  The
//        de-duplicated links are then emitted twice, as (src, count) grouped
//        by row bucket and as (dst, count) grouped by column bucket, into a
//        region reserved from the window's emission cursor.
//     C  row / column aggregation: one item per row bucket and per column
//        bucket gathers its runs from every link bucket into an LDS table
//        id -> (packets, links), giving stats 3-5 and 6-8.
//   Partial results of B and C combine into the window's output with 64-bit
//   atomic add (counts) and max (maxima): exact and order-independent.
#ifndef NSGC_PLAN_H_
#define NSGC_PLAN_H_

#include <stdint.h>

#define NSGC_BLOCK 512          // threads per workgroup in every kernel
#define NSGC_MAX_SEG 1024       // segments staged in LDS at a time (phases B, C)

struct nsgc_small_desc {        // 16 bytes
  int64_t in_begin;             // index of the window's first packet
  uint32_t n;                   // packets
  uint32_t out_index;           // window index in out_stats
};

struct nsgc_win_desc {          // 64 bytes
  int64_t in_begin;             // index of the window's first packet
  int64_t ws;                   // element offset of the window in keys/emit arrays
  int64_t tilemeta;             // u32 offset of the tile bucket starts [ntiles][B+1]
  int64_t lbmeta;               // u32 offset of the link-bucket records [B][R+C+3]
  uint32_t n;                   // packets (< 2^32)
  uint32_t out_index;           // window index in out_stats
  uint32_t ntiles;              // partition tiles
  uint32_t counter;             // index of the window's emission cursor
  uint8_t logB, logR, logC, pad0;
  uint32_t pad1[3];
};

// Link-bucket record (u32 words), stride R + C + 3:
//   [0]                 emission base, relative to the window's ws offset
//   [1 .. R+1]          row-bucket starts within the emission (R+1 entries)
//   [R+2 .. R+C+2]      column-bucket starts within the emission (C+1 entries)

struct nsgc_dev_plan {          // header of the device plan buffer
  const uint32_t* src;
  const uint32_t* dst;
  unsigned long long* out;      // 9 x u64 per window
  unsigned long long* keys;     // partitioned packed keys
  unsigned long long* emit_row; // (src << 32 | count) per link
  unsigned long long* emit_col; // (dst << 32 | count) per link
  uint32_t* tilemeta;
  uint32_t* lbmeta;
  uint32_t* counters;
  const nsgc_small_desc* small;
  const nsgc_win_desc* win;
  const uint32_t* prefA;        // [num_part + 1] first phase-A item of each window
  const uint32_t* prefB;        // [num_part + 1] first phase-B item
  const uint32_t* prefC;        // [num_part + 1] first phase-C item
  uint32_t num_small;
  uint32_t num_part;
  uint32_t itemsA, itemsB, itemsC;
  uint32_t tile_log2;
  uint32_t link_slots_log2;
  uint32_t rc_slots_log2;
  uint32_t small_slots_log2;
  uint32_t pad[3];
};

#endif  // NSGC_PLAN_H_
