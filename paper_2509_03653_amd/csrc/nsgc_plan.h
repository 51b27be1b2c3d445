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
//     A  partition: tiles of 2^tile_log2 packets; each packet becomes the
//        hashed link key row_hash(src) << 32 | col_hash(dst) (a bijection of
//        the pair), each tile is reordered by link bucket (top bits of the
//        key's position mix) and written to the window's key region, with
//        per-tile bucket starts.  All later phases work on these hashed
//        identities, so they never hash again.
//     B  link aggregation: one item per link bucket gathers its segments from
//        every tile into an LDS hash table (key -> packet count).  This gives
//        A's non-zeros: sum, count and max per bucket (stats 0-2).  The
//        bucket's links are then combined per source and per destination
//        and emitted as (row_hash(src), packets, links) grouped by row
//        bucket and (col_hash(dst), packets, links) grouped by column bucket
//        (the top bits of the hashed id), into the bucket's own
//        emission region (as many slots as it has packets).  A source with
//        many links thus leaves one entry per link bucket, not one per link.
//     C  row / column aggregation: one item per row bucket and per column
//        bucket gathers its runs from every link bucket into an LDS table
//        id -> (packets, links), giving stats 3-5 and 6-8.
//   Every phase-B and phase-C item stores its bucket's totals (counts and
//   maxima); k_finish combines them per window by sums and maxima, which is
//   exact because buckets partition the links, sources and destinations.
//   Row-complete windows: before A, a sample of each window's sources marks
//   the heavy ones (table `heavy`).  A puts every link of a light source s
//   in bucket top(row_hash(s)) and spreads a heavy source's links over the
//   other buckets, top(row_hash(s)) ^ x with x in 1..B-1 from the
//   destination hash.  So a source met in bucket b with top(row_hash) == b
//   has all its links there: B combines the bucket's links per source and
//   stores the totals of those sources (partR); every other source leaves one
//   entry (packets, links) per bucket for C.  The id EMPTY32 and buckets
//   that sweep keep per-link row entries.
#ifndef NSGC_PLAN_H_
#define NSGC_PLAN_H_

#include <stdint.h>

#define NSGC_BLOCK 512          // threads per workgroup in every kernel
#define NSGC_UNROLL 8           // elements per thread in flight in the B/C gathers

// A phase-B emission entry packs an id with the links and packets it stands
// for: id << 32 | links << 19 | packets.  A link bucket holds at most 4096
// links, so the link field never overflows; a triple with more packets than
// the packet field holds is emitted as several entries that sum to it (phase C
// adds them up).  Since links <= packets no triple needs more entries than it
// has packets, so an emission region of one slot per packet suffices.
// Work-queue counters per kernel, one per 128-byte line (see ItemQueue).
#define NSGC_QCLASSES 8
#define NSGC_QSTRIDE 32
// Batches of at most this many phase-C items have them ordered large first.
#define NSGC_ORDER_MAX 16384
#define NSGC_ENT_PACKET_BITS 19
#define NSGC_ENT_LINK_BITS 13
// Phase B one wavefront per link bucket (k_links_wave): LDS table slots per
// wavefront, and the most row (or column) buckets such a window may have.
#define NSGC_WAVE_SLOTS_LOG2 9
#define NSGC_WAVE_MAX_RC 256
// Row-complete windows (tune row_complete): slots of a window's table of
// heavy sources (sets of four ids, the set picked by the hashed id's low
// bits), the sample of packets it is drawn from, and the LDS row table of
// each phase-B wavefront.
#define NSGC_HEAVY_SLOTS 512
#define NSGC_HEAVY_SAMPLE 4096
#define NSGC_WAVE_ROW_SLOTS 256

struct nsgc_small_desc {        // 16 bytes
  int64_t in_begin;             // index of the window's first packet
  uint32_t n;                   // packets
  uint32_t out_index;           // window index in out_stats
};

struct nsgc_win_desc {          // 64 bytes
  int64_t in_begin;             // index of the window's first packet
  int64_t ws;                   // element offset of the window in keys/emit arrays
  int64_t tilemeta;             // u32 offset of the tile bucket starts [B+1][ntiles]
  int64_t lbmeta;               // u32 offset of the link-bucket records (below)
  uint32_t n;                   // packets (< 2^32)
  uint32_t out_index;           // window index in out_stats
  uint32_t ntiles;              // partition tiles
  uint32_t counter;             // index of the window among partitioned windows
  uint8_t logB, logR, logC;
  uint8_t wave;                 // 1: phase B runs one wavefront per link bucket
  uint8_t rows;                 // 1: row-complete (wavefront windows only, logB >= 1)
  uint8_t pad0[3];
  uint32_t pad1[2];
};

// Tile bucket starts, bucket-major: word b * ntiles + t holds the number of
// keys of tile t whose link bucket is < b (b = 0..B), so bucket b of tile t
// is [start(b,t), start(b+1,t)) within the tile's region.  The emission
// region of link bucket b starts at sum over t of start(b,t), the number of
// the window's packets in buckets below b, and has one slot per packet of b.
//
// Link-bucket records of a window (u32 words), bucket-major so that a phase-C
// item reads contiguous vectors over the link buckets b:
//   [b]                                   emission base of link bucket b
//   [B + r * B + b], r = 0..R             row-bucket r start in b's emission
//   [B + (R+1) * B + c * B + b], c = 0..C column-bucket c start
// A window's record block holds B * (R + C + 3) words.

struct nsgc_dev_plan {          // header of the device plan buffer
  const uint32_t* src;
  const uint32_t* dst;
  unsigned long long* out;      // 9 x u64 per window
  unsigned long long* keys;     // partitioned packed keys
  unsigned long long* emit_row; // row entries (src, links, packets), packed below
  unsigned long long* emit_col; // column entries (dst, links, packets)
  uint32_t* tilemeta;
  uint32_t* lbmeta;
  uint32_t* rcsize;             // [itemsC] size of each phase-C item (packets of its row or
                                //   column bucket in the window's first tile, by phase A)
  uint32_t* order;              // [itemsC] phase-C items, large ones first
  uint32_t* partB;              // [itemsB][4] link-bucket totals: packets, links, max, invalid
  uint32_t* partC;              // [itemsC][4] row/column-bucket totals: ids, max packets,
                                //   max links, invalid
  const nsgc_small_desc* small;
  const nsgc_win_desc* win;
  const uint32_t* prefA;        // [num_part + 1] first phase-A item of each window
  const uint32_t* prefB;        // [num_part + 1] first phase-B item
  const uint32_t* prefC;        // [num_part + 1] first phase-C item
  const uint32_t* itemwinB;     // [itemsB] window (index among partitioned) of each phase-B item
  const uint32_t* mapBb;        // phase-B items of workgroup windows (null: items 0..itemsBb)
  const uint32_t* mapBw;        // phase-B items of wavefront windows (null: items 0..itemsBw)
  const uint32_t* itemwinC;     // [itemsC] window of each phase-C item
  uint32_t num_small;
  uint32_t num_part;
  uint32_t itemsA, itemsB, itemsC;
  uint32_t itemsBb, itemsBw;    // phase-B items of workgroup / wavefront windows
  uint32_t tile_log2;
  uint32_t link_slots_log2;
  uint32_t rc_slots_log2;
  uint32_t small_slots_log2;
  uint32_t max_sweeps_log2;     // overflow sweeps allowed before a bucket is abandoned
  uint32_t combine_probes;      // 0: per-link emission; else probe limit of the combining table
  uint32_t order_items;         // 1: phase C takes its items in the order of `order`
  // Entity outputs (zero / null for the statistics entry points).  In entity
  // mode destinations are hashed like sources, row and column buckets
  // coincide (R = C), and each phase-C row item also aggregates the column
  // bucket of the same index, so that it can count the union of the two.
  uint32_t entity;
  long long* ent_links;         // rows (src, dst, packets), or null
  long long* ent_src;           // rows (s, r(s), f(s)), or null
  long long* ent_dst;           // rows (d, c(d), g(d)), or null
  unsigned long long* ent_cur;  // [windows][3] next free row of each list
  const unsigned long long* ent_end;  // [windows][3] end of each window's rows
  long long* ent_counts;        // [windows][4] nsgc_entity_counts
  uint32_t* partU;              // [itemsC] union count of each merged phase-C item
  // Row-complete windows (null when the batch has none).
  uint32_t* heavy;              // [num_part][NSGC_HEAVY_SLOTS] heavy sources, 4-way sets
  uint32_t* partR;              // [itemsB][4] complete sources of a bucket: count, max packets,
                                //   max links, 0
  // Work-queue counters of the small, B (workgroup), C and B (wavefront)
  // kernels.  Uploaded as zero with every plan.
  uint32_t queue[4][NSGC_QCLASSES * NSGC_QSTRIDE];
};

#endif  // NSGC_PLAN_H_
