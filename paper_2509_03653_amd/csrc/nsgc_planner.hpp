// Host planner: window offsets -> tiers, bucket counts, work items and
// workspace layout.  Pure host C++ (no HIP calls), so it can be exercised
// without a device.
#ifndef NSGC_PLANNER_HPP_
#define NSGC_PLANNER_HPP_

#include <cstddef>
#include <cstdint>
#include <vector>

#include "nsgc.h"
#include "nsgc_plan.h"

namespace nsgc {

// Workspace regions of one batch, as byte offsets from the workspace base.
struct WsLayout {
  size_t keys = 0, emit_row = 0, emit_col = 0, tilemeta = 0, lbmeta = 0, rcsize = 0, order = 0,
         partB = 0, partC = 0, partU = 0, stats = 0, large = 0, partR = 0, heavy = 0;
  size_t total = 0;
};

// A window of the large-window tier (computed by sorting, nsgc_large.hpp).
struct LargeWindow {
  int64_t in_begin;
  uint64_t n;
  uint32_t out_index;
};

struct HostPlan {
  std::vector<nsgc_small_desc> small;
  std::vector<LargeWindow> large;
  uint64_t large_max = 0;      // packets of the largest large window
  std::vector<nsgc_win_desc> win;
  std::vector<uint32_t> prefA, prefB, prefC;
  std::vector<uint32_t> itemwinB, itemwinC;   // window of each phase-B / phase-C item
  std::vector<uint32_t> mapBb, mapBw;         // phase-B items by kernel (empty: identity)
  uint32_t itemsBb = 0, itemsBw = 0;
  uint32_t wave_rc_max = 0;    // largest row or column bucket count of a wavefront window
  uint32_t num_rows = 0;       // row-complete windows (tune row_complete)
  int64_t ws_elems = 0;        // packets of the partitioned windows
  int64_t tilemeta_words = 0;  // u32 words of tile bucket starts
  int64_t lbmeta_words = 0;    // u32 words of link-bucket records
  uint32_t itemsA = 0, itemsB = 0, itemsC = 0;
  uint32_t tile_log2 = 14, link_slots_log2 = 12, rc_slots_log2 = 12, small_slots_log2 = 11;
  uint32_t max_sweeps_log2 = 24;
  uint32_t combine_probes = 0;
  std::vector<int32_t> tier;   // per window: 0 empty, 1 small, 2 partitioned, 3 large
  // Entity outputs (make_plan with entity = true): per window and list the
  // first and the end row, and the caller's device arrays.
  bool entity = false;
  std::vector<uint64_t> ent_cur, ent_end;   // [windows][3]
  void* ent_links = nullptr;
  void* ent_src = nullptr;
  void* ent_dst = nullptr;
  void* ent_counts = nullptr;

  WsLayout layout() const;
  size_t plan_bytes() const;
  // Write the device plan (header + arrays) into host memory `buf` (at least
  // plan_bytes()), with array pointers relative to the device address
  // `dev_plan` and workspace pointers relative to `dev_ws`.
  void serialize(void* buf, uint64_t dev_plan, uint64_t dev_ws, const uint32_t* src,
                 const uint32_t* dst, void* out) const;
};

// Checks offsets: >= 0, non-decreasing, every window < 2^32 packets.
int validate_offsets(const int64_t* offsets, int64_t num_windows);

// Builds the plan.  Returns NSGC_OK or NSGC_ERR_* (offsets must be valid).
int make_plan(const int64_t* offsets, int64_t num_windows, const nsgc_tune& tune,
              HostPlan* plan, bool entity = false, bool allow_large = true);

void default_tune(nsgc_tune* t);
int check_tune(const nsgc_tune& t);

// Smallest k with 2^k >= x (x >= 1).
int ceil_log2(uint64_t x);

// Upper bound of plan_bytes() for any batch of <= max_packets packets in <=
// max_windows windows planned with `t`.
size_t plan_bound(int64_t max_packets, int64_t max_windows, const nsgc_tune& t);


}  // namespace nsgc

#endif  // NSGC_PLANNER_HPP_
