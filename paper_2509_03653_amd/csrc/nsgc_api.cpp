// C ABI of the window-statistics library (declared in include/nsgc.h).
//
// Host side of every call: validate the arguments, plan the batch (tiers,
// bucket counts, items, workspace layout), upload the plan through a pinned
// staging buffer with one async copy, and launch the persistent kernels on the
// caller's stream.  Workspaces and plan buffers are cached per (device,
// stream) so calls on different streams can overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "nsgc.h"
#include "nsgc_anon.hpp"
#include "nsgc_large.hpp"
#include "nsgc_planner.hpp"

namespace nsgc {
hipError_t launch_small(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s);
hipError_t launch_partition(const nsgc_dev_plan* P, uint32_t tile_log2, uint32_t max_link_buckets,
                            bool rows, uint32_t grid, size_t lds, hipStream_t s);
hipError_t launch_links(const nsgc_dev_plan* P, bool combine, uint32_t max_rc_buckets, uint32_t grid,
                        size_t lds, hipStream_t s);
hipError_t launch_links_wave(const nsgc_dev_plan* P, uint32_t hist, uint32_t rows,
                             uint32_t order_block, uint32_t grid, size_t lds, hipStream_t s);
hipError_t launch_heavy(const nsgc_dev_plan* P, uint32_t grid, hipStream_t s);
size_t lds_heavy_bytes();
hipError_t launch_order(const nsgc_dev_plan* P, hipStream_t s);
hipError_t launch_finish(const nsgc_dev_plan* P, uint32_t grid, hipStream_t s);
hipError_t launch_rowcol_ent(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s);
size_t lds_rc_ent_bytes(uint32_t slots_log2);
hipError_t launch_rowcol(const nsgc_dev_plan* P, uint32_t grid, size_t lds, hipStream_t s);
size_t lds_small_bytes(uint32_t slots_log2);
size_t lds_part_bytes(uint32_t max_link_buckets, uint32_t tile_log2, uint32_t max_rc_buckets);
size_t lds_link_bytes(uint32_t slots_log2, uint32_t max_rc_buckets);
size_t lds_rc_bytes(uint32_t slots_log2);
size_t lds_links_wave_bytes(uint32_t hist, uint32_t rows);
hipError_t allow_large_lds(size_t bytes);
hipError_t resident_blocks(int which, uint32_t tile_log2, size_t lds, int* blocks);
}  // namespace nsgc

using namespace nsgc;

namespace {

thread_local int t_last_hip_error = 0;

int hip_fail(hipError_t e) {
  t_last_hip_error = int(e);
  return NSGC_ERR_HIP;
}

#define NSGC_HIP(expr)                       \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

constexpr int kStages = 4;

// Device buffers and staging of one (device, stream) pair.  A call works on
// its slot under the slot's own lock; slots are never deleted (nsgc_release
// frees their buffers), so a slot pointer stays valid once looked up.
struct Slot {
  std::mutex mu;
  char* plan_dev = nullptr;
  size_t plan_cap = 0;
  char* ws = nullptr;
  size_t ws_cap = 0;
  char* stage[kStages] = {};
  size_t stage_cap[kStages] = {};
  hipEvent_t ev[kStages] = {};
  bool ev_used[kStages] = {};
  int next = 0;
  hipEvent_t phase_ev[6] = {};  // timing events of nsgc_window_stats_timed
};

// State of the fixed-scratch form on one device: a host staging buffer for
// its plan (ordinary host memory, sized once), the event after its last plan
// copy (the staging buffer is rewritten only once that copy has read it) and
// the event after its last launch (a call on another stream waits for it on
// the device, since every call shares the device's one scratch array).
struct FixedState {
  std::mutex mu;
  std::vector<char> stage;
  hipEvent_t copied = nullptr;
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool used = false;
};

struct DevCtx {
  int device = 0;
  int cus = 256;
  size_t lds_limit = 65536;
  std::map<hipStream_t, Slot*> slots;
  // resident workgroups per CU by (kernel, tile_log2, dynamic LDS bytes)
  std::map<std::tuple<int, uint32_t, size_t>, int> resident;
  FixedState fixed;
};

// Guards the process-wide state below (device contexts, their slot maps and
// occupancy cache, the tuning and the plain-mode switch).  Calls hold it only
// to look these up; planning, uploads and launches run under the lock of the
// call's slot (or graph, or the device's fixed scratch), so calls on
// different streams plan and enqueue concurrently.  Lock order: g_mu before a
// slot's lock, and no code holding a slot's lock takes g_mu.
std::mutex g_mu;
std::map<int, DevCtx*> g_devs;
nsgc_tune g_tune;
bool g_tune_set = false;
bool g_plain_mode = false;   // nsgc_set_plain_mode: route nsgc_window_stats through the plain form

const nsgc_tune& current_tune() {
  if (!g_tune_set) {
    default_tune(&g_tune);
    g_tune_set = true;
  }
  return g_tune;
}

int get_ctx(DevCtx** out) {
  int dev = 0;
  NSGC_HIP(hipGetDevice(&dev));
  auto it = g_devs.find(dev);
  if (it != g_devs.end()) {
    *out = it->second;
    return NSGC_OK;
  }
  DevCtx* c = new DevCtx;
  c->device = dev;
  hipDeviceProp_t prop;
  NSGC_HIP(hipGetDeviceProperties(&prop, dev));
  c->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->lds_limit = prop.sharedMemPerBlock > 0 ? size_t(prop.sharedMemPerBlock) : 65536;
  // gfx950 gives a workgroup up to the whole 160 KB LDS of its compute unit
  int per_cu = 0;
  if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      per_cu > 0)
    c->lds_limit = std::max(c->lds_limit, size_t(per_cu));
  NSGC_HIP(allow_large_lds(c->lds_limit));
  g_devs[dev] = c;
  *out = c;
  return NSGC_OK;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// Grow a device buffer; waits for `s` first since queued work may still use it.
int ensure_device(char** buf, size_t* cap, size_t need, hipStream_t s) {
  if (*cap >= need && *buf) return NSGC_OK;
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  size_t want = std::max(need, *cap + *cap / 4);
  if (*buf) {
    NSGC_HIP(hipStreamSynchronize(s));
    NSGC_HIP(hipFree(*buf));
    *buf = nullptr;
    *cap = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = hipMalloc(&p, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return NSGC_ERR_NO_MEMORY;
    }
    want = need;
  }
  *buf = static_cast<char*>(p);
  *cap = want;
  return NSGC_OK;
}

// A staging buffer that no queued copy still reads.
int take_stage(Slot* sl, size_t need, hipStream_t s, int* idx) {
  const int k = sl->next;
  if (sl->ev_used[k]) NSGC_HIP(hipEventSynchronize(sl->ev[k]));
  if (!sl->ev[k]) NSGC_HIP(hipEventCreateWithFlags(&sl->ev[k], hipEventDisableTiming));
  if (sl->stage_cap[k] < need) {
    if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
    if (sl->stage[k]) NSGC_HIP(hipHostFree(sl->stage[k]));
    sl->stage[k] = nullptr;
    sl->stage_cap[k] = 0;
    const size_t want = std::max<size_t>(need * 2, 4096);
    void* p = nullptr;
    NSGC_HIP(hipHostMalloc(&p, want, hipHostMallocDefault));
    sl->stage[k] = static_cast<char*>(p);
    sl->stage_cap[k] = want;
  }
  *idx = k;
  sl->next = (k + 1) % kStages;
  return NSGC_OK;
}

// The wavefront phase-B kernel's two sizes of per-wavefront row and column
// counters: batches whose wavefront windows have at most 64 row and column
// buckets get the smaller LDS footprint and more resident wavefronts.
constexpr uint32_t kWaveHist[2] = {64 + 1, NSGC_WAVE_MAX_RC + 1};
inline int wave_class(uint32_t rc_max) { return rc_max <= 64 ? 0 : 1; }

struct Launch {
  uint32_t grid_small, grid_part, grid_link, grid_rc, grid_finish, grid_rce;  // persistent grids
  uint32_t grid_linkw[2][2];                           // per wave_class, row tables
  uint32_t grid_heavy;
  bool combine;                                        // phase-B emission combines per id
  size_t lds_small, lds_part, lds_link, lds_rc, lds_rce;
  size_t lds_linkw[2][2];
  uint32_t max_link_buckets, max_rc_buckets;
};

// Workgroups per CU that can actually be resident (registers and LDS), at
// most `want`: persistent workgroups beyond that would only queue.
int resident_cap(DevCtx* c, int which, uint32_t tile_log2, size_t lds, int want, uint32_t* grid) {
  const auto key = std::make_tuple(which, tile_log2, lds);
  auto it = c->resident.find(key);
  if (it == c->resident.end()) {
    int n = 0;
    NSGC_HIP(resident_blocks(which, tile_log2, lds, &n));
    it = c->resident.emplace(key, std::max(n, 1)).first;
  }
  *grid = uint32_t(c->cus) * uint32_t(std::min(want, it->second));
  return NSGC_OK;
}

int launch_params(DevCtx* c, const nsgc_tune& t, Launch* out) {
  Launch L;
  L.max_link_buckets = 1u << t.max_link_buckets_log2;
  L.max_rc_buckets = 1u << t.max_rc_buckets_log2;
  const uint32_t small_log2 =
      uint32_t(std::max(ceil_log2(uint64_t(std::max(t.small_max, 1)) * 2), 6));
  const uint32_t tile = uint32_t(t.tile_log2);
  L.lds_small = lds_small_bytes(small_log2);
  L.lds_part = lds_part_bytes(L.max_link_buckets, tile, L.max_rc_buckets);
  L.lds_link = lds_link_bytes(uint32_t(t.link_slots_log2), L.max_rc_buckets);
  L.lds_rc = lds_rc_bytes(uint32_t(t.rc_slots_log2));
  for (int k = 0; k < 2; ++k)
    for (int r = 0; r < 2; ++r) L.lds_linkw[k][r] = lds_links_wave_bytes(kWaveHist[k], uint32_t(r));
  const size_t m = std::max(std::max(std::max(L.lds_small, L.lds_part), std::max(L.lds_link, L.lds_rc)),
                            std::max(L.lds_linkw[1][1], lds_heavy_bytes()));
  if (m > c->lds_limit) return NSGC_ERR_INVALID_ARG;
  int rc;
  const int want = t.blocks_per_cu;
  if ((rc = resident_cap(c, 0, tile, L.lds_small, want, &L.grid_small)) != NSGC_OK) return rc;
  if ((rc = resident_cap(c, 1, tile, L.lds_part, want, &L.grid_part)) != NSGC_OK) return rc;
  L.combine = t.combine_probes > 0;
  if ((rc = resident_cap(c, L.combine ? 4 : 2, tile, L.lds_link, want, &L.grid_link)) != NSGC_OK)
    return rc;
  if ((rc = resident_cap(c, 3, tile, L.lds_rc, want, &L.grid_rc)) != NSGC_OK) return rc;
  // the wavefront kernel runs four small workgroups per CU for every one of
  // the workgroup kernels' 512-thread workgroups
  for (int k = 0; k < 2; ++k)
    for (int r = 0; r < 2; ++r)
      if ((rc = resident_cap(c, r ? 7 : 5, tile, L.lds_linkw[k][r], 4 * want, &L.grid_linkw[k][r])) !=
          NSGC_OK)
        return rc;
  L.grid_finish = uint32_t(c->cus) * 4;
  L.grid_heavy = uint32_t(c->cus);   // one workgroup per row-complete window
  // the entity outputs' phase C (two tables per workgroup)
  L.lds_rce = lds_rc_ent_bytes(uint32_t(std::min(t.rc_slots_log2, 12)));
  L.grid_rce = 0;
  if (L.lds_rce <= c->lds_limit &&
      (rc = resident_cap(c, 6, tile, L.lds_rce, want, &L.grid_rce)) != NSGC_OK)
    return rc;
  *out = L;
  return NSGC_OK;
}

// Which kernels a plan needs: bit 0 the small-window kernel, bit 1 phases A
// and C, bit 2 phase B by workgroups, bit 3 phase B by wavefronts, bit 4 the
// wavefront kernel's larger counters (see wave_class), bit 5 row-complete
// windows (the heavy-source sample and the wavefront kernel's row tables).
constexpr int kVariants = 64;
int plan_variant(const HostPlan& hp) {
  return (hp.small.empty() ? 0 : 1) | (hp.win.empty() ? 0 : 2) | (hp.itemsBb ? 4 : 0) |
         (hp.itemsBw ? 8 : 0) | (hp.itemsBw && wave_class(hp.wave_rc_max) ? 16 : 0) |
         (hp.num_rows ? 32 : 0);
}

// Enqueue the kernels of one uploaded plan.  With `fixed_grid` (graph
// capture) every kernel of `variant` is launched with the full persistent
// grid; otherwise grids are trimmed to the item counts and empty phases are
// skipped.
// The buffers the large-window tier works on directly (it takes no plan).
struct LargeArgs {
  const uint32_t* src;
  const uint32_t* dst;
  unsigned long long* out;   // nsgc_stats array
  char* ws;                  // the workspace (its large-tier region per the plan's layout)
  uint32_t grid;
};

int enqueue_kernels(const HostPlan& hp, const nsgc_dev_plan* dplan, const Launch& L,
                    uint32_t tile_log2, hipStream_t s, bool fixed_grid, int variant,
                    const hipEvent_t* ev = nullptr, const LargeArgs* la = nullptr) {
  auto grid = [&](uint32_t items, uint32_t cap) { return fixed_grid ? cap : std::min(items, cap); };
  auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
  const bool small = fixed_grid ? (variant & 1) != 0 : !hp.small.empty();
  const bool part = fixed_grid ? (variant & 2) != 0 : !hp.win.empty();
  const bool linkb = fixed_grid ? (variant & 4) != 0 : hp.itemsBb > 0;
  const bool linkw = fixed_grid ? (variant & 8) != 0 : hp.itemsBw > 0;
  const bool rows = fixed_grid ? (variant & 32) != 0 : hp.num_rows > 0;
  NSGC_HIP(mark(0));
  if (small)
    NSGC_HIP(launch_small(dplan, grid(uint32_t(hp.small.size()), L.grid_small), L.lds_small, s));
  NSGC_HIP(mark(1));
  if (rows) NSGC_HIP(launch_heavy(dplan, grid(uint32_t(hp.win.size()), L.grid_heavy), s));
  if (part)
    NSGC_HIP(launch_partition(dplan, tile_log2, L.max_link_buckets, rows, grid(hp.itemsA, L.grid_part),
                              L.lds_part, s));
  NSGC_HIP(mark(2));
  // The phase-C order depends only on the partition's sizes: with wavefront
  // phase-B items it is computed by an extra workgroup of that kernel, beside
  // phase B, instead of by k_order after it.
  const bool order_in_b = part && !hp.entity && linkw;
  if (linkw) {
    const int wc = fixed_grid ? ((variant & 16) ? 1 : 0) : wave_class(hp.wave_rc_max);
    const int r = rows ? 1 : 0;
    NSGC_HIP(launch_links_wave(dplan, kWaveHist[wc], uint32_t(r), order_in_b ? 1u : 0u,
                               grid((hp.itemsBw + 3) / 4, L.grid_linkw[wc][r]), L.lds_linkw[wc][r],
                               s));
  }
  if (linkb)
    NSGC_HIP(launch_links(dplan, L.combine && !hp.entity, L.max_rc_buckets,
                          grid(hp.itemsBb, L.grid_link), L.lds_link, s));
  NSGC_HIP(mark(3));
  if (part && hp.entity) {
    NSGC_HIP(launch_rowcol_ent(dplan, grid(hp.itemsC, L.grid_rce), L.lds_rce, s));
  } else if (part) {
    if (!order_in_b) NSGC_HIP(launch_order(dplan, s));
    NSGC_HIP(launch_rowcol(dplan, grid(hp.itemsC, L.grid_rc), L.lds_rc, s));
  }
  if (part) NSGC_HIP(launch_finish(dplan, grid(uint32_t(hp.win.size()), L.grid_finish), s));
  NSGC_HIP(mark(4));
  if (!hp.large.empty()) {
    if (!la) return NSGC_ERR_INTERNAL;
    char* region = la->ws + hp.layout().large;
    for (const LargeWindow& lw : hp.large)
      NSGC_HIP(large_window_stats(la->src + lw.in_begin, la->dst + lw.in_begin, lw.n, region,
                                  la->out + (unsigned long long)lw.out_index * 9, la->grid, s));
  }
  NSGC_HIP(mark(5));
  return NSGC_OK;
}

int validate_common(const uint32_t* src, const uint32_t* dst, const int64_t* offsets,
                    int64_t num_windows, const void* out) {
  if (num_windows < 0) return NSGC_ERR_INVALID_ARG;
  if (num_windows == 0) return NSGC_OK;
  if (!offsets || !out) return NSGC_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(out) % 8 != 0) return NSGC_ERR_INVALID_ARG;
  const int rc = validate_offsets(offsets, num_windows);
  if (rc != NSGC_OK) return rc;
  if (offsets[num_windows] > offsets[0] && (!src || !dst)) return NSGC_ERR_INVALID_ARG;
  return NSGC_OK;
}

int get_slot(DevCtx* c, hipStream_t s, Slot** out) {
  auto it = c->slots.find(s);
  if (it != c->slots.end()) {
    *out = it->second;
    return NSGC_OK;
  }
  Slot* sl = new Slot;
  c->slots[s] = sl;
  *out = sl;
  return NSGC_OK;
}

// Upload one plan into slot `sl` and launch it.
int run_plan(DevCtx* c, Slot* sl, const HostPlan& hp, const Launch& L, const uint32_t* src,
             const uint32_t* dst, void* out, hipStream_t s, const hipEvent_t* ev = nullptr) {
  int rc;
  const size_t pbytes = hp.plan_bytes();
  const WsLayout lay = hp.layout();
  if ((rc = ensure_device(&sl->plan_dev, &sl->plan_cap, pbytes, s)) != NSGC_OK) return rc;
  if ((rc = ensure_device(&sl->ws, &sl->ws_cap, lay.total, s)) != NSGC_OK) return rc;
  int k = 0;
  if ((rc = take_stage(sl, pbytes, s, &k)) != NSGC_OK) return rc;
  hp.serialize(sl->stage[k], reinterpret_cast<uint64_t>(sl->plan_dev),
               reinterpret_cast<uint64_t>(sl->ws), src, dst, out);
  NSGC_HIP(hipMemcpyAsync(sl->plan_dev, sl->stage[k], pbytes, hipMemcpyHostToDevice, s));
  NSGC_HIP(hipEventRecord(sl->ev[k], s));
  sl->ev_used[k] = true;
  const LargeArgs la = {src, dst, static_cast<unsigned long long*>(out), sl->ws,
                        uint32_t(c->cus) * 8};
  return enqueue_kernels(hp, reinterpret_cast<const nsgc_dev_plan*>(sl->plan_dev), L,
                         hp.tile_log2, s, false, 0, ev, &la);
}

// Upper bound of the workspace for any batch within the limits (`large`: the
// batch may use the large-window tier).
size_t workspace_bound(int64_t max_packets, int64_t max_windows, const nsgc_tune& t,
                       bool large = true) {
  const uint64_t P = uint64_t(std::max<int64_t>(max_packets, 0));
  const uint64_t W = uint64_t(std::max<int64_t>(max_windows, 1));
  int lt = 1 << 30, rt = 1 << 30;
  for (int k = 0; k <= 32; ++k) {
    lt = std::min(lt, t.cls[k].link_target);
    if (t.cls[k].wave_target > 0) lt = std::min(lt, t.cls[k].wave_target);
    rt = std::min(rt, std::min(t.cls[k].row_target, t.cls[k].col_target));
  }
  const uint64_t MB = uint64_t(1) << t.max_link_buckets_log2;
  const uint64_t MRC = uint64_t(1) << t.max_rc_buckets_log2;
  const uint64_t T = uint64_t(1) << t.tile_log2;
  const uint64_t bmax = std::min<uint64_t>(MB, 2 * P / uint64_t(lt) + 1);
  const uint64_t rmax = std::min<uint64_t>(MRC, 2 * P / uint64_t(rt) + 1);
  const uint64_t tilemeta = (P / T + W) * (bmax + 2);
  const uint64_t lbmeta = (std::min<uint64_t>(bmax * W, 2 * P / uint64_t(lt) + W)) * (2 * rmax + 3);
  // phase-C items: R_w + C_w < 4 n_w / rt + 4 per window, at most 2 * MRC
  const uint64_t items = std::min<uint64_t>(4 * P / uint64_t(rt) + 4 * W, 2 * W * MRC);
  // bucket totals: 16 B per phase-B and per phase-C item
  const uint64_t bitems = std::min<uint64_t>(2 * P / uint64_t(lt) + 2 * W, W * MB);
  size_t b = size_t(P * 24 + (tilemeta + lbmeta + 2 * items) * 4 + (bitems + items) * 16 + 10 * 256);
  // row-complete windows: source totals per phase-B item and a heavy table per window
  if (t.row_complete) b += size_t(bitems * 16 + W * NSGC_HEAVY_SLOTS * 4 + 2 * 256);
  // a large window's region comes on top of the partitioned windows' regions
  if (large && t.large_min_log2 < 33 && P >= (uint64_t(1) << t.large_min_log2))
    b += large_window_bytes(P) + 256;
  return b;
}

// What a call on (current device, s) reads from the shared state, looked up
// under g_mu: the tuning in force (entity calls adjust it), the device
// context, the stream's slot, the launch shapes and the plain-mode switch.
struct CallCtx {
  nsgc_tune t;
  DevCtx* c = nullptr;
  Slot* sl = nullptr;
  Launch L;
  bool plain = false;
};

int begin_call(hipStream_t s, CallCtx* cc, bool entity = false, bool launch = true) {
  std::lock_guard<std::mutex> lock(g_mu);
  cc->t = current_tune();
  if (entity) {
    cc->t.combine_probes = 0;                              // links are listed by the per-link emission
    cc->t.rc_slots_log2 = std::min(cc->t.rc_slots_log2, 12);   // two phase-C tables per workgroup
  }
  cc->plain = g_plain_mode;
  int rc;
  if ((rc = get_ctx(&cc->c)) != NSGC_OK) return rc;
  if ((rc = get_slot(cc->c, s, &cc->sl)) != NSGC_OK) return rc;
  return launch ? launch_params(cc->c, cc->t, &cc->L) : NSGC_OK;
}

// The batched form (caller holds the slot's lock, arguments validated,
// num_windows > 0).
int batched_locked(const CallCtx& cc, const uint32_t* src, const uint32_t* dst,
                   const int64_t* window_offsets, int64_t num_windows, nsgc_stats* out_stats,
                   hipStream_t s) {
  HostPlan hp;
  int rc;
  if ((rc = make_plan(window_offsets, num_windows, cc.t, &hp)) != NSGC_OK) return rc;
  return run_plan(cc.c, cc.sl, hp, cc.L, src, dst, out_stats, s);
}

// The plain form: one plan and one launch sequence per window (caller holds
// the slot's lock, arguments validated, num_windows > 0).
int plain_locked(const CallCtx& cc, const uint32_t* src, const uint32_t* dst,
                 const int64_t* window_offsets, int64_t num_windows, nsgc_stats* out_stats,
                 hipStream_t s) {
  const nsgc_tune& t = cc.t;
  DevCtx* c = cc.c;
  Slot* sl = cc.sl;
  const Launch& L = cc.L;
  int rc;

  // One plan per window, all uploaded with one copy; the windows then run one
  // launch sequence each, in order, sharing one workspace.
  std::vector<HostPlan> plans(static_cast<size_t>(num_windows));
  std::vector<size_t> at(static_cast<size_t>(num_windows));
  size_t pbytes = 0, wsmax = 0;
  for (int64_t w = 0; w < num_windows; ++w) {
    if ((rc = make_plan(window_offsets + w, 1, t, &plans[size_t(w)])) != NSGC_OK) return rc;
    at[size_t(w)] = pbytes;
    pbytes += (plans[size_t(w)].plan_bytes() + 255) / 256 * 256;
    wsmax = std::max(wsmax, plans[size_t(w)].layout().total);
  }
  if ((rc = ensure_device(&sl->plan_dev, &sl->plan_cap, pbytes, s)) != NSGC_OK) return rc;
  if ((rc = ensure_device(&sl->ws, &sl->ws_cap, wsmax, s)) != NSGC_OK) return rc;
  int k = 0;
  if ((rc = take_stage(sl, pbytes, s, &k)) != NSGC_OK) return rc;
  for (int64_t w = 0; w < num_windows; ++w)
    plans[size_t(w)].serialize(sl->stage[k] + at[size_t(w)],
                               reinterpret_cast<uint64_t>(sl->plan_dev + at[size_t(w)]),
                               reinterpret_cast<uint64_t>(sl->ws), src, dst, out_stats + w);
  NSGC_HIP(hipMemcpyAsync(sl->plan_dev, sl->stage[k], pbytes, hipMemcpyHostToDevice, s));
  NSGC_HIP(hipEventRecord(sl->ev[k], s));
  sl->ev_used[k] = true;
  for (int64_t w = 0; w < num_windows; ++w) {
    const LargeArgs la = {src, dst, reinterpret_cast<unsigned long long*>(out_stats + w), sl->ws,
                          uint32_t(c->cus) * 8};
    rc = enqueue_kernels(plans[size_t(w)],
                         reinterpret_cast<const nsgc_dev_plan*>(sl->plan_dev + at[size_t(w)]), L,
                         plans[size_t(w)].tile_log2, s, false, 0, nullptr, &la);
    if (rc != NSGC_OK) return rc;
  }
  return NSGC_OK;
}

// Pre-size the workspace, plan buffer and staging ring of (current device, s).
int reserve_call(int64_t max_packets, int64_t max_windows, hipStream_t s) {
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  CallCtx cc;
  int rc;
  if ((rc = begin_call(s, &cc, false, false)) != NSGC_OK) return rc;
  Slot* sl = cc.sl;
  std::lock_guard<std::mutex> lock(sl->mu);
  const size_t pb = plan_bound(max_packets, max_windows, cc.t);
  if ((rc = ensure_device(&sl->plan_dev, &sl->plan_cap, pb, s)) != NSGC_OK) return rc;
  if ((rc = ensure_device(&sl->ws, &sl->ws_cap, workspace_bound(max_packets, max_windows, cc.t), s)) !=
      NSGC_OK)
    return rc;
  for (int k = 0; k < kStages; ++k) {
    int idx = 0;
    if ((rc = take_stage(sl, pb, s, &idx)) != NSGC_OK) return rc;
  }
  return NSGC_OK;
}


}  // namespace

namespace nsgc {

int validate_call(const uint32_t* src, const uint32_t* dst, const int64_t* offsets,
                  int64_t num_windows, const void* out) {
  return validate_common(src, dst, offsets, num_windows, out);
}

int record_hip_error(int e) { return hip_fail(hipError_t(e)); }

// The batched form on caller-provided device buffers: `plan_dev` (plan_cap
// bytes) receives the plan and `ws` (ws_cap bytes) serves as the workspace.
// Nothing is allocated on the device or in pinned host memory: the plan is
// staged in the device context's host buffer, sized once at the first call
// on the device.  Batches whose plan or workspace exceed the buffers return
// NSGC_ERR_TOO_LARGE with nothing enqueued.
int run_fixed_scratch(const uint32_t* src, const uint32_t* dst, const int64_t* window_offsets,
                      int64_t num_windows, nsgc_stats* out_stats, void* stream, char* plan_dev,
                      size_t plan_cap, char* ws, size_t ws_cap) {
  int rc = validate_common(src, dst, window_offsets, num_windows, out_stats);
  if (rc != NSGC_OK || num_windows == 0) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  nsgc_tune t;
  DevCtx* c = nullptr;
  Launch L;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    t = current_tune();
    if ((rc = get_ctx(&c)) != NSGC_OK) return rc;
    if ((rc = launch_params(c, t, &L)) != NSGC_OK) return rc;
  }
  HostPlan hp;
  if ((rc = make_plan(window_offsets, num_windows, t, &hp)) != NSGC_OK) return rc;
  const size_t pbytes = hp.plan_bytes();
  const WsLayout lay = hp.layout();
  if (pbytes > plan_cap || lay.total > ws_cap) return NSGC_ERR_TOO_LARGE;
  FixedState& f = c->fixed;
  std::lock_guard<std::mutex> lock(f.mu);
  if (!f.copied) NSGC_HIP(hipEventCreateWithFlags(&f.copied, hipEventDisableTiming));
  if (!f.done) NSGC_HIP(hipEventCreateWithFlags(&f.done, hipEventDisableTiming));
  if (f.stage.size() < plan_cap) f.stage.resize(plan_cap);
  // the previous call's plan copy must have read the staging buffer
  if (f.used) NSGC_HIP(hipEventSynchronize(f.copied));
  hp.serialize(f.stage.data(), reinterpret_cast<uint64_t>(plan_dev), reinterpret_cast<uint64_t>(ws),
               src, dst, out_stats);
  // every call on the device shares its scratch: order after the last one
  if (f.used && f.last_stream != s) NSGC_HIP(hipStreamWaitEvent(s, f.done, 0));
  NSGC_HIP(hipMemcpyAsync(plan_dev, f.stage.data(), pbytes, hipMemcpyHostToDevice, s));
  NSGC_HIP(hipEventRecord(f.copied, s));
  const LargeArgs la = {src, dst, reinterpret_cast<unsigned long long*>(out_stats), ws,
                        uint32_t(c->cus) * 8};
  rc = enqueue_kernels(hp, reinterpret_cast<const nsgc_dev_plan*>(plan_dev), L, hp.tile_log2, s,
                       false, 0, nullptr, &la);
  if (rc != NSGC_OK) return rc;
  NSGC_HIP(hipEventRecord(f.done, s));
  f.last_stream = s;
  f.used = true;
  return NSGC_OK;
}

}  // namespace nsgc

// ---------------------------------------------------------------------------

extern "C" {

const char* nsgc_status_string(int status) {
  switch (status) {
    case NSGC_OK: return "ok";
    case NSGC_ERR_INVALID_ARG: return "invalid argument";
    case NSGC_ERR_BAD_OFFSETS: return "bad window offsets (negative, decreasing, or a window of 2^32 or more packets)";
    case NSGC_ERR_NO_MEMORY: return "device workspace allocation failed";
    case NSGC_ERR_HIP: return "HIP runtime error";
    case NSGC_ERR_INTERNAL: return "internal error";
    case NSGC_ERR_CAPTURING: return "called on a stream that is being captured";
    case NSGC_ERR_TOO_LARGE: return "batch does not fit the fixed scratch of nsgc_window_stats_noalloc";
    default: return "unknown status";
  }
}

int nsgc_last_hip_error(void) { return t_last_hip_error; }

int nsgc_window_stats(const uint32_t* src, const uint32_t* dst, const int64_t* window_offsets,
                      int64_t num_windows, nsgc_stats* out_stats, void* stream) {
  int rc = validate_common(src, dst, window_offsets, num_windows, out_stats);
  if (rc != NSGC_OK || num_windows == 0) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // The plan travels through a rotating staging ring and a per-stream
  // workspace that later calls reuse, so a captured call could not be
  // replayed safely: capture the graph form (nsgc_graph_*) instead.
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  CallCtx cc;
  if ((rc = begin_call(s, &cc)) != NSGC_OK) return rc;
  std::lock_guard<std::mutex> lock(cc.sl->mu);
  if (cc.plain) return plain_locked(cc, src, dst, window_offsets, num_windows, out_stats, s);
  return batched_locked(cc, src, dst, window_offsets, num_windows, out_stats, s);
}

int nsgc_window_stats_plain(const uint32_t* src, const uint32_t* dst,
                            const int64_t* window_offsets, int64_t num_windows,
                            nsgc_stats* out_stats, void* stream) {
  int rc = validate_common(src, dst, window_offsets, num_windows, out_stats);
  if (rc != NSGC_OK || num_windows == 0) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  CallCtx cc;
  if ((rc = begin_call(s, &cc)) != NSGC_OK) return rc;
  std::lock_guard<std::mutex> lock(cc.sl->mu);
  return plain_locked(cc, src, dst, window_offsets, num_windows, out_stats, s);
}

namespace {

// Host offsets of one entity list: num_windows + 1 non-decreasing values >= 0.
int check_list_offsets(const int64_t* off, int64_t num_windows, const void* list) {
  if (!off) return NSGC_ERR_INVALID_ARG;
  if (off[0] < 0) return NSGC_ERR_BAD_OFFSETS;
  for (int64_t w = 0; w < num_windows; ++w)
    if (off[w + 1] < off[w]) return NSGC_ERR_BAD_OFFSETS;
  if (off[num_windows] > off[0] && !list) return NSGC_ERR_INVALID_ARG;
  return NSGC_OK;
}

int entities_call(const uint32_t* src, const uint32_t* dst, const int64_t* window_offsets,
                  int64_t num_windows, const int64_t* const* list_off, void* const* lists,
                  nsgc_entity_counts* counts, void* stream) {
  int rc = validate_common(src, dst, window_offsets, num_windows, counts);
  if (rc != NSGC_OK || num_windows == 0) return rc;
  if (list_off)
    for (int k = 0; k < 3; ++k)
      if ((rc = check_list_offsets(list_off[k], num_windows, lists[k])) != NSGC_OK) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  CallCtx cc;
  if ((rc = begin_call(s, &cc, true)) != NSGC_OK) return rc;
  std::lock_guard<std::mutex> lock(cc.sl->mu);
  HostPlan hp;
  if ((rc = make_plan(window_offsets, num_windows, cc.t, &hp, true)) != NSGC_OK) return rc;
  hp.ent_cur.assign(size_t(num_windows) * 3, 0);
  hp.ent_end.assign(size_t(num_windows) * 3, 0);
  if (list_off) {
    for (int64_t w = 0; w < num_windows; ++w)
      for (int k = 0; k < 3; ++k) {
        hp.ent_cur[size_t(w) * 3 + k] = uint64_t(list_off[k][w]);
        hp.ent_end[size_t(w) * 3 + k] = uint64_t(list_off[k][w + 1]);
      }
    hp.ent_links = lists[0];
    hp.ent_src = lists[1];
    hp.ent_dst = lists[2];
  }
  hp.ent_counts = counts;
  if (!hp.win.empty() && cc.L.grid_rce == 0) return NSGC_ERR_INVALID_ARG;
  return run_plan(cc.c, cc.sl, hp, cc.L, src, dst, nullptr, s);
}

}  // namespace

int nsgc_window_entity_counts(const uint32_t* src, const uint32_t* dst,
                              const int64_t* window_offsets, int64_t num_windows,
                              nsgc_entity_counts* counts, void* stream) {
  return entities_call(src, dst, window_offsets, num_windows, nullptr, nullptr, counts, stream);
}

int nsgc_window_entities(const uint32_t* src, const uint32_t* dst,
                         const int64_t* window_offsets, int64_t num_windows,
                         const int64_t* link_offsets, int64_t* links,
                         const int64_t* source_offsets, int64_t* sources,
                         const int64_t* destination_offsets, int64_t* destinations,
                         nsgc_entity_counts* counts, void* stream) {
  const int64_t* offs[3] = {link_offsets, source_offsets, destination_offsets};
  void* lists[3] = {links, sources, destinations};
  return entities_call(src, dst, window_offsets, num_windows, offs, lists, counts, stream);
}

int nsgc_anonymize(const uint32_t* src, const uint32_t* dst, int64_t num_packets, uint64_t seed,
                   uint32_t* anon_src, uint32_t* anon_dst, uint64_t* num_addresses, void* stream) {
  if (num_packets < 0 || num_packets >= (int64_t(1) << 31)) return NSGC_ERR_INVALID_ARG;
  if (!num_addresses || reinterpret_cast<uintptr_t>(num_addresses) % 8 != 0)
    return NSGC_ERR_INVALID_ARG;
  if (num_packets > 0 && (!src || !dst || !anon_src || !anon_dst)) return NSGC_ERR_INVALID_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  CallCtx cc;
  int rc;
  if ((rc = begin_call(s, &cc, false, false)) != NSGC_OK) return rc;
  DevCtx* c = cc.c;
  Slot* sl = cc.sl;
  std::lock_guard<std::mutex> lock(sl->mu);
  const unsigned long long n = (unsigned long long)num_packets;
  if ((rc = ensure_device(&sl->ws, &sl->ws_cap, anonymize_bytes(n), s)) != NSGC_OK) return rc;
  NSGC_HIP(anonymize(src, dst, n, seed, anon_src, anon_dst,
                     reinterpret_cast<unsigned long long*>(num_addresses), sl->ws,
                     uint32_t(c->cus) * 8, s));
  return NSGC_OK;
}

int nsgc_set_plain_mode(int on) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_plain_mode = on != 0;
  return NSGC_OK;
}

int nsgc_get_plain_mode(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  return g_plain_mode ? 1 : 0;
}

int nsgc_window_stats_timed(const uint32_t* src, const uint32_t* dst,
                            const int64_t* window_offsets, int64_t num_windows,
                            nsgc_stats* out_stats, void* stream, float* phase_ms) {
  if (!phase_ms) return NSGC_ERR_INVALID_ARG;
  int rc = validate_common(src, dst, window_offsets, num_windows, out_stats);
  if (rc != NSGC_OK) return rc;
  for (int i = 0; i < 5; ++i) phase_ms[i] = 0.0f;
  if (num_windows == 0) return NSGC_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return NSGC_ERR_CAPTURING;
  CallCtx cc;
  if ((rc = begin_call(s, &cc)) != NSGC_OK) return rc;
  Slot* sl = cc.sl;
  std::lock_guard<std::mutex> lock(sl->mu);
  HostPlan hp;
  if ((rc = make_plan(window_offsets, num_windows, cc.t, &hp)) != NSGC_OK) return rc;
  for (int i = 0; i < 6; ++i)
    if (!sl->phase_ev[i]) NSGC_HIP(hipEventCreate(&sl->phase_ev[i]));
  if ((rc = run_plan(cc.c, sl, hp, cc.L, src, dst, out_stats, s, sl->phase_ev)) != NSGC_OK) return rc;
  NSGC_HIP(hipEventSynchronize(sl->phase_ev[5]));
  for (int i = 0; i < 5; ++i)
    NSGC_HIP(hipEventElapsedTime(&phase_ms[i], sl->phase_ev[i], sl->phase_ev[i + 1]));
  return NSGC_OK;
}

int nsgc_reserve(int64_t max_packets, int64_t max_windows) {
  if (max_packets < 0 || max_windows < 0) return NSGC_ERR_INVALID_ARG;
  return reserve_call(max_packets, max_windows, nullptr);
}

int nsgc_reserve_stream(int64_t max_packets, int64_t max_windows, void* stream) {
  if (max_packets < 0 || max_windows < 0) return NSGC_ERR_INVALID_ARG;
  return reserve_call(max_packets, max_windows, static_cast<hipStream_t>(stream));
}

int nsgc_release(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0;
  NSGC_HIP(hipGetDevice(&dev));
  auto it = g_devs.find(dev);
  if (it == g_devs.end()) return NSGC_OK;
  NSGC_HIP(hipDeviceSynchronize());
  // the slots stay (a call may hold a pointer to one); their buffers go
  for (auto& kv : it->second->slots) {
    Slot* sl = kv.second;
    std::lock_guard<std::mutex> slock(sl->mu);
    if (sl->plan_dev) (void)hipFree(sl->plan_dev);
    if (sl->ws) (void)hipFree(sl->ws);
    sl->plan_dev = sl->ws = nullptr;
    sl->plan_cap = sl->ws_cap = 0;
    for (int k = 0; k < kStages; ++k) {
      if (sl->stage[k]) (void)hipHostFree(sl->stage[k]);
      if (sl->ev[k]) (void)hipEventDestroy(sl->ev[k]);
      sl->stage[k] = nullptr;
      sl->stage_cap[k] = 0;
      sl->ev[k] = nullptr;
      sl->ev_used[k] = false;
    }
    for (int k = 0; k < 6; ++k) {
      if (sl->phase_ev[k]) (void)hipEventDestroy(sl->phase_ev[k]);
      sl->phase_ev[k] = nullptr;
    }
    sl->next = 0;
  }
  return NSGC_OK;
}

int nsgc_default_tune(nsgc_tune* out) {
  if (!out) return NSGC_ERR_INVALID_ARG;
  default_tune(out);
  return NSGC_OK;
}

int nsgc_get_tune(nsgc_tune* out) {
  if (!out) return NSGC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  *out = current_tune();
  return NSGC_OK;
}

int nsgc_set_tune(const nsgc_tune* tune) {
  if (!tune) return NSGC_ERR_INVALID_ARG;
  const int rc = check_tune(*tune);
  if (rc != NSGC_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  g_tune = *tune;
  g_tune_set = true;
  return NSGC_OK;
}

int nsgc_plan_sizes(const int64_t* window_offsets, int64_t num_windows, int64_t* plan_bytes,
                    int64_t* workspace_bytes, int64_t* plan_bound_bytes,
                    int64_t* workspace_bound_bytes) {
  if (num_windows < 0) return NSGC_ERR_INVALID_ARG;
  if (num_windows > 0 && !window_offsets) return NSGC_ERR_INVALID_ARG;
  if (num_windows > 0) {
    const int rc = validate_offsets(window_offsets, num_windows);
    if (rc != NSGC_OK) return rc;
  }
  nsgc_tune t;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    t = current_tune();
  }
  HostPlan hp;
  const int rc = make_plan(window_offsets, num_windows, t, &hp);
  if (rc != NSGC_OK) return rc;
  const int64_t P = num_windows > 0 ? window_offsets[num_windows] - window_offsets[0] : 0;
  if (plan_bytes) *plan_bytes = int64_t(hp.plan_bytes());
  if (workspace_bytes) *workspace_bytes = int64_t(hp.layout().total);
  if (plan_bound_bytes) *plan_bound_bytes = int64_t(plan_bound(P, num_windows, t));
  if (workspace_bound_bytes) *workspace_bound_bytes = int64_t(workspace_bound(P, num_windows, t));
  return NSGC_OK;
}

int nsgc_plan_inspect(const int64_t* window_offsets, int64_t num_windows, int32_t* tier,
                      int32_t* log2_link_buckets, int32_t* log2_row_buckets,
                      int32_t* log2_col_buckets, int64_t* tiles, int64_t* workspace_bytes) {
  if (num_windows < 0) return NSGC_ERR_INVALID_ARG;
  if (num_windows > 0 && !window_offsets) return NSGC_ERR_INVALID_ARG;
  if (num_windows > 0) {
    const int rc = validate_offsets(window_offsets, num_windows);
    if (rc != NSGC_OK) return rc;
  }
  nsgc_tune t;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    t = current_tune();
  }
  HostPlan hp;
  const int rc = make_plan(window_offsets, num_windows, t, &hp);
  if (rc != NSGC_OK) return rc;
  size_t m = 0;
  for (int64_t w = 0; w < num_windows; ++w) {
    if (tier) tier[w] = hp.tier[size_t(w)];
    const bool part = hp.tier[size_t(w)] == 2;
    const nsgc_win_desc* d = part ? &hp.win[m] : nullptr;
    if (log2_link_buckets) log2_link_buckets[w] = d ? d->logB : -1;
    if (log2_row_buckets) log2_row_buckets[w] = d ? d->logR : -1;
    if (log2_col_buckets) log2_col_buckets[w] = d ? d->logC : -1;
    if (tiles) tiles[w] = d ? int64_t(d->ntiles) : 0;
    if (part) ++m;
  }
  if (workspace_bytes) *workspace_bytes = int64_t(hp.layout().total);
  return NSGC_OK;
}

// ---------------------------------------------------------------------------
// Graph form.
// ---------------------------------------------------------------------------

}  // extern "C"

struct nsgc_graph {
  std::mutex mu;   // launches of one graph object (plans, instances, workspace)
  int device = 0;
  nsgc_tune tune;
  Launch L;
  int64_t max_packets = 0, max_windows = 0;
  hipStream_t capture = nullptr;
  // two instances so the host can plan batch i+1 while batch i runs
  struct Inst {
    char* plan_dev = nullptr;
    size_t plan_cap = 0;
    char* stage = nullptr;
    hipGraph_t graph[kVariants] = {};     // indexed by plan variant (see plan_variant)
    hipGraphExec_t exec[kVariants] = {};
    // the plan-upload node of each variant, resized to the plan at every
    // launch (null: the node keeps uploading plan_cap bytes)
    hipGraphNode_t copy[kVariants] = {};
    hipEvent_t done = nullptr;
    hipStream_t stream = nullptr;  // stream of the last launch
    bool used = false;
  } inst[2];
  int next = 0;
  char* ws = nullptr;
  size_t ws_cap = 0;
};

namespace {

int capture_instance(nsgc_graph* g, nsgc_graph::Inst& in, int variant) {
  NSGC_HIP(hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipMemcpyAsync(in.plan_dev, in.stage, in.plan_cap, hipMemcpyHostToDevice,
                                g->capture);
  HostPlan empty;
  int rc = NSGC_OK;
  if (e == hipSuccess) {
    rc = enqueue_kernels(empty, reinterpret_cast<const nsgc_dev_plan*>(in.plan_dev), g->L,
                         uint32_t(g->tune.tile_log2), g->capture, true, variant);
  }
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(g->capture, &graph);
  if (e != hipSuccess) return hip_fail(e);
  if (rc != NSGC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e2 != hipSuccess) return hip_fail(e2);
  in.graph[variant] = graph;
  NSGC_HIP(hipGraphInstantiate(&in.exec[variant], graph, nullptr, nullptr, 0));
  // The plan-upload node, so that each launch copies only its plan: the
  // bound it was captured with is sized for the graph's largest batch.
  size_t nn = 0;
  if (hipGraphGetNodes(graph, nullptr, &nn) == hipSuccess && nn > 0) {
    std::vector<hipGraphNode_t> nodes(nn);
    if (hipGraphGetNodes(graph, nodes.data(), &nn) == hipSuccess) {
      for (size_t i = 0; i < nn; ++i) {
        hipGraphNodeType type;
        if (hipGraphNodeGetType(nodes[i], &type) == hipSuccess && type == hipGraphNodeTypeMemcpy) {
          in.copy[variant] = nodes[i];
          break;
        }
      }
    }
  }
  (void)hipGetLastError();   // no node found: every launch uploads plan_cap bytes
  return NSGC_OK;
}

void destroy_graph(nsgc_graph* g) {
  for (auto& in : g->inst) {
    if (in.done) (void)hipEventSynchronize(in.done);
    for (int v = 0; v < kVariants; ++v) {
      if (in.exec[v]) (void)hipGraphExecDestroy(in.exec[v]);
      if (in.graph[v]) (void)hipGraphDestroy(in.graph[v]);
    }
    if (in.plan_dev) (void)hipFree(in.plan_dev);
    if (in.stage) (void)hipHostFree(in.stage);
    if (in.done) (void)hipEventDestroy(in.done);
  }
  if (g->ws) (void)hipFree(g->ws);
  if (g->capture) (void)hipStreamDestroy(g->capture);
  delete g;
}

}  // namespace

extern "C" {

int nsgc_graph_create(int64_t max_packets, int64_t max_windows, nsgc_graph** out) {
  if (!out || max_packets < 0 || max_windows < 1) return NSGC_ERR_INVALID_ARG;
  *out = nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  DevCtx* c = nullptr;
  int rc;
  if ((rc = get_ctx(&c)) != NSGC_OK) return rc;
  nsgc_graph* g = new nsgc_graph;
  g->device = c->device;
  g->tune = current_tune();
  g->max_packets = max_packets;
  g->max_windows = max_windows;
  if ((rc = launch_params(c, g->tune, &g->L)) != NSGC_OK) {
    destroy_graph(g);
    return rc;
  }
  hipError_t e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
  if (e != hipSuccess) {
    destroy_graph(g);
    return hip_fail(e);
  }
  const size_t pb = plan_bound(max_packets, max_windows, g->tune);
  for (auto& in : g->inst) {
    void* p = nullptr;
    if ((e = hipMalloc(&p, pb)) != hipSuccess) { destroy_graph(g); return NSGC_ERR_NO_MEMORY; }
    in.plan_dev = static_cast<char*>(p);
    in.plan_cap = pb;
    if ((e = hipHostMalloc(&p, pb, hipHostMallocDefault)) != hipSuccess) {
      destroy_graph(g);
      return hip_fail(e);
    }
    in.stage = static_cast<char*>(p);
    std::memset(in.stage, 0, pb);
    if ((e = hipEventCreateWithFlags(&in.done, hipEventDisableTiming)) != hipSuccess) {
      destroy_graph(g);
      return hip_fail(e);
    }
  }
  if ((rc = ensure_device(&g->ws, &g->ws_cap,
                          workspace_bound(max_packets, max_windows, g->tune, false),
                          g->capture)) != NSGC_OK) {
    destroy_graph(g);
    return rc;
  }
  *out = g;
  return NSGC_OK;
}

int nsgc_graph_launch(nsgc_graph* g, const uint32_t* src, const uint32_t* dst,
                      const int64_t* window_offsets, int64_t num_windows, nsgc_stats* out_stats,
                      void* stream) {
  if (!g) return NSGC_ERR_INVALID_ARG;
  int rc = validate_common(src, dst, window_offsets, num_windows, out_stats);
  if (rc != NSGC_OK || num_windows == 0) return rc;
  if (num_windows > g->max_windows) return NSGC_ERR_INVALID_ARG;
  if (window_offsets[num_windows] - window_offsets[0] > g->max_packets) return NSGC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g->mu);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  NSGC_HIP(hipGetDevice(&dev));
  if (dev != g->device) return NSGC_ERR_INVALID_ARG;
  HostPlan hp;   // a captured graph has no large-window tier (its launches are fixed)
  if ((rc = make_plan(window_offsets, num_windows, g->tune, &hp, false, false)) != NSGC_OK)
    return rc;
  if (hp.plan_bytes() > g->inst[0].plan_cap) return NSGC_ERR_INTERNAL;
  const size_t need = hp.layout().total;
  if (need > g->ws_cap) {
    // wait for both instances before moving the shared workspace
    for (auto& in : g->inst)
      if (in.used) NSGC_HIP(hipEventSynchronize(in.done));
    if ((rc = ensure_device(&g->ws, &g->ws_cap, need, s)) != NSGC_OK) return rc;
  }
  nsgc_graph::Inst& in = g->inst[g->next];
  if (in.used) NSGC_HIP(hipEventSynchronize(in.done));
  const int variant = plan_variant(hp);
  if (!in.exec[variant] && (rc = capture_instance(g, in, variant)) != NSGC_OK) return rc;
  hp.serialize(in.stage, reinterpret_cast<uint64_t>(in.plan_dev), reinterpret_cast<uint64_t>(g->ws),
               src, dst, out_stats);
  // Both instances share the workspace: a launch on another stream than the
  // other instance's last one waits (on the device) for that launch to end.
  const nsgc_graph::Inst& other = g->inst[g->next ^ 1];
  if (other.used && other.stream != s) NSGC_HIP(hipStreamWaitEvent(s, other.done, 0));
  if (in.copy[variant])   // upload this plan's bytes only
    NSGC_HIP(hipGraphExecMemcpyNodeSetParams1D(in.exec[variant], in.copy[variant], in.plan_dev,
                                               in.stage, hp.plan_bytes(), hipMemcpyHostToDevice));
  NSGC_HIP(hipGraphLaunch(in.exec[variant], s));
  NSGC_HIP(hipEventRecord(in.done, s));
  in.stream = s;
  in.used = true;
  g->next ^= 1;
  return NSGC_OK;
}

int nsgc_graph_destroy(nsgc_graph* g) {
  if (!g) return NSGC_ERR_INVALID_ARG;
  destroy_graph(g);   // no launch of g may overlap (see nsgc.h)
  return NSGC_OK;
}

}  // extern "C"
