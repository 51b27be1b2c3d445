// Host planner (see nsgc_plan.h for the tiers and phases it lays out).
#include "nsgc_planner.hpp"

#include "nsgc_large.hpp"

#include <algorithm>
#include <cstring>

namespace nsgc {

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

int ceil_log2(uint64_t x) {
  int k = 0;
  while ((uint64_t(1) << k) < x) ++k;
  return k;
}

void default_tune(nsgc_tune* t) {
  std::memset(t, 0, sizeof(*t));
  t->small_max = 1024;
  t->tile_log2 = 14;
  t->link_slots_log2 = 12;
  t->rc_slots_log2 = 12;
  t->blocks_per_cu = 3;
  t->max_link_buckets_log2 = 11;
  t->max_rc_buckets_log2 = 10;
  t->max_sweeps_log2 = 24;
  t->combine_probes = 0;
  t->large_min_log2 = 24;
  t->row_complete = 0;
  // Per size class (windows of [2^k, 2^(k+1)) packets): below 2^23 packets a
  // link bucket holds at most as many packets as its LDS table has slots (at
  // 2^23, twice as many), so it sweeps only when nearly all its packets are
  // distinct links.  A row or column bucket of a window of 2^19 packets or
  // more holds up to four times as many packets as its table has slots: its
  // ids are distinct sources (destinations), of which large windows of
  // heavy-tailed traffic have far fewer than packets (2^23-packet windows
  // measured 0.03-0.1 distinct ids per packet), and the larger phase-C items
  // and longer phase-B segments measured 11% faster per batch than twice as
  // many buckets.  Windows below 2^19 packets keep the smaller buckets, which
  // measured faster there.
  for (int k = 0; k <= 32; ++k) {
    nsgc_tune_class& c = t->cls[k];
    c.link_target = k < 19 ? 2048 : k < 23 ? 4096 : 8192;
    c.row_target = c.col_target = k < 19 ? 4096 : 16384;
    c.wave_target = 256;
  }
}

int check_tune(const nsgc_tune& t) {
  if (t.small_max < 0 || t.small_max > 2048) return NSGC_ERR_INVALID_ARG;
  if (t.tile_log2 < 11 || t.tile_log2 > 14) return NSGC_ERR_INVALID_ARG;
  if (t.link_slots_log2 < 10 || t.link_slots_log2 > 12) return NSGC_ERR_INVALID_ARG;
  if (t.rc_slots_log2 < 10 || t.rc_slots_log2 > 13) return NSGC_ERR_INVALID_ARG;
  if (t.blocks_per_cu < 1 || t.blocks_per_cu > 16) return NSGC_ERR_INVALID_ARG;
  if (t.max_link_buckets_log2 < 0 || t.max_link_buckets_log2 > 12) return NSGC_ERR_INVALID_ARG;
  if (t.max_rc_buckets_log2 < 0 || t.max_rc_buckets_log2 > 12) return NSGC_ERR_INVALID_ARG;
  if (t.max_sweeps_log2 < 0 || t.max_sweeps_log2 > 24) return NSGC_ERR_INVALID_ARG;
  if (t.combine_probes < 0 || t.combine_probes > 64) return NSGC_ERR_INVALID_ARG;
  if (t.large_min_log2 < 20 || t.large_min_log2 > 33) return NSGC_ERR_INVALID_ARG;
  if (t.row_complete < 0 || t.row_complete > 1) return NSGC_ERR_INVALID_ARG;
  for (int k = 0; k <= 32; ++k) {
    const nsgc_tune_class& c = t.cls[k];
    if (c.link_target < 64 || c.row_target < 64 || c.col_target < 64) return NSGC_ERR_INVALID_ARG;
    if (c.wave_target != 0 && (c.wave_target < 64 || c.wave_target > 2048)) return NSGC_ERR_INVALID_ARG;
  }
  return NSGC_OK;
}

int validate_offsets(const int64_t* offsets, int64_t num_windows) {
  if (offsets[0] < 0) return NSGC_ERR_BAD_OFFSETS;
  for (int64_t w = 0; w < num_windows; ++w) {
    const int64_t n = offsets[w + 1] - offsets[w];
    if (offsets[w + 1] < offsets[w]) return NSGC_ERR_BAD_OFFSETS;
    if (n > int64_t(0xFFFFFFFFll)) return NSGC_ERR_BAD_OFFSETS;
  }
  return NSGC_OK;
}

int make_plan(const int64_t* offsets, int64_t num_windows, const nsgc_tune& tune,
              HostPlan* p, bool entity, bool allow_large) {
  p->large.clear();
  p->large_max = 0;
  p->entity = entity;
  p->ent_cur.clear();
  p->ent_end.clear();
  p->small.clear();
  p->win.clear();
  p->prefA.clear();
  p->prefB.clear();
  p->prefC.clear();
  p->itemwinB.clear();
  p->itemwinC.clear();
  p->mapBb.clear();
  p->mapBw.clear();
  p->itemsBb = p->itemsBw = 0;
  p->wave_rc_max = 0;
  p->num_rows = 0;
  p->tier.assign(size_t(num_windows), 0);
  p->ws_elems = p->tilemeta_words = p->lbmeta_words = 0;
  p->tile_log2 = uint32_t(tune.tile_log2);
  p->link_slots_log2 = uint32_t(tune.link_slots_log2);
  p->rc_slots_log2 = uint32_t(tune.rc_slots_log2);
  p->max_sweeps_log2 = uint32_t(tune.max_sweeps_log2);
  p->combine_probes = uint32_t(tune.combine_probes);
  p->small_slots_log2 = uint32_t(std::max(ceil_log2(uint64_t(std::max(tune.small_max, 1)) * 2), 6));

  const uint64_t tile = uint64_t(1) << tune.tile_log2;
  uint64_t a = 0, b = 0, c = 0;
  for (int64_t w = 0; w < num_windows; ++w) {
    const uint64_t n = uint64_t(offsets[w + 1] - offsets[w]);
    if (n <= uint64_t(tune.small_max)) {
      nsgc_small_desc s;
      s.in_begin = offsets[w];
      s.n = uint32_t(n);
      s.out_index = uint32_t(w);
      p->small.push_back(s);
      p->tier[size_t(w)] = n == 0 ? 0 : 1;
      continue;
    }
    if (allow_large && !entity && tune.large_min_log2 < 33 &&
        n >= (uint64_t(1) << tune.large_min_log2)) {
      p->large.push_back({offsets[w], n, uint32_t(w)});
      p->large_max = std::max(p->large_max, n);
      p->tier[size_t(w)] = 3;
      continue;
    }
    p->tier[size_t(w)] = 2;
    int cls = 0;
    while (cls < 32 && (uint64_t(1) << (cls + 1)) <= n) ++cls;
    const nsgc_tune_class& tc = tune.cls[cls];
    const int capB = tune.max_link_buckets_log2, capRC = tune.max_rc_buckets_log2;
    nsgc_win_desc d;
    std::memset(&d, 0, sizeof d);
    d.in_begin = offsets[w];
    d.n = uint32_t(n);
    d.out_index = uint32_t(w);
    d.logB = uint8_t(std::min(ceil_log2((n + uint64_t(tc.link_target) - 1) / uint64_t(tc.link_target)), capB));
    d.logR = uint8_t(std::min(ceil_log2((n + uint64_t(tc.row_target) - 1) / uint64_t(tc.row_target)), capRC));
    d.logC = uint8_t(std::min(ceil_log2((n + uint64_t(tc.col_target) - 1) / uint64_t(tc.col_target)), capRC));
    if (entity) d.logR = d.logC = std::max(d.logR, d.logC);   // merged phase-C items
    // one wavefront per link bucket when the window's buckets fit its tables
    if (tc.wave_target > 0 && (1u << d.logR) <= NSGC_WAVE_MAX_RC && (1u << d.logC) <= NSGC_WAVE_MAX_RC) {
      const int lw = ceil_log2((n + uint64_t(tc.wave_target) - 1) / uint64_t(tc.wave_target));
      if (lw <= capB) {
        d.logB = uint8_t(lw);
        d.wave = 1;
        p->wave_rc_max = std::max(p->wave_rc_max, 1u << std::max(d.logR, d.logC));
      }
    }
    // row-complete: wavefront windows of two or more link buckets
    if (tune.row_complete && d.wave && !entity && d.logB >= 1) {
      d.rows = 1;
      ++p->num_rows;
    }
    d.ntiles = uint32_t((n + tile - 1) / tile);
    d.counter = uint32_t(p->win.size());
    d.ws = p->ws_elems;
    d.tilemeta = p->tilemeta_words;
    d.lbmeta = p->lbmeta_words;
    const uint64_t B = uint64_t(1) << d.logB, R = uint64_t(1) << d.logR, C = uint64_t(1) << d.logC;
    p->ws_elems += int64_t(n);
    p->tilemeta_words += int64_t(uint64_t(d.ntiles) * (B + 1));
    p->lbmeta_words += int64_t(B * (R + C + 3));
    p->prefA.push_back(uint32_t(a));
    p->prefB.push_back(uint32_t(b));
    p->prefC.push_back(uint32_t(c));
    const uint32_t wi = uint32_t(p->win.size());
    p->itemwinB.insert(p->itemwinB.end(), size_t(B), wi);
    std::vector<uint32_t>& m = d.wave ? p->mapBw : p->mapBb;
    for (uint64_t i = 0; i < B; ++i) m.push_back(uint32_t(b + i));
    p->itemwinC.insert(p->itemwinC.end(), size_t(R + C), wi);
    a += d.ntiles;
    b += B;
    c += R + C;
    if (a > 0xFFFFFFFFull || b > 0xFFFFFFFFull || c > 0xFFFFFFFFull) return NSGC_ERR_INVALID_ARG;
    p->win.push_back(d);
  }
  p->prefA.push_back(uint32_t(a));
  p->prefB.push_back(uint32_t(b));
  p->prefC.push_back(uint32_t(c));
  p->itemsA = uint32_t(a);
  p->itemsB = uint32_t(b);
  p->itemsC = uint32_t(c);
  p->itemsBb = uint32_t(p->mapBb.size());
  p->itemsBw = uint32_t(p->mapBw.size());
  // a kernel that takes every phase-B item needs no map
  if (p->itemsBb == p->itemsB) p->mapBb.clear();
  if (p->itemsBw == p->itemsB) p->mapBw.clear();
  return NSGC_OK;
}

WsLayout HostPlan::layout() const {
  WsLayout L;
  const size_t e = size_t(ws_elems) * 8;
  size_t o = 0;
  L.keys = o;      o = align_up(o + e, 256);
  L.emit_row = o;  o = align_up(o + e, 256);
  L.emit_col = o;  o = align_up(o + e, 256);
  L.tilemeta = o;  o = align_up(o + size_t(tilemeta_words) * 4, 256);
  L.lbmeta = o;    o = align_up(o + size_t(lbmeta_words) * 4, 256);
  L.rcsize = o;    o = align_up(o + size_t(itemsC) * 4, 256);
  L.order = o;     o = align_up(o + size_t(itemsC) * 4, 256);
  L.partB = o;     o = align_up(o + size_t(itemsB) * 16, 256);
  L.partC = o;     o = align_up(o + size_t(itemsC) * 16, 256);
  if (num_rows) {
    L.partR = o;   o = align_up(o + size_t(itemsB) * 16, 256);
    L.heavy = o;   o = align_up(o + win.size() * NSGC_HEAVY_SLOTS * 4, 256);
  }
  if (entity) {
    L.partU = o;   o = align_up(o + size_t(itemsC) * 4, 256);
    L.stats = o;   o = align_up(o + tier.size() * 72, 256);
  }
  if (!large.empty()) {   // shared by the large windows, one after another
    L.large = o;   o = align_up(o + large_window_bytes(large_max), 256);
  }
  L.total = std::max<size_t>(o, 256);
  return L;
}

namespace {
struct PlanOffsets {
  size_t small, win, prefA, prefB, prefC, itemwinB, itemwinC, mapBb, mapBw, entcur, entend, total;
};
PlanOffsets plan_offsets(size_t ns, size_t nm, size_t nb, size_t nc, size_t nbb = 0,
                         size_t nbw = 0, size_t nent = 0) {
  PlanOffsets o;
  size_t x = align_up(sizeof(nsgc_dev_plan), 64);
  o.small = x; x = align_up(x + ns * sizeof(nsgc_small_desc), 64);
  o.win = x;   x = align_up(x + nm * sizeof(nsgc_win_desc), 64);
  o.prefA = x; x = align_up(x + (nm + 1) * 4, 64);
  o.prefB = x; x = align_up(x + (nm + 1) * 4, 64);
  o.prefC = x; x = align_up(x + (nm + 1) * 4, 64);
  o.itemwinB = x; x = align_up(x + nb * 4, 64);
  o.itemwinC = x; x = align_up(x + nc * 4, 64);
  o.mapBb = x; x = align_up(x + nbb * 4, 64);
  o.mapBw = x; x = align_up(x + nbw * 4, 64);
  o.entcur = x; x = align_up(x + nent * 8, 64);
  o.entend = x; x = align_up(x + nent * 8, 64);
  o.total = x;
  return o;
}
}  // namespace

size_t HostPlan::plan_bytes() const {
  return plan_offsets(small.size(), win.size(), itemwinB.size(), itemwinC.size(), mapBb.size(),
                      mapBw.size(), ent_cur.size()).total;
}

size_t plan_bound(int64_t max_packets, int64_t max_windows, const nsgc_tune& t) {
  const uint64_t P = uint64_t(std::max<int64_t>(max_packets, 0));
  const uint64_t W = uint64_t(std::max<int64_t>(max_windows, 1));
  uint64_t lt = ~uint64_t(0), rt = ~uint64_t(0);
  for (int k = 0; k <= 32; ++k) {
    lt = std::min<uint64_t>(lt, uint64_t(t.cls[k].link_target));
    rt = std::min<uint64_t>(rt, uint64_t(std::min(t.cls[k].row_target, t.cls[k].col_target)));
  }
  // A bucket count is the power of two at or above ceil(n_w / target) < n_w /
  // target + 1, so B_w < 2 n_w / lt + 2 and R_w + C_w < 4 n_w / rt + 4; each
  // count is also at most its cap (2^max_link_buckets_log2, 2^max_rc_buckets_log2)
  // per window.
  const uint64_t capB = uint64_t(1) << t.max_link_buckets_log2;
  const uint64_t capRC = uint64_t(1) << t.max_rc_buckets_log2;
  const uint64_t nb = std::min<uint64_t>(2 * P / lt + 2 * W, W * capB);
  const uint64_t nc = std::min<uint64_t>(4 * P / rt + 4 * W, 2 * W * capRC);
  // the wavefront buckets (wave_target >= 64) may outnumber the workgroup ones
  uint64_t wt = ~uint64_t(0);
  for (int k = 0; k <= 32; ++k)
    if (t.cls[k].wave_target > 0) wt = std::min<uint64_t>(wt, uint64_t(t.cls[k].wave_target));
  const uint64_t nbw = wt == ~uint64_t(0) ? 0 : std::min<uint64_t>(2 * P / wt + 2 * W, W * capB);
  const uint64_t nb_all = std::max(nb, nbw);
  return plan_offsets(size_t(W), size_t(W), size_t(nb_all), size_t(nc), size_t(nb_all),
                      size_t(nb_all)).total + 1024;
}

void HostPlan::serialize(void* buf, uint64_t dev_plan, uint64_t dev_ws, const uint32_t* src,
                         const uint32_t* dst, void* out) const {
  const PlanOffsets o = plan_offsets(small.size(), win.size(), itemwinB.size(), itemwinC.size(),
                                     mapBb.size(), mapBw.size(), ent_cur.size());
  const WsLayout L = layout();
  char* base = static_cast<char*>(buf);
  std::memset(base, 0, align_up(sizeof(nsgc_dev_plan), 64));
  nsgc_dev_plan h;
  std::memset(&h, 0, sizeof h);
  h.src = src;
  h.dst = dst;
  h.out = static_cast<unsigned long long*>(out);
  h.keys = reinterpret_cast<unsigned long long*>(dev_ws + L.keys);
  h.emit_row = reinterpret_cast<unsigned long long*>(dev_ws + L.emit_row);
  h.emit_col = reinterpret_cast<unsigned long long*>(dev_ws + L.emit_col);
  h.tilemeta = reinterpret_cast<uint32_t*>(dev_ws + L.tilemeta);
  h.lbmeta = reinterpret_cast<uint32_t*>(dev_ws + L.lbmeta);
  h.rcsize = reinterpret_cast<uint32_t*>(dev_ws + L.rcsize);
  h.order = reinterpret_cast<uint32_t*>(dev_ws + L.order);
  h.partB = reinterpret_cast<uint32_t*>(dev_ws + L.partB);
  h.partC = reinterpret_cast<uint32_t*>(dev_ws + L.partC);
  if (num_rows) {
    h.partR = reinterpret_cast<uint32_t*>(dev_ws + L.partR);
    h.heavy = reinterpret_cast<uint32_t*>(dev_ws + L.heavy);
  }
  h.small = reinterpret_cast<const nsgc_small_desc*>(dev_plan + o.small);
  h.win = reinterpret_cast<const nsgc_win_desc*>(dev_plan + o.win);
  h.prefA = reinterpret_cast<const uint32_t*>(dev_plan + o.prefA);
  h.prefB = reinterpret_cast<const uint32_t*>(dev_plan + o.prefB);
  h.prefC = reinterpret_cast<const uint32_t*>(dev_plan + o.prefC);
  h.itemwinB = reinterpret_cast<const uint32_t*>(dev_plan + o.itemwinB);
  h.itemwinC = reinterpret_cast<const uint32_t*>(dev_plan + o.itemwinC);
  h.mapBb = mapBb.empty() ? nullptr : reinterpret_cast<const uint32_t*>(dev_plan + o.mapBb);
  h.mapBw = mapBw.empty() ? nullptr : reinterpret_cast<const uint32_t*>(dev_plan + o.mapBw);
  h.itemsBb = itemsBb;
  h.itemsBw = itemsBw;
  h.num_small = uint32_t(small.size());
  h.num_part = uint32_t(win.size());
  h.itemsA = itemsA;
  h.itemsB = itemsB;
  h.itemsC = itemsC;
  h.tile_log2 = tile_log2;
  h.link_slots_log2 = link_slots_log2;
  h.rc_slots_log2 = rc_slots_log2;
  h.small_slots_log2 = small_slots_log2;
  h.max_sweeps_log2 = max_sweeps_log2;
  h.combine_probes = combine_probes;
  h.order_items = itemsC <= NSGC_ORDER_MAX && !entity ? 1u : 0u;
  if (entity) {
    // the statistics go to the workspace; the entity counts to the caller
    h.out = reinterpret_cast<unsigned long long*>(dev_ws + L.stats);
    h.entity = 1;
    h.partU = reinterpret_cast<uint32_t*>(dev_ws + L.partU);
    h.ent_links = static_cast<long long*>(ent_links);
    h.ent_src = static_cast<long long*>(ent_src);
    h.ent_dst = static_cast<long long*>(ent_dst);
    h.ent_counts = static_cast<long long*>(ent_counts);
    h.ent_cur = reinterpret_cast<unsigned long long*>(dev_plan + o.entcur);
    h.ent_end = reinterpret_cast<const unsigned long long*>(dev_plan + o.entend);
  }
  std::memcpy(base, &h, sizeof h);
  if (!small.empty()) std::memcpy(base + o.small, small.data(), small.size() * sizeof(nsgc_small_desc));
  if (!win.empty()) std::memcpy(base + o.win, win.data(), win.size() * sizeof(nsgc_win_desc));
  std::memcpy(base + o.prefA, prefA.data(), prefA.size() * 4);
  std::memcpy(base + o.prefB, prefB.data(), prefB.size() * 4);
  std::memcpy(base + o.prefC, prefC.data(), prefC.size() * 4);
  if (!itemwinB.empty()) std::memcpy(base + o.itemwinB, itemwinB.data(), itemwinB.size() * 4);
  if (!itemwinC.empty()) std::memcpy(base + o.itemwinC, itemwinC.data(), itemwinC.size() * 4);
  if (!mapBb.empty()) std::memcpy(base + o.mapBb, mapBb.data(), mapBb.size() * 4);
  if (!mapBw.empty()) std::memcpy(base + o.mapBw, mapBw.data(), mapBw.size() * 4);
  if (!ent_cur.empty()) std::memcpy(base + o.entcur, ent_cur.data(), ent_cur.size() * 8);
  if (!ent_end.empty()) std::memcpy(base + o.entend, ent_end.data(), ent_end.size() * 8);
}

}  // namespace nsgc
