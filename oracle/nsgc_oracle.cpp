// Window-statistics ORACLE -- test infrastructure only.
//
// This is the plain, slow, obviously correct CPU definition of what the HIP
// library computes.  Only the tests, the smoke check and the bench's CPU
// baseline may call it; the product path never does.  It shares no code,
// header, constant or helper with the HIP library.
//
// What it computes (paper, Section IV "Graph Analytics" and Table III, with
// the caption's rule that the reverse queries swap src and dst):
//
//   For one window, the packets are a multiset of (src, dst) pairs.  The
//   traffic matrix A is the multigraph's count matrix (Section V, last
//   paragraph, reads the packets as a multi-graph):
//       A(s, d) = number of packets with source s and destination d.
//   Row view:    r(s) = sum_d A(s,d)         (packets from source s)
//                f(s) = #{d : A(s,d) > 0}    (fan-out of source s)
//   Column view: c(d) = sum_s A(s,d)         (packets to destination d)
//                g(d) = #{s : A(s,d) > 0}    (fan-in of destination d)
//
//   stat[0] valid packets          = sum of A                  (Table III row 1)
//   stat[1] unique links           = nnz(A)                    (row 2)
//   stat[2] max link packets       = max of A                  (row 4)
//   stat[3] unique sources         = #{s : r(s) > 0}           (row 5)
//   stat[4] max source packets     = max r                     (row 7)
//   stat[5] max source fan-out     = max f                     (row 9)
//   stat[6] unique destinations    = #{d : c(d) > 0}           (reverse of row 5)
//   stat[7] max destination packets= max c                     (reverse of row 7)
//   stat[8] max destination fan-in = max g                     (reverse of row 9)
//
// The maximum over an empty set is 0, so an empty window gives nine zeros.
// Every pair in the window counts as one valid packet: there is no validity
// mask at this layer.
//
// Implementation: one std::map for A keyed by (src, dst), then one std::map
// per view built from A's entries.  Windows are independent; the optional
// thread count only spreads whole windows over threads.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <map>
#include <set>
#include <thread>
#include <utility>
#include <vector>

namespace {

struct Totals {
  uint64_t packets = 0;   // sum of A over the row (or column)
  uint64_t links = 0;     // number of non-zero entries in the row (or column)
};

void one_window(const uint32_t* src, const uint32_t* dst, int64_t begin, int64_t end,
                uint64_t out[9]) {
  // A(s, d), keyed by the ordered pair (s, d).
  std::map<std::pair<uint32_t, uint32_t>, uint64_t> A;
  for (int64_t i = begin; i < end; ++i) A[std::make_pair(src[i], dst[i])] += 1;

  std::map<uint32_t, Totals> rows;     // s -> (r(s), f(s))
  std::map<uint32_t, Totals> cols;     // d -> (c(d), g(d))
  uint64_t valid = 0, max_link = 0;
  for (const auto& e : A) {
    const uint32_t s = e.first.first;
    const uint32_t d = e.first.second;
    const uint64_t a = e.second;       // a > 0 for every stored entry
    valid += a;
    max_link = std::max(max_link, a);
    rows[s].packets += a;
    rows[s].links += 1;
    cols[d].packets += a;
    cols[d].links += 1;
  }

  uint64_t max_r = 0, max_f = 0, max_c = 0, max_g = 0;
  for (const auto& e : rows) {
    max_r = std::max(max_r, e.second.packets);
    max_f = std::max(max_f, e.second.links);
  }
  for (const auto& e : cols) {
    max_c = std::max(max_c, e.second.packets);
    max_g = std::max(max_g, e.second.links);
  }

  out[0] = valid;
  out[1] = static_cast<uint64_t>(A.size());
  out[2] = max_link;
  out[3] = static_cast<uint64_t>(rows.size());
  out[4] = max_r;
  out[5] = max_f;
  out[6] = static_cast<uint64_t>(cols.size());
  out[7] = max_c;
  out[8] = max_g;
}

// Globally unique IP addresses of one window (Section IV, "Graph Analytics"
// paragraph: the unique values of each column with the values common to both
// counted once): the size of the union of the source and destination sets.
uint64_t unique_ips(const uint32_t* src, const uint32_t* dst, int64_t begin, int64_t end) {
  std::set<uint32_t> ips;
  for (int64_t i = begin; i < end; ++i) {
    ips.insert(src[i]);
    ips.insert(dst[i]);
  }
  return static_cast<uint64_t>(ips.size());
}

// ---- anonymization (Section IV, "IP Address Anonymization") ----------------
// The paper lists the unique addresses of the source and destination columns,
// draws a random permutation of 0..N-1 by shuffling that sequence, and maps
// the i-th unique address to the i-th value of the permutation.  Here the
// unique addresses are listed in ascending order (what a sort-based unique
// returns) and the shuffle is a seeded pseudo-random permutation, so that
// the mapping is reproducible:
//   b = the smallest even bit count with 2^b >= max(N, 4), h = b / 2;
//   E(x) on [0, 2^b): split x into halves L = x >> h, R = x mod 2^h and run
//     four Feistel rounds (L, R) <- (R, L xor F_r(R)), r = 0..3, with
//     F_r(R) = mix(seed xor (r + 1) * 0x9E3779B97F4A7C15 xor R) mod 2^h,
//     where mix is the SplitMix64 output function; E(x) = L * 2^h + R;
//   pi(i) = the first of E(i), E(E(i)), ... that is below N (cycle walking,
//     Black and Rogaway, "Ciphers with arbitrary finite domains", 2002).
// A Feistel network is a bijection for any round function, and cycle walking
// restricts a bijection of [0, 2^b) to one of [0, N).

uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t feistel(uint64_t x, int h, uint64_t seed) {
  const uint64_t mask = (uint64_t(1) << h) - 1;
  uint64_t L = x >> h, R = x & mask;
  for (uint64_t r = 0; r < 4; ++r) {
    const uint64_t f = splitmix_mix(seed ^ ((r + 1) * 0x9E3779B97F4A7C15ull) ^ R) & mask;
    const uint64_t t = L ^ f;
    L = R;
    R = t;
  }
  return (L << h) | R;
}

uint64_t permute(uint64_t i, uint64_t N, uint64_t seed) {
  if (N <= 1) return i;
  int b = 2;
  while ((uint64_t(1) << b) < N) b += 2;
  uint64_t y = feistel(i, b / 2, seed);
  while (y >= N) y = feistel(y, b / 2, seed);
  return y;
}

}  // namespace

extern "C" {

// pi(i) of the anonymization's permutation of [0, N) for `seed` (see above).
uint64_t nsgc_oracle_permute(uint64_t i, uint64_t N, uint64_t seed) { return permute(i, N, seed); }

// The unique addresses of src[0..n) and dst[0..n) in ascending order; returns
// their number N (out must hold 2n values).
int64_t nsgc_oracle_unique_addresses(const uint32_t* src, const uint32_t* dst, int64_t n,
                                     uint32_t* out) {
  std::set<uint32_t> ips;
  for (int64_t i = 0; i < n; ++i) {
    ips.insert(src[i]);
    ips.insert(dst[i]);
  }
  int64_t k = 0;
  for (uint32_t v : ips) out[k++] = v;
  return k;
}

// Anonymization of n packets: every address x of either column becomes
// pi(rank of x among the unique addresses in ascending order).  Writes the
// two anonymized columns and N; returns 0, or -1 for bad arguments.
int nsgc_oracle_anonymize(const uint32_t* src, const uint32_t* dst, int64_t n, uint64_t seed,
                          uint32_t* asrc, uint32_t* adst, uint64_t* num_ips) {
  if (n < 0 || (n > 0 && (!src || !dst || !asrc || !adst)) || !num_ips) return -1;
  std::set<uint32_t> ips;
  for (int64_t i = 0; i < n; ++i) {
    ips.insert(src[i]);
    ips.insert(dst[i]);
  }
  const uint64_t N = ips.size();
  std::map<uint32_t, uint64_t> id;
  uint64_t rank = 0;
  for (uint32_t v : ips) id[v] = permute(rank++, N, seed);
  for (int64_t i = 0; i < n; ++i) {
    asrc[i] = static_cast<uint32_t>(id[src[i]]);
    adst[i] = static_cast<uint32_t>(id[dst[i]]);
  }
  *num_ips = N;
  return 0;
}

// Nine statistics per window for windows [offsets[w], offsets[w+1]).
// src, dst, offsets and out are host pointers; out holds 9*num_windows
// values in the order listed above.  threads <= 1 runs single-threaded.
// Returns 0, -1 for bad arguments (null pointers, negative count, decreasing
// or negative offsets); on error out is left untouched.
int nsgc_oracle_window_stats(const uint32_t* src, const uint32_t* dst,
                             const int64_t* offsets, int64_t num_windows, uint64_t* out,
                             int threads) {
  if (num_windows < 0) return -1;
  if (num_windows == 0) return 0;
  if (!offsets || !out) return -1;
  if (offsets[0] < 0) return -1;
  for (int64_t w = 0; w < num_windows; ++w)
    if (offsets[w + 1] < offsets[w]) return -1;
  if (offsets[num_windows] > offsets[0] && (!src || !dst)) return -1;

  if (threads <= 1 || num_windows == 1) {
    for (int64_t w = 0; w < num_windows; ++w)
      one_window(src, dst, offsets[w], offsets[w + 1], out + 9 * w);
    return 0;
  }
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    for (;;) {
      const int64_t w = next.fetch_add(1);
      if (w >= num_windows) break;
      one_window(src, dst, offsets[w], offsets[w + 1], out + 9 * w);
    }
  };
  const int n = static_cast<int>(std::min<int64_t>(threads, num_windows));
  std::vector<std::thread> pool;
  pool.reserve(n);
  for (int t = 0; t < n; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  return 0;
}

// |{sources} U {destinations}| per window for windows [offsets[w], offsets[w+1]):
// out[w] receives the count.  Same argument rules and return values as
// nsgc_oracle_window_stats.
int nsgc_oracle_unique_ips(const uint32_t* src, const uint32_t* dst, const int64_t* offsets,
                           int64_t num_windows, uint64_t* out, int threads) {
  if (num_windows < 0) return -1;
  if (num_windows == 0) return 0;
  if (!offsets || !out) return -1;
  if (offsets[0] < 0) return -1;
  for (int64_t w = 0; w < num_windows; ++w)
    if (offsets[w + 1] < offsets[w]) return -1;
  if (offsets[num_windows] > offsets[0] && (!src || !dst)) return -1;
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    for (;;) {
      const int64_t w = next.fetch_add(1);
      if (w >= num_windows) break;
      out[w] = unique_ips(src, dst, offsets[w], offsets[w + 1]);
    }
  };
  const int n = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(threads, num_windows)));
  if (n == 1) {
    worker();
    return 0;
  }
  std::vector<std::thread> pool;
  pool.reserve(n);
  for (int t = 0; t < n; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  return 0;
}

// The per-entity vectors of one window (Table III rows 3, 6 and 8 and their
// reverses), as sorted lists.  Used by tests that check intermediate results.
// Each output array must hold at least (end - begin) entries; the returned
// counts say how many were written.  Returns 0 or -1.
int nsgc_oracle_window_entities(const uint32_t* src, const uint32_t* dst, int64_t begin,
                                int64_t end, uint64_t* link_keys, uint64_t* link_counts,
                                int64_t* n_links, uint32_t* row_ids, uint64_t* row_packets,
                                uint64_t* row_links, int64_t* n_rows, uint32_t* col_ids,
                                uint64_t* col_packets, uint64_t* col_links,
                                int64_t* n_cols) {
  if (begin < 0 || end < begin) return -1;
  if (end > begin && (!src || !dst)) return -1;
  std::map<std::pair<uint32_t, uint32_t>, uint64_t> A;
  for (int64_t i = begin; i < end; ++i) A[std::make_pair(src[i], dst[i])] += 1;
  std::map<uint32_t, Totals> rows, cols;
  int64_t k = 0;
  for (const auto& e : A) {
    link_keys[k] = (static_cast<uint64_t>(e.first.first) << 32) | e.first.second;
    link_counts[k] = e.second;
    ++k;
    rows[e.first.first].packets += e.second;
    rows[e.first.first].links += 1;
    cols[e.first.second].packets += e.second;
    cols[e.first.second].links += 1;
  }
  *n_links = k;
  k = 0;
  for (const auto& e : rows) {
    row_ids[k] = e.first;
    row_packets[k] = e.second.packets;
    row_links[k] = e.second.links;
    ++k;
  }
  *n_rows = k;
  k = 0;
  for (const auto& e : cols) {
    col_ids[k] = e.first;
    col_packets[k] = e.second.packets;
    col_links[k] = e.second.links;
    ++k;
  }
  *n_cols = k;
  return 0;
}

}  // extern "C"
