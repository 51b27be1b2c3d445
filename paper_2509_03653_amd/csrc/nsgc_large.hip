// Large-window tier: the nine statistics of one very large window by sorting
// instead of LDS hashing (Table III rows 1-9 and their src/dst reverse).
//
// A window of hundreds of millions of packets would need many levels of hash
// partitioning before its buckets fit LDS tables; sorting reaches the same
// groups directly:
//   1. each packet becomes its hashed link key row_hash(src) << 32 |
//      col_hash(dst) (a bijection of the pair), and the keys are radix-sorted;
//   2. equal keys are now adjacent: a link is a run of equal keys (its length
//      is A(s, d)), and a source is a run of equal high halves, which covers
//      its links contiguously (r(s) = run length in packets, f(s) = number of
//      link runs inside);
//   3. one element per link, (col_hash(dst) << 32 | A(s, d)), sorted by the
//      high half, groups the links by destination: c(d) is the sum of the low
//      halves of a run, g(d) its length.
// Run starts are found by comparing neighbours, numbered by exclusive scans,
// and compacted; run lengths and sums are then differences of neighbouring
// starts.  Every step is a plain data-parallel pass, so the tier has no
// overflow path and no dependence on the data's skew.
#include <hip/hip_runtime.h>

#include "nsgc_device.hpp"
#include "nsgc_large.hpp"
#include "nsgc_sort.hpp"

namespace nsgc {

namespace {

constexpr uint32_t LT = 256;   // threads per workgroup of the element-wise passes

__global__ __launch_bounds__(LT) void k_lw_keys(const uint32_t* __restrict__ src,
                                                const uint32_t* __restrict__ dst, u64 n,
                                                u64* __restrict__ keys) {
  for (u64 i = u64(blockIdx.x) * LT + threadIdx.x; i < n; i += u64(gridDim.x) * LT)
    keys[i] = link_key(src[i], dst[i]);
}

// Run starts of the sorted keys: link runs (whole key) and source runs (high
// half), as 0/1 flags (scanned in place afterwards into run numbers).
__global__ __launch_bounds__(LT) void k_lw_flags(const u64* __restrict__ k, u64 n,
                                                 uint32_t* __restrict__ fl,
                                                 uint32_t* __restrict__ fr) {
  for (u64 i = u64(blockIdx.x) * LT + threadIdx.x; i < n; i += u64(gridDim.x) * LT) {
    const u64 a = k[i];
    const u64 p = i ? k[i - 1] : ~a;   // the first element always starts both runs
    fl[i] = a != p;
    fr[i] = (a >> 32) != (p >> 32);
  }
}

// Compaction of the run starts: link run j starts at ls[j], source run j at
// rs[j]; the end markers ls[nl] = rs[nr] = n.
__global__ __launch_bounds__(LT) void k_lw_compact(const u64* __restrict__ k, u64 n,
                                                   const uint32_t* __restrict__ li,
                                                   const uint32_t* __restrict__ ri,
                                                   uint32_t* __restrict__ ls,
                                                   uint32_t* __restrict__ rs,
                                                   const uint32_t* __restrict__ nl,
                                                   const uint32_t* __restrict__ nr) {
  for (u64 i = u64(blockIdx.x) * LT + threadIdx.x; i < n; i += u64(gridDim.x) * LT) {
    const u64 a = k[i];
    const u64 p = i ? k[i - 1] : ~a;
    if (a != p) ls[li[i]] = uint32_t(i);
    if ((a >> 32) != (p >> 32)) rs[ri[i]] = uint32_t(i);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ls[*nl] = uint32_t(n);
    rs[*nr] = uint32_t(n);
  }
}

__device__ __forceinline__ void atomic_max64(u64* p, u64 v) {
  if (v) __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per link: its packets A(s, d) (run length) for the maximum, and the column
// element col_hash(dst) << 32 | A(s, d).
__global__ __launch_bounds__(LT) void k_lw_links(const u64* __restrict__ k,
                                                 const uint32_t* __restrict__ ls,
                                                 const uint32_t* __restrict__ nl,
                                                 u64* __restrict__ cols, u64* __restrict__ out) {
  __shared__ uint32_t red[LT / 64];
  const uint32_t m = *nl;
  uint32_t mx = 0;
  for (u64 j = u64(blockIdx.x) * LT + threadIdx.x; j < m; j += u64(gridDim.x) * LT) {
    const uint32_t a = ls[j], len = ls[j + 1] - a;
    mx = max(mx, len);
    cols[j] = (k[a] << 32) | len;
  }
  mx = wave_max(mx);
  if (lane_id() == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < LT / 64; ++w) mx = max(mx, red[w]);
    atomic_max64(out + 2, mx);
  }
}

// Per source run: r(s) = run length, f(s) = link runs inside (the difference
// of the link numbers at its start and at the next source's start).
__global__ __launch_bounds__(LT) void k_lw_rows(const uint32_t* __restrict__ rs,
                                                const uint32_t* __restrict__ li,
                                                const uint32_t* __restrict__ nl,
                                                const uint32_t* __restrict__ nr, u64 n,
                                                u64* __restrict__ out) {
  __shared__ uint32_t red[2][LT / 64];
  const uint32_t m = *nr, links = *nl;
  uint32_t mp = 0, mf = 0;
  for (u64 j = u64(blockIdx.x) * LT + threadIdx.x; j < m; j += u64(gridDim.x) * LT) {
    const uint32_t a = rs[j], b = rs[j + 1];
    mp = max(mp, b - a);
    mf = max(mf, (b < n ? li[b] : links) - li[a]);
  }
  mp = wave_max(mp);
  mf = wave_max(mf);
  if (lane_id() == 0) {
    red[0][threadIdx.x >> 6] = mp;
    red[1][threadIdx.x >> 6] = mf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < LT / 64; ++w) {
      mp = max(mp, red[0][w]);
      mf = max(mf, red[1][w]);
    }
    atomic_max64(out + 4, mp);
    atomic_max64(out + 5, mf);
  }
}

// Column runs over the column elements sorted by their high half: start flags
// and the packets of each element (both scanned in place afterwards).
__global__ __launch_bounds__(LT) void k_lw_colflags(const u64* __restrict__ c,
                                                    const uint32_t* __restrict__ nl,
                                                    uint32_t* __restrict__ fc,
                                                    uint32_t* __restrict__ pk) {
  const uint32_t m = *nl;
  for (u64 i = u64(blockIdx.x) * LT + threadIdx.x; i < m; i += u64(gridDim.x) * LT) {
    const u64 a = c[i];
    const u64 p = i ? c[i - 1] : ~a;
    fc[i] = (a >> 32) != (p >> 32);
    pk[i] = uint32_t(a);
  }
}

__global__ __launch_bounds__(LT) void k_lw_colcompact(const u64* __restrict__ c,
                                                      const uint32_t* __restrict__ ci,
                                                      const uint32_t* __restrict__ pc,
                                                      uint32_t* __restrict__ cs,
                                                      uint32_t* __restrict__ cp,
                                                      const uint32_t* __restrict__ nl,
                                                      const uint32_t* __restrict__ nc, u64 n) {
  const uint32_t m = *nl;
  for (u64 i = u64(blockIdx.x) * LT + threadIdx.x; i < m; i += u64(gridDim.x) * LT) {
    const u64 a = c[i];
    const u64 p = i ? c[i - 1] : ~a;
    if ((a >> 32) != (p >> 32)) {
      cs[ci[i]] = uint32_t(i);
      cp[ci[i]] = pc[i];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cs[*nc] = m;
    cp[*nc] = uint32_t(n);
  }
}

// Per destination run: g(d) = run length in links, c(d) = packets in it.
__global__ __launch_bounds__(LT) void k_lw_cols(const uint32_t* __restrict__ cs,
                                                const uint32_t* __restrict__ cp,
                                                const uint32_t* __restrict__ nc,
                                                u64* __restrict__ out) {
  __shared__ uint32_t red[2][LT / 64];
  const uint32_t m = *nc;
  uint32_t mc = 0, mg = 0;
  for (u64 j = u64(blockIdx.x) * LT + threadIdx.x; j < m; j += u64(gridDim.x) * LT) {
    mg = max(mg, cs[j + 1] - cs[j]);
    mc = max(mc, cp[j + 1] - cp[j]);
  }
  mc = wave_max(mc);
  mg = wave_max(mg);
  if (lane_id() == 0) {
    red[0][threadIdx.x >> 6] = mc;
    red[1][threadIdx.x >> 6] = mg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < LT / 64; ++w) {
      mc = max(mc, red[0][w]);
      mg = max(mg, red[1][w]);
    }
    atomic_max64(out + 7, mc);
    atomic_max64(out + 8, mg);
  }
}

// Copy two device counts (scan totals whose scratch is about to be reused).
__global__ void k_lw_save(const uint32_t* nl, const uint32_t* nr, uint32_t* to) {
  if (threadIdx.x == 0) {
    to[0] = *nl;
    to[1] = *nr;
  }
}

// Zero the window's statistics before the maxima are merged into them.
__global__ void k_lw_zero(u64* out) {
  if (threadIdx.x < 9) out[threadIdx.x] = 0;
}

// The counts: packets, links, sources, destinations.
__global__ void k_lw_counts(u64* out, u64 n, const uint32_t* nl, const uint32_t* nr,
                            const uint32_t* nc) {
  if (threadIdx.x == 0) {
    out[0] = n;
    out[1] = *nl;
    out[3] = *nr;
    out[6] = *nc;
  }
}

}  // namespace

size_t large_window_bytes(u64 n) {
  const size_t words = 16 + 4 * size_t(n + 1) +
                       std::max(radix_sort_scratch_words(n), 2 * scan_scratch_words(n)) + 256;
  return 2 * size_t(n) * 8 + words * 4 + 1024;
}

hipError_t large_window_stats(const uint32_t* src, const uint32_t* dst, u64 n, void* ws,
                              unsigned long long* out, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_lw_zero, dim3(1), dim3(64), 0, s, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  // workspace: two key buffers, four u32 arrays of n + 1, sort / scan scratch
  u64* K = static_cast<u64*>(ws);
  u64* T = K + n;
  uint32_t* counts = reinterpret_cast<uint32_t*>(T + n);   // 16 words: saved run counts
  uint32_t* A = counts + 16;
  uint32_t* Bv = A + (n + 1);
  uint32_t* Cv = Bv + (n + 1);
  uint32_t* Dv = Cv + (n + 1);
  uint32_t* scratch = Dv + (n + 1);
  uint32_t* scratch2 = scratch + scan_scratch_words(n);   // second scan of a pass
  const uint32_t g = uint32_t(std::min<u64>((n + LT - 1) / LT, grid));

  hipLaunchKernelGGL(k_lw_keys, dim3(g), dim3(LT), 0, s, src, dst, n, K);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  u64* S = nullptr;
  if ((e = radix_sort_u64(K, T, n, 0, 64, scratch, grid, s, &S)) != hipSuccess) return e;
  u64* O = S == K ? T : K;   // free for the column elements

  // link runs (A) and source runs (B): flags, then run numbers
  hipLaunchKernelGGL(k_lw_flags, dim3(g), dim3(LT), 0, s, S, n, A, Bv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = exclusive_scan_u32(A, n, scratch, s)) != hipSuccess) return e;
  if ((e = exclusive_scan_u32(Bv, n, scratch2, s)) != hipSuccess) return e;
  const uint32_t* nl = scan_total(scratch, n);
  const uint32_t* nr = scan_total(scratch2, n);
  hipLaunchKernelGGL(k_lw_compact, dim3(g), dim3(LT), 0, s, S, n, A, Bv, Cv, Dv, nl, nr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lw_links, dim3(g), dim3(LT), 0, s, S, Cv, nl, O, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lw_rows, dim3(g), dim3(LT), 0, s, Dv, A, nl, nr, n, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  // keep the link and source counts: the scratch that holds them is reused
  hipLaunchKernelGGL(k_lw_save, dim3(1), dim3(64), 0, s, nl, nr, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t* nl2 = counts;
  const uint32_t* nr2 = counts + 1;
  // Columns: sort the column elements by their high half.  Only the first
  // `links` slots hold elements; the count is read back (one wait for the
  // stream) so that the sort and the scans cover just those, a small share of
  // the window's packets when links repeat.
  uint32_t links = 0;
  if ((e = hipMemcpyAsync(&links, counts, sizeof links, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if (links == 0 || links > n) return hipErrorInvalidValue;
  const uint32_t gl = uint32_t(std::min<u64>((u64(links) + LT - 1) / LT, grid));
  u64* C = nullptr;
  if ((e = radix_sort_u64(O, S, links, 32, 64, scratch, grid, s, &C)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lw_colflags, dim3(gl), dim3(LT), 0, s, C, nl2, A, Bv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = exclusive_scan_u32(A, links, scratch, s)) != hipSuccess) return e;
  if ((e = exclusive_scan_u32(Bv, links, scratch2, s)) != hipSuccess) return e;
  const uint32_t* nc = scan_total(scratch, links);
  hipLaunchKernelGGL(k_lw_colcompact, dim3(gl), dim3(LT), 0, s, C, A, Bv, Cv, Dv, nl2, nc, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lw_cols, dim3(g), dim3(LT), 0, s, Cv, Dv, nc, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_lw_counts, dim3(1), dim3(64), 0, s, out, n, nl2, nr2, nc);
  return hipGetLastError();
}

}  // namespace nsgc
