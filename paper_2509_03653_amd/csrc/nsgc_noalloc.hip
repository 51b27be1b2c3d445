// Fixed-scratch entry point: the batched form with its plan and workspace in
// a statically sized device array instead of allocated buffers, for callers
// that cannot allocate device memory.
//
// The array is a file-scope __device__ variable, so each GPU that loads this
// code object holds its own copy at its own address for the life of the
// process.  Host code never passes the variable's name to a kernel or a copy
// (on the host it is only a stand-in for the symbol): the device address is
// looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "nsgc.h"

namespace nsgc {
int run_fixed_scratch(const uint32_t* src, const uint32_t* dst, const int64_t* window_offsets,
                      int64_t num_windows, nsgc_stats* out_stats, void* stream, char* plan_dev,
                      size_t plan_cap, char* ws, size_t ws_cap);
int validate_call(const uint32_t* src, const uint32_t* dst, const int64_t* offsets,
                  int64_t num_windows, const void* out);
int record_hip_error(int e);
}

namespace {

static __device__ __align__(256) unsigned char scratch[NSGC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;   // device -> device address of `scratch`

// The device address of this device's array (looked up on first use).
int scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return nsgc::record_hip_error(int(e));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return NSGC_OK;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return nsgc::record_hip_error(int(e));
  if (p == nullptr) return NSGC_ERR_INTERNAL;
  g_scratch_ptr[dev] = static_cast<char*>(p);
  *out = static_cast<char*>(p);
  return NSGC_OK;
}

}  // namespace

extern "C" int nsgc_window_stats_noalloc(const uint32_t* src, const uint32_t* dst,
                                         const int64_t* window_offsets, int64_t num_windows,
                                         nsgc_stats* out_stats, void* stream) {
  int rc = nsgc::validate_call(src, dst, window_offsets, num_windows, out_stats);
  if (rc != NSGC_OK || num_windows == 0) return rc;
  char* base = nullptr;
  if ((rc = scratch_address(&base)) != NSGC_OK) return rc;
  constexpr size_t plan = NSGC_NOALLOC_PLAN_BYTES;
  static_assert(NSGC_NOALLOC_PLAN_BYTES % 256 == 0 && NSGC_NOALLOC_PLAN_BYTES < NSGC_NOALLOC_SCRATCH_BYTES,
                "plan region");
  return nsgc::run_fixed_scratch(src, dst, window_offsets, num_windows, out_stats, stream, base,
                                 plan, base + plan, size_t(NSGC_NOALLOC_SCRATCH_BYTES) - plan);
}
