// The CCCS entry point that allocates nothing (mgc_cccs_noalloc): its scratch
// (projection partials, channel right-hand sides and solutions) lives in a
// file-scope device array of fixed size that every GPU the library runs on
// holds until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mgcccs.h"
#include "internal.h"

namespace {
constexpr int MAX_DEVICES = 64;
// one copy per device; host code uses only the addresses in g_scratch
static __device__ __align__(256) unsigned char scratch[MGC_NOALLOC_SCRATCH_BYTES];
void* g_scratch[MAX_DEVICES] = {};
std::mutex g_lock;
}  // namespace

extern "C" mgc_status mgc_cccs_noalloc(mgc_grid g, void* u, const void* f, mgc_precision prec) {
  if (!g) return mgc::set_error(MGC_EINVAL, "null handle");
  const int dev = mgc::handle_device(g);
  if (dev < 0 || dev >= MAX_DEVICES) return mgc::set_error(MGC_EINVAL, "device index out of range");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_scratch[dev]) {
      // first call on this device: the array's device address, taken with
      // that device current
      int cur = 0;
      if (hipGetDevice(&cur) != hipSuccess) return mgc::set_error(MGC_EHIP, "hipGetDevice failed");
      if (cur != dev && hipSetDevice(dev) != hipSuccess) return mgc::set_error(MGC_EHIP, "hipSetDevice failed");
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (cur != dev) (void)hipSetDevice(cur);
      if (e != hipSuccess || !p) return mgc::set_error(MGC_EHIP, "hipGetSymbolAddress of the scratch array failed");
      g_scratch[dev] = p;
    }
    ptr = g_scratch[dev];
  }
  return mgc::cccs_with_scratch(g, u, f, prec, ptr, MGC_NOALLOC_SCRATCH_BYTES);
}
