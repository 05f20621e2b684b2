// D-GAMP-CT iterations for callers that cannot allocate device memory (code
// under stream capture, tight serving loops, harnesses that forbid
// hipMalloc): dgamp_iterate_noalloc runs exactly the kernels of
// dgamp_iterate, with the iteration workspace taken from a fixed device array
// of this library instead of a caller buffer.
//
// The array `scratch` below is a device variable.  In host code its name is
// only a host-side stand-in: passing it to a kernel would make the kernel
// dereference a host address.  Its device address is obtained once per
// device (hipGetSymbolAddress, with that device current) and cached; every
// kernel argument and every copy uses that address.  Each GPU the library
// runs on holds its own copy until the process ends; all calls on one GPU
// share it, so calls that overlap on one GPU (different streams, or threads)
// race on it.  The iteration writes every workspace word it reads before
// reading it within a call, so nothing needs clearing between calls.
#include <mutex>

#include "dg_internal.h"

namespace dg {

static constexpr size_t kNoallocScratchBytes = (size_t)48 << 20;  // 48 MiB per device
static constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up on the first
// call per device).
static dg_status scratch_address(void** out) {
  int dev = -1;
  DG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("dgamp_iterate_noalloc: device index out of range");
    return DG_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    DG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("dgamp_iterate_noalloc: no device address for the scratch array");
      return DG_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" size_t dg_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

extern "C" dg_status dgamp_iterate_noalloc(const dg_plan* plan, const float* y,
                                           const dgamp_opts* opts, dgamp_state* st,
                                           float* mu_out, double* log, void* stream) {
  DG_ARG_CHECK(plan && y && opts && st, "dgamp_iterate_noalloc: null argument");
  const size_t need = dg_workspace_bytes(plan, DG_OP_DGAMP);
  if (need > kNoallocScratchBytes) {
    set_error("dgamp_iterate_noalloc: this plan's iteration workspace (" +
              std::to_string(need) + " bytes) exceeds the fixed scratch array (" +
              std::to_string(kNoallocScratchBytes) + " bytes); use dgamp_iterate");
    return DG_ERR_ARG;
  }
  void* work = nullptr;
  dg_status rc = scratch_address(&work);
  if (rc != DG_OK) return rc;
  return dgamp_iterate(plan, y, opts, st, mu_out, log, work, stream);
}
