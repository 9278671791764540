// Allocation-free variant of ipr_solve for callers that cannot allocate
// device memory (serving loops and harnesses that forbid it): the workspace
// is a fixed device array of the library instead of the caller's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ipr.h"
#include "ipr_host.h"

using namespace ipr;

namespace {

// The workspace of ipr_solve_noalloc: one copy per device, held until the
// process ends. Its name is a host-side stand-in in host code; kernels get
// the device address from hipGetSymbolAddress (scratch_ptr below).
__device__ __align__(256) unsigned char scratch[IPR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_ptr(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(IPR_EARG, "ipr_solve_noalloc: device %d beyond the supported %d", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(IPR_EHIP, "ipr_solve_noalloc: no device address for the scratch array");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return IPR_OK;
}

struct NoAllocScope {  // read_scalars and the phase timer skip their allocations
  NoAllocScope() { g_no_alloc = true; }
  ~NoAllocScope() { g_no_alloc = false; }
};

}  // namespace

extern "C" int ipr_solve_noalloc(const double* dA, double* dC, int n, int p, double tol,
                                 const ipr_schedule* s, ipr_result* out, hipStream_t stream) {
  g_last_error.clear();
  ipr_schedule sd;
  ipr_schedule_default(&sd);
  const ipr_schedule& sc = s ? *s : sd;
  if (n < 1 || p < 1 || p > 64)
    return fail(IPR_EARG, "ipr_solve_noalloc: need n >= 1 and 1 <= p <= 64");
  if (sc.timing)
    return fail(IPR_EARG, "ipr_solve_noalloc: schedule.timing needs device events (not created "
                "here); use ipr_solve");
  const size_t need = ipr_workspace_size(n, p, 1, &sc);
  if (need > (size_t)IPR_NOALLOC_SCRATCH_BYTES)
    return fail(IPR_EARG, "ipr_solve_noalloc: n = %d, p = %d needs %zu bytes of workspace, the "
                "fixed scratch holds %zu", n, p, need, (size_t)IPR_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if (int rc = scratch_ptr(&ws)) return rc;
  NoAllocScope scope;
  return ipr_solve(dA, dC, n, p, tol, s, out, ws, IPR_NOALLOC_SCRATCH_BYTES, stream);
}
