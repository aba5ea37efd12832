// resolvent_apply_noalloc: resolvent_apply for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  Its workspace is a fixed array in device memory
// that the library's code object defines; each GPU the library runs on holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/resolvent.h"
#include "runtime_internal.h"

namespace {

constexpr size_t kScratchBytes = RESOLVENT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The workspace of every no-allocation call on a device.  In host code this name stands for a host-side shadow,
// not a device address: the device address comes from hipGetSymbolAddress, once per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first call on that device.
int scratch_on_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return res_fail(RES_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return res_fail(RES_EINVAL, "device index beyond the supported range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return res_fail(RES_EHIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RES_OK;
}

}  // namespace

extern "C" int resolvent_apply_noalloc(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run,
                                       int32_t k, const void* f_hat, void* u_hat, void* stream) {
  void* base = nullptr;
  const int rc = scratch_on_current_device(&base);
  if (rc != RES_OK) return rc;
  return res_apply_in_scratch(op, grid, run, k, f_hat, u_hat, base, kScratchBytes, stream);
}
