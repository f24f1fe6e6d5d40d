// ppf_execute_noalloc: the batch PPF without any device allocation, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, hosts that forbid it). The two-pass path's presum workspace is a
// fixed device array of this file instead of a per-stream hipMalloc
// allocation; the fused and matrix-core paths use no workspace at all.

#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ppf.h"
#include "ppf_internal.h"

namespace {

// 32 MiB: 2^22 complex FP32 presums. Each GPU the library runs on holds its
// own copy until the process ends.
constexpr size_t kScratchBytes = (size_t)PPF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Host code must not pass `scratch` itself to a kernel: in host code it is a
// stand-in, not a device address. Each device's address is looked up once,
// with that device current, and kept here.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    ppf_internal_set_error(PPF_ERR_HIP, "hipGetDevice failed");
    return PPF_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    ppf_internal_set_error(PPF_ERR_UNSUPPORTED, "device index beyond the static workspace table");
    return PPF_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ppf_internal_set_error(PPF_ERR_HIP, "hipGetSymbolAddress of the static workspace failed");
      return PPF_ERR_HIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PPF_OK;
}

}  // namespace

extern "C" int ppf_execute_noalloc(ppf_plan_t plan, const void* in, void* out, long long nspectra) {
  if (!plan) {
    ppf_internal_set_error(PPF_ERR_INVALID, "plan is NULL");
    return PPF_ERR_INVALID;
  }
  void* ws = nullptr;
  const int st = scratch_ptr(&ws);
  if (st != PPF_OK) return st;
  return ppf_internal_execute_in(plan, in, out, nspectra, ws, kScratchBytes);
}
