// Planned matvec for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
// the matvec workspace comes from a fixed device array of this translation
// unit instead of a caller buffer.  The array is part of this unit's code
// object, so it exists on a device from the first call there until the
// process ends; programs that never call this entry point never load it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "common.h"
#include "hmv.h"
#include "plan.h"

namespace hmv {
namespace {

// Status block (256 bytes) plus the spectra of x and y of one planned
// matvec: 448 MiB holds every split-FFT plan up to n = 4096 at P = 33 220
// (385 MiB there) and every smaller shape.
constexpr int64_t kNoAllocBytes = int64_t(448) << 20;
static_assert(HMV_NOALLOC_BYTES == kNoAllocBytes, "header and library disagree on the size");

static __device__ __align__(256) char scratch[kNoAllocBytes];

// Device address of `scratch` on each device, resolved once per device with
// that device current.  The host-side name `scratch` is only a stand-in for
// the symbol; every use below goes through the resolved address.
std::mutex g_mu;
char* g_ptr[64] = {};

int scratch_on_current_device(int dev, char** out) {
  if (dev < 0 || dev >= 64) return fail_with(HMV_EDEVICE, "no-alloc scratch: device index");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return status_from_hip(e, "no-alloc scratch address");
    if (!ptr) return fail_with(HMV_EDEVICE, "no-alloc scratch address: null");
    g_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_ptr[dev];
  return HMV_OK;
}

}  // namespace
}  // namespace hmv

extern "C" {

int hmv_plan_matvec_noalloc(const hmv_plan* plan, const uint64_t* x, uint64_t* y, void* status,
                            void* stream) {
  using namespace hmv;
  if (!plan || !x || !y) return HMV_EINVAL;
  const int64_t need = kStatusBytes + plan->mv_scratch;
  if (need > kNoAllocBytes) {
    char msg[160];
    std::snprintf(msg, sizeof(msg),
                  "no-alloc matvec: the plan needs %lld bytes of workspace, the fixed scratch "
                  "holds %lld",
                  (long long)need, (long long)kNoAllocBytes);
    return fail_with(HMV_ENOMEM, msg);
  }
  clear_stale_error();
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return status_from_hip(e, "no-alloc matvec: current device");
  if (dev != plan->device)
    return fail_with(HMV_EINVAL, "no-alloc matvec: the plan belongs to another device");
  char* base = nullptr;
  const int rc = scratch_on_current_device(dev, &base);
  if (rc != HMV_OK) return rc;
  DevStatus* st = status ? static_cast<DevStatus*>(status) : reinterpret_cast<DevStatus*>(base);
  return plan_matvec_parts(plan, x, y, st, base + kStatusBytes, kNoAllocBytes - kStatusBytes,
                           static_cast<hipStream_t>(stream), nullptr, true);
}

}  // extern "C"
