// Status block maintenance (a fill kernel rather than a memset, so that a
// captured graph holds no memset node).
#include "common.h"
#include "kernels.h"

namespace hmv {

__global__ void k_clear_status(DevStatus* st) {
  uint64_t* p = reinterpret_cast<uint64_t*>(st);
  if (threadIdx.x < sizeof(DevStatus) / 8) p[threadIdx.x] = 0ull;
}

hipError_t launch_clear_status(DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace hmv
