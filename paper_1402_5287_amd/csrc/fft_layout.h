// Layout of the binary64 root tables, shared by the host generator and the
// device FFT engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmv {

// ---------------------------------------------------------------- twiddles
// One table per (R, Ns), R in {2,4,8,16}, Ns in {1,16,256,4096}:
// entries [k][r-1] = exp(-2 pi i r k / (R Ns)), k < Ns, 1 <= r < R.
__host__ __device__ constexpr int64_t tw_offset(int R, int Ns) {
  int64_t off = 0;
  const int radices[4] = {2, 4, 8, 16};
  const int spans[4] = {1, 16, 256, 4096};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      if (radices[a] == R && spans[b] == Ns) return off;
      off += (int64_t)spans[b] * (radices[a] - 1);
    }
  return off;
}
constexpr int64_t kTwEntries = (1 + 3 + 7 + 15) * (1 + 16 + 256 + 4096);
// real-input packing roots exp(-2 pi i k / 16384), k = 0..8192
constexpr int kRealTwN = 16384;
constexpr int64_t kRealTwEntries = kRealTwN / 2 + 1;
}  // namespace hmv
