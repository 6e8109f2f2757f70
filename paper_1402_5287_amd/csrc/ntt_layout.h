// Constants and table layout of the transforms modulo p = 2^64 - 2^32 + 1,
// shared by the host generator and the device engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmv {

constexpr uint64_t kGoldP = 0xFFFFFFFF00000001ull;

// (R, Ns) tables: entries [k][r-1] = w_{R Ns}^(r k), k < Ns, 1 <= r < R.  Unlike
// the binary64 tables (root-major), a thread's R-1 roots of 8 bytes are
// contiguous here, so that they load as a few wide loads.
__host__ __device__ constexpr int64_t ntt_tw_offset(int R, int Ns) {
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
constexpr int64_t kNttTwEntries = (1 + 3 + 7 + 15) * (1 + 16 + 256 + 4096);
// split roots w_{16384}^s, s < 8192 (radix-2 split of the index axis)
constexpr int kNttSplitN = 16384;
constexpr int64_t kNttSplitEntries = kNttSplitN / 2;

}  // namespace hmv
