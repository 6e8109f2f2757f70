// Layout of the binary64 root tables, shared by the host generator and the
// device FFT engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmv {

// ---------------------------------------------------------------- twiddles
// One table per (R, Ns), R in {2,4,8,16}, Ns in {1,8,16,64,256,512,4096}
// (the spans of radix-16 passes and of radix-8 passes):
// entries [r-1][k] = exp(-2 pi i r k / (R Ns)), 1 <= r < R, k < Ns.  Root-major:
// the lanes of a wave (consecutive k) read one root index from consecutive
// entries, a few cache lines per load instead of one line per lane.
constexpr int kTwSpans = 7;
__host__ __device__ constexpr int tw_span(int b) {
  return b == 0 ? 1 : b == 1 ? 8 : b == 2 ? 16 : b == 3 ? 64 : b == 4 ? 256 : b == 5 ? 512 : 4096;
}
__host__ __device__ constexpr int64_t tw_offset(int R, int Ns) {
  int64_t off = 0;
  for (int a = 1; a <= 4; ++a)
    for (int b = 0; b < kTwSpans; ++b) {
      if ((1 << a) == R && tw_span(b) == Ns) return off;
      off += (int64_t)tw_span(b) * ((1 << a) - 1);
    }
  return off;
}
constexpr int64_t kTwEntries = (1 + 3 + 7 + 15) * (1 + 8 + 16 + 64 + 256 + 512 + 4096);
// real-input packing roots exp(-2 pi i k / 16384), k = 0..8192
constexpr int kRealTwN = 16384;
constexpr int64_t kRealTwEntries = kRealTwN / 2 + 1;
constexpr int64_t kRealTwEntries2 = kRealTwN / 4 + 1;
// radix-3 step of the limb transforms of 3K points (K a power of two, at most
// kR3MaxK): exp(-2 pi i s / (3 kR3MaxK)), s < kR3MaxK; a transform of 3K
// points reads every (kR3MaxK / K)-th entry
constexpr int kR3MaxLogK = 11;
constexpr int kR3MaxK = 1 << kR3MaxLogK;
constexpr int64_t kR3Entries = kR3MaxK;
}  // namespace hmv
