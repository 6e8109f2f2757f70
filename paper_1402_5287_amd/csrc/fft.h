// Binary64 complex FFT engine for one work-group, data resident in LDS.
//
// Transform: X[f] = sum_t x[t] exp(sign * 2 pi i t f / N), sign = -1 forward,
// +1 inverse (unnormalised).  Stockham autosort passes: radix 16 while at
// least 16 points remain, then one tail pass of radix 2, 4 or 8.  A pass of
// radix R with span Ns (the product of the earlier radices) reads element
// b + r N/R, multiplies it by the tabulated root exp(sign 2 pi i r k / (R Ns))
// with k = b mod Ns, runs an R-point DFT and writes element
// (b - k) R + k + r Ns.  The output comes out in natural order.
//
// Radix-16 DFTs are two radix-4 stages with one internal twiddle; radix-4
// uses only +-1 and +-i.  Along every data path each binary stage therefore
// carries at most one inexact multiplication by a tabulated or constant root,
// which is the operation model of the error bound used to pick the limb width.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_layout.h"

namespace hmv {


// The tables live in the code object of the one translation unit that
// includes this header (the split-FFT kernels); the host fills them once per
// device with hipMemcpyToSymbol.  Page-aligned, so that where they land does
// not depend on the size of the code around them.
__device__ __align__(4096) double2 g_tw[kTwEntries];
__device__ __align__(4096) double2 g_rtw[kRealTwEntries];
// the even entries of g_rtw (roots of order kRealTwN / 2), so that the
// common even strides read consecutive entries
__device__ __align__(4096) double2 g_rtw2[kRealTwEntries2];

// exp(-2 pi i s / (3 kR3MaxK)), s < kR3MaxK
__device__ __align__(4096) double2 g_r3tw[kR3Entries];

// exp(-2 pi i k rs / kRealTwN)
__device__ __forceinline__ double2 real_root(int k, int rs) {
  return (rs & 1) ? g_rtw[k * rs] : g_rtw2[k * (rs >> 1)];
}

// exp(-2 pi i s / 3K), K = 2^LOGK, s < K
template <int LOGK>
__device__ __forceinline__ double2 r3_root(int s) {
  return g_r3tw[s << (kR3MaxLogK - LOGK)];
}
// sqrt(3)/2 and sqrt(3), correctly rounded
constexpr double kSqrt3h = 0.86602540378443864676;
constexpr double kSqrt3 = 1.73205080756887729353;

// ---------------------------------------------------------------- complex ops
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
// multiply by sign*i  (sign = +-1): exact
__device__ __forceinline__ double2 mul_si(double2 a, int sign) {
  return sign > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// 4-point DFT in place
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3, int sign) {
  const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const double2 t2 = cadd(a1, a3), t3 = mul_si(csub(a1, a3), sign);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// cos / sin of 2 pi m / 16 for m = 1, 2, 3 (correctly rounded constants)
constexpr double kC16_1 = 0.92387953251128673848;   // cos(pi/8)
constexpr double kS16_1 = 0.38268343236508978178;   // sin(pi/8)
constexpr double kC16_2 = 0.70710678118654757274;   // cos(pi/4)

// multiply by exp(sign * 2 pi i m / 16) for m in 0..9 used by the radix-16 split
__device__ __forceinline__ double2 rot16(double2 a, int m, int sign) {
  double c, s;
  switch (m) {
    case 0: return a;
    case 1: c = kC16_1; s = kS16_1; break;
    case 2: c = kC16_2; s = kC16_2; break;
    case 3: c = kS16_1; s = kC16_1; break;
    case 4: return mul_si(a, sign);
    case 6: c = -kC16_2; s = kC16_2; break;
    case 9: c = -kC16_1; s = -kS16_1; break;
    default: c = 1.0; s = 0.0; break;
  }
  s = sign > 0 ? s : -s;
  return make_double2(a.x * c - a.y * s, a.x * s + a.y * c);
}

template <int R>
__device__ __forceinline__ void dft(double2* v, int sign);

template <>
__device__ __forceinline__ void dft<1>(double2*, int) {}

template <>
__device__ __forceinline__ void dft<2>(double2* v, int) {
  const double2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<4>(double2* v, int sign) {
  dft4(v[0], v[1], v[2], v[3], sign);
}

template <>
__device__ __forceinline__ void dft<8>(double2* v, int sign) {
  double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3, sign);
  dft4(o0, o1, o2, o3, sign);
  // exp(sign 2 pi i k / 8), k = 0..3
  o1 = rot16(o1, 2, sign);
  o2 = mul_si(o2, sign);
  o3 = rot16(o3, 6, sign);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <>
__device__ __forceinline__ void dft<16>(double2* v, int sign) {
  // X[k1 + 4 k2] = sum_n2 w16^(n2 k1) w4^(n2 k2) DFT4_n1(v[n2 + 4 n1])[k1]
  double2 u[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    double2 a0 = v[n2], a1 = v[n2 + 4], a2 = v[n2 + 8], a3 = v[n2 + 12];
    dft4(a0, a1, a2, a3, sign);
    u[n2][0] = a0;
    u[n2][1] = rot16(a1, n2, sign);
    u[n2][2] = rot16(a2, 2 * n2, sign);
    u[n2][3] = rot16(a3, 3 * n2, sign);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    double2 a0 = u[0][k1], a1 = u[1][k1], a2 = u[2][k1], a3 = u[3][k1];
    dft4(a0, a1, a2, a3, sign);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

// LDS slot of element i: one spare slot after every 16 elements.  Strided
// accesses (stride 16 and 256 points) then fall on distinct bank groups,
// and every per-element offset inside a pass is a constant that the LDS
// instructions take as an immediate.  An N-point buffer needs
// lds_points(N) slots.
__device__ __forceinline__ int lds_slot(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_points(int N) { return N + (N >> 4); }
// lds_slot(i + r * s) for a stride s that is a multiple of 16, given
// si = lds_slot(i): the slot step per r is the constant s + s/16
__device__ __forceinline__ int lds_step(int si, int r, int s) { return si + r * (s + (s >> 4)); }

// One Stockham pass over N points held in buf (LDS).  Requires
// blockDim.x * NB >= N / R.  Ends with a barrier.
template <int R, int NB>
__device__ __forceinline__ void stockham_pass(double2* buf, int N, int Ns, int sign) {
  const int nbf = N / R;
  const int T = blockDim.x;
  const double2* tw = g_tw + tw_offset(R, Ns);
  double2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * T;
    if (b < nbf) {
      const int k = b & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[i][r] = buf[(nbf & 15) == 0 ? lds_step(lds_slot(b), r, nbf) : lds_slot(b + r * nbf)];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 w = tw[(r - 1) * Ns + k];
          if (sign > 0) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * T;
    if (b < nbf) {
      const int k = b & (Ns - 1);
      dft<R>(v[i], sign);
      const int base = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r)
        buf[(Ns & 15) == 0 ? lds_step(lds_slot(base), r, Ns) : lds_slot(base + r * Ns)] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform of N = 2^logN points (2 <= N <= 8192) in buf (element i in
// slot lds_slot(i)).  Requires
// blockDim.x >= N / 16 (blockDim.x >= 1 for N < 16).  Caller must have
// synchronised after filling buf; ends with a barrier.
__device__ __forceinline__ void fft_lds(double2* buf, int logN, int sign) {
  const int N = 1 << logN;
  int Ns = 1;
  const int a = logN >> 2, rem = logN & 3;
  for (int p = 0; p < a; ++p) {
    stockham_pass<16, 1>(buf, N, Ns, sign);
    Ns <<= 4;
  }
  if (rem == 1) stockham_pass<2, 8>(buf, N, Ns, sign);
  else if (rem == 2) stockham_pass<4, 4>(buf, N, Ns, sign);
  else if (rem == 3) stockham_pass<8, 2>(buf, N, Ns, sign);
}

// fft_lds with the size known at compile time (every pass's span, table
// offset and slot steps become constants).
template <int LOGN>
__device__ __forceinline__ void fft_lds_t(double2* buf, int sign) {
  constexpr int N = 1 << LOGN, A = LOGN >> 2, REM = LOGN & 3;
  int Ns = 1;
#pragma unroll
  for (int p = 0; p < A; ++p) {
    stockham_pass<16, 1>(buf, N, Ns, sign);
    Ns <<= 4;
  }
  if constexpr (REM == 1) stockham_pass<2, 8>(buf, N, Ns, sign);
  else if constexpr (REM == 2) stockham_pass<4, 4>(buf, N, Ns, sign);
  else if constexpr (REM == 3) stockham_pass<8, 2>(buf, N, Ns, sign);
}

// ------------------------------------------------------------------------
// Two independent transforms in one work-group, of NA = 2^LA points in bufA
// and NB = 2^LB points in bufB (each with its own lds_slot layout), run pass
// by pass together: pass p has span 16^p in both, radix 16 while four or more
// bits remain, then the tail radix, and radix 1 (no work) once a transform
// is done.  The butterflies of A come first in one index space, then those of
// B; thread t takes indices t, t + T, ...  T = blockDim.x.

template <int R, int N>
__device__ __forceinline__ void pair_read(const double2* buf, int b, int Ns, int sign,
                                          double2* v) {
  constexpr int nbf = N / R;
  const int k = b & (Ns - 1);
#pragma unroll
  for (int r = 0; r < R; ++r)
    v[r] = buf[(nbf & 15) == 0 ? lds_step(lds_slot(b), r, nbf) : lds_slot(b + r * nbf)];
  if (Ns > 1) {
    const double2* tw = g_tw + tw_offset(R, Ns);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 w = tw[(r - 1) * Ns + k];
      if (sign > 0) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
  }
}

template <int R>
__device__ __forceinline__ void pair_write(double2* buf, int b, int Ns, int sign, double2* v) {
  const int k = b & (Ns - 1);
  dft<R>(v, sign);
  const int base = (b - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r)
    buf[(Ns & 15) == 0 ? lds_step(lds_slot(base), r, Ns) : lds_slot(base + r * Ns)] = v[r];
}

template <int RA, int RB, int NA, int NB, int T>
__device__ __forceinline__ void stockham_pass_pair(double2* bufA, double2* bufB, int Ns,
                                                   int sign) {
  constexpr int nbA = RA > 1 ? NA / RA : 0, nbB = RB > 1 ? NB / RB : 0;
  constexpr int IT = (nbA + nbB + T - 1) / T;
  constexpr int RM = RA > RB ? RA : RB;
  const int t = threadIdx.x;
  double2 v[IT][RM];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int u = t + i * T;
    if constexpr (nbA > 0) {
      if (u < nbA) pair_read<RA, NA>(bufA, u, Ns, sign, v[i]);
    }
    if constexpr (nbB > 0) {
      if (u >= nbA && u < nbA + nbB) pair_read<RB, NB>(bufB, u - nbA, Ns, sign, v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int u = t + i * T;
    if constexpr (nbA > 0) {
      if (u < nbA) pair_write<RA>(bufA, u, Ns, sign, v[i]);
    }
    if constexpr (nbB > 0) {
      if (u >= nbA && u < nbA + nbB) pair_write<RB>(bufB, u - nbA, Ns, sign, v[i]);
    }
  }
  __syncthreads();
}

// radix of pass p of a 2^LG-point transform (1 once it is done)
__host__ __device__ constexpr int pass_radix(int LG, int p) {
  return p < LG / 4 ? 16 : (p == LG / 4 && (LG & 3)) ? (1 << (LG & 3)) : 1;
}

template <int LA, int LB, int T, int p = 0>
__device__ __forceinline__ void fft_pair_lds(double2* bufA, double2* bufB, int sign) {
  constexpr int RA = pass_radix(LA, p), RB = pass_radix(LB, p);
  if constexpr (RA > 1 || RB > 1) {
    stockham_pass_pair<RA, RB, (1 << LA), (1 << LB), T>(bufA, bufB, 1 << (4 * p), sign);
    fft_pair_lds<LA, LB, T, p + 1>(bufA, bufB, sign);
  }
}

// ------------------------------------------------------------------------
// Register-resident variant.  For N >= 16 the Ta = N/16 active threads each
// hold 16 elements, element t + Ta*j in v[j]; for N < 16 thread 0 holds all
// N.  The first pass reads its radix-16 inputs straight from registers and
// the last pass writes its outputs straight back, in the same layout and in
// natural order; LDS (N points) carries only the exchanges in between.  The
// layout is also the input layout of the next transform's first pass, so a
// pointwise product can sit between a forward and an inverse transform with
// no LDS round trip.  Every thread of the block must call it.

template <int R>
__device__ __forceinline__ void last_pass_to_regs(const double2* buf, int N, int sign, int t,
                                                  int Ta, double2* v) {
  const int Ns = N / R;            // span before the pass == butterflies in it
  const double2* tw = g_tw + tw_offset(R, Ns);
#pragma unroll
  for (int i = 0; i < 16 / R; ++i) {
    const int b = t + i * Ta;      // butterfly index; k = b since b < Ns
    double2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
      u[r] = buf[(Ns & 15) == 0 ? lds_step(lds_slot(b), r, Ns) : lds_slot(b + r * Ns)];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 w = tw[(r - 1) * Ns + b];
      if (sign > 0) w.y = -w.y;
      u[r] = cmul(u[r], w);
    }
    dft<R>(u, sign);
#pragma unroll
    for (int r = 0; r < R; ++r) v[i + r * (16 / R)] = u[r];
  }
}

template <int LOGN>
__device__ __forceinline__ void fft_regs(double2* v, double2* buf, int sign) {
  constexpr int N = 1 << LOGN;
  const int t = threadIdx.x;
  if constexpr (N <= 16) {
    if (t == 0) dft<N>(v, sign);
    return;
  } else {
    constexpr int Ta = N >> 4;
    constexpr int A = LOGN >> 2, REM = LOGN & 3;
    const bool act = t < Ta;
    if (act) {
      dft<16>(v, sign);
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[17 * t + r] = v[r];     // lds_slot(16 t + r)
    }
    __syncthreads();
    constexpr int NMID = (REM ? A : A - 1) - 1;
    int Ns = 16;
#pragma unroll
    for (int p = 0; p < NMID; ++p) {
      stockham_pass<16, 1>(buf, N, Ns, sign);
      Ns <<= 4;
    }
    if (act) last_pass_to_regs<(REM == 0 ? 16 : (1 << REM))>(buf, N, sign, t, Ta, v);
    __syncthreads();
  }
}

// The same contract with 8 elements per thread, for N = 8^P >= 64 points:
// thread t < Ta = N/8 holds element t + Ta j in v[j]; all passes radix 8
// (twice as many threads as fft_regs for the same N, half the registers
// per thread).  Every thread of the block must call it.
template <int LOGN>
__device__ __forceinline__ void fft_regs8(double2* v, double2* buf, int sign) {
  static_assert(LOGN % 3 == 0 && LOGN >= 6, "N must be a power of 8, at least 64");
  constexpr int N = 1 << LOGN, Ta = N >> 3;
  const int t = threadIdx.x;
  const bool act = t < Ta;
  if (act) {
    dft<8>(v, sign);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[8 * t + (t >> 1) + r] = v[r];   // lds_slot(8 t + r)
  }
  __syncthreads();
  constexpr int NMID = LOGN / 3 - 2;
  int Ns = 8;
#pragma unroll
  for (int p = 0; p < NMID; ++p) {
    stockham_pass<8, 1>(buf, N, Ns, sign);
    Ns <<= 3;
  }
  if (act) {
    // last pass, span N/8: butterfly t writes elements t + Ta r, natural order
    const double2* tw = g_tw + tw_offset(8, Ta);
    double2 u[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
      u[r] = buf[(Ta & 15) == 0 ? lds_step(lds_slot(t), r, Ta) : lds_slot(t + r * Ta)];
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      double2 w = tw[(r - 1) * Ta + t];
      if (sign > 0) w.y = -w.y;
      u[r] = cmul(u[r], w);
    }
    dft<8>(u, sign);
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = u[r];
  }
  __syncthreads();
}

// fft_regs (R = 16 elements per thread) or fft_regs8 (R = 8).
template <int LOGN, int R>
__device__ __forceinline__ void fft_regs_r(double2* v, double2* buf, int sign) {
  if constexpr (R == 8) fft_regs8<LOGN>(v, buf, sign);
  else fft_regs<LOGN>(v, buf, sign);
}

}  // namespace hmv
