// Number-theoretic transforms modulo the prime p = 2^64 - 2^32 + 1.
//
// Used where exactness must not depend on a floating-point error bound: the
// limb-axis and index-axis transforms of the NTT path and the limb-axis
// transforms under the Karatsuba-style recursion.  p - 1 = 2^32 (2^32 - 1),
// so p has roots of unity of every power-of-two order up to 2^32; all roots
// used here are powers of one primitive 2^32-th root, so the roots of every
// transform size are mutually consistent.  Residues are kept in [0, p).
//
// The engine mirrors the binary64 one: Stockham radix-16 passes (two
// radix-4 stages) plus one radix-2/4/8 tail, data in LDS with the same
// XOR swizzle, and a register-resident variant for the index-axis pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_layout.h"

namespace hmv {

// roots: the same (R, Ns) table layout as the binary64 engine, forward
// (w^(r k)) and inverse (w^(-r k)); the split roots w_{16384}^s for
// s = 0..8191 (forward, then inverse).  Filled once per device by the host.
// The radix-16 internal roots are powers of two (gl_shl below).
__device__ uint64_t g_ntw[2 * kNttTwEntries];
__device__ uint64_t g_nsplit[2 * kNttSplitEntries];

__device__ __forceinline__ uint64_t gl_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  if (s < a) s += 0xFFFFFFFFull;        // wrapped: 2^64 = 2^32 - 1 (mod p)
  return s >= kGoldP ? s - kGoldP : s;
}

__device__ __forceinline__ uint64_t gl_sub(uint64_t a, uint64_t b) {
  return a >= b ? a - b : a + (kGoldP - b);
}

// lo + hi 2^64 reduced mod p, for any 64-bit lo and hi
__device__ __forceinline__ uint64_t gl_fold(uint64_t lo, uint64_t hi) {
  const uint64_t hh = hi >> 32, hl = hi & 0xFFFFFFFFull;
  // lo + hl 2^64 + hh 2^96 = lo + hl (2^32 - 1) - hh  (mod p)
  uint64_t t = lo >= hh ? lo - hh : lo - hh + kGoldP;
  const uint64_t u = (hl << 32) - hl;
  uint64_t s = t + u;
  if (s < t) s += 0xFFFFFFFFull;
  return s >= kGoldP ? s - kGoldP : s;
}

__device__ __forceinline__ uint64_t gl_mul(uint64_t a, uint64_t b) {
  return gl_fold(a * b, __umul64hi(a, b));
}

// x 2^E mod p for a constant E < 192, with 2^96 = -1 and 2^64 = 2^32 - 1
// (mod p): shifts and one folding step instead of a 64 x 64-bit product.
// Every 16th root of unity mod p is a power of two (2 has order 192), so
// the radix-16 internal roots take this form.
template <int E>
__device__ __forceinline__ uint64_t gl_shl(uint64_t x) {
  static_assert(E >= 0 && E < 192, "exponent out of range");
  if constexpr (E >= 96) {
    const uint64_t r = gl_shl<E - 96>(x);
    return r ? kGoldP - r : 0;
  } else if constexpr (E == 0) {
    return x;
  } else if constexpr (E < 64) {
    return gl_fold(x << E, x >> (64 - E));
  } else {
    return gl_sub(gl_shl<E - 32>(x), gl_shl<E - 64>(x));
  }
}

// w16 = 2^156 (mod p) is the 16th root of unity of the transforms (the
// primitive 2^32-th root 7^((p-1)/2^32) raised to 2^28; the host checks the
// tables against it), so w16^m = 2^(156 m mod 192) forward and
// 2^(36 m mod 192) inverse.
constexpr int kNttRootExp16 = 156;
template <int INV>
__host__ __device__ constexpr int r16_exp(int m) {
  return ((INV ? 192 - kNttRootExp16 : kNttRootExp16) * m) % 192;
}
template <int INV, int M>
__device__ __forceinline__ uint64_t mul_r16(uint64_t x) {
  return gl_shl<r16_exp<INV>(M)>(x);
}

// balanced digit -> residue
__device__ __forceinline__ uint64_t gl_from_int(int64_t d) {
  return d >= 0 ? (uint64_t)d : kGoldP - (uint64_t)(-d);
}

// residue -> centred integer in (-p/2, p/2)
__device__ __forceinline__ int64_t gl_centre(uint64_t v) {
  return v > (kGoldP >> 1) ? -(int64_t)(kGoldP - v) : (int64_t)v;
}

// 4-point transform, in place, in the direction INV (w4 = w16^4)
template <int INV>
__device__ __forceinline__ void ndft4(uint64_t& a0, uint64_t& a1, uint64_t& a2, uint64_t& a3) {
  const uint64_t t0 = gl_add(a0, a2), t1 = gl_sub(a0, a2);
  const uint64_t t2 = gl_add(a1, a3), t3 = mul_r16<INV, 4>(gl_sub(a1, a3));
  a0 = gl_add(t0, t2);
  a2 = gl_sub(t0, t2);
  a1 = gl_add(t1, t3);
  a3 = gl_sub(t1, t3);
}

template <int R, int INV>
__device__ __forceinline__ void ndft(uint64_t* v);

template <>
__device__ __forceinline__ void ndft<1, 0>(uint64_t*) {}
template <>
__device__ __forceinline__ void ndft<1, 1>(uint64_t*) {}

template <int INV>
__device__ __forceinline__ void ndft2(uint64_t* v) {
  const uint64_t a = v[0], b = v[1];
  v[0] = gl_add(a, b);
  v[1] = gl_sub(a, b);
}
template <>
__device__ __forceinline__ void ndft<2, 0>(uint64_t* v) { ndft2<0>(v); }
template <>
__device__ __forceinline__ void ndft<2, 1>(uint64_t* v) { ndft2<1>(v); }

template <>
__device__ __forceinline__ void ndft<4, 0>(uint64_t* v) { ndft4<0>(v[0], v[1], v[2], v[3]); }
template <>
__device__ __forceinline__ void ndft<4, 1>(uint64_t* v) { ndft4<1>(v[0], v[1], v[2], v[3]); }

template <int INV>
__device__ __forceinline__ void ndft8(uint64_t* v) {
  uint64_t e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  uint64_t o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  ndft4<INV>(e0, e1, e2, e3);
  ndft4<INV>(o0, o1, o2, o3);
  o1 = mul_r16<INV, 2>(o1);
  o2 = mul_r16<INV, 4>(o2);
  o3 = mul_r16<INV, 6>(o3);
  v[0] = gl_add(e0, o0); v[4] = gl_sub(e0, o0);
  v[1] = gl_add(e1, o1); v[5] = gl_sub(e1, o1);
  v[2] = gl_add(e2, o2); v[6] = gl_sub(e2, o2);
  v[3] = gl_add(e3, o3); v[7] = gl_sub(e3, o3);
}
template <>
__device__ __forceinline__ void ndft<8, 0>(uint64_t* v) { ndft8<0>(v); }
template <>
__device__ __forceinline__ void ndft<8, 1>(uint64_t* v) { ndft8<1>(v); }

// internal root w16^(n2 k) applied after the first radix-4 stage
template <int INV, int N2, int K>
__device__ __forceinline__ uint64_t tw16(uint64_t x) {
  if constexpr (N2 == 0 || K == 0) return x;
  else return mul_r16<INV, N2 * K>(x);
}

template <int INV, int N2>
__device__ __forceinline__ void ndft16_col(const uint64_t* v, uint64_t (&u)[4][4]) {
  uint64_t a0 = v[N2], a1 = v[N2 + 4], a2 = v[N2 + 8], a3 = v[N2 + 12];
  ndft4<INV>(a0, a1, a2, a3);
  u[N2][0] = a0;
  u[N2][1] = tw16<INV, N2, 1>(a1);
  u[N2][2] = tw16<INV, N2, 2>(a2);
  u[N2][3] = tw16<INV, N2, 3>(a3);
}

template <int INV>
__device__ __forceinline__ void ndft16(uint64_t* v) {
  uint64_t u[4][4];
  ndft16_col<INV, 0>(v, u);
  ndft16_col<INV, 1>(v, u);
  ndft16_col<INV, 2>(v, u);
  ndft16_col<INV, 3>(v, u);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    uint64_t a0 = u[0][k1], a1 = u[1][k1], a2 = u[2][k1], a3 = u[3][k1];
    ndft4<INV>(a0, a1, a2, a3);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}
template <>
__device__ __forceinline__ void ndft<16, 0>(uint64_t* v) { ndft16<0>(v); }
template <>
__device__ __forceinline__ void ndft<16, 1>(uint64_t* v) { ndft16<1>(v); }

__device__ __forceinline__ int nswz(int i) { return i ^ ((i >> 4) & 15); }

// One Stockham pass mod p over N points in LDS.  inv selects the inverse
// roots.  Requires blockDim.x * NB >= N / R.  Ends with a barrier.
template <int R, int NB, int INV>
__device__ __forceinline__ void ntt_pass(uint64_t* buf, int N, int Ns) {
  constexpr int inv = INV;
  const int nbf = N / R;
  const int T = blockDim.x;
  const uint64_t* tw = g_ntw + (inv ? kNttTwEntries : 0) + ntt_tw_offset(R, Ns);
  uint64_t v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * T;
    if (b < nbf) {
      const int k = b & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[nswz(b + r * nbf)];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = gl_mul(v[i][r], tw[k * (R - 1) + (r - 1)]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * T;
    if (b < nbf) {
      const int k = b & (Ns - 1);
      ndft<R, INV>(v[i]);
      const int base = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[nswz(base + r * Ns)] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform of N = 2^logN points (N <= 8192) in LDS, natural order, in
// the direction INV.  Requires blockDim.x >= N / 16.
template <int INV>
__device__ __forceinline__ void ntt_lds(uint64_t* buf, int logN) {
  const int N = 1 << logN;
  int Ns = 1;
  const int a = logN >> 2, rem = logN & 3;
  for (int p = 0; p < a; ++p) {
    ntt_pass<16, 1, INV>(buf, N, Ns);
    Ns <<= 4;
  }
  if (rem == 1) ntt_pass<2, 8, INV>(buf, N, Ns);
  else if (rem == 2) ntt_pass<4, 4, INV>(buf, N, Ns);
  else if (rem == 3) ntt_pass<8, 2, INV>(buf, N, Ns);
}

// Register-resident variant (layout as the binary64 fft_regs: for N >= 16
// thread t < N/16 holds element t + (N/16) j in v[j]; for N < 16 thread 0
// holds all N).
template <int R, int INV>
__device__ __forceinline__ void ntt_last_to_regs(const uint64_t* buf, int N, int t, int Ta,
                                                 uint64_t* v) {
  constexpr int inv = INV;
  const int Ns = N / R;
  const uint64_t* tw = g_ntw + (inv ? kNttTwEntries : 0) + ntt_tw_offset(R, Ns);
#pragma unroll
  for (int i = 0; i < 16 / R; ++i) {
    const int b = t + i * Ta;
    uint64_t u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = buf[nswz(b + r * Ns)];
#pragma unroll
    for (int r = 1; r < R; ++r) u[r] = gl_mul(u[r], tw[b * (R - 1) + (r - 1)]);
    ndft<R, INV>(u);
#pragma unroll
    for (int r = 0; r < R; ++r) v[i + r * (16 / R)] = u[r];
  }
}

template <int LOGN, int INV>
__device__ __forceinline__ void ntt_regs(uint64_t* v, uint64_t* buf) {
  constexpr int N = 1 << LOGN;
  const int t = threadIdx.x;
  if constexpr (N <= 16) {
    if (t == 0) ndft<N, INV>(v);
    return;
  } else {
    constexpr int Ta = N >> 4;
    constexpr int A = LOGN >> 2, REM = LOGN & 3;
    const bool act = t < Ta;
    if (act) {
      ndft<16, INV>(v);
#pragma unroll
      for (int r = 0; r < 16; ++r) buf[nswz(16 * t + r)] = v[r];
    }
    __syncthreads();
    constexpr int NMID = (REM ? A : A - 1) - 1;
    int Ns = 16;
#pragma unroll
    for (int p = 0; p < NMID; ++p) {
      ntt_pass<16, 1, INV>(buf, N, Ns);
      Ns <<= 4;
    }
    if (act) ntt_last_to_regs<(REM == 0 ? 16 : (1 << REM)), INV>(buf, N, t, Ta, v);
    __syncthreads();
  }
}

}  // namespace hmv
