// Host generation of the binary64 root-of-unity tables and the rigorous
// error bound that fixes the limb width.
#pragma once
#include <stdint.h>

namespace hmv {

// exp(-2 pi i m / N), N a power of two, computed in long double with an
// octant reduction and rounded to binary64.
void unit_root(int64_t m, int64_t N, double* re, double* im);

// Fill the Stockham table (2 * kTwEntries doubles), the real-packing
// table (2 * kRealTwEntries doubles: exp(-2 pi i k / 16384), k <= 8192) and
// the radix-3 table (2 * kR3Entries doubles: exp(-2 pi i s / (3 kR3MaxK))).
// Returns the largest |table - root| observed against the long double values
// (the radix-8/16 constants and sqrt(3)/2 included), plus a margin for the
// long double evaluation itself: the beta of the error bound.
double gen_fft_tables(double* tw, double* rtw, double* r3);

// Percival-type bound on the max-norm error of a binary64 FFT convolution
// z = IFFT(FFT(a) . FFT(b)) with transforms of 2^k points:
//   ||a||_2 ||b||_2 ((1+eps)^(3k) (1+eps sqrt5)^(3k+1) (1+beta)^(3k) - 1),
// eps = 2^-53, evaluated through log1p / expm1 in long double so that terms
// like 1 + 2^-53 are not lost.
double fft_conv_bound(double norm_a, double norm_b, int k, double beta);

// ---------------------------------------------------------------- mod p
// Arithmetic modulo p = 2^64 - 2^32 + 1 on the host (reference for tables).
uint64_t gold_mul(uint64_t a, uint64_t b);
uint64_t gold_pow(uint64_t a, uint64_t e);
uint64_t gold_inv(uint64_t a);
// w_M = g^((p-1)/M) with M a power of two <= 2^32, taken as a power of one
// primitive 2^32-th root so that all sizes are consistent (g = 7 generates
// the multiplicative group).
uint64_t gold_root(int64_t M);
// Fill the NTT tables: forward and inverse (R, Ns) tables (2 kNttTwEntries),
// the 16 internal roots forward then inverse (32), the split roots forward
// then inverse (2 kNttSplitEntries).
void gen_ntt_tables(uint64_t* tw, uint64_t* r16, uint64_t* split);

}  // namespace hmv
