// Root-of-unity tables and the FFT error bound (host code).
#include "tables.h"

#include <cmath>
#include <cstdint>

#include "fft_layout.h"
#include "ntt_layout.h"

namespace hmv {

void unit_root(int64_t m, int64_t N, double* re, double* im) {
  m %= N;
  if (m < 0) m += N;
  long double c, s;               // cos, sin of 2 pi m / N
  if (N < 8) {
    const long double th = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)N;
    c = cosl(th);
    s = sinl(th);
    if (2 * m == N) { c = -1.0L; s = 0.0L; }
    if (m == 0) { c = 1.0L; s = 0.0L; }
    if (4 * m == N) { c = 0.0L; s = 1.0L; }
    if (4 * m == 3 * N) { c = 0.0L; s = -1.0L; }
  } else {
    const int64_t q4 = N / 4, q8 = N / 8;
    const int64_t quad = m / q4;
    int64_t r = m - quad * q4;            // 0 <= r < N/4
    bool swap = false;
    if (r > q8) { r = q4 - r; swap = true; }
    const long double th = 2.0L * 3.141592653589793238462643383279502884L * (long double)r / (long double)N;
    long double cb = cosl(th), sb = sinl(th);
    if (r == 0) { cb = 1.0L; sb = 0.0L; }
    if (swap) { const long double t = cb; cb = sb; sb = t; }
    // angle = quad * pi/2 + phi, (cb, sb) = (cos phi, sin phi)
    switch (quad) {
      case 0: c = cb; s = sb; break;
      case 1: c = -sb; s = cb; break;
      case 2: c = -cb; s = -sb; break;
      default: c = sb; s = -cb; break;
    }
  }
  *re = (double)c;
  *im = (double)(-s);
}

double gen_fft_tables(double* tw, double* rtw) {
  long double worst = 0.0L;
  auto track = [&](int64_t m, int64_t N, double re, double im) {
    const long double th = 2.0L * 3.141592653589793238462643383279502884L * (long double)(m % N) / (long double)N;
    const long double dr = (long double)re - cosl(th), di = (long double)im + sinl(th);
    const long double e = sqrtl(dr * dr + di * di);
    if (e > worst) worst = e;
  };
  for (int k = 0; k < kRealTwN / 2 + 1; ++k) {
    double re, im;
    unit_root(k, kRealTwN, &re, &im);
    rtw[2 * k] = re;
    rtw[2 * k + 1] = im;
    track(k, kRealTwN, re, im);
  }
  for (int a = 1; a <= 4; ++a)
    for (int b = 0; b < kTwSpans; ++b) {
      const int R = 1 << a, Ns = tw_span(b);
      double* t = tw + 2 * tw_offset(R, Ns);
      for (int k = 0; k < Ns; ++k)
        for (int r = 1; r < R; ++r) {
          double re, im;
          unit_root((int64_t)r * k, (int64_t)R * Ns, &re, &im);
          t[2 * ((r - 1) * Ns + k)] = re;
          t[2 * ((r - 1) * Ns + k) + 1] = im;
          track((int64_t)r * k, (int64_t)R * Ns, re, im);
        }
    }
  // constants of the radix-8/16 kernels: cos(pi/8), sin(pi/8), cos(pi/4)
  {
    const double c[3] = {0.92387953251128673848, 0.38268343236508978178, 0.70710678118654757274};
    const long double ex[3] = {cosl(3.141592653589793238462643383279502884L / 8),
                               sinl(3.141592653589793238462643383279502884L / 8),
                               sqrtl(2.0L) / 2};
    for (int i = 0; i < 3; ++i) {
      const long double e = fabsl((long double)c[i] - ex[i]) * sqrtl(2.0L);
      if (e > worst) worst = e;
    }
  }
  // the long double reference itself is within a few 2^-64 of the true root
  return (double)(worst + ldexpl(1.0L, -60));
}

double fft_conv_bound(double norm_a, double norm_b, int k, double beta) {
  const long double eps = ldexpl(1.0L, -53);
  const long double lg = 3.0L * k * log1pl(eps) + (3.0L * k + 1.0L) * log1pl(eps * sqrtl(5.0L)) +
                         3.0L * k * log1pl((long double)beta);
  const long double f = expm1l(lg);
  // a relative margin for the evaluation of the bound itself
  return (double)((long double)norm_a * (long double)norm_b * f * (1.0L + ldexpl(1.0L, -20)));
}

uint64_t gold_mul(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) % kGoldP);
}

uint64_t gold_pow(uint64_t a, uint64_t e) {
  uint64_t r = 1;
  a %= kGoldP;
  while (e) {
    if (e & 1) r = gold_mul(r, a);
    a = gold_mul(a, a);
    e >>= 1;
  }
  return r;
}

uint64_t gold_inv(uint64_t a) { return gold_pow(a, kGoldP - 2); }

uint64_t gold_root(int64_t M) {
  const uint64_t w32 = gold_pow(7, (kGoldP - 1) >> 32);   // primitive 2^32-th root
  return gold_pow(w32, (uint64_t(1) << 32) / (uint64_t)M);
}

void gen_ntt_tables(uint64_t* tw, uint64_t* r16, uint64_t* split) {
  const int radices[4] = {2, 4, 8, 16};
  const int spans[4] = {1, 16, 256, 4096};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const int R = radices[a], Ns = spans[b];
      const uint64_t w = gold_root((int64_t)R * Ns), wi = gold_inv(w);
      uint64_t* f = tw + ntt_tw_offset(R, Ns);
      uint64_t* g = tw + kNttTwEntries + ntt_tw_offset(R, Ns);
      for (int k = 0; k < Ns; ++k)
        for (int r = 1; r < R; ++r) {
          f[k * (R - 1) + (r - 1)] = gold_pow(w, (uint64_t)r * k);
          g[k * (R - 1) + (r - 1)] = gold_pow(wi, (uint64_t)r * k);
        }
    }
  const uint64_t w16 = gold_root(16), w16i = gold_inv(w16);
  for (int m = 0; m < 16; ++m) {
    r16[m] = gold_pow(w16, m);
    r16[16 + m] = gold_pow(w16i, m);
  }
  const uint64_t ws = gold_root(kNttSplitN), wsi = gold_inv(ws);
  uint64_t f = 1, g = 1;
  for (int s = 0; s < kNttSplitEntries; ++s) {
    split[s] = f;
    split[kNttSplitEntries + s] = g;
    f = gold_mul(f, ws);
    g = gold_mul(g, wsi);
  }
}

}  // namespace hmv
