// Root-of-unity tables and the FFT error bound (host code).
#include "tables.h"

#include <cmath>
#include <cstdint>
#include <vector>

#include "fft_layout.h"
#include "ntt_layout.h"

namespace hmv {

namespace {
constexpr long double kPiL = 3.141592653589793238462643383279502884L;

// cos and sin (long double) of the first-octant angles 2 pi r / kRootRes,
// r = 0 .. kRootRes / 8.  Every table size N divides kRootRes, and for N a
// power of two the angle 2 pi r / N is computed to the same long double as
// 2 pi (r kRootRes / N) / kRootRes (scaling by a power of two is exact), so
// the roots come out bit for bit as if evaluated directly; the cosines and
// sines are evaluated once each instead of once per table entry.
constexpr int64_t kRootRes = 65536;
struct Octant {
  long double c[kRootRes / 8 + 1], s[kRootRes / 8 + 1];
};
const Octant& octant() {
  static const Octant* t = [] {
    Octant* o = new Octant;
    for (int64_t r = 0; r <= kRootRes / 8; ++r) {
      const long double th = 2.0L * kPiL * (long double)r / (long double)kRootRes;
      o->c[r] = r == 0 ? 1.0L : cosl(th);
      o->s[r] = r == 0 ? 0.0L : sinl(th);
    }
    return o;
  }();
  return *t;
}

// the root exp(-2 pi i m / N) rounded to doubles; *base = its first-octant
// index at kRootRes resolution (its rounding error is that entry's), or -1
// when it is exact or was evaluated directly
void unit_root_base(int64_t m, int64_t N, double* re, double* im, int64_t* base) {
  m %= N;
  if (m < 0) m += N;
  *base = -1;
  long double c, s;               // cos, sin of 2 pi m / N
  if (N < 8) {
    const long double th = 2.0L * kPiL * (long double)m / (long double)N;
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
    long double cb, sb;
    if (kRootRes % N == 0) {
      const int64_t rr = r * (kRootRes / N);
      cb = octant().c[rr];
      sb = octant().s[rr];
      if (rr != 0) *base = rr;
    } else {
      const long double th = 2.0L * kPiL * (long double)r / (long double)N;
      cb = cosl(th);
      sb = sinl(th);
      if (r == 0) { cb = 1.0L; sb = 0.0L; }
    }
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
}  // namespace

void unit_root(int64_t m, int64_t N, double* re, double* im) {
  int64_t base;
  unit_root_base(m, N, re, im, &base);
}

double gen_fft_tables(double* tw, double* rtw, double* r3) {
  // worst rounding error of the roots: per first-octant entry (the other
  // entries are exact sign changes and swaps of it), over the entries used
  long double worst = 0.0L;
  std::vector<char> used(kRootRes / 8 + 1, 0);
  auto root = [&](int64_t m, int64_t N, double* re, double* im) {
    int64_t base;
    unit_root_base(m, N, re, im, &base);
    if (base >= 0) {
      used[base] = 1;
    } else {
      const long double th = 2.0L * kPiL * (long double)(m % N) / (long double)N;
      const long double dr = (long double)*re - cosl(th), di = (long double)*im + sinl(th);
      const long double e = sqrtl(dr * dr + di * di);
      if (e > worst) worst = e;
    }
  };
  for (int k = 0; k < kRealTwN / 2 + 1; ++k) {
    double re, im;
    root(k, kRealTwN, &re, &im);
    rtw[2 * k] = re;
    rtw[2 * k + 1] = im;
  }
  for (int k = 0; k < kR3Entries; ++k) {
    double re, im;
    root(k, 3 * (int64_t)kR3MaxK, &re, &im);
    r3[2 * k] = re;
    r3[2 * k + 1] = im;
  }
  for (int a = 1; a <= 4; ++a)
    for (int b = 0; b < kTwSpans; ++b) {
      const int R = 1 << a, Ns = tw_span(b);
      double* t = tw + 2 * tw_offset(R, Ns);
      for (int k = 0; k < Ns; ++k)
        for (int r = 1; r < R; ++r) {
          double re, im;
          root((int64_t)r * k, (int64_t)R * Ns, &re, &im);
          t[2 * ((r - 1) * Ns + k)] = re;
          t[2 * ((r - 1) * Ns + k) + 1] = im;
        }
    }
  for (int64_t r = 0; r <= kRootRes / 8; ++r)
    if (used[r]) {
      const long double dc = (long double)(double)octant().c[r] - octant().c[r];
      const long double ds = (long double)(double)octant().s[r] - octant().s[r];
      const long double e = sqrtl(dc * dc + ds * ds);
      if (e > worst) worst = e;
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
    // sqrt(3)/2 of the radix-3 step (the inverse multiplies by its double,
    // sqrt(3), whose relative error is the same)
    const long double e3 = fabsl((long double)0.86602540378443864676 - sqrtl(3.0L) / 2);
    if (e3 > worst) worst = e3;
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
      // w^k and w^(-k) step by one multiplication per k, their r-th powers
      // by one per r (exact modular arithmetic: the same values as powering)
      uint64_t wk = 1, wik = 1;
      for (int k = 0; k < Ns; ++k) {
        uint64_t pf = wk, pg = wik;
        for (int r = 1; r < R; ++r) {
          f[k * (R - 1) + (r - 1)] = pf;
          g[k * (R - 1) + (r - 1)] = pg;
          pf = gold_mul(pf, wk);
          pg = gold_mul(pg, wik);
        }
        wk = gold_mul(wk, w);
        wik = gold_mul(wik, wi);
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
