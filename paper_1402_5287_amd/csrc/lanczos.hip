// Lanczos tridiagonalisation over planned matvecs (Section 1: the Lanczos
// iteration multiplies one symmetric matrix by a sequence of vectors and
// reduces it to a tridiagonal matrix whose eigenvalues QR iterations find).
//
// Fixed point with P fractional bits throughout; every scalar and entry is
// one rounding (to nearest, ties to even, at 2^-P) of an exact expression:
//   w       = A q_j                                    (planned matvec)
//   alpha_j = rne(sum_i q_j,i w_i)
//   r_i     = rne(w_i - alpha_j q_j,i - beta_j q_j-1,i)
//   nu      = rne(sum_i r_i^2); stop when nu < 2^-120
//   rho     = 1/sqrt(nu) by a fixed Newton iteration on mu = nu 4^-s in
//             [1/4, 1):  y <- rne((3 y 2^p - y rne(mu_p rne(y y))) / 2) at a
//             working precision p that doubles (64 bits first, 9 steps from
//             y = 3/2; then min(P, 2p - 8), one step per level, two at P;
//             mu_p = mu rounded to p bits), then rho = y 2^-s
//   beta_j+1 = rne(nu rho),   q_j+1,i = rne(r_i rho) clamped to [-1, 1]
//
// The exact expressions are big-integer sums of products.  A work-group
// holds each operand's magnitude as 32-bit limbs in LDS and sums the limb
// products column by column (the low and high halves of every 64-bit limb
// product in their own columns, signed int64 column sums); the shared
// carry / round / pack step (limb width 32) then turns the column sums into
// the rounded result.  Dot products sum the columns of many entries per
// work-group, then add them into one shared column array with integer
// atomics.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <new>
#include <vector>

#include "common.h"
#include "hmv.h"
#include "kernels.h"
#include "plan.h"

namespace hmv {
namespace {

constexpr int kLzThreads = 256;
constexpr int kLzLimbs = 2 * kMaxWords;              // 32-bit limbs of one number
// Column sums: the NC columns are cut into nbk = ceil(NC / kLzBlk) blocks of
// kLzBlk; thread t owns block t and block t + ceil(nbk / 2).  A product's
// column k has min(k + 1, NC - 1 - k) terms, rising then falling, so every
// thread pairs a block of the rising half with the block of the falling half
// whose length complements it, and all threads do about the same number of
// limb products.
constexpr int kLzBlk = 6;
constexpr int kLzCols = 2 * kLzBlk;                   // columns per thread
constexpr int kLzMaxNC = kLzCols * kLzThreads;
static_assert(kLzMaxNC >= 4 * kMaxWords + 2, "column blocks cover the widest sum");
constexpr int kStopBytes = 256;                       // stop flag and step count

struct LzShared {
  uint64_t wbuf[kMaxWords];                           // words of the number being loaded
  uint32_t mag[5][kLzLimbs];                          // magnitudes (32-bit limbs)
  int64_t coef[kLzMaxNC + 2];                         // column sums
  int64_t cs[kLzThreads + 8];                         // carry scratch (carry_lds_bytes)
  uint64_t out[kMaxWords];                            // a rounded result
  uint32_t red[32];
  int first_nz;
};

// LDS of the update kernel: two operands at a time, the column sums, the
// carry scratch, and the rounded result in the words buffer's place (the
// last load ends before the carry writes it): about 42 KB, three work-groups
// per CU.
struct LzCombShared {
  union {
    uint64_t wbuf[kMaxWords];
    uint64_t out[kMaxWords];
  };
  uint32_t mag[2][kLzLimbs];
  int64_t coef[kLzMaxNC + 2];
  int64_t cs[kLzThreads + 8];
  uint32_t red[32];
  int first_nz;
};

// LDS of the dot-product kernel: its two operands and the column sums only
// (about 39 KB, against about 63 KB of LzShared), so that four work-groups
// fit on a CU.
struct LzDotShared {
  uint64_t wbuf[kMaxWords];
  uint32_t mag[2][kLzLimbs];
  int64_t coef[kLzMaxNC + 2];
  int first_nz;
};

// Loads W two's complement words and stores the magnitude's 2W 32-bit limbs
// in mag; returns the sign (+1 / -1; +1 for zero).  Every thread calls it.
template <class SH>
__device__ int lz_load(const uint64_t* src, int W, SH& sh, uint32_t* mag) {
  const int T = blockDim.x, t = threadIdx.x;
  if (t == 0) sh.first_nz = W;
  for (int q = t; q < W; q += T) sh.wbuf[q] = src[q];
  __syncthreads();
  const bool neg = (sh.wbuf[W - 1] >> 63) != 0;
  if (neg) {
    for (int q = t; q < W; q += T)
      if (sh.wbuf[q]) atomicMin(&sh.first_nz, q);
  }
  __syncthreads();
  const int f = sh.first_nz;
  for (int q = t; q < W; q += T) {
    uint64_t v = sh.wbuf[q];
    if (neg) v = q < f ? 0ull : (q == f ? 0ull - v : ~v);
    mag[2 * q] = (uint32_t)v;
    mag[2 * q + 1] = (uint32_t)(v >> 32);
  }
  __syncthreads();
  return neg ? -1 : 1;
}

// First column of this thread's block q (0: block t, 1: block t + half), or
// -1 if the thread has no such block.
__device__ __forceinline__ int lz_block_start(int q, int NC, int t) {
  const int nbk = (NC + kLzBlk - 1) / kLzBlk, half = (nbk + 1) / 2;
  const int blk = q == 0 ? t : t + half;
  const bool own = q == 0 ? t < half : blk < nbk;
  return own ? blk * kLzBlk : -1;
}

__device__ __forceinline__ int lz_block_start(int q, int NC) {
  return lz_block_start(q, NC, (int)threadIdx.x);
}

// Adds sgn * a * b (magnitudes of na, nb limbs) to the column sums lo / hi
// of this thread's blocks (columns < NC): column k's sum of the limb
// products a_i b_(k-i) is kept as lo_k + hi_k 2^32 (hi belongs to column
// k + 1).  For a block k0 .. k0 + kLzBlk - 1 the b limbs a step needs,
// b[k0 + c - i], shift by one place from one i to the next, so a window of
// kLzBlk registers holds them (one new limb per step, steps unrolled in
// groups of kLzBlk so that every slot is a fixed register) and a step costs
// two LDS reads for kLzBlk independent limb products.  Out-of-range limbs
// read as zero.
// (t: the thread's index among the threads that share the product; every
// block of the NC columns belongs to one of them when they number at least
// half the blocks.)
__device__ __forceinline__ void lz_product(const uint32_t* a, int na, const uint32_t* b, int nb,
                                           int sgn, int NC, int64_t* lo, int64_t* hi,
                                           int t = -1) {
  constexpr int B = kLzBlk;
  if (t < 0) t = (int)threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int k0 = lz_block_start(q, NC, t);
    if (k0 < 0) continue;
    const int ilo = max(0, k0 - nb + 1), ihi = min(na - 1, k0 + B - 1);
    if (ilo > ihi) continue;
    const int i0 = ilo - ilo % B;
    // al / ah: sums of the products of a's low / high 16 bits (below
    // kLzLimbs 2^48 < 2^59), one 64-bit multiply-add each
    uint64_t al[B], ah[B];
    uint32_t w[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      al[c] = ah[c] = 0;
      const int j = k0 + c - i0;                 // slot c holds b[k0 + c - i] for i = i0
      w[c] = (c > 0 && j >= 0 && j < nb) ? b[j] : 0u;
    }
    for (int ib = i0; ib <= ihi; ib += B) {
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int i = ib + u;
        const int j = k0 - i;                    // the new limb, for column k0: slot (-i) mod B
        w[(B - u) % B] = (j >= 0 && j < nb) ? b[j] : 0u;
        const uint32_t ai = i <= ihi ? a[i] : 0u;
        const uint32_t alo = ai & 0xffffu, ahi = ai >> 16;
#pragma unroll
        for (int c = 0; c < B; ++c) {
          const uint32_t wc = w[(c - u + B) % B];
          al[c] += (uint64_t)alo * wc;
          ah[c] += (uint64_t)ahi * wc;
        }
      }
    }
    // column value al + ah 2^16 as lo (column k) + hi 2^32 (column k + 1)
#pragma unroll
    for (int c = 0; c < B; ++c) {
      const uint64_t l = (al[c] & 0xffffffffull) + ((ah[c] & 0xffffull) << 16);
      const uint64_t h = (al[c] >> 32) + (ah[c] >> 16);
      lo[q * B + c] += sgn * (int64_t)l;
      hi[q * B + c] += sgn * (int64_t)h;
    }
  }
}

// coef[k] = lo_k + hi_(k-1) for k < NC (the per-thread sums written out):
// within a block directly, across a block boundary after a barrier (the
// first column of every block receives from exactly one block).
template <class SH>
__device__ void lz_store_cols(const int64_t* lo, const int64_t* hi, int NC, SH& sh) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int k0 = lz_block_start(q, NC);
    if (k0 < 0) continue;
#pragma unroll
    for (int c = 0; c < kLzBlk; ++c)
      if (k0 + c < NC) sh.coef[k0 + c] = lo[q * kLzBlk + c] + (c > 0 ? hi[q * kLzBlk + c - 1] : 0);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int k0 = lz_block_start(q, NC);
    if (k0 >= 0 && k0 + kLzBlk < NC) sh.coef[k0 + kLzBlk] += hi[q * kLzBlk + kLzBlk - 1];
  }
  __syncthreads();
}

// coef += sgn * |m| 2^shift (m: n limbs), split at the 32-bit column
// boundaries (two passes, so that no two threads add to one column at once).
template <class SH>
__device__ void lz_add_shifted(const uint32_t* m, int n, int sgn, int shift, int NC, SH& sh) {
  const int T = blockDim.x, t = threadIdx.x;
  const int q = shift >> 5, r = shift & 31;
  for (int pass = 0; pass < 2; ++pass) {
    for (int l = t; l < n; l += T) {
      const uint64_t v = (uint64_t)m[l] << r;
      const int k = q + l + pass;
      const int64_t part = pass == 0 ? (int64_t)(v & 0xffffffffull) : (int64_t)(v >> 32);
      if (k < NC) sh.coef[k] += sgn * part;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void lz_zero(int64_t* lo, int64_t* hi) {
#pragma unroll
  for (int c = 0; c < kLzCols; ++c) lo[c] = hi[c] = 0;
}

// ------------------------------------------------------------------ kernels
// One work-group per entry i:
//   out_i = rne(ew w_i 2^P + sum_t sg_t a_t u_t,i), clamped to [-1, 1] if asked
// (a_t scalars, u_t vectors; terms with a null pointer are left out).
struct LzCombine {
  const uint64_t* w;
  int ew;
  const uint64_t* a[2];
  const uint64_t* u[2];
  int sg[2];
  uint64_t* out;
  int clamp;
};

template <class SH>
__device__ void lz_clamp_store(SH& sh, int P, int W, uint64_t* dst) {
  // floor(v / 2^P) from bits [P, P + 64) (and all higher words equal to its
  // sign extension); v > 2^P or v < -2^P become +-2^P
  const int T = blockDim.x, t = threadIdx.x;
  const int pq = P >> 6, pr = P & 63;
  const uint64_t lo = sh.out[pq] >> pr;
  const uint64_t hi = (pr && pq + 1 < W) ? sh.out[pq + 1] << (64 - pr) : 0ull;
  const int64_t q = (int64_t)(lo | hi);
  const uint64_t ext = q < 0 ? ~0ull : 0ull;
  bool wide = false;
  for (int m = pq + 2; m < W; ++m)
    if (sh.out[m] != ext) wide = true;
  if (pr == 0 && pq + 1 < W && sh.out[pq + 1] != ext) wide = true;
  if (pr && pq + 1 < W && ((int64_t)sh.out[pq + 1] >> pr) != (int64_t)ext) wide = true;
  bool rem = false;
  for (int m = 0; m <= pq && m < W; ++m) {
    const uint64_t v = m < pq ? sh.out[m] : (pr ? sh.out[m] & ((1ull << pr) - 1) : 0ull);
    if (v) rem = true;
  }
  int cl = 0;
  if (wide) cl = q < 0 ? -1 : 1;
  else if (q >= 2 || (q == 1 && rem)) cl = 1;
  else if (q <= -2) cl = -1;
  for (int m = t; m < W; m += T) {
    uint64_t v = sh.out[m];
    if (cl > 0) v = m == pq ? (1ull << pr) : 0ull;
    if (cl < 0) v = m < pq ? 0ull : (m == pq ? (~0ull << pr) : ~0ull);
    dst[m] = v;
  }
}

__global__ void __launch_bounds__(kLzThreads) k_lz_combine(LzCombine cmb, int n, int P, int W,
                                                           const int* stop) {
  __shared__ LzCombShared sh;
  const int i = blockIdx.x;
  if (i >= n || *stop) return;
  const int NL = 2 * W, NC = 2 * NL + 2;
  int64_t lo[kLzCols], hi[kLzCols];
  lz_zero(lo, hi);
  for (int tm = 0; tm < 2; ++tm) {
    if (!cmb.a[tm]) continue;
    const int sa = lz_load(cmb.a[tm], W, sh, sh.mag[0]);
    const int su = lz_load(cmb.u[tm] + (int64_t)i * W, W, sh, sh.mag[1]);
    lz_product(sh.mag[0], NL, sh.mag[1], NL, cmb.sg[tm] * sa * su, NC, lo, hi);
    __syncthreads();
  }
  lz_store_cols(lo, hi, NC, sh);
  if (cmb.ew) {
    const int sw = lz_load(cmb.w + (int64_t)i * W, W, sh, sh.mag[0]);
    lz_add_shifted(sh.mag[0], NL, sw, P, NC, sh);
  }
  uint64_t* dst = cmb.out + (int64_t)i * W;
  carry_round_pack_fit(sh.coef, NC, 32, P, W, sh.cs, cmb.clamp ? sh.out : dst, sh.red);
  if (cmb.clamp) lz_clamp_store(sh, P, W, dst);
}

// The same update for few entries, in two kernels.  Part: n S work-groups;
// work-group g takes slice g mod S of the limbs of the scalar a[t] (all
// terms t) times entry i = g / S of u[t], and adds its column sums into the
// entry's own column array ccols + i NC (integer atomics, exact in any
// order).  Final: one work-group per entry takes the columns (and zeroes them
// for the next update), adds w, and carries, rounds and stores as above.
__global__ void __launch_bounds__(kLzThreads) k_lz_combine_part(LzCombine cmb, int n, int W,
                                                                int slices, int64_t* ccols,
                                                                const int* stop) {
  __shared__ LzDotShared sh;
  const int g = blockIdx.x;
  const int i = g / slices, sl = g - i * slices;
  if (i >= n || *stop) return;
  const int NL = 2 * W, NC = 2 * NL + 2;
  const int pl = (NL + slices - 1) / slices, a0 = min(NL, sl * pl);
  const int na = min(NL, a0 + pl) - a0;
  if (na <= 0) return;
  const int NCs = na + NL + 1;                       // this slice's columns, from column a0
  int64_t lo[kLzCols], hi[kLzCols];
  lz_zero(lo, hi);
  for (int tm = 0; tm < 2; ++tm) {
    if (!cmb.a[tm]) continue;
    const int sa = lz_load(cmb.a[tm], W, sh, sh.mag[0]);
    const int su = lz_load(cmb.u[tm] + (int64_t)i * W, W, sh, sh.mag[1]);
    lz_product(sh.mag[0] + a0, na, sh.mag[1], NL, cmb.sg[tm] * sa * su, NCs, lo, hi);
    __syncthreads();
  }
  lz_store_cols(lo, hi, NCs, sh);
  int64_t* dst = ccols + (int64_t)i * NC + a0;
  for (int k = threadIdx.x; k < NCs; k += blockDim.x)
    if (sh.coef[k])
      atomicAdd(reinterpret_cast<unsigned long long*>(dst + k), (unsigned long long)sh.coef[k]);
}

__global__ void __launch_bounds__(kLzThreads) k_lz_combine_final(LzCombine cmb, int n, int P,
                                                                 int W, int64_t* ccols,
                                                                 const int* stop) {
  __shared__ LzCombShared sh;
  const int i = blockIdx.x;
  if (i >= n || *stop) return;
  const int NL = 2 * W, NC = 2 * NL + 2;
  int64_t* src = ccols + (int64_t)i * NC;
  for (int k = threadIdx.x; k < NC; k += blockDim.x) {
    sh.coef[k] = src[k];
    src[k] = 0;
  }
  __syncthreads();
  if (cmb.ew) {
    const int sw = lz_load(cmb.w + (int64_t)i * W, W, sh, sh.mag[0]);
    lz_add_shifted(sh.mag[0], NL, sw, P, NC, sh);
  }
  uint64_t* dst = cmb.out + (int64_t)i * W;
  carry_round_pack_fit(sh.coef, NC, 32, P, W, sh.cs, cmb.clamp ? sh.out : dst, sh.red);
  if (cmb.clamp) lz_clamp_store(sh, P, W, dst);
}

// Dot product, first stage: the column sums of sgn |u_i| |v_i| added into the
// shared columns cols[k] (64-bit integer atomics: exact, so the order of the
// work-groups does not matter).  With slices = 1, work-group g takes the
// entries [g per, (g + 1) per); with slices = S > 1 (few entries), work-group
// g takes slice g mod S of the limbs of u_i, i = g / S, times all of v_i, so
// that n S work-groups share the products.
__global__ void __launch_bounds__(kLzThreads) k_lz_dot_part(const uint64_t* u, const uint64_t* v,
                                                            int n, int W, int per, int slices,
                                                            int64_t* cols, const int* stop) {
  __shared__ LzDotShared sh;
  const int g = blockIdx.x;
  if (*stop) return;
  const int NL = 2 * W, NC = 2 * NL + 2;
  int64_t lo[kLzCols], hi[kLzCols];
  lz_zero(lo, hi);
  if (slices > 1) {                                  // uniform
    const int i = g / slices, sl = g - i * slices;
    if (i >= n) return;                              // whole work-groups
    const int su = lz_load(u + (int64_t)i * W, W, sh, sh.mag[0]);
    const int sv = lz_load(v + (int64_t)i * W, W, sh, sh.mag[1]);
    const int pl = (NL + slices - 1) / slices, a0 = min(NL, sl * pl);
    const int na = min(NL, a0 + pl) - a0;
    if (na <= 0) return;
    const int NCs = na + NL + 1;                     // this slice's columns, from column a0
    lz_product(sh.mag[0] + a0, na, sh.mag[1], NL, su * sv, NCs, lo, hi);
    __syncthreads();
    lz_store_cols(lo, hi, NCs, sh);
    for (int k = threadIdx.x; k < NCs; k += blockDim.x)
      if (sh.coef[k])
        atomicAdd(reinterpret_cast<unsigned long long*>(cols + a0 + k),
                  (unsigned long long)sh.coef[k]);
    return;
  }
  const int i0 = g * per, i1 = min(n, i0 + per);
  for (int i = i0; i < i1; ++i) {
    const int su = lz_load(u + (int64_t)i * W, W, sh, sh.mag[0]);
    const int sv = lz_load(v + (int64_t)i * W, W, sh, sh.mag[1]);
    lz_product(sh.mag[0], NL, sh.mag[1], NL, su * sv, NC, lo, hi);
    __syncthreads();
  }
  lz_store_cols(lo, hi, NC, sh);
  for (int k = threadIdx.x; k < NC; k += blockDim.x)
    if (sh.coef[k])
      atomicAdd(reinterpret_cast<unsigned long long*>(cols + k), (unsigned long long)sh.coef[k]);
}

// Second stage (one work-group): the shared column sums, rounded:
// out = rne(sum_i u_i v_i); the columns are zeroed again for the next dot
// product.  count (if not null) counts the steps.
__global__ void __launch_bounds__(kLzThreads) k_lz_dot_final(int64_t* cols, int P, int W,
                                                             uint64_t* out, const int* stop,
                                                             int* count) {
  __shared__ LzShared sh;
  if (*stop) return;
  const int NC = 4 * W + 2;
  for (int k = threadIdx.x; k < NC; k += blockDim.x) {
    sh.coef[k] = cols[k];
    cols[k] = 0;
  }
  __syncthreads();
  carry_round_pack_fit(sh.coef, NC, 32, P, W, sh.cs, out, sh.red);
  if (count && threadIdx.x == 0) *count += 1;
}

// The scalars of a step run on G work-groups of a cooperative launch.  Each
// work-group keeps every operand in its own LDS and repeats the small
// operations itself (identical results, no communication).  A product of at
// least kLzDistLimbs limbs is split: work-group g multiplies its slice of a
// by b and adds its columns into a shared column array with integer atomics;
// after one grid barrier every work-group reads the full sums back and
// carries them itself.  Three arrays rotate: during product j the
// work-groups zero array (j + 1) mod 3, which product j - 2 used and which
// every work-group finished reading before the barrier of product j - 1.
constexpr int kLzDistLimbs = 128;
struct LzDist {
  int64_t* cols;     // 3 x kLzMaxNC column sums
  int k;             // distributed products so far (the rotation)
};

// sh.coef[0 .. NC) = the column sums of sgn * a * b (nl limbs each).
__device__ void lz_product_cols(LzShared& sh, const uint32_t* a, const uint32_t* b, int nl,
                                int sgn, int NC, LzDist& dist) {
  const int G = gridDim.x, g = blockIdx.x, T = blockDim.x, t = threadIdx.x;
  if (G == 1 || nl < kLzDistLimbs) {
    // few columns leave most threads without a block: then S groups of
    // T / S threads take one slice of a's limbs each and add their columns
    // into sh.coef with 64-bit LDS atomics
    const int half = ((NC + kLzBlk - 1) / kLzBlk + 1) / 2;
    int S = 1;
    while (S < 16 && 2 * S <= nl && (T / (2 * S)) >= half) S *= 2;
    if (S == 1) {
      int64_t lo[kLzCols], hi[kLzCols];
      lz_zero(lo, hi);
      lz_product(a, nl, b, nl, sgn, NC, lo, hi);
      __syncthreads();
      lz_store_cols(lo, hi, NC, sh);
      return;
    }
    for (int k = t; k < NC; k += T) sh.coef[k] = 0;
    __syncthreads();
    const int Tg = T / S, grp = t / Tg, tl = t - grp * Tg;
    const int pl = (nl + S - 1) / S, a0 = min(nl, grp * pl), na = min(nl, a0 + pl) - a0;
    if (na > 0) {
      const int NCs = na + nl + 1;               // this slice's columns, from column a0
      int64_t lo[kLzCols], hi[kLzCols];
      lz_zero(lo, hi);
      lz_product(a + a0, na, b, nl, sgn, NCs, lo, hi, tl);
      unsigned long long* cf = reinterpret_cast<unsigned long long*>(sh.coef + a0);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k0 = lz_block_start(q, NCs, tl);
        if (k0 < 0) continue;
#pragma unroll
        for (int c = 0; c < kLzBlk; ++c) {
          if (k0 + c < NCs) atomicAdd(cf + k0 + c, (unsigned long long)lo[q * kLzBlk + c]);
          if (k0 + c + 1 < NCs) atomicAdd(cf + k0 + c + 1, (unsigned long long)hi[q * kLzBlk + c]);
        }
      }
    }
    __syncthreads();
    return;
  }
  int64_t* cur = dist.cols + (int64_t)(dist.k % 3) * kLzMaxNC;
  int64_t* nxt = dist.cols + (int64_t)((dist.k + 1) % 3) * kLzMaxNC;
  ++dist.k;
  const int chunk = (kLzMaxNC + G - 1) / G;
  for (int e = g * chunk + t; e < min(kLzMaxNC, (g + 1) * chunk); e += T) nxt[e] = 0;
  const int per = (nl + G - 1) / G, a0 = min(nl, g * per), na = min(nl, a0 + per) - a0;
  if (na > 0) {
    const int NCs = na + nl + 1;                 // this slice's columns, from column a0
    int64_t lo[kLzCols], hi[kLzCols];
    lz_zero(lo, hi);
    lz_product(a + a0, na, b, nl, sgn, NCs, lo, hi);
    __syncthreads();
    lz_store_cols(lo, hi, NCs, sh);
    for (int k = t; k < NCs; k += T)
      if (sh.coef[k])
        atomicAdd(reinterpret_cast<unsigned long long*>(cur + a0 + k),
                  (unsigned long long)sh.coef[k]);
  }
  // release the zeroing stores and the atomics, meet, acquire the sums (the
  // work-groups sit on different XCDs, whose L2s the fences keep coherent)
  __threadfence();
  cooperative_groups::this_grid().sync();
  __threadfence();
  for (int k = t; k < NC; k += T) sh.coef[k] = cur[k];
  __syncthreads();
}

// A product of two numbers already in LDS (magnitudes mag[nx], mag[ny], nl
// limbs each; nx < 0 for none) plus an optional shifted term addsgn
// mag[addm] 2^addshift, rounded at `round` bits (0: exact); the result goes
// to sh.out (W words).
__device__ void lz_scalar_op(LzShared& sh, int W, int nl, int nx, int ny, int sgn, int addm,
                             int addsgn, int addshift, int round, LzDist& dist) {
  const int NC = 2 * nl + 2;
  if (nx >= 0) {
    lz_product_cols(sh, sh.mag[nx], sh.mag[ny], nl, sgn, NC, dist);
  } else {
    for (int k = threadIdx.x; k < NC; k += blockDim.x) sh.coef[k] = 0;
    __syncthreads();
  }
  if (addm >= 0) lz_add_shifted(sh.mag[addm], nl, addsgn, addshift, NC, sh);
  carry_round_pack_fit(sh.coef, NC, 32, round, W, sh.cs, sh.out, sh.red);
}

// mag[dst] = rne(A 2^(sl - sr)) as 2W = NL limbs, for A = mag[src] (its
// first na limbs; A >= 0; sl or sr is 0): the value that the carry step
// gives for the column sums of A shifted, rounded at sr bits, but cut
// straight from the limbs (one funnel shift per limb, the round and sticky
// bits, an increment that ripples through the lowest all-ones limbs), with
// no column array.  src may be dst.  Every thread calls it.
__device__ void lz_shift_round(LzShared& sh, int src, int na, int dst, int sl, int sr, int NL) {
  constexpr int kPer = (kLzLimbs + kLzThreads - 1) / kLzThreads;
  const int T = blockDim.x, t = threadIdx.x;
  const uint32_t* a = sh.mag[src];
  uint32_t* o = sh.mag[dst];
  auto bits32 = [&](int64_t b) -> uint32_t {        // bits [b, b + 32) of A
    if (b <= -32) return 0u;
    if (b < 0) return na > 0 ? a[0] << (-b) : 0u;
    const int64_t q = b >> 5;
    const int r = (int)(b & 31);
    const uint32_t lo = q < na ? a[q] >> r : 0u;
    const uint32_t hi = (r && q + 1 < na) ? a[q + 1] << (32 - r) : 0u;
    return lo | hi;
  };
  const int d = sl - sr;
  uint32_t ov[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = t + T * j;
    ov[j] = k < NL ? bits32(32 * (int64_t)k - d) : 0u;
  }
  int up = 0;
  if (d < 0) {                                       // uniform
    // round bit r - 1, sticky bits below it, last kept bit r
    const int r = -d, rq = (r - 1) >> 5, rr = (r - 1) & 31;
    int st = 0;
    for (int l = t; l <= rq && l < na; l += T) {
      const uint32_t v = l < rq ? a[l] : (a[l] & ((1u << rr) - 1u));
      if (v) st = 1;
    }
    const int sticky = __syncthreads_or(st);
    const int rbit = rq < na ? (int)((a[rq] >> rr) & 1u) : 0;
    const int lsb = (int)(bits32(r) & 1u);
    up = rbit && (sticky || lsb);
  }
  if (t == 0) sh.first_nz = NL;
  __syncthreads();                                   // A read in full (src may be dst)
  int fno = NL;                                      // first limb that is not all ones
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = t + T * j;
    if (k < NL) {
      o[k] = ov[j];
      if (ov[j] != 0xffffffffu && k < fno) fno = k;
    }
  }
  if (up) {                                          // uniform
    if (fno < NL) atomicMin(&sh.first_nz, fno);
    __syncthreads();
    const int f = sh.first_nz;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int k = t + T * j;
      if (k < NL && k <= f) o[k] = k < f ? 0u : ov[j] + 1u;
    }
  }
  __syncthreads();
}

// The first Newton levels on 64-bit words, by one thread, with every size
// and shift fixed at compile time (the words stay in registers): NW words
// hold every operand of the level at PB bits (below 2^(PB+6) <= 2^(64 NW)),
// products take 2 NW words.  Same roundings as the general steps, every
// value non-negative: mu_PB >= 2^(PB-2) and, after the first step,
// mu y^2 <= 2^(2 PB) (1 + tiny) < 3 2^(2 PB).
template <int NW>
__device__ __forceinline__ void lz_mulw(const uint64_t (&a)[NW], const uint64_t (&b)[NW],
                                        uint64_t (&r)[2 * NW]) {
#pragma unroll
  for (int i = 0; i < 2 * NW; ++i) r[i] = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const unsigned __int128 v = (unsigned __int128)a[i] * b[j] + r[i + j] + c;
      r[i + j] = (uint64_t)v;
      c = (uint64_t)(v >> 64);
    }
    r[i + NW] = c;
  }
}

// q = rne(v / 2^K), 0 < K <= 64 NW, the quotient below 2^(64 NW)
template <int NW, int K>
__device__ __forceinline__ void lz_rnew(const uint64_t (&v)[2 * NW], uint64_t (&q)[NW]) {
  constexpr int ws = K >> 6, bs = K & 63;
  constexpr int rw = (K - 1) >> 6, rb = (K - 1) & 63;
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    const uint64_t lo = v[m + ws];
    const uint64_t hi = m + ws + 1 < 2 * NW ? v[m + ws + 1] : 0ull;
    q[m] = bs ? (lo >> bs) | (hi << ((64 - bs) & 63)) : lo;
  }
  const uint64_t rbit = (v[rw] >> rb) & 1u;
  bool sticky = rb ? (v[rw] & ((1ull << rb) - 1)) != 0 : false;
#pragma unroll
  for (int m = 0; m < rw; ++m) sticky = sticky || v[m] != 0;
  uint64_t c = (rbit && (sticky || (q[0] & 1u))) ? 1u : 0u;
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    q[m] += c;
    c = (c && q[m] == 0) ? 1u : 0u;
  }
}

// steps Newton steps at PB bits: t1 = rne(y y / 2^PB), t2 = rne(mu t1 /
// 2^PB), y = rne((3 y 2^PB - y t2) / 2^(PB+1))
template <int NW, int PB>
__device__ void lz_newton_words(uint64_t (&y)[NW], const uint64_t (&mu)[NW], int steps) {
  static_assert(PB + 6 <= 64 * NW && PB + 1 <= 64 * NW, "the level fits its words");
  for (int it = 0; it < steps; ++it) {
    uint64_t pr[2 * NW], t1[NW], t2[NW];
    lz_mulw<NW>(y, y, pr);
    lz_rnew<NW, PB>(pr, t1);
    lz_mulw<NW>(mu, t1, pr);
    lz_rnew<NW, PB>(pr, t2);
    lz_mulw<NW>(y, t2, pr);                      // y t2
    uint64_t y3[NW];                             // 3 y, below 2^(PB+6)
    {
      uint64_t c = 0;
#pragma unroll
      for (int m = 0; m < NW; ++m) {
        const unsigned __int128 v = (unsigned __int128)y[m] * 3u + c;
        y3[m] = (uint64_t)v;
        c = (uint64_t)(v >> 64);
      }
    }
    // S = 3 y 2^PB - y t2 (>= 0)
    uint64_t S[2 * NW];
    constexpr int ws = PB >> 6, bs = PB & 63;
    uint64_t borrow = 0;
#pragma unroll
    for (int m = 0; m < 2 * NW; ++m) {
      const int src = m - ws;
      const uint64_t lo = src >= 0 && src < NW ? y3[src] : 0ull;
      const uint64_t lo1 = src - 1 >= 0 && src - 1 < NW ? y3[src - 1] : 0ull;
      const uint64_t a = bs ? (lo << bs) | (lo1 >> ((64 - bs) & 63)) : lo;
      const uint64_t d = a - pr[m];
      const uint64_t b1 = a < pr[m];
      S[m] = d - borrow;
      borrow = b1 | (d < borrow);
    }
    lz_rnew<NW, PB + 1>(S, y);
  }
}

// One thread: the Newton steps of level PB on y = mag[2], mu_PB = mag[4]
// (the first 2 NW limbs of each; the limbs above are zero and stay so).
template <int NW, int PB>
__device__ void lz_newton_level(LzShared& sh, int steps) {
  uint64_t y[NW], mu[NW];
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    y[m] = ((uint64_t)sh.mag[2][2 * m + 1] << 32) | sh.mag[2][2 * m];
    mu[m] = ((uint64_t)sh.mag[4][2 * m + 1] << 32) | sh.mag[4][2 * m];
  }
  lz_newton_words<NW, PB>(y, mu, steps);
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    sh.mag[2][2 * m] = (uint32_t)y[m];
    sh.mag[2][2 * m + 1] = (uint32_t)(y[m] >> 32);
  }
}

// Limbs that hold the values of a Newton step at working precision p (every
// operand below 2^(p+4) in magnitude, with one limb to spare).
__device__ __forceinline__ int lz_newton_limbs(int p) { return (p + 4 + 31) / 32 + 1; }

// The Newton levels (working precision, steps): p = min(P, 64) for 9 steps
// from y = 3/2, then p = min(P, 2p - 8) for one step each, two at p = P.
constexpr int kNewtonStartBits = 64, kNewtonStartSteps = 9, kNewtonFinalSteps = 2;

__global__ void __launch_bounds__(kLzThreads) k_lz_scalars(const uint64_t* nu, int P, int W,
                                                           uint64_t* rho, uint64_t* beta,
                                                           int* stop, int64_t* dcols,
                                                           int* dctr) {
  __shared__ LzShared sh;
  __shared__ int top;
  if (*stop) return;
  const int T = blockDim.x, t = threadIdx.x;
  const bool lead = blockIdx.x == 0;             // the work-group that writes results
  LzDist dist{dcols, *dctr};
  const int k_start = dist.k;
  const int NLF = 2 * W;                         // full-precision limbs
  // mag[0] = N (nu's integer; nu >= 0)
  lz_load(nu, W, sh, sh.mag[0]);
  if (t == 0) top = -1;
  __syncthreads();
  for (int l = t; l < NLF; l += T)
    if (sh.mag[0][l]) atomicMax(&top, l);
  __syncthreads();
  const int64_t bits = top < 0 ? 0 : 32 * (int64_t)top + (32 - __clz((int)sh.mag[0][top]));
  // stop when nu < 2^-120, i.e. N < 2^(P - 120)
  if (top < 0 || bits - 1 < (int64_t)P - 120) {
    if (lead) {
      for (int m = t; m < W; m += T) beta[m] = 0ull;
      __syncthreads();
      if (t == 0) *stop = 1;
    }
    return;
  }
  const int b = (int)(bits - P);                 // 2^(b-1) <= nu < 2^b
  const int s = b >= 0 ? (b + 1) / 2 : -((-b) / 2);   // ceil(b / 2)
  // mag[1] = M: mu = nu 4^-s at P bits, rounded when s > 0
  lz_shift_round(sh, 0, NLF, 1, s > 0 ? 0 : -2 * s, s > 0 ? 2 * s : 0, NLF);
  int p = P < kNewtonStartBits ? P : kNewtonStartBits, prev = 0;
  for (;;) {
    const int nl = lz_newton_limbs(p);
    const int steps = prev == 0 ? kNewtonStartSteps : (p == P ? kNewtonFinalSteps : 1);
    // mag[2] = y: 3/2 at the first level, else y shifted up by p - prev bits
    if (prev == 0) {
      for (int l = t; l < NLF; l += T) sh.mag[2][l] = 0u;
      __syncthreads();
      if (t == 0) {                              // 3 * 2^(p-1): bits p - 1 and p
        sh.mag[2][(p - 1) >> 5] |= 1u << ((p - 1) & 31);
        sh.mag[2][p >> 5] |= 1u << (p & 31);
      }
      __syncthreads();
    } else {
      lz_shift_round(sh, 2, nl, 2, p - prev, 0, NLF);
    }
    // mag[4] = mu_p: M rounded to p bits
    lz_shift_round(sh, 1, NLF, 4, 0, p < P ? P - p : 0, NLF);
    // the levels up to 456 bits (every one of them below P) in one thread
    const bool small = (prev == 0 && p == 64) || (P > 456 && (p == 120 || p == 232 || p == 456));
    if (small) {
      if (t == 0) {
        if (p == 64) lz_newton_level<2, 64>(sh, steps);
        else if (p == 120) lz_newton_level<2, 120>(sh, steps);
        else if (p == 232) lz_newton_level<4, 232>(sh, steps);
        else lz_newton_level<8, 456>(sh, steps);
      }
      __syncthreads();
    }
    for (int it = 0; it < (small ? 0 : steps); ++it) {
      // t1 = rne(y y)          -> mag[3]
      lz_scalar_op(sh, W, nl, 2, 2, 1, -1, 1, 0, p, dist);
      lz_load(sh.out, W, sh, sh.mag[3]);
      // t2 = rne(mu_p t1)      -> mag[3]
      lz_scalar_op(sh, W, nl, 4, 3, 1, -1, 1, 0, p, dist);
      const int s2 = lz_load(sh.out, W, sh, sh.mag[3]);
      // y = rne((3 y 2^p - y t2) / 2): 3 y 2^p as y 2^(p+1) + y 2^p
      {
        const int NC = 2 * nl + 2;
        lz_product_cols(sh, sh.mag[2], sh.mag[3], nl, -s2, NC, dist);
        lz_add_shifted(sh.mag[2], nl, 1, p + 1, NC, sh);
        lz_add_shifted(sh.mag[2], nl, 1, p, NC, sh);
        carry_round_pack_fit(sh.coef, NC, 32, p + 1, W, sh.cs, sh.out, sh.red);
      }
      lz_load(sh.out, W, sh, sh.mag[2]);
    }
    if (p == P) break;
    prev = p;
    p = 2 * p - 8 < P ? 2 * p - 8 : P;
  }
  // rho = y 2^-s (mag[2] -> mag[4] and rho)
  if (s > 0) lz_scalar_op(sh, W, NLF, -1, -1, 1, 2, 1, 0, s, dist);
  else lz_scalar_op(sh, W, NLF, -1, -1, 1, 2, 1, -s, 0, dist);
  if (lead)
    for (int m = t; m < W; m += T) rho[m] = sh.out[m];
  lz_load(sh.out, W, sh, sh.mag[4]);
  // beta = rne(N rho)
  lz_scalar_op(sh, W, NLF, 0, 4, 1, -1, 1, 0, P, dist);
  if (lead) {
    for (int m = t; m < W; m += T) beta[m] = sh.out[m];
    // every work-group read the counter before the first grid barrier
    if (t == 0 && dist.k != k_start) *dctr = dist.k;
  }
}

__global__ void k_lz_init(int* stop, uint64_t* zero, int W, int64_t* cols, int NC,
                          int64_t* dcols, int64_t* ccols, int64_t nccols) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    stop[0] = 0;
    stop[1] = 0;
    stop[2] = 0;                                 // the rotation of the distributed products
  }
  for (int m = threadIdx.x; m < W; m += blockDim.x) zero[m] = 0ull;
  for (int k = threadIdx.x; k < NC; k += blockDim.x) cols[k] = 0;
  for (int k = threadIdx.x; k < 3 * kLzMaxNC; k += blockDim.x) dcols[k] = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nccols;
       k += (int64_t)gridDim.x * blockDim.x)
    ccols[k] = 0;
}

__global__ void k_lz_count(const int* stop, int32_t* steps_done) {
  if (threadIdx.x == 0) *steps_done = stop[1];
}

__global__ void k_lz_copy(const uint64_t* src, uint64_t* dst, int64_t words, const int* stop) {
  if (*stop) return;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < words;
       m += (int64_t)gridDim.x * blockDim.x)
    dst[m] = src[m];
}

// Work-groups of the scalar kernel: up to 32, all resident at once (16 to 32
// take the same time per step; 64 wait longer at each grid barrier of a
// split product, 8 multiply too much each).
hipError_t lz_scalars_grid(int* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_lz_scalars,
                                                     kLzThreads, 0);
  if (e != hipSuccess) return e;
  *grid = std::max(1, std::min(32, per_cu * cus));
  return hipSuccess;
}

struct LzLayout {
  int W, G, per, slices, NC;
  int64_t off_stop, off_zero, off_nu, off_rho, off_vec[3], off_cols, off_dcols, off_ccols, nccols,
      off_mv, bytes;
};

LzLayout lz_layout(const hmv_plan* p) {
  LzLayout L{};
  const int64_t n = p->n;
  L.W = (int)words_of(p->P);
  L.NC = 4 * L.W + 2;
  // dot products: one work-group per entry up to 1024 entries, and for fewer
  // than 512 entries each product split over up to 16 work-groups
  L.slices = n >= 512 ? 1 : (int)std::min<int64_t>(16, 1024 / n);
  L.G = L.slices > 1 ? (int)(n * L.slices) : (int)(n < 1024 ? n : 1024);
  L.per = (int)((n + L.G - 1) / L.G);
  int64_t o = kStatusBytes;
  L.off_stop = o;
  o += kStopBytes;
  L.off_zero = o;
  o += align_up(8 * (int64_t)L.W);
  L.off_nu = o;
  o += align_up(8 * (int64_t)L.W);
  L.off_rho = o;
  o += align_up(8 * (int64_t)L.W);
  for (int k = 0; k < 3; ++k) {
    L.off_vec[k] = o;
    o += align_up(8 * n * L.W);
  }
  L.off_cols = o;
  o += align_up(8 * (int64_t)L.NC);
  L.off_dcols = o;
  o += align_up(8 * 3 * (int64_t)kLzMaxNC);
  // per-entry column arrays of the split updates (fewer than 512 entries)
  L.nccols = L.slices > 1 ? n * (int64_t)L.NC : 0;
  L.off_ccols = o;
  o += align_up(8 * L.nccols);
  L.off_mv = o;
  o += kStatusBytes + p->mv_scratch;
  L.bytes = o;
  return L;
}

// An entry update: one work-group per entry, or for fewer than 512 entries
// the split form (n S partial work-groups, then one per entry).
void lz_launch_combine(const LzCombine& c, int n, int P, int W, const LzLayout& L,
                       int64_t* ccols, const int* stop, hipStream_t s) {
  if (L.slices > 1) {
    hipLaunchKernelGGL(k_lz_combine_part, dim3(n * L.slices), dim3(kLzThreads), 0, s, c, n, W,
                       L.slices, ccols, stop);
    hipLaunchKernelGGL(k_lz_combine_final, dim3(n), dim3(kLzThreads), 0, s, c, n, P, W, ccols,
                       stop);
  } else {
    hipLaunchKernelGGL(k_lz_combine, dim3(n), dim3(kLzThreads), 0, s, c, n, P, W, stop);
  }
}

}  // namespace
}  // namespace hmv

extern "C" {

int64_t hmv_lanczos_workspace_bytes(const hmv_plan* p) {
  if (!p) return HMV_EINVAL;
  return hmv::lz_layout(p).bytes;
}

int hmv_lanczos(const hmv_plan* p, const uint64_t* q1, int32_t steps, uint64_t* alpha,
                uint64_t* beta, int32_t* steps_done, uint64_t* basis, void* ws, int64_t ws_bytes,
                void* stream) {
  using namespace hmv;
  if (!p || !q1 || !alpha || !beta || !steps_done || !ws || steps < 1) return HMV_EINVAL;
  if (p->kind != HMV_HANKEL) return HMV_EINVAL;     // a symmetric matrix
  const LzLayout L = lz_layout(p);
  if (ws_bytes < L.bytes) return HMV_ENOMEM;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  DevStatus* st = reinterpret_cast<DevStatus*>(base);
  int* stop = reinterpret_cast<int*>(base + L.off_stop);
  uint64_t* zero = reinterpret_cast<uint64_t*>(base + L.off_zero);
  uint64_t* nu = reinterpret_cast<uint64_t*>(base + L.off_nu);
  uint64_t* rho = reinterpret_cast<uint64_t*>(base + L.off_rho);
  uint64_t* vec[3];
  for (int k = 0; k < 3; ++k) vec[k] = reinterpret_cast<uint64_t*>(base + L.off_vec[k]);
  int64_t* cols = reinterpret_cast<int64_t*>(base + L.off_cols);
  int64_t* dcols = reinterpret_cast<int64_t*>(base + L.off_dcols);
  int* dctr = stop + 2;
  int sgrid = 0;
  hipError_t ge = lz_scalars_grid(&sgrid);
  if (ge != hipSuccess) return status_from_hip(ge, "lanczos: scalar grid");
  char* mv = base + L.off_mv;
  const int n = (int)p->n, W = L.W, P = p->P;
  const int64_t nw = (int64_t)n * W;
  hipError_t e = launch_clear_status(st, s);
  if (e != hipSuccess) return status_from_hip(e, "lanczos: clear status");
  int64_t* ccols = reinterpret_cast<int64_t*>(base + L.off_ccols);
  hipLaunchKernelGGL(k_lz_init, dim3(L.nccols > 0 ? 64 : 1), dim3(256), 0, s, stop, zero, W, cols,
                     L.NC, dcols, ccols, L.nccols);
  e = hipMemcpyAsync(vec[0], q1, 8 * nw, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return status_from_hip(e, "lanczos: start vector");
  // vec[q] = q_j, vec[qp] = q_(j-1) (zero at first), vec[wv] = w, then r
  int q = 0, qp = 1, wv = 2;
  // q_0 is never read: beta_1 = 0 leaves its term out of the first update
  for (int j = 0; j < steps; ++j) {
    const uint64_t* beta_j = j == 0 ? zero : beta + (int64_t)(j - 1) * W;
    uint64_t* alpha_j = alpha + (int64_t)j * W;
    uint64_t* beta_j1 = beta + (int64_t)j * W;
    if (basis) {
      hipLaunchKernelGGL(k_lz_copy, dim3(256), dim3(256), 0, s, vec[q], basis + (int64_t)j * nw,
                         nw, stop);
    }
    // w = A q_j
    int rc = plan_matvec_parts(p, vec[q], vec[wv], st, mv + kStatusBytes, p->mv_scratch, s,
                               nullptr, false);
    if (rc != HMV_OK) return rc;
    // alpha_j = rne(q . w)
    hipLaunchKernelGGL(k_lz_dot_part, dim3(L.G), dim3(kLzThreads), 0, s, vec[q], vec[wv], n, W,
                       L.per, L.slices, cols, stop);
    hipLaunchKernelGGL(k_lz_dot_final, dim3(1), dim3(kLzThreads), 0, s, cols, P, W, alpha_j,
                       stop, stop + 1);
    // r = rne(w - alpha q_j - beta_j q_j-1), in place of w
    LzCombine c{};
    c.w = vec[wv];
    c.ew = 1;
    c.a[0] = alpha_j;
    c.u[0] = vec[q];
    c.sg[0] = -1;
    c.a[1] = j == 0 ? nullptr : beta_j;
    c.u[1] = vec[qp];
    c.sg[1] = -1;
    c.out = vec[wv];
    c.clamp = 0;
    lz_launch_combine(c, n, P, W, L, ccols, stop, s);
    // nu = rne(r . r); rho, beta_j+1 (or the stop)
    hipLaunchKernelGGL(k_lz_dot_part, dim3(L.G), dim3(kLzThreads), 0, s, vec[wv], vec[wv], n, W,
                       L.per, L.slices, cols, stop);
    hipLaunchKernelGGL(k_lz_dot_final, dim3(1), dim3(kLzThreads), 0, s, cols, P, W, nu, stop,
                       nullptr);
    {
      const uint64_t* a_nu = nu;
      void* args[] = {(void*)&a_nu, (void*)&P, (void*)&W, (void*)&rho, (void*)&beta_j1,
                      (void*)&stop, (void*)&dcols, (void*)&dctr};
      e = hipLaunchCooperativeKernel((const void*)k_lz_scalars, dim3(sgrid), dim3(kLzThreads),
                                     args, 0, s);
      if (e != hipSuccess) return status_from_hip(e, "lanczos: scalars");
    }
    // q_j+1 = clamp(rne(rho r)), in place of q_j-1
    LzCombine d{};
    d.w = nullptr;
    d.ew = 0;
    d.a[0] = rho;
    d.u[0] = vec[wv];
    d.sg[0] = 1;
    d.out = vec[qp];
    d.clamp = 1;
    lz_launch_combine(d, n, P, W, L, ccols, stop, s);
    e = hipGetLastError();
    if (e != hipSuccess) return status_from_hip(e, "lanczos step");
    const int nq = qp;
    qp = q;
    q = nq;
  }
  hipLaunchKernelGGL(k_lz_count, dim3(1), dim3(64), 0, s, stop, steps_done);
  return status_from_hip(hipGetLastError(), "lanczos: step count");
}

}  // extern "C"
