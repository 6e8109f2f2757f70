// Device helpers shared by every path: number format, balanced limb split,
// block-wide scans, and the exact carry / round-to-nearest-even / pack step.
//
// Number format: value = X * 2^-P, X an integer with |X| <= 2^P, stored as W
// little-endian uint64 words in two's complement (W = ceil((P+64)/64)).
// Limbs (Section 3: a number as a sum of limb terms a = sum_k B^k a_k):
// balanced base-2^w digits d_e in [-2^(w-1), 2^(w-1)), X = sum_e d_e 2^(w e),
// L = ceil((P+2)/w) digits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmv {

// ---------------------------------------------------------------------------
// device status block: the first 256 bytes of every workspace
// ---------------------------------------------------------------------------
struct DevStatus {
  uint32_t flags;          // ST_* bits, OR-ed by kernels
  uint32_t pad0;
  uint64_t max_err_bits;   // bit pattern of the largest |c - round(c)| seen (FP64 path)
  uint64_t spare[30];
};
static_assert(sizeof(DevStatus) == 256, "status block is 256 bytes");
enum : uint32_t { ST_RANGE = 1u, ST_BOUND = 2u, ST_SPIN = 4u, ST_OVERFLOW = 8u };

__device__ inline void status_or(DevStatus* st, uint32_t f) {
  if (st) atomicOr(&st->flags, f);
}

// Record the work-group's largest rounding distance m (each thread passes its
// own, m >= 0).  One atomic per work-group at most, and none when the value
// already recorded is at least as large: thousands of work-groups updating
// one word would otherwise serialise on it.  Non-negative doubles order like
// their bit patterns.  `slots` = 16 LDS doubles; ends with a barrier.
__device__ inline void status_max_err(DevStatus* st, double m, double* slots) {
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0 && st) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, slots[k]);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(&st->max_err_bits);
    if (bits > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(dst, bits);
  }
}

// Copy W words from global memory into LDS.  Each thread issues its loads
// four at a time (clamped, always in bounds) before storing any of them, so
// they are in flight together.  The caller synchronises afterwards.
__device__ inline void load_words(const uint64_t* __restrict__ src, int W, uint64_t* dst) {
  const int T = blockDim.x, t = threadIdx.x;
  for (int q0 = t; q0 < W; q0 += 4 * T) {
    uint64_t r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u * T;
      r[u] = src[q < W ? q : W - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u * T;
      if (q < W) dst[q] = r[u];
    }
  }
}

// ---------------------------------------------------------------------------
// block-wide exclusive scan of an associative operator on small codes.
// op(a, b) means "a first, then b".  blockDim.x must be a multiple of 64.
// `lds` needs 32 uint32 slots.
// ---------------------------------------------------------------------------
template <class Op>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t ident, Op op, uint32_t* lds) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc = op(o, inc);
  }
  __syncthreads();
  if (lane == 63) lds[wv] = inc;
  __syncthreads();
  if (t == 0) {
    uint32_t acc = ident;
    for (int k = 0; k < nw; ++k) {
      uint32_t tot = lds[k];
      lds[k] = acc;              // exclusive prefix of wave k
      acc = op(acc, tot);
    }
  }
  __syncthreads();
  uint32_t prev = __shfl_up(inc, 1, 64);
  if (lane == 0) prev = ident;
  uint32_t res = op(lds[wv], prev);
  __syncthreads();
  return res;
}

// carry function of the balancing pass: 0 = kill (out 0), 1 = generate
// (out 1), 2 = propagate (out = in).
struct BalOp {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return b == 2u ? a : b; }
};

// carry function of the word pass: maps kappa in {-1,0,1} (index kappa+1) to
// kappa' in {-1,0,1}; 2 bits per entry.  Identity = 0b100100.
struct WordOp {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uint32_t mid = (a >> (2 * i)) & 3u;
      r |= ((b >> (2 * mid)) & 3u) << (2 * i);
    }
    return r;
  }
};
constexpr uint32_t kWordIdent = 0x24u;

// ---------------------------------------------------------------------------
// range check of one number held in LDS: |X| <= 2^P  (block-wide, uniform).
// X fits iff every bit >= P equals the sign bit, or X == 2^P exactly.
// ---------------------------------------------------------------------------
__device__ inline bool number_in_range(const uint64_t* wd, int W, int P) {
  const uint64_t sign = (wd[W - 1] >> 63) ? ~0ull : 0ull;
  int ok_hi = 1, ok_sp = (sign == 0ull);
  for (int q = threadIdx.x; q < W; q += blockDim.x) {
    const uint64_t word = wd[q];
    const int lo = q * 64;
    uint64_t mask;
    if (lo >= P) mask = ~0ull;
    else if (P < lo + 64) mask = ~0ull << (P - lo);
    else mask = 0ull;
    if ((word & mask) != (sign & mask)) ok_hi = 0;
    const uint64_t expect = (q == (P >> 6)) ? (1ull << (P & 63)) : 0ull;
    if (word != expect) ok_sp = 0;
  }
  ok_hi = __syncthreads_and(ok_hi);
  ok_sp = __syncthreads_and(ok_sp);
  return ok_hi || ok_sp;
}

// raw (unsigned) w-bit field e of the sign-extended two's complement number
__device__ inline uint32_t raw_digit(const uint64_t* wd, int W, uint64_t signw, int w, int e) {
  const int bit = e * w, q = bit >> 6, r = bit & 63;
  uint64_t v = (q < W ? wd[q] : signw) >> r;
  if (r + w > 64) v |= (q + 1 < W ? wd[q + 1] : signw) << (64 - r);
  return (uint32_t)(v & ((1ull << w) - 1ull));
}

// Balanced digits of the number in `wd` (LDS, W words).  Threads own
// contiguous chunks of ceil(L / blockDim) digits; store(e, d) is called once
// per digit.  The balancing carry c_{e+1} = [u_e + c_e >= 2^(w-1)] is resolved
// with a block scan of generate / propagate / kill codes.  `lds` = 32 slots.
template <class Store>
__device__ inline void split_balanced(const uint64_t* wd, int W, int w, int L, Store store,
                                      uint32_t* lds) {
  const uint64_t signw = (wd[W - 1] >> 63) ? ~0ull : 0ull;
  const int per = (L + blockDim.x - 1) / blockDim.x;
  const int e0 = threadIdx.x * per;
  const int e1 = min(L, e0 + per);
  const uint32_t half = 1u << (w - 1);
  BalOp op;
  uint32_t f = 2u;
  for (int e = e0; e < e1; ++e) {
    const uint32_t u = raw_digit(wd, W, signw, w, e);
    const uint32_t g = u >= half ? 1u : (u == half - 1u ? 2u : 0u);
    f = op(f, g);
  }
  const uint32_t cin = block_exclusive_scan(f, 2u, op, lds);
  int c = (cin == 1u) ? 1 : 0;
  for (int e = e0; e < e1; ++e) {
    const int u = (int)raw_digit(wd, W, signw, w, e);
    const int s = u + c;
    int d;
    if (s >= (int)half) { d = s - (1 << w); c = 1; } else { d = s; c = 0; }
    store(e, d);
  }
}

// ---------------------------------------------------------------------------
// Exact carry, round and pack
// ---------------------------------------------------------------------------
constexpr int kCarryMaxPer = 16;

// LDS words needed by carry_round_pack: NWS words for S plus NWS small carries.
__host__ __device__ inline int carry_words(int NC, int w, int P, int W) {
  const int a = (int)(((int64_t)w * (NC - 1)) / 64) + 3;
  const int b = (P >> 6) + W + 2;
  return a > b ? a : b;
}
__host__ __device__ inline int carry_lds_bytes(int NC, int w, int P, int W) {
  return carry_words(NC, w, P, W) * 12;
}

__device__ inline __int128 word_column(const int64_t* coef, int NC, int w, int q) {
  // A_q = sum_{e: floor(we/64)=q} lo(coef_e 2^r) + sum_{e: floor(we/64)=q-1} hi(coef_e 2^r)
  __int128 acc = 0;
  int elo = (64 * q + w - 1) / w, ehi = min(NC, (64 * (q + 1) + w - 1) / w);
  for (int e = elo; e < ehi; ++e) {
    const int r = w * e - 64 * q;
    const unsigned __int128 V = (unsigned __int128)(__int128)coef[e] << r;
    acc += (__int128)(uint64_t)V;
  }
  if (q >= 1) {
    elo = (64 * (q - 1) + w - 1) / w;
    ehi = min(NC, (64 * q + w - 1) / w);
    for (int e = elo; e < ehi; ++e) {
      const int r = w * e - 64 * (q - 1);
      const __int128 V = (__int128)((unsigned __int128)(__int128)coef[e] << r);
      acc += (__int128)(V >> 64);
    }
  }
  return acc;
}

// Exact carry, round and pack.
// S = sum_{e < NC} coef[e] * 2^(w e) with int64 coefficients (LDS).
// Y = round-half-even(S / 2^P) is written as W two's complement words to y.
// sw: LDS scratch of carry_lds_bytes() bytes; red: 32 uint32 LDS slots.
// S is cut into 64-bit columns A_q = v_q + c_q 2^64 (v_q unsigned, c_q a
// small signed carry); word q then holds v_q + c_{q-1} + kappa_q where the
// ripple carry kappa in {-1, 0, 1} is resolved by a block scan of the maps
// kappa_q -> kappa_{q+1}.
__device__ inline void carry_round_pack(const int64_t* coef, int NC, int w, int P, int W,
                                        uint64_t* sw, int NWS, uint64_t* __restrict__ y,
                                        uint32_t* red) {
  const int T = blockDim.x, t = threadIdx.x;
  const int per = (NWS + T - 1) / T;
  const int q0 = min(NWS, t * per), q1 = min(NWS, q0 + per);
  int32_t* cv = reinterpret_cast<int32_t*>(sw + NWS);     // c_{q-1} per word q
  int64_t cprev = 0;
  if (q0 >= 1 && q0 < q1) cprev = (int64_t)(word_column(coef, NC, w, q0 - 1) >> 64);
  WordOp op;
  uint32_t f = kWordIdent;
  for (int q = q0; q < q1; ++q) {
    const __int128 A = word_column(coef, NC, w, q);
    const uint64_t v = (uint64_t)A;
    sw[q] = v;
    cv[q] = (int32_t)cprev;
    uint32_t g = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const __int128 s = (__int128)v + cprev + (i - 1);
      const int kap = (int)(s >> 64);           // -1, 0 or 1
      g |= (uint32_t)(kap + 1) << (2 * i);
    }
    f = op(f, g);
    cprev = (int64_t)(A >> 64);
  }
  const uint32_t fin = block_exclusive_scan(f, kWordIdent, op, red);
  int kappa = (int)(fin >> 2 & 3u) - 1;        // applied to kappa_0 = 0 (index 1)
  for (int q = q0; q < q1; ++q) {
    const __int128 s = (__int128)sw[q] + cv[q] + kappa;
    sw[q] = (uint64_t)s;
    kappa = (int)(s >> 64);
  }
  __syncthreads();
  // round half to even at bit P
  const int pb = P - 1;
  const int bitP1 = (int)((sw[pb >> 6] >> (pb & 63)) & 1ull);
  const int qlsb = (int)((sw[P >> 6] >> (P & 63)) & 1ull);
  int st = 0;
  for (int q = t; q <= (pb >> 6); q += T) {
    uint64_t word = sw[q];
    if (q == (pb >> 6)) word &= (pb & 63) ? ((1ull << (pb & 63)) - 1ull) : 0ull;
    if (word) st = 1;
  }
  const int sticky = __syncthreads_or(st);
  const int up = bitP1 && (sticky || qlsb);
  // words of floor(S / 2^P); the increment ripples through low all-ones words
  if (t == 0) red[0] = (uint32_t)W;
  __syncthreads();
  const int sh = P & 63, base = P >> 6;
  for (int m = t; m < W; m += T) {
    const uint64_t lo = sw[base + m] >> sh;
    const uint64_t hi = sh ? (sw[base + m + 1] << (64 - sh)) : 0ull;
    if ((lo | hi) != ~0ull) atomicMin(&red[0], (uint32_t)m);
  }
  __syncthreads();
  const int first = (int)red[0];
  for (int m = t; m < W; m += T) {
    uint64_t ym = (sw[base + m] >> sh) | (sh ? (sw[base + m + 1] << (64 - sh)) : 0ull);
    if (up) {
      if (m < first) ym = 0ull;
      else if (m == first) ym += 1ull;
    }
    y[m] = ym;
  }
  __syncthreads();
}

}  // namespace hmv
