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

// Per-row status of the rounding step.  ST_BOUND is raised when a
// coefficient is out of its range (`bad`) or lies more than 1/4 from its
// nearest integer.  Every thread folds its largest
// rounding distance into one of 16 LDS slots (LDS atomics on 16 addresses,
// so at most 16 threads contend for one); the bound flag rides on the
// barrier.  Thread 0 then publishes both with at most one global atomic
// each, the max-error one only when it raises the recorded value (thousands
// of work-groups updating one word would otherwise serialise on it).
// Non-negative doubles order like their bit patterns.
struct RowStatus {
  unsigned long long err[16];
};
// before the work-group's first barrier
__device__ inline void row_status_init(RowStatus* rs) {
  if (threadIdx.x < 16) rs->err[threadIdx.x] = 0ull;
}
// every thread; ends with a barrier
__device__ __forceinline__ void row_status_publish(RowStatus* rs, double err, int bad, DevStatus* st) {
  // a maximum per wavefront first (err >= 0, so its bits order as unsigned),
  // then one LDS atomic per wave
  unsigned long long eb = (unsigned long long)__double_as_longlong(err);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long q = (unsigned long long)__shfl_xor((long long)eb, o, 64);
    eb = q > eb ? q : eb;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(&rs->err[(threadIdx.x >> 6) & 15], eb);
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0 && st) {
    unsigned long long bits = rs->err[0];
#pragma unroll
    for (int k = 1; k < 16; ++k) bits = rs->err[k] > bits ? rs->err[k] : bits;
    // a non-returning atomic: the work-group does not wait for it
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(&st->max_err_bits);
    if (bits) atomicMax(dst, bits);
    // a rounding distance above 1/4 is far outside the proven bound: the
    // nearest integer may not be the exact coefficient, so y is not trusted
    if (bad || __longlong_as_double((long long)bits) > 0.25) status_or(st, ST_BOUND);
  }
}

// Every exact coefficient of the binary64 path is below this in magnitude
// (the planner's constraint n L 4^(w-1) < 2^50), so round_to_int applies.
constexpr double kCoefLimit = 1125899906842624.0;   // 2^50

// Nearest integer of v (ties to even) for |v| < 2^51, as a double and as an
// int64: adding 1.5 * 2^52 leaves the rounded value in the low mantissa bits.
__device__ __forceinline__ int64_t round_to_int(double v, double* rounded) {
  const double kMagic = 6755399441055744.0;        // 1.5 * 2^52
  const double t = v + kMagic;
  *rounded = t - kMagic;
  return (int64_t)(__double_as_longlong(t) - __double_as_longlong(kMagic));
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

// load_words with `between()` run after the first loads are issued and
// before their values reach LDS, so that independent LDS work overlaps the
// global-memory latency.
template <class F>
__device__ __forceinline__ void load_words_then(const uint64_t* __restrict__ src, int W,
                                                uint64_t* dst, F between) {
  const int T = blockDim.x, t = threadIdx.x;
  uint64_t r[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = t + u * T;
    r[u] = src[q < W ? q : W - 1];
  }
  between();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = t + u * T;
    if (q < W) dst[q] = r[u];
  }
  if (4 * T < W) load_words(src + 4 * T, W - 4 * T, dst + 4 * T);
}

// ---------------------------------------------------------------------------
// block-wide exclusive scan of an associative operator on small codes.
// op(a, b) means "a first, then b".  blockDim.x must be a multiple of 64.
// `lds` needs 32 uint32 slots; the caller synchronises before writing them
// again.
// ---------------------------------------------------------------------------
template <class Op>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t ident, Op op, uint32_t* lds) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc = op(o, inc);
  }
  __syncthreads();                 // earlier readers of lds are done
  if (lane == 63) lds[wv] = inc;
  __syncthreads();
  // every wave composes the totals of the waves before it (at most 15)
  uint32_t acc = ident;
  for (int k = 0; k < wv; ++k) acc = op(acc, lds[k]);
  uint32_t prev = __shfl_up(inc, 1, 64);
  if (lane == 0) prev = ident;
  return op(acc, prev);
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

// The same test spread over every wave of the work-group, with no barrier
// of its own.  rf: two LDS flags (every high bit equals the sign bit; the
// number is 2^P) that thread 0 sets with range_flags_init before the
// barrier which publishes the words; a wave holding a word that breaks a
// test clears its flag.  After a later barrier range_flags_ok(rf) tells
// whether the number is in range.
__device__ inline void range_flags_init(uint32_t* rf) {
  if (threadIdx.x == 0) {
    rf[0] = 1u;
    rf[1] = 1u;
  }
}

__device__ inline void range_check_block(const uint64_t* wd, int W, int P, uint32_t* rf) {
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
  const bool lead = (threadIdx.x & 63) == 0;
  if (!__all(ok_hi) && lead) rf[0] = 0u;
  if (!__all(ok_sp) && lead) rf[1] = 0u;
}

__device__ inline bool range_flags_ok(const uint32_t* rf) { return (rf[0] | rf[1]) != 0u; }

// raw (unsigned) w-bit field e of the sign-extended two's complement number
__device__ inline uint32_t raw_digit(const uint64_t* wd, int W, uint64_t signw, int w, int e) {
  const int bit = e * w, q = bit >> 6, r = bit & 63;
  uint64_t v = (q < W ? wd[q] : signw) >> r;
  if (r + w > 64) v |= (q + 1 < W ? wd[q + 1] : signw) << (64 - r);
  return (uint32_t)(v & ((1ull << w) - 1ull));
}

// Digits a thread keeps in registers while splitting (chunks of at most this
// many digits; longer chunks read their fields from LDS twice).
constexpr int kSplitRegs = 16;

// Balanced digits of the number in `wd` (LDS, W words).  Threads own
// contiguous chunks of ceil(L / blockDim) digits; store(e, d) is called once
// per digit.  The balancing carry c_{e+1} = [u_e + c_e >= 2^(w-1)] is resolved
// with a block scan of generate / propagate / kill codes.  `lds` = 32 slots.
// A chunk of at most kSplitRegs digits is kept in registers; each field is
// cut with one funnel shift from the aligned pair of 32-bit words that holds
// it (w < 32), and all of a thread's reads are independent, so they are in
// flight together.
template <class Store>
__device__ __forceinline__ void split_balanced(const uint64_t* wd, int W, int w, int L, Store store,
                                               uint32_t* lds) {
  const uint64_t signw = (wd[W - 1] >> 63) ? ~0ull : 0ull;
  const int per = (L + blockDim.x - 1) / blockDim.x;
  const int e0 = threadIdx.x * per;
  const int e1 = min(L, e0 + per);
  const uint32_t half = 1u << (w - 1);
  BalOp op;
  uint32_t f = 2u;
  if (per <= kSplitRegs) {                       // uniform
    const int cnt = e1 > e0 ? e1 - e0 : 0;
    const uint32_t mask = (1u << w) - 1u;
    const uint32_t* wd32 = reinterpret_cast<const uint32_t*>(wd);
    const uint32_t sg = (uint32_t)signw;
    const int nd = 2 * W;                        // 32-bit words of the number
    uint32_t u[kSplitRegs];
    // field e: bits [e w, e w + w), past the words the sign fill; the
    // addresses are clamped into the words, so every read is in bounds
#pragma unroll
    for (int j = 0; j < kSplitRegs; ++j) {
      const int b = (e0 + j) * w, d = b >> 5;
      const uint32_t lo = wd32[d < nd ? d : nd - 1];
      const uint32_t hi = wd32[d + 1 < nd ? d + 1 : nd - 1];
      u[j] = __builtin_amdgcn_alignbit(d + 1 < nd ? hi : sg, d < nd ? lo : sg, (uint32_t)b & 31u) &
             mask;
    }
#pragma unroll
    for (int j = 0; j < kSplitRegs; ++j) {
      if (j < cnt) {
        const uint32_t g = u[j] >= half ? 1u : (u[j] == half - 1u ? 2u : 0u);
        f = op(f, g);
      }
    }
    const uint32_t cin = block_exclusive_scan(f, 2u, op, lds);
    int c = (cin == 1u) ? 1 : 0;
#pragma unroll
    for (int j = 0; j < kSplitRegs; ++j) {
      if (j < cnt) {
        const int sv = (int)u[j] + c;
        const bool hi = sv >= (int)half;
        store(e0 + j, hi ? sv - (1 << w) : sv);
        c = hi ? 1 : 0;
      }
    }
    return;
  }
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
// LDS scratch of carry_round_pack for a work-group of T threads.
__host__ __device__ inline int carry_lds_bytes(int T) { return 8 * T + 64; }

// Exact carry, round and pack.
// S = sum_{e < NC} coef[e] 2^(w e) with int64 coefficients in LDS, |coef| <
// 2^62.  Y = round-half-even(S / 2^P) is written as W two's complement
// words to y.  coef is overwritten with the limbs of S; cs: LDS scratch of
// carry_lds_bytes(blockDim.x) bytes; red: 32 uint32 LDS slots.
//
// Thread t owns a chunk of E consecutive coefficients (E odd, so that the
// strided LDS accesses spread over the banks, and E w >= 60).
//  1. Each chunk is normalised on its own: limbs in [0, 2^w) (floor
//     division), leaving a carry C_t with |C_t| < 2^55 for the next chunk.
//  2. Chunk t adds C_{t-1}: limbs R' = (R + C_{t-1}) mod 2^(w E) and an
//     outgoing carry c in {-1, 0, 1} (|C_{t-1}| < 2^(w E)).  One more unit
//     kappa in {-1, 0, 1} arriving from below changes what leaves the chunk
//     only if R' is 0 (kappa = -1 borrows through it) or 2^(w E) - 1
//     (kappa = 1 carries through it), so the map kappa -> outgoing carry is
//     (c - [R' = 0], c, c + [R' all ones]).  A block scan composes these
//     maps, which gives every chunk its kappa.
//  3. A chunk with kappa != 0 adds it to R' (the unit ripples through the
//     low limbs that are all ones, or all zeros for a borrow); the top chunk
//     keeps what leaves the limbs plus its own C (S = sum limbs 2^(w e) +
//     top 2^(w NC)).
// Then the round bit (P-1), the sticky OR below it and bit P decide the
// round-half-even increment of floor(S / 2^P), whose words are cut from the
// limbs; the increment ripples through the lowest all-ones words.
// P = 0 asks for S itself, unrounded: its W low words (the caller sizes W
// for the whole sum; the floating-point interface keeps exact sums).
// Limbs a thread keeps in registers during the carry passes; a longer chunk
// (only for very large P at small widths) or a width outside 8..24 runs the
// passes from LDS.
constexpr int kCarryRegs = 32;

// chunk length of carry_round_pack for NC coefficients over T threads
__host__ __device__ inline int carry_chunk(int NC, int w, int T) {
  const int kmin = (60 + w - 1) / w;
  int E = (NC + T - 1) / T;
  if (E < kmin) E = kmin;
  return E | 1;
}

// Steps 1-3 with the chunk in registers, REGS >= E limbs per thread, for
// 8 <= w <= 24.  The limbs are kept as uint32.  From step 2 on the carry
// shrinks by w bits per limb: after four limbs it fits 32 bits (|C| <
// 2^55), and the rest of the chain runs in 32-bit arithmetic.  Returns the
// sticky flag of this thread's limbs; the top value goes to
// cs[blockDim.x].
template <int REGS>
__device__ __forceinline__ int carry_limbs_regs(int64_t* coef, int NC, int w, int E, int ep,
                                                int rp, int64_t* cs, uint32_t* red) {
  const int T = blockDim.x, t = threadIdx.x;
  const int64_t mask = (int64_t(1) << w) - 1;
  const uint32_t mask32 = (uint32_t)mask;
  const int nch = (NC + E - 1) / E;
  const int e0 = t * E, e1 = min(NC, e0 + E);
  const bool own = t < nch;
  const int len = own ? e1 - e0 : 0;
  uint32_t r[REGS];
  // 1. chunk-local normalisation (in place in v, whose registers the limbs
  //    then reuse)
  int64_t cown = 0;
  {
    int64_t v[REGS];
#pragma unroll
    for (int j = 0; j < REGS; ++j) v[j] = coef[e0 + j < NC ? e0 + j : NC - 1];
#pragma unroll
    for (int j = 0; j < REGS; ++j) {
      const int64_t c = v[j] + cown;
      const bool in = j < len;
      v[j] = in ? (c & mask) : 0;
      cown = in ? (c >> w) : cown;
    }
#pragma unroll
    for (int j = 0; j < REGS; ++j) r[j] = (uint32_t)v[j];
  }
  if (own) cs[t] = cown;
  __syncthreads();
  const int64_t cin = (own && t > 0) ? cs[t - 1] : 0;
  // 2. add the incoming carry once; all-zero / all-ones flags of the result
  int64_t c64 = cin;
  int32_t c32 = 0;
  bool allz = true, allo = true;
#pragma unroll
  for (int j = 0; j < REGS; ++j) {
    const bool in = j < len;
    uint32_t rn;
    if (j < 4) {
      const int64_t v = (int64_t)r[j] + c64;
      rn = (uint32_t)(v & mask);
      c64 = in ? (v >> w) : c64;
      if (j == 3) c32 = (int32_t)c64;
    } else {
      const int32_t v = (int32_t)r[j] + c32;
      rn = (uint32_t)v & mask32;
      c32 = in ? (v >> w) : c32;
    }
    r[j] = in ? rn : r[j];
    allz = allz && (!in || rn == 0u);
    allo = allo && (!in || rn == mask32);
  }
  // the outgoing carry: in {-1, 0, 1} for every chunk but the top one, whose
  // carry may be large when it is shorter than four limbs (then it is c64)
  const int64_t cfin = len > 3 ? (int64_t)c32 : c64;
  const int c0 = (int)cfin;
  uint32_t g = kWordIdent;
  if (own && t < nch - 1) {
    const int cm = c0 - (allz ? 1 : 0), cp = c0 + (allo ? 1 : 0);
    g = (uint32_t)(cm + 1) | ((uint32_t)(c0 + 1) << 2) | ((uint32_t)(cp + 1) << 4);
  }
  const uint32_t pre = block_exclusive_scan(g, kWordIdent, WordOp(), red);
  const int kap = own && t > 0 ? (int)((pre >> 2) & 3u) - 1 : 0;   // the map applied to 0
  // 3. the extra unit (rare: a whole chunk of zeros or of ones above it)
  int64_t carry = cfin;
  if (kap != 0) {
    int k = kap;
#pragma unroll
    for (int j = 0; j < REGS; ++j) {
      if (j < len) {
        const int64_t v = (int64_t)r[j] + k;
        r[j] = (uint32_t)(v & mask);
        k = (int)(v >> w);
      }
    }
    carry += k;
  }
  // sticky bit: any 1 below the round bit (none when ep < 0)
  const uint32_t rpmask = (uint32_t)((int64_t(1) << rp) - 1);
  int st = 0;
#pragma unroll
  for (int j = 0; j < REGS; ++j) {
    const int e = e0 + j;
    const uint32_t low = e < ep ? r[j] : (e == ep ? (r[j] & rpmask) : 0u);
    if (j < len && low) st = 1;
  }
  if (own) {
#pragma unroll
    for (int j = 0; j < REGS; ++j)
      if (j < len) coef[e0 + j] = (int64_t)r[j];
  }
  if (own && t == nch - 1) cs[T] = carry + cown;   // the top chunk's own C too
  return st;
}

// Steps 1-3 from LDS: chunks longer than kCarryRegs limbs, and widths
// outside 8..24 (64-bit arithmetic throughout).
__device__ __forceinline__ int carry_limbs_lds(int64_t* coef, int NC, int w, int E, int ep, int rp,
                                      int64_t* cs, uint32_t* red) {
  const int T = blockDim.x, t = threadIdx.x;
  const int64_t mask = (int64_t(1) << w) - 1;
  const int nch = (NC + E - 1) / E;
  const int e0 = t * E, e1 = min(NC, e0 + E);
  const bool own = t < nch;
  int64_t cown = 0;
  if (own) {
    for (int e = e0; e < e1; ++e) {
      const int64_t c = coef[e] + cown;
      coef[e] = c & mask;
      cown = c >> w;
    }
    cs[t] = cown;
  }
  __syncthreads();
  const int64_t cin = (own && t > 0) ? cs[t - 1] : 0;
  int64_t c = cin;
  bool allz = true, allo = true;
  if (own) {
    for (int e = e0; e < e1; ++e) {
      const int64_t v = coef[e] + c;
      coef[e] = v & mask;
      c = v >> w;
      allz = allz && coef[e] == 0;
      allo = allo && coef[e] == mask;
    }
  }
  const int c0 = (int)c;                           // in {-1, 0, 1} below the top chunk
  uint32_t g = kWordIdent;
  if (own && t < nch - 1) {
    const int cm = c0 - (allz ? 1 : 0), cp = c0 + (allo ? 1 : 0);
    g = (uint32_t)(cm + 1) | ((uint32_t)(c0 + 1) << 2) | ((uint32_t)(cp + 1) << 4);
  }
  const uint32_t pre = block_exclusive_scan(g, kWordIdent, WordOp(), red);
  const int kap = own && t > 0 ? (int)((pre >> 2) & 3u) - 1 : 0;
  int64_t carry = c;
  const int64_t rpmask = (int64_t(1) << rp) - 1;
  int st = 0;
  if (own) {
    int k = kap;
    for (int e = e0; e < e1; ++e) {
      if (k != 0) {
        const int64_t v = coef[e] + k;
        coef[e] = v & mask;
        k = (int)(v >> w);
      }
      const int64_t low = e < ep ? coef[e] : (e == ep ? (coef[e] & rpmask) : 0);
      if (low) st = 1;
    }
    carry += k;
    if (t == nch - 1) cs[T] = carry + cown;
  }
  return st;
}

// The carry, the rounding and the output words.
template <int REGS>
__device__ __forceinline__ void carry_round_pack(int64_t* coef, int NC, int w, int P, int W, int64_t* cs,
                                        uint64_t* __restrict__ y, uint32_t* red) {
  const int T = blockDim.x, t = threadIdx.x;
  const int E = carry_chunk(NC, w, T);
  // round bit P-1 sits in limb ep at bit rp (no rounding with P = 0: ep = -1
  // leaves no limb below the round bit)
  const bool exact = P <= 0;
  const int ep = exact ? -1 : (P - 1) / w, rp = exact ? 0 : (P - 1) - ep * w;
  int st;
  // (one register form only: a second one inlined beside it made the
  // compiler keep both sets of limbs live)
  if (E > REGS || w < 8 || w > 24) st = carry_limbs_lds(coef, NC, w, E, ep, rp, cs, red);
  else st = carry_limbs_regs<REGS>(coef, NC, w, E, ep, rp, cs, red);
  if (t == 0) red[31] = (uint32_t)W;               // first word that is not all ones
  const int sticky = __syncthreads_or(st);
  const int64_t top = cs[T];
  const int64_t ncw = (int64_t)NC * w;             // > P: every bit below P+1 is in a limb
  const int rbit = exact ? 0 : (int)((coef[ep] >> rp) & 1);
  const int el = exact ? 0 : P / w;
  const int lsb = exact ? 0 : (int)((coef[el] >> (P - el * w)) & 1);
  const int up = rbit && (sticky || lsb);
  // words of floor(S / 2^P): bits [P + 64 m, P + 64 m + 64) of S; for
  // w >= 8 at most 64 / w + 2 <= 10 limbs overlap a word
  auto word_at = [&](int b) -> uint64_t {
    if (b >= ncw) return (uint64_t)(top >> (b - ncw < 63 ? b - ncw : 63));
    const int e = b / w;
    const int off = b - e * w;
    // only the low 64 bits are kept, and every shift is below 64
    if (w < 8) {                                    // more limbs per word than the window
      uint64_t acc = (uint64_t)coef[e] >> off;
      int nb = w - off, k = e + 1;
      for (; nb < 64 && k < NC; ++k, nb += w) acc |= (uint64_t)coef[k] << nb;
      if (nb < 64) acc |= (uint64_t)top << nb;
      return acc;
    }
    int64_t l[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) l[j] = coef[e + j < NC ? e + j : NC - 1];
    uint64_t acc = (uint64_t)l[0] >> off;
    int nb = w - off;
#pragma unroll
    for (int j = 1; j < 10; ++j) {
      if (nb < 64) {
        const uint64_t v = e + j < NC ? (uint64_t)l[j] : (uint64_t)top;
        acc |= v << nb;
        nb = e + j < NC ? nb + w : 64;
      }
    }
    return acc;
  };
  // floor words go straight out; with a round-up increment the words below
  // the first one that is not all ones become 0 and that one gains 1
  int firstme = W;
  for (int m = t; m < W; m += T) {
    const uint64_t um = word_at(P + 64 * m);
    y[m] = um;
    if (um != ~0ull && m < firstme) firstme = m;
  }
  // the first word that is not all ones: a minimum per wavefront first, then
  // one LDS atomic per wave (every thread on one address serialises); up is
  // uniform over the block
  if (up) {
    int fm = firstme;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) fm = min(fm, __shfl_xor(fm, o, 64));
    if ((t & 63) == 0 && fm < W) atomicMin(&red[31], (uint32_t)fm);
  }
  __syncthreads();
  if (up) {
    const int first = (int)red[31];
    for (int m = t; m <= first && m < W; m += T)
      y[m] = m < first ? 0ull : word_at(P + 64 * m) + 1ull;
  }
  __syncthreads();
}

template <class... A>
__device__ __forceinline__ void carry_round_pack_fit(int64_t* coef, int NC, int w, A... rest) {
  const int E = carry_chunk(NC, w, blockDim.x);     // uniform
  if (E <= 9) carry_round_pack<9>(coef, NC, w, rest...);
  else if (E <= 13) carry_round_pack<13>(coef, NC, w, rest...);
  else if (E <= 17) carry_round_pack<17>(coef, NC, w, rest...);
  else if (E <= 25) carry_round_pack<25>(coef, NC, w, rest...);
  else carry_round_pack<kCarryRegs>(coef, NC, w, rest...);
}

}  // namespace hmv
