// Floating-point interface.  The paper's numbers are floating multiprecision
// values: a mantissa of b bits (Section 2) and, in the limb form of Section 3,
// a per-number factor B_0 in front of the limb sum.  Here a number is a
// significand M with |M| < 2^P (P significant bits, W = ceil((P+64)/64)
// two's complement words) and an int32 exponent e: value M 2^(e-P).  The
// product is the exact sum, rounded once to P significant bits with ties to
// even.
//
// It runs on the fixed-point path.  Every entry of h is aligned to the
// largest exponent E_h of h and every entry of x to the largest exponent
// E_x of that x, as integers with Q = P + D fractional bits, where D is the
// exponent spread the plan admits:
//     h_k = H_k 2^(E_h - Q),  H_k = M_k 2^(D - (E_h - e_k)),  |H_k| < 2^Q,
// exactly, as long as E_h - e_k <= D.  The fixed-point plan at precision Q
// then gives the exact integer sums S_i = sum_j H_{i+j} X_j (its carry step
// in exact mode), and y_i = S_i 2^(E_h + E_x - 2Q) is rounded to P
// significant bits.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <new>

#include "common.h"
#include "hmv.h"
#include "kernels.h"
#include "plan.h"

namespace hmv {
namespace {

constexpr int kFxThreads = 256;

// Clears the status block and starts exps: exps[0] = largest exponent of a
// nonzero entry, exps[1] = smallest, exps[2] = 1 if a significand needs
// more than P bits (one launch for both).
__global__ void k_f_clear(DevStatus* st, int* exps) {
  uint64_t* p = reinterpret_cast<uint64_t*>(st);
  if (threadIdx.x < sizeof(DevStatus) / 8) p[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) {
    exps[0] = INT_MIN;
    exps[1] = INT_MAX;
    exps[2] = 0;
  }
}

// Is each number nonzero, and does |M| < 2^P hold (every bit from P up equal
// to the sign, and M != -2^P)?  A wavefront takes the numbers r = its index,
// its index + the wavefronts of the grid, ...; the work-group combines its
// wavefronts in LDS and makes one atomic update of each kind (one update
// per number, all on the same words, would run one after another).
__global__ void __launch_bounds__(kFxThreads) k_f_exp_range(const uint64_t* __restrict__ sig,
                                                            const int32_t* __restrict__ exp,
                                                            int count, int W, int P, int* exps) {
  constexpr int kWaves = kFxThreads / 64;
  __shared__ int red[3][kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int pw = P >> 6, pb = P & 63;
  int emax = INT_MIN, emin = INT_MAX, bad = 0;
  for (int r = blockIdx.x * kWaves + wv; r < count; r += gridDim.x * kWaves) {
    const uint64_t* m = sig + (int64_t)r * W;
    const uint64_t signw = (m[W - 1] >> 63) ? ~0ull : 0ull;
    int nz = 0, wide = 0, low_zero = 1;
#pragma unroll 4
    for (int q = lane; q < W; q += 64) {
      const uint64_t v = m[q];
      if (v) nz = 1;
      // bits at and above P must all equal the sign bit
      const uint64_t hi = q > pw ? v : (q == pw ? (pb ? v >> pb : v) : 0ull);
      const uint64_t ref = q > pw ? signw : (q == pw ? (pb ? signw >> pb : signw) : 0ull);
      if (q >= pw && hi != ref) wide = 1;
      // bits below P all zero (with a negative sign: M = -2^P)
      const uint64_t lowbits = q < pw ? v : (q == pw ? (pb ? v & ((1ull << pb) - 1) : 0ull) : 0ull);
      if (lowbits) low_zero = 0;
    }
    if (__any(nz)) {                        // uniform over the wavefront
      if (__any(wide) || (signw && __all(low_zero))) bad = 1;
      const int e = exp[r];
      emax = max(emax, e);
      emin = min(emin, e);
    }
  }
  if (lane == 0) {
    red[0][wv] = emax;
    red[1][wv] = emin;
    red[2][wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = INT_MIN, b = INT_MAX, c = 0;
    for (int k = 0; k < kWaves; ++k) {
      a = max(a, red[0][k]);
      b = min(b, red[1][k]);
      c |= red[2][k];
    }
    if (a != INT_MIN) {
      atomicMax(&exps[0], a);
      atomicMin(&exps[1], b);
    }
    if (c) atomicOr(&exps[2], 1);
  }
}

// One work-group per number: out = M shifted left by D - (E - e) bits into Wq
// words; zero for a zero significand; an exponent outside the window
// (E - e > D) or an over-wide significand sets the range flag.
__global__ void __launch_bounds__(kFxThreads) k_f_to_fixed(const uint64_t* __restrict__ sig,
                                                           const int32_t* __restrict__ exp,
                                                           int count, int Wp, int D, int Wq,
                                                           const int* __restrict__ exps,
                                                           uint64_t* __restrict__ out,
                                                           DevStatus* st) {
  __shared__ int nz;
  const int r = blockIdx.x;
  if (r >= count) return;
  const uint64_t* m = sig + (int64_t)r * Wp;
  uint64_t* o = out + (int64_t)r * Wq;
  if (threadIdx.x == 0) nz = 0;
  __syncthreads();
  int mine = 0;
  for (int q = threadIdx.x; q < Wp; q += blockDim.x)
    if (m[q]) mine = 1;
  if (mine) nz = 1;
  __syncthreads();
  const int64_t d = nz ? (int64_t)exps[0] - exp[r] : 0;
  const bool ok = d >= 0 && d <= D;
  if (threadIdx.x == 0 && ((nz && !ok) || (nz && exps[2]))) status_or(st, ST_RANGE);
  const int s = (nz && ok) ? (int)(D - d) : 0;
  const uint64_t signw = (m[Wp - 1] >> 63) ? ~0ull : 0ull;
  auto word = [&](int q) -> uint64_t {      // word q of M, sign-extended
    if (q < 0) return 0ull;
    return q < Wp ? m[q] : signw;
  };
  const int qs = s >> 6, bs = s & 63;
  for (int q = threadIdx.x; q < Wq; q += blockDim.x) {
    uint64_t v = 0ull;
    if (nz && ok) {
      // bits [64 q - s, 64 q - s + 64) of M
      const int q0 = q - qs;
      v = bs ? (word(q0) << bs) | (word(q0 - 1) >> (64 - bs)) : word(q0);
    }
    o[q] = v;
  }
}

// LDS operations of a wavefront complete in issue order, so lanes of one
// wavefront exchange LDS words with no barrier; the fences keep the
// compiler's order of the accesses around the exchange.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One wavefront per row (blockDim.x / 64 rows per work-group, each with its
// own We + Wp words of LDS; no block barrier): the exact sum S (We words,
// two's complement) to P significant bits, ties to even; significand in Wp
// words, exponent E_h + E_x - 2Q + shift + P (zero: 0 and exponent 0).
// Lane l owns the words q = l, l + 64, ...; first / last words with a
// property are wavefront minima / maxima of each lane's first / last hit.
__global__ void __launch_bounds__(kFxThreads) k_f_from_exact(const uint64_t* __restrict__ S,
                                                             int count, int We, int P, int Wp,
                                                             int64_t ebase, const int* __restrict__ exps,
                                                             uint64_t* __restrict__ ysig,
                                                             int32_t* __restrict__ yexp,
                                                             DevStatus* st) {
  extern __shared__ uint64_t lds[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = blockIdx.x * (int)(blockDim.x >> 6) + wv;
  if (r >= count) return;                   // whole wavefronts; nothing waits on them
  uint64_t* mag = lds + (int64_t)wv * (We + Wp);
  uint64_t* res = mag + We;
  const uint64_t* src = S + (int64_t)r * We;
  const bool neg = (src[We - 1] >> 63) != 0;
  int f = We;                                // first nonzero word
#pragma unroll 4
  for (int q = lane; q < We; q += 64) {
    const uint64_t v = src[q];
    mag[q] = v;
    if (v && f == We) f = q;
  }
  f = wave_min(f);
  // magnitude: -S = ~S + 1, i.e. zeros below the first nonzero word f, -S_f
  // there and ~S above (each lane rewrites its own words)
  int hw = -1;                               // highest nonzero word
  for (int q = lane; q < We; q += 64) {
    uint64_t v = mag[q];
    if (neg) {
      v = q < f ? 0ull : (q == f ? (0ull - v) : ~v);
      mag[q] = v;
    }
    if (v) hw = q;
  }
  hw = wave_max(hw);
  wave_sync();
  uint64_t* outs = ysig + (int64_t)r * Wp;
  if (hw < 0) {                              // S = 0
    for (int q = lane; q < Wp; q += 64) outs[q] = 0ull;
    if (lane == 0) yexp[r] = 0;
    return;
  }
  const int64_t b = 64 * (int64_t)hw + (64 - __clzll((long long)mag[hw]));   // bit length
  int64_t shift = b - P;
  auto bits_at = [&](int64_t p) -> uint64_t {   // bits [p, p + 64) of the magnitude
    if (p >= 64 * (int64_t)We) return 0ull;
    if (p <= -64) return 0ull;
    if (p < 0) return mag[0] << (-p);
    const int64_t q = p >> 6;
    const int o = (int)(p & 63);
    const uint64_t lo = mag[q] >> o;
    const uint64_t hi = (o && q + 1 < We) ? mag[q + 1] << (64 - o) : 0ull;
    return lo | hi;
  };
  // round bit, sticky bits below it and the last kept bit
  int up = 0;
  if (shift > 0) {
    const int64_t rb = shift - 1;
    const int rq = (int)(rb >> 6), ro = (int)(rb & 63);
    int st_mine = 0;
    for (int q = lane; q <= rq; q += 64) {
      const uint64_t v = q < rq ? mag[q] : (ro ? mag[q] & ((1ull << ro) - 1) : 0ull);
      if (v) st_mine = 1;
    }
    const int sticky = __any(st_mine);
    const int rbit = (int)((mag[rq] >> ro) & 1ull);
    const int lsb = (int)((bits_at(shift) & 1ull));
    up = rbit && (sticky || lsb);
  }
  // P significant bits: bits [shift, shift + P) of the magnitude
  const int pw = P >> 6, pb = P & 63;
  int fno = Wp;                              // first word that is not all ones
  for (int q = lane; q < Wp; q += 64) {
    uint64_t v = bits_at(shift + 64 * (int64_t)q);
    if (q > pw || (q == pw && pb == 0)) v = 0ull;
    else if (q == pw) v &= (1ull << pb) - 1;
    res[q] = v;
    if (v != ~0ull && fno == Wp) fno = q;
  }
  if (up) {                                  // uniform over the wavefront
    // increment: the words below the first one that is not all ones become 0
    fno = wave_min(fno);
    for (int q = lane; q <= fno && q < Wp; q += 64) res[q] = q < fno ? 0ull : res[q] + 1ull;
    wave_sync();
    // a carry into bit P: the significand was 2^P - 1, now 2^P -> 2^(P-1)
    if ((res[pw] >> pb) & 1ull) {
      for (int q = lane; q < Wp; q += 64) res[q] = 0ull;
      wave_sync();
      if (lane == 0) res[(P - 1) >> 6] = 1ull << ((P - 1) & 63);
      shift += 1;
    }
    wave_sync();
  }
  // sign: two's complement over Wp words
  if (neg) {
    int fr = Wp;
    for (int q = lane; q < Wp; q += 64)
      if (res[q] && fr == Wp) fr = q;
    fr = wave_min(fr);
    for (int q = lane; q < Wp; q += 64) {
      const uint64_t v = res[q];
      outs[q] = q < fr ? 0ull : (q == fr ? (0ull - v) : ~v);
    }
  } else {
    for (int q = lane; q < Wp; q += 64) outs[q] = res[q];
  }
  if (lane == 0) {
    const int64_t e = ebase + (int64_t)exps[0] + shift + P;
    if (e > INT_MAX || e < INT_MIN) status_or(st, ST_OVERFLOW);
    yexp[r] = (int32_t)(e > INT_MAX ? INT_MAX : (e < INT_MIN ? INT_MIN : e));
  }
}

// status cleared, then the exponent range of `count` numbers into exps
hipError_t clear_and_exp_range(const uint64_t* sig, const int32_t* exp, int count, int W, int P,
                               int* exps, DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_f_clear, dim3(1), dim3(64), 0, s, st, exps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || count <= 0) return e;
  const int per = kFxThreads / 64;
  const int blocks = (count + per - 1) / per;
  hipLaunchKernelGGL(k_f_exp_range, dim3(blocks < 256 ? blocks : 256), dim3(kFxThreads), 0, s,
                     sig, exp, count, W, P, exps);
  return hipGetLastError();
}

hipError_t to_fixed(const uint64_t* sig, const int32_t* exp, int count, int Wp, int D, int Wq,
                    const int* exps, uint64_t* out, DevStatus* st, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_f_to_fixed, dim3(count), dim3(kFxThreads), 0, s, sig, exp, count, Wp, D,
                     Wq, exps, out, st);
  return hipGetLastError();
}

hipError_t from_exact(const uint64_t* S, int count, int We, int P, int Wp, int64_t ebase,
                      const int* exps, uint64_t* ysig, int32_t* yexp, DevStatus* st,
                      hipStream_t s) {
  // one wavefront per row, up to four per work-group within 64 KiB of LDS
  const size_t per_row = sizeof(uint64_t) * (size_t)(We + Wp);
  if (per_row > 64 * 1024) return hipErrorInvalidValue;
  if (count <= 0) return hipSuccess;
  int rows = (int)((64 * 1024) / per_row);
  rows = rows < kFxThreads / 64 ? rows : kFxThreads / 64;
  hipLaunchKernelGGL(k_f_from_exact, dim3((count + rows - 1) / rows), dim3(64 * rows),
                     per_row * rows, s, S, count, We, P, Wp, ebase, exps, ysig, yexp, st);
  return hipGetLastError();
}

// Sizes of the floating-point layer around a fixed-point plan at Q = P + D.
struct FSizes {
  int32_t Q;
  int Wp, Wq, We;
  int64_t inner_plan, inner_ws;          // fixed-point plan memory and workspace
  int64_t plan_ws;                       // workspace of hmv_fplan_h
  int64_t mv_ws;                         // workspace of hmv_fplan_matvec
  int64_t off_fixed, off_exact;          // matvec workspace: converted x, exact sums
  int64_t off_inner;                     // inner status block + scratch
};

constexpr int64_t kExpBytes = 256;       // exponent range block (after the status block)

bool fsizes(int kind, int64_t n, int32_t P, int32_t D, FSizes* z) {
  if (!valid_kind(kind) || n < 1 || n > HMV_MAX_N || P < 2 || D < 0) return false;
  if ((int64_t)P + D > HMV_MAX_P) return false;
  z->Q = P + D;
  z->Wp = (int)words_of(P);
  z->Wq = (int)words_of(z->Q);
  // |S| < n 2^(2Q) <= 2^(2Q + 14): 2Q + 15 bits and a sign
  z->We = (int)((2 * (int64_t)z->Q + 16 + 63) / 64) + 1;
  z->inner_plan = hmv_plan_bytes(kind, n, z->Q, HMV_AUTO);
  z->inner_ws = hmv_workspace_bytes(kind, n, z->Q, HMV_AUTO);
  if (z->inner_plan < 0 || z->inner_ws < 0) return false;
  const int64_t hl = kind == HMV_CIRCULANT ? n : 2 * n - 1;
  // plan: status | exponent block | converted h | inner workspace
  z->plan_ws = kStatusBytes + kExpBytes + align_up(hl * z->Wq * 8) + z->inner_ws;
  z->off_fixed = kStatusBytes + kExpBytes;
  z->off_exact = z->off_fixed + align_up(n * z->Wq * 8);
  z->off_inner = z->off_exact + align_up(n * (int64_t)z->We * 8);
  z->mv_ws = z->off_inner + z->inner_ws;
  return true;
}

}  // namespace
}  // namespace hmv

struct hmv_fplan {
  int kind = 0;
  int64_t n = 0;
  int32_t P = 0, D = 0;
  int32_t Eh = 0;                 // largest exponent of h
  hmv::FSizes z{};
  hmv_plan* inner = nullptr;      // fixed-point plan at Q = P + D
};

extern "C" {

int64_t hmv_fplan_bytes(int kind, int64_t n, int32_t P, int32_t spread) {
  hmv::FSizes z;
  if (!hmv::fsizes(kind, n, P, spread, &z)) return HMV_EINVAL;
  return z.inner_plan;
}

int64_t hmv_fplan_workspace_bytes(int kind, int64_t n, int32_t P, int32_t spread) {
  hmv::FSizes z;
  if (!hmv::fsizes(kind, n, P, spread, &z)) return HMV_EINVAL;
  return z.plan_ws > z.mv_ws ? z.plan_ws : z.mv_ws;
}

int hmv_fplan_h(hmv_fplan** out, int kind, const uint64_t* h_sig, const int32_t* h_exp,
                int64_t n, int32_t P, int32_t spread, void* plan_mem, int64_t plan_bytes, void* ws,
                int64_t ws_bytes, void* stream) {
  using namespace hmv;
  if (!out || !h_sig || !h_exp || !plan_mem || !ws) return HMV_EINVAL;
  *out = nullptr;
  FSizes z;
  if (!fsizes(kind, n, P, spread, &z)) return HMV_EINVAL;
  if (plan_bytes < z.inner_plan || ws_bytes < z.plan_ws) return HMV_ENOMEM;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  DevStatus* st = reinterpret_cast<DevStatus*>(base);
  int* exps = reinterpret_cast<int*>(base + kStatusBytes);
  uint64_t* Hq = reinterpret_cast<uint64_t*>(base + kStatusBytes + kExpBytes);
  const int64_t hl = kind == HMV_CIRCULANT ? n : 2 * n - 1;
  char* inner_ws = base + z.plan_ws - z.inner_ws;
  hipError_t e = clear_and_exp_range(h_sig, h_exp, (int)hl, z.Wp, P, exps, st, s);
  int host[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(host, exps, sizeof(host), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return status_from_hip(e, "float plan: exponent range of h");
  if (host[2]) return fail_with(HMV_ERANGE, "float plan: a significand of h needs more than P bits");
  const bool allzero = host[0] == INT_MIN;
  if (!allzero && (int64_t)host[0] - host[1] > spread)
    return fail_with(HMV_ERANGE, "float plan: the exponents of h span more than the spread");
  e = to_fixed(h_sig, h_exp, (int)hl, z.Wp, spread, z.Wq, exps, Hq, st, s);
  if (e != hipSuccess) return status_from_hip(e, "float plan: alignment of h");
  hmv_fplan* p = new (std::nothrow) hmv_fplan();
  if (!p) return HMV_ENOMEM;
  p->kind = kind;
  p->n = n;
  p->P = P;
  p->D = spread;
  p->Eh = allzero ? 0 : host[0];
  p->z = z;
  const int rc = plan_h_impl(&p->inner, kind, Hq, n, z.Q, HMV_AUTO, plan_mem, plan_bytes,
                             inner_ws, z.inner_ws, stream, true);
  if (rc != HMV_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return HMV_OK;
}

int hmv_fplan_matvec(const hmv_fplan* p, const uint64_t* x_sig, const int32_t* x_exp,
                     uint64_t* y_sig, int32_t* y_exp, void* ws, int64_t ws_bytes, void* stream) {
  using namespace hmv;
  if (!p || !x_sig || !x_exp || !y_sig || !y_exp || !ws) return HMV_EINVAL;
  const FSizes& z = p->z;
  if (ws_bytes < z.mv_ws) return HMV_ENOMEM;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  DevStatus* st = reinterpret_cast<DevStatus*>(base);
  int* exps = reinterpret_cast<int*>(base + kStatusBytes);
  uint64_t* Xq = reinterpret_cast<uint64_t*>(base + z.off_fixed);
  uint64_t* Se = reinterpret_cast<uint64_t*>(base + z.off_exact);
  const int n = (int)p->n;
  hipError_t e = clear_and_exp_range(x_sig, x_exp, n, z.Wp, p->P, exps, st, s);
  if (e == hipSuccess) e = to_fixed(x_sig, x_exp, n, z.Wp, p->D, z.Wq, exps, Xq, st, s);
  if (e != hipSuccess) return status_from_hip(e, "float matvec: alignment of x");
  // exact sums S_i = sum_j H_{i+j} X_j (carry step without rounding)
  char* inner = base + z.off_inner;
  int rc = plan_matvec_parts(p->inner, Xq, Se, st, inner + kStatusBytes,
                             z.inner_ws - kStatusBytes, s, nullptr, false, z.We);
  if (rc != HMV_OK) return rc;
  // y_i = S_i 2^(E_h + E_x - 2Q), rounded to P significant bits
  const int64_t ebase = (int64_t)p->Eh - 2 * (int64_t)z.Q;
  e = from_exact(Se, n, z.We, p->P, z.Wp, ebase, exps, y_sig, y_exp, st, s);
  return status_from_hip(e, "float matvec: rounding");
}

int hmv_fplan_info(const hmv_fplan* p, hmv_plan_info_t* info, int32_t* Q, int32_t* Eh) {
  if (!p) return HMV_EINVAL;
  if (Q) *Q = p->z.Q;
  if (Eh) *Eh = p->Eh;
  return info ? hmv_plan_info(p->inner, info) : HMV_OK;
}

int hmv_fplan_destroy(hmv_fplan* p) {
  if (p) hmv_plan_destroy(p->inner);
  delete p;
  return HMV_OK;
}

}  // extern "C"
