// GPU schoolbook path: the plain sum y_i = sum_j a_{i+j-1} x_j of Section 2
// (Preliminaries, the schoolbook product after eq. (3)), carried out on
// balanced limbs.  Each entry becomes a polynomial in z = 2^w with small
// integer coefficients, and row i accumulates
//     s_i[e] = sum_j sum_c hd[i+j][c] * xd[j][e-c]
// exactly in binary64: the host picks w so that n * L * 4^(w-1) < 2^53, so
// every product and every partial sum is an integer below 2^53 and no
// rounding happens.  The exact coefficients then go through the shared
// carry / round / pack step.
#include "common.h"
#include "kernels.h"

namespace hmv {

// One work-group per number: range check, balanced split, digits as doubles.
// Row r of the output takes input number src_row(r): identity, or for the
// circulant embedding the gather t -> (n-1-t) mod n.
__global__ void __launch_bounds__(256) k_split_digits_f64(const uint64_t* __restrict__ in, int W,
                                                           int P, int w, int L, int count,
                                                           int gather_n, double* __restrict__ out,
                                                           int ld, DevStatus* st) {
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  const int r = blockIdx.x;
  if (r >= count) return;
  int src = r;
  if (gather_n > 0) src = ((gather_n - 1 - r) % gather_n + gather_n) % gather_n;
  for (int q = threadIdx.x; q < W; q += blockDim.x) wd[q] = in[(int64_t)src * W + q];
  __syncthreads();
  if (!number_in_range(wd, W, P)) {
    if (threadIdx.x == 0) status_or(st, ST_RANGE);
  }
  double* o = out + (int64_t)r * ld;
  for (int e = L + threadIdx.x; e < ld; e += blockDim.x) o[e] = 0.0;   // zero digits past L
  split_balanced(wd, W, w, L, [&](int e, int d) { o[e] = (double)d; }, red);
}

// One work-group per RI consecutive output rows, 512 threads.  Per j the
// work-group stages the row x[j] in LDS.  Lane l of wavefront v owns the RE
// consecutive outputs e = e0 .. e0+RE-1, e0 = 64 RE v + RE l, for each of
// the RI rows: an RI x RE register tile.  Step c adds h[i+j][c] x[e-c] to
// every output; from one step to the next the x digits a lane needs shift
// by one place, so a window of RE registers holds them and each step loads
// just one new digit from the LDS.  The steps run in blocks of RE, which
// makes every window slot a compile-time register.  h[i+j][c] is the same
// on every lane (scalar loads through the constant cache).  A wavefront's
// steps cover the c that reach its outputs, widened to whole blocks: the
// extra terms are zero, since x sits between zero pads of 65 RE digits and
// the rows of h carry zero digits past L.  Afterwards each row's sums
// (exact integers) go through the carry / round / pack step, the
// coefficients in the same LDS.
template <int RI, int RE>
__global__ void __launch_bounds__(kSchoolThreads) k_school_tile(const double* __restrict__ hd,
                                                                const double* __restrict__ xd,
                                                                int n, int L, int ld, int w,
                                                                int P, int W, int out_reverse,
                                                                uint64_t* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int PAD = 65 * RE;
  double* xs = reinterpret_cast<double*>(smem);               // PAD | L digits | PAD
  __shared__ uint32_t red[32];
  const int i0 = blockIdx.x * RI;
  const int T = blockDim.x, t = threadIdx.x;
  // the wavefront index is the same on all its lanes: say so, so that the
  // step loop and the h addresses stay scalar
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int NC = 2 * L - 1;
  const int E0 = wave * 64 * RE;
  const int e0 = E0 + lane * RE;
  const bool busy = E0 < NC;                                  // uniform per wavefront
  const int clo = max(0, E0 - L + 1), chi = min(L - 1, E0 + 64 * RE - 1);
  const int c0 = clo - clo % RE;                              // whole blocks from c0
  const int nblk = (chi - c0) / RE + 1;
  // rows past n - 1 read row n - 1 (their sums are not written)
  int hr[RI];
#pragma unroll
  for (int q = 0; q < RI; ++q) hr[q] = min(i0 + q, n - 1);
  double acc[RI][RE];
#pragma unroll
  for (int q = 0; q < RI; ++q)
#pragma unroll
    for (int r = 0; r < RE; ++r) acc[q][r] = 0.0;
  for (int m = t; m < PAD; m += T) {
    xs[m] = 0.0;
    xs[PAD + L + m] = 0.0;
  }
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    const double* xrow = xd + (int64_t)j * ld;
    for (int c = t; c < L; c += T) xs[PAD + c] = xrow[c];
    __syncthreads();
    if (busy) {
      const double* xp = xs + PAD + e0;                       // xp[d] = x[e0 + d]
      const double* hrow[RI];
#pragma unroll
      for (int q = 0; q < RI; ++q) hrow[q] = hd + (int64_t)(hr[q] + j) * ld;
      // slot (d mod RE) holds x[e0 + d]; before step c0 the slots hold
      // d = r - c0 for r = 1 .. RE-1 (c0 is a multiple of RE)
      double win[RE];
      win[0] = 0.0;
#pragma unroll
      for (int r = 1; r < RE; ++r) win[r] = xp[r - c0];
      for (int bk = 0; bk < nblk; ++bk) {
        const int cb = c0 + bk * RE;
        const double* xb = xp - cb;
#pragma unroll
        for (int u = 0; u < RE; ++u) {
          win[(RE - u) % RE] = xb[-u];                        // d = -(cb + u)
#pragma unroll
          for (int q = 0; q < RI; ++q) {
            const double hv = hrow[q][cb + u];
#pragma unroll
            for (int r = 0; r < RE; ++r)
              acc[q][r] = fma(hv, win[(r - u + RE) % RE], acc[q][r]);
          }
        }
      }
    }
  }
  // the coefficients of all RI rows into the LDS (the register tile is
  // indexed at compile time), then carry / round / pack row by row
  int64_t* coef = reinterpret_cast<int64_t*>(smem);
  int64_t* cs = coef + RI * NC;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RI; ++q)
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const int e = e0 + r;
      if (busy && e < NC) coef[q * NC + e] = (int64_t)acc[q][r];
    }
  __syncthreads();
  for (int q = 0; q < RI && i0 + q < n; ++q) {                // uniform
    const int i = i0 + q;
    const int row = out_reverse ? (n - 1 - i) : i;
    carry_round_pack_fit(coef + q * NC, NC, w, P, W, cs, y + (int64_t)row * W, red);
  }
}

// Register tile of the schoolbook kernel: RE outputs per lane (64 RE per
// wavefront, 8 wavefronts), RE odd (the lanes' LDS reads, RE doubles apart,
// then fall on distinct banks) or 16, the least that covers the 2L - 1
// outputs; RI rows per work-group: 4 where their coefficients fit the LDS
// (the multiply-adds per LDS read and per h load are RI RE and RE), else 2.
struct SchoolTile {
  int RI, RE;
};

SchoolTile school_tile(int L) {
  const int NC = 2 * L - 1;
  int RE = 1;
  while (RE < 15 && RE * kSchoolThreads < NC) RE += 2;
  if (RE * kSchoolThreads < NC) RE = 16;
  for (int RI = 4; RI >= 2; RI >>= 1) {
    const size_t carry = (size_t)RI * NC * 8 + (size_t)carry_lds_bytes(kSchoolThreads);
    if (carry <= 160 * 1024) return {RI, RE};
  }
  return {0, 0};
}

size_t school_lds_bytes(int L, int w, int P, int W) {
  (void)w;
  (void)P;
  (void)W;
  const SchoolTile tl = school_tile(L);
  const int NC = 2 * L - 1;
  const size_t a = (size_t)(L + 2 * 65 * tl.RE) * 8;
  const size_t b = (size_t)tl.RI * NC * 8 + (size_t)carry_lds_bytes(kSchoolThreads);
  return a > b ? a : b;
}

hipError_t launch_split_digits_f64(const uint64_t* in, int W, int P, int w, int L, int count,
                                   int gather_n, double* out, int ld, DevStatus* st,
                                   hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_digits_f64, dim3(count), dim3(256), 0, s, in, W, P, w, L, count,
                     gather_n, out, ld, st);
  return hipGetLastError();
}

template <int RI, int RE>
hipError_t school_tile_t(const double* hd, const double* xd, int n, int L, int ld, int w, int P,
                         int W, int out_reverse, uint64_t* y, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_school_tile<RI, RE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_school_tile<RI, RE>), dim3((n + RI - 1) / RI), dim3(kSchoolThreads), lds,
                     s, hd, xd, n, L, ld, w, P, W, out_reverse, y);
  return hipGetLastError();
}

hipError_t launch_school_rows(const double* hd, const double* xd, int n, int L, int ld, int w,
                              int P, int W, int out_reverse, uint64_t* y, hipStream_t s) {
  const SchoolTile tl = school_tile(L);
  const size_t lds = school_lds_bytes(L, w, P, W);
#define HMV_ST(ri, re)                                                                     \
  if (tl.RI == ri && tl.RE == re)                                                          \
    return school_tile_t<ri, re>(hd, xd, n, L, ld, w, P, W, out_reverse, y, lds, s);
  HMV_ST(4, 1) HMV_ST(4, 3) HMV_ST(4, 5) HMV_ST(4, 7) HMV_ST(4, 9) HMV_ST(4, 11) HMV_ST(4, 13)
  HMV_ST(4, 15) HMV_ST(4, 16)
  HMV_ST(2, 9) HMV_ST(2, 11) HMV_ST(2, 13) HMV_ST(2, 15) HMV_ST(2, 16)
#undef HMV_ST
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ MFMA form
// The same sums as integer matrix products on the matrix cores.  With 8-bit
// balanced limbs (int8), for output row i
//     G_i[c][d] = sum_j h[i+j][c] x[j][d]          (an L x L product over j)
//     s_i[e]    = sum_{c + d = e} G_i[c][d]        (its anti-diagonal sums).
// G_i's entries are below n 2^14 < 2^31 in magnitude, so int32 accumulation
// is exact; the anti-diagonal sums are int64.  The digits are stored limb
// major (Ht[c][r] = digit c of h row r, Xt[d][j]), so that both operands of
// v_mfma_i32_32x32x32_i8 read 16 consecutive bytes of the index axis per
// lane; lanes 0-31 take the first 16 bytes of each 32-byte step and lanes
// 32-63 the next 16, for A and B alike (the sum over k does not depend on
// which lane carries which k).  A work-group (4 wavefronts) computes one row
// i over tiles of 256 c x 128 d, each wavefront 128 x 64 (4 x 2 products of
// 32 x 32), with the index axis staged through LDS 64 bytes at a time (two
// buffers: the next stage's loads are in flight during the products).  Row
// i's operand starts at index i, which need not be 8-byte aligned: each
// stage loads 24 aligned bytes per 16 and shifts them by i mod 8 bytes.
// After a tile, every lane adds its 128 products into s_i (int64 LDS
// atomics); after all tiles the carry / round / pack step runs on s_i.
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef int v16i32 __attribute__((ext_vector_type(16)));
constexpr int kSmTileC = 256, kSmTileD = 128, kSmStage = 64, kSmRow = 80;
constexpr int kSmStageBytes = (kSmTileC + kSmTileD) * kSmRow;

// One work-group per number: range check, balanced 8-bit split into int8
// digits, row-major out[r][0 .. Lp) with zeros from L on.
__global__ void __launch_bounds__(256) k_split_digits_i8(const uint64_t* __restrict__ in, int W,
                                                          int P, int L, int Lp, int count,
                                                          int gather_n, int8_t* __restrict__ out,
                                                          DevStatus* st) {
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  const int r = blockIdx.x;
  if (r >= count) return;
  int src = r;
  if (gather_n > 0) src = ((gather_n - 1 - r) % gather_n + gather_n) % gather_n;
  for (int q = threadIdx.x; q < W; q += blockDim.x) wd[q] = in[(int64_t)src * W + q];
  __syncthreads();
  if (!number_in_range(wd, W, P)) {
    if (threadIdx.x == 0) status_or(st, ST_RANGE);
  }
  int8_t* o = out + (int64_t)r * Lp;
  for (int e = L + threadIdx.x; e < Lp; e += blockDim.x) o[e] = 0;
  split_balanced(wd, W, 8, L, [&](int e, int d) { o[e] = (int8_t)d; }, red);
}

// dst[c][r] = src[r][c] for r < R, 0 for R <= r < Rp; 64 x 64 byte tiles.
__global__ void __launch_bounds__(256) k_transpose_i8(const int8_t* __restrict__ src, int R,
                                                       int Lp, int8_t* __restrict__ dst, int Rp) {
  __shared__ uint8_t tile[64][68];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int t = threadIdx.x, row = t >> 2, part = (t & 3) * 16;
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (r0 + row < R) v = *reinterpret_cast<const uint4*>(src + (int64_t)(r0 + row) * Lp + c0 + part);
  const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 16; ++q) tile[row][part + q] = (uint8_t)(w4[q >> 2] >> (8 * (q & 3)));
  __syncthreads();
  // thread: destination row c0 + row, bytes r0 + part .. + 15
  uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int q = 0; q < 16; ++q) o[q >> 2] |= (uint32_t)tile[part + q][row] << (8 * (q & 3));
  *reinterpret_cast<uint4*>(dst + (int64_t)(c0 + row) * Rp + r0 + part) =
      make_uint4(o[0], o[1], o[2], o[3]);
}

// Global loads of one stage (index bytes j0 .. j0 + 63 of every operand row).
__device__ __forceinline__ void school_mfma_gload(const int8_t* __restrict__ Ht,
                                                  const int8_t* __restrict__ Xt, int R2, int n64,
                                                  int c0, int d0, int ib, int j0, int t,
                                                  uint2 (&ra)[4][3], uint4 (&rb)[2]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int piece = t + 256 * q, row = piece >> 2, off = (piece & 3) * 16;
    const uint2* a = reinterpret_cast<const uint2*>(Ht + (int64_t)(c0 + row) * R2 + ib + j0 + off);
    ra[q][0] = a[0];
    ra[q][1] = a[1];
    ra[q][2] = a[2];
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int piece = t + 256 * q, row = piece >> 2, off = (piece & 3) * 16;
    rb[q] = *reinterpret_cast<const uint4*>(Xt + (int64_t)(d0 + row) * n64 + j0 + off);
  }
}

// The stage into LDS, the A pieces shifted by shq * 4 + shr bytes.
__device__ __forceinline__ void school_mfma_lstore(unsigned char* buf, int shq, int shr, int t,
                                                   const uint2 (&ra)[4][3],
                                                   const uint4 (&rb)[2]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int piece = t + 256 * q, row = piece >> 2, off = (piece & 3) * 16;
    const uint32_t d0 = ra[q][0].x, d1 = ra[q][0].y, d2 = ra[q][1].x, d3 = ra[q][1].y,
                   d4 = ra[q][2].x, d5 = ra[q][2].y;
    uint4 o;
    if (shq) {
      o.x = __builtin_amdgcn_alignbyte(d2, d1, shr);
      o.y = __builtin_amdgcn_alignbyte(d3, d2, shr);
      o.z = __builtin_amdgcn_alignbyte(d4, d3, shr);
      o.w = __builtin_amdgcn_alignbyte(d5, d4, shr);
    } else {
      o.x = __builtin_amdgcn_alignbyte(d1, d0, shr);
      o.y = __builtin_amdgcn_alignbyte(d2, d1, shr);
      o.z = __builtin_amdgcn_alignbyte(d3, d2, shr);
      o.w = __builtin_amdgcn_alignbyte(d4, d3, shr);
    }
    *reinterpret_cast<uint4*>(buf + row * kSmRow + off) = o;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int piece = t + 256 * q, row = piece >> 2, off = (piece & 3) * 16;
    *reinterpret_cast<uint4*>(buf + (kSmTileC + row) * kSmRow + off) = rb[q];
  }
}

__global__ void __launch_bounds__(256) k_school_mfma(const int8_t* __restrict__ Ht,
                                                      const int8_t* __restrict__ Xt, int n,
                                                      int L, int Lp, int R2, int n64, int P,
                                                      int W, int out_reverse,
                                                      uint64_t* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t red[32];
  const int NCp = 2 * Lp - 1;
  int64_t* S = reinterpret_cast<int64_t*>(smem + 2 * kSmStageBytes);
  int64_t* cs = S + NCp;
  const int i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wc = wave & 1, wd = wave >> 1;
  for (int e = t; e < NCp; e += blockDim.x) S[e] = 0;
  const int sh = i & 7, ib = i - sh, shq = sh >> 2, shr = sh & 3;
  const int nst = n64 / kSmStage;
  const int ntd = Lp / kSmTileD, ntiles = (Lp / kSmTileC) * ntd;
  for (int tile = 0; tile < ntiles; ++tile) {
    const int c0 = (tile / ntd) * kSmTileC, d0 = (tile % ntd) * kSmTileD;
    v16i32 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;
    // staging: A pieces t + 256 q (row piece / 4, 16 bytes at (piece % 4) 16),
    // 24 aligned bytes each for the shift; B pieces likewise, aligned.  The
    // last stage loads and stores one stage more (a repeat of itself) into
    // the buffer nobody reads any more, which keeps the loop free of
    // conditions around the staging registers.
    uint2 ra[4][3];
    uint4 rb[2];
    school_mfma_gload(Ht, Xt, R2, n64, c0, d0, ib, 0, t, ra, rb);
    school_mfma_lstore(smem, shq, shr, t, ra, rb);
    __syncthreads();
    for (int stage = 0; stage < nst; ++stage) {
      const unsigned char* cur = smem + (stage & 1) * kSmStageBytes;
      school_mfma_gload(Ht, Xt, R2, n64, c0, d0, ib, min(stage + 1, nst - 1) * kSmStage, t, ra,
                        rb);
#pragma unroll
      for (int ks = 0; ks < kSmStage / 32; ++ks) {
        const int kb = ks * 32 + (lane >> 5) * 16;
        v4i32 a[4], b[2];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          a[cb] = *reinterpret_cast<const v4i32*>(cur + (wc * 128 + cb * 32 + (lane & 31)) * kSmRow + kb);
#pragma unroll
        for (int db = 0; db < 2; ++db)
          b[db] = *reinterpret_cast<const v4i32*>(
              cur + (kSmTileC + wd * 64 + db * 32 + (lane & 31)) * kSmRow + kb);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int db = 0; db < 2; ++db)
            acc[cb][db] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[cb], b[db], acc[cb][db], 0, 0, 0);
      }
      school_mfma_lstore(smem + ((stage + 1) & 1) * kSmStageBytes, shq, shr, t, ra, rb);
      __syncthreads();
    }
    // anti-diagonal sums: product (m, nn) of block (cb, db) is G[c][d] with
    // c = c0 + 128 wc + 32 cb + m, d = d0 + 64 wd + 32 db + nn
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), nn = lane & 31;
          const int e = c0 + 128 * wc + 32 * cb + m + d0 + 64 * wd + 32 * db + nn;
          atomicAdd(reinterpret_cast<unsigned long long*>(&S[e]),
                    (unsigned long long)(int64_t)acc[cb][db][r]);
        }
  }
  __syncthreads();
  const int row = out_reverse ? (n - 1 - i) : i;
  carry_round_pack_fit(S, 2 * L - 1, 8, P, W, cs, y + (int64_t)row * W, red);
}

size_t school_mfma_lds_bytes(int Lp) {
  return (size_t)2 * kSmStageBytes + (size_t)(2 * Lp - 1) * 8 + (size_t)carry_lds_bytes(256) + 16;
}

hipError_t launch_split_digits_i8(const uint64_t* in, int W, int P, int L, int Lp, int count,
                                  int gather_n, int8_t* out, DevStatus* st, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_digits_i8, dim3(count), dim3(256), 0, s, in, W, P, L, Lp, count,
                     gather_n, out, st);
  return hipGetLastError();
}

hipError_t launch_transpose_i8(const int8_t* src, int R, int Lp, int8_t* dst, int Rp,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_i8, dim3(Lp / 64, Rp / 64), dim3(256), 0, s, src, R, Lp, dst,
                     Rp);
  return hipGetLastError();
}

hipError_t launch_school_mfma(const int8_t* Ht, const int8_t* Xt, int n, int L, int Lp, int R2,
                              int n64, int P, int W, int out_reverse, uint64_t* y,
                              hipStream_t s) {
  const size_t lds = school_mfma_lds_bytes(Lp);
  hipError_t e = hipFuncSetAttribute((const void*)k_school_mfma,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_school_mfma, dim3(n), dim3(256), lds, s, Ht, Xt, n, L, Lp, R2, n64, P, W,
                     out_reverse, y);
  return hipGetLastError();
}

}  // namespace hmv
