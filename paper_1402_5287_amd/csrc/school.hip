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
// major (Hs[c][r] = digit c of h row r, Xt[d][j]), so that both operands of
// v_mfma_i32_32x32x32_i8 read 16 consecutive bytes of the index axis per
// lane; lanes 0-31 take the first 16 bytes of each 32-byte step and lanes
// 32-63 the next 16, for A and B alike (the sum over k does not depend on
// which lane carries which k).  A work-group (8 wavefronts, or 4 at the
// largest precisions) computes one row i over tiles of 256 c x 256 d (256 x
// 128), each wavefront 128 x 64 (4 x 2 products of 32 x 32), with the index
// axis staged through LDS 64 bytes at a time (two LDS buffers; the loads of
// a stage are issued two (four) stages ahead into a ring of register
// sets).  Row i's operand starts at index i; h's digits
// are kept in 16 copies, copy s shifted by s rows, so that row i reads copy
// i mod 16 from a 16-byte aligned index and every load is one aligned
// 16-byte access (about 16 x 36 MB at n = 4096, P = 33 220).
// After the tiles that feed one band of anti-diagonals, every lane adds its
// 128 sums into s_i (int64 LDS atomics); after all tiles the carry / round /
// pack step runs on s_i.
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef int v16i32 __attribute__((ext_vector_type(16)));
// Tiles: 256 c x 64 WD d per work-group of 2 x WD wavefronts, 128 c x 64 d
// per wavefront (4 x 2 products of 32 x 32; with 4 x 4 the accumulators
// alone fill the 256 accumulation registers and the kernel spills).  WD = 4
// (8 wavefronts, two per SIMD) where the LDS holds its larger stages, else
// 2.  A stage holds 64 index bytes of every operand row, rows 80 bytes apart
// (16 bytes of padding spread the lanes' 16-byte reads over all banks).
constexpr int kSmTileC = 256, kSmStage = 64, kSmRow = 80;
__host__ __device__ constexpr int sm_stage_bytes(int WD) { return (kSmTileC + 64 * WD) * kSmRow; }

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

// Global loads of one stage (index bytes j0 .. j0 + 63 of every operand
// row) by the T = 128 WD threads: pieces t + T q, row piece / 4, 16 bytes
// at (piece % 4) 16; PA = 1024 / T pieces of A, 2 of B per thread.  Ha is
// the copy of h's digits shifted so that row i's index bytes start at the
// 16-byte aligned ib.
template <int WD>
__device__ __forceinline__ void school_mfma_gload(const int8_t* __restrict__ Ha,
                                                  const int8_t* __restrict__ Xt, int R2, int n64,
                                                  int c0, int d0, int ib, int j0, int t,
                                                  v4i32 (&ra)[8 / WD], v4i32 (&rb)[2]) {
  constexpr int T = 128 * WD;
#pragma unroll
  for (int q = 0; q < 8 / WD; ++q) {
    const int piece = t + T * q, row = piece >> 2, off = (piece & 3) * 16;
    ra[q] = *reinterpret_cast<const v4i32*>(Ha + (int64_t)(c0 + row) * R2 + ib + j0 + off);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int piece = t + T * q, row = piece >> 2, off = (piece & 3) * 16;
    rb[q] = *reinterpret_cast<const v4i32*>(Xt + (int64_t)(d0 + row) * n64 + j0 + off);
  }
}

// The stage into LDS.
template <int WD>
__device__ __forceinline__ void school_mfma_lstore(unsigned char* buf, int t,
                                                   const v4i32 (&ra)[8 / WD],
                                                   const v4i32 (&rb)[2]) {
  constexpr int T = 128 * WD;
#pragma unroll
  for (int q = 0; q < 8 / WD; ++q) {
    const int piece = t + T * q, row = piece >> 2, off = (piece & 3) * 16;
    *reinterpret_cast<v4i32*>(buf + row * kSmRow + off) = ra[q];
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int piece = t + T * q, row = piece >> 2, off = (piece & 3) * 16;
    *reinterpret_cast<v4i32*>(buf + (kSmTileC + row) * kSmRow + off) = rb[q];
  }
}

// The products of one stage (two 32-byte steps) from the buffer at cur:
// wavefront (wc, wd) covers c rows 128 wc .. + 127, d rows 64 wd .. + 63.
__device__ __forceinline__ void school_mfma_stage(const unsigned char* cur, int wc, int wd,
                                                  int lane, v16i32 (&acc)[4][2]) {
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
}

template <int WD, int NSET>
__global__ void __launch_bounds__(128 * WD) k_school_mfma(const int8_t* __restrict__ Hs,
                                                           const int8_t* __restrict__ Xt, int n,
                                                           int L, int Lp, int R2, int n64, int P,
                                                           int W, int out_reverse, int group,
                                                           uint64_t* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t red[32];
  constexpr int SB = sm_stage_bytes(WD), TD = 64 * WD, RD = kSmTileC / TD;
  const int NCp = 2 * Lp - 1;
  int64_t* S = reinterpret_cast<int64_t*>(smem + 2 * SB);
  int64_t* cs = S + NCp;
  const int i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wc = wave & 1, wd = wave >> 1;
  for (int e = t; e < NCp; e += blockDim.x) S[e] = 0;
  const int ib = i & ~15;                    // row i reads copy i % 16 from ib on
  const int8_t* Ha = Hs + (int64_t)(i & 15) * Lp * R2;
  const int nst = n64 / kSmStage;
  const int ntc = Lp / kSmTileC, ntd = Lp / TD;
  // Tiles in order of c0 + d0 = TD g (g = RD ct + dt): the tiles of one g
  // feed the same anti-diagonals, so with group != 0 (the host checked that
  // the sum over a group stays below 2^31) their products accumulate in the
  // registers and reach s_i once per g.
  v16i32 acc[4][2];
  const int ng = RD * (ntc - 1) + ntd;
  for (int g = 0; g < ng; ++g) {
    const int ct_lo = g - ntd + 1 > 0 ? (g - ntd + RD) / RD : 0;
    const int ct_hi = min(ntc - 1, g / RD);
    for (int ct = ct_lo; ct <= ct_hi; ++ct) {
      const int dt = g - RD * ct;
      const int c0 = ct * kSmTileC, d0 = dt * TD;
      if (ct == ct_lo || !group) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;
      }
      // A ring of NSET register sets: set u % NSET holds stage u.  While
      // stage s computes, the loads of stage s + NSET go to the set that
      // held stage s (already in LDS), and stage s + 1, loaded NSET - 1
      // stages earlier, goes to LDS after the products.  Past the last
      // stage the loads repeat it and the stores go to the buffer nobody
      // reads any more, which keeps the ring free of conditions.
      v4i32 ra[NSET][8 / WD];
      v4i32 rb[NSET][2];
#pragma unroll
      for (int u = 0; u < NSET; ++u)
        school_mfma_gload<WD>(Ha, Xt, R2, n64, c0, d0, ib, min(u, nst - 1) * kSmStage, t, ra[u],
                              rb[u]);
      school_mfma_lstore<WD>(smem, t, ra[0], rb[0]);
      __syncthreads();
      for (int s0 = 0; s0 < nst; s0 += NSET) {
#pragma unroll
        for (int u = 0; u < NSET; ++u) {
          const int stage = s0 + u;
          if (stage < nst) {                                 // uniform
            school_mfma_gload<WD>(Ha, Xt, R2, n64, c0, d0, ib,
                                  min(stage + NSET, nst - 1) * kSmStage, t, ra[u], rb[u]);
            school_mfma_stage(smem + (stage & 1) * SB, wc, wd, lane, acc);
            school_mfma_lstore<WD>(smem + ((stage + 1) & 1) * SB, t, ra[(u + 1) % NSET],
                                   rb[(u + 1) % NSET]);
            __syncthreads();
          }
        }
      }
      if (ct == ct_hi || !group) {
        // anti-diagonal sums: product (m, nn) of block (cb, db) is G[c][d]
        // with c = c0 + 128 wc + 32 cb + m, d = d0 + 64 wd + 32 db + nn,
        // m = 8 (r / 4) + 4 (lane / 32) + r % 4, nn = lane % 32: one base per
        // lane and a constant offset per (cb, db, r), which the LDS atomic
        // takes as an immediate
        unsigned long long* Sb = reinterpret_cast<unsigned long long*>(
            S + (c0 + 128 * wc + d0 + 64 * wd + 4 * (lane >> 5) + (lane & 31)));
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int db = 0; db < 2; ++db)
#pragma unroll
            for (int r = 0; r < 16; ++r)
              atomicAdd(Sb + (32 * cb + 32 * db + 8 * (r >> 2) + (r & 3)),
                        (unsigned long long)(int64_t)acc[cb][db][r]);
      }
    }
  }
  __syncthreads();
  const int row = out_reverse ? (n - 1 - i) : i;
  carry_round_pack_fit(S, 2 * L - 1, 8, P, W, cs, y + (int64_t)row * W, red);
}

size_t school_mfma_lds_bytes_wd(int Lp, int WD) {
  return (size_t)2 * sm_stage_bytes(WD) + (size_t)(2 * Lp - 1) * 8 +
         (size_t)carry_lds_bytes(128 * WD) + 16;
}

// the smaller form (WD = 2) decides whether the MFMA path applies at all
size_t school_mfma_lds_bytes(int Lp) { return school_mfma_lds_bytes_wd(Lp, 2); }

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

hipError_t launch_school_mfma(const int8_t* Hs, const int8_t* Xt, int n, int L, int Lp, int R2,
                              int n64, int P, int W, int out_reverse, uint64_t* y,
                              hipStream_t s) {
  // a group's int32 sums stay exact: at most Lp/256 tiles of products below
  // n 2^14 each
  const int group = (int64_t)(Lp / kSmTileC) * n * 16384 < (int64_t(1) << 31) ? 1 : 0;
  const bool wide = school_mfma_lds_bytes_wd(Lp, 4) <= (size_t)kSchoolMfmaMaxLds;
  const size_t lds = school_mfma_lds_bytes_wd(Lp, wide ? 4 : 2);
  const void* fn = wide ? (const void*)k_school_mfma<4, 2> : (const void*)k_school_mfma<2, 4>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (wide)
    hipLaunchKernelGGL((k_school_mfma<4, 2>), dim3(n), dim3(512), lds, s, Hs, Xt, n, L, Lp, R2,
                       n64, P, W, out_reverse, group, y);
  else
    hipLaunchKernelGGL((k_school_mfma<2, 4>), dim3(n), dim3(256), lds, s, Hs, Xt, n, L, Lp, R2,
                       n64, P, W, out_reverse, group, y);
  return hipGetLastError();
}

}  // namespace hmv
