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

}  // namespace hmv
