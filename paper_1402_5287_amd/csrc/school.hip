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
  split_balanced(wd, W, w, L, [&](int e, int d) { o[e] = (double)d; }, red);
}

// One work-group per output row.  Dynamic LDS: hs[L] | xs[L + 128] with
// xs[64 + m] = x digit m and zeros around it (a wave reads x digits e - c in
// [-63, L + 62] for its uniform c range), later reused for the int64
// coefficients and the carry words.
__global__ void __launch_bounds__(512) k_school_row(const double* __restrict__ hd,
                                                    const double* __restrict__ xd, int n, int L,
                                                    int ld, int w, int P, int W, int out_reverse,
                                                    uint64_t* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* hs = reinterpret_cast<double*>(smem);
  double* xs = hs + L;
  __shared__ uint32_t red[32];
  const int i = blockIdx.x;
  if (i >= n) return;
  const int T = blockDim.x, t = threadIdx.x;
  const int NC = 2 * L - 1;
  constexpr int K = kSchoolMaxK;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int m = t; m < L + 128; m += T) xs[m] = 0.0;
  const int lane0 = t & ~63;
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    const double* hrow = hd + (int64_t)(i + j) * ld;
    const double* xrow = xd + (int64_t)j * ld;
    for (int c = t; c < L; c += T) {
      hs[c] = hrow[c];
      xs[64 + c] = xrow[c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int ew0 = lane0 + T * k;          // first e of this wave
      if (ew0 >= NC) break;
      const int e = t + T * k;
      const int clo = max(0, ew0 - L + 1);
      const int chi = min(L - 1, ew0 + 63);
      double a = acc[k];
      const double* xp = xs + 64 + e;
      for (int c = clo; c <= chi; ++c) a = fma(hs[c], xp[-c], a);
      acc[k] = a;
    }
  }
  __syncthreads();
  int64_t* coef = reinterpret_cast<int64_t*>(smem);
  int64_t* cs = coef + NC;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = t + T * k;
    if (e < NC) coef[e] = (int64_t)acc[k];
  }
  __syncthreads();
  const int row = out_reverse ? (n - 1 - i) : i;
  carry_round_pack_fit(coef, NC, w, P, W, cs, y + (int64_t)row * W, red);
}

size_t school_lds_bytes(int L, int w, int P, int W) {
  const int NC = 2 * L - 1;
  const size_t a = (size_t)(2 * L + 128) * 8;
  const size_t b = (size_t)NC * 8 + (size_t)carry_lds_bytes(kSchoolThreads);
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

hipError_t launch_school_rows(const double* hd, const double* xd, int n, int L, int ld, int w,
                              int P, int W, int out_reverse, uint64_t* y, hipStream_t s) {
  const size_t lds = school_lds_bytes(L, w, P, W);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_school_row,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_school_row, dim3(n), dim3(kSchoolThreads), lds, s, hd, xd, n, L, ld, w, P, W,
                     out_reverse, y);
  return hipGetLastError();
}

}  // namespace hmv
