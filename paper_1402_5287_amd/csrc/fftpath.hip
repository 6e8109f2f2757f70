// Split-FFT path (Section 3, the decomposition approach, in its exact form).
//
// Every number becomes a polynomial in z = 2^w with balanced limb digits, so
// the Hankel product becomes the bivariate correlation
//     S_i(z) = sum_j H_{i+j}(z) X_j(z),
// an index-axis correlation times a limb-axis linear convolution.  Both run
// as one 2-D binary64 FFT (Section 2: a product with a circulant embedding is
// a componentwise product of transforms), every output coefficient is
// rounded to its integer (exact because the proven error bound is below 1/2)
// and the exact carry step gives y.
//
//   limb axis   real FFT of N_z = 2M points per number, done as an M-point
//               complex FFT plus the real-input packing step
//   index axis  complex FFT of N_t >= 2n-1 points per limb frequency; x is
//               reversed so the correlation becomes a convolution and rows
//               n-1 .. 2n-2 of the cyclic result are exactly S_0 .. S_{n-1}
//
// Spectra between passes live in HBM in column tiles of 8 complex values:
// element (row, k) of a [rows][C] half-plane sits at ((k/8) rows + row) 8 + k%8,
// so a row pass writes and reads whole 128-byte lines and a column pass
// reads one 16-byte slot per line while the 7 neighbouring columns of the
// tile run on the same XCD (column order is remapped per XCD) and hit in its L2.
#include <mutex>
#include <vector>

#include "common.h"
#include "fft.h"
#include "kernels.h"
#include "tables.h"

namespace hmv {

namespace {
std::mutex g_tab_mu;
bool g_tab_ready[64] = {};
double g_beta = -1.0;
std::vector<double> g_tw_host, g_rtw_host;

void ensure_host_tables() {
  if (g_beta < 0.0) {
    g_tw_host.assign(2 * kTwEntries, 0.0);
    g_rtw_host.assign(2 * kRealTwEntries, 0.0);
    g_beta = gen_fft_tables(g_tw_host.data(), g_rtw_host.data());
  }
}
}  // namespace

double fft_twiddle_beta() {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  ensure_host_tables();
  return g_beta;
}

hipError_t fft_tables_init() {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (g_tab_ready[dev]) return hipSuccess;
  ensure_host_tables();
  e = hipMemcpyToSymbol(HIP_SYMBOL(g_tw), g_tw_host.data(), sizeof(double) * g_tw_host.size());
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(g_rtw), g_rtw_host.data(), sizeof(double) * g_rtw_host.size());
  if (e != hipSuccess) return e;
  g_tab_ready[dev] = true;
  return hipSuccess;
}

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int xcd_column(int b, int grid) {
  // work-groups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous run of columns so tile neighbours share its L2
  const int q = grid >> 3;
  return (b & 7) * q + (b >> 3);
}

__device__ __forceinline__ int64_t tile_index(int k, int row, int rows) {
  return ((int64_t)(k >> 3) * rows + row) * 8 + (k & 7);
}

__device__ __forceinline__ int gather_row(int r, int gather_n) {
  if (gather_n <= 0) return r;
  int s = (gather_n - 1 - r) % gather_n;
  return s < 0 ? s + gather_n : s;
}

// ------------------------------------------------------------------ kernels

// Sum of squared balanced digits of every h entry, for each candidate width
// w in [wlo, whi]: the Euclidean limb norm that enters the error bound.
__global__ void __launch_bounds__(256) k_h_norms(const uint64_t* __restrict__ h, int W, int P,
                                                 int rows, int gather_n, int wlo, int whi,
                                                 unsigned long long* __restrict__ norms,
                                                 DevStatus* st) {
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  __shared__ unsigned long long part[4];
  const int r = blockIdx.x;
  if (r >= rows) return;
  const int src = gather_row(r, gather_n);
  for (int q = threadIdx.x; q < W; q += blockDim.x) wd[q] = h[(int64_t)src * W + q];
  __syncthreads();
  if (!number_in_range(wd, W, P) && threadIdx.x == 0) status_or(st, ST_RANGE);
  for (int w = wlo; w <= whi; ++w) {
    const int L = (P + 2 + w - 1) / w;
    unsigned long long acc = 0;
    split_balanced(wd, W, w, L, [&](int, int d) { acc += (unsigned long long)((int64_t)d * d); }, red);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long s = 0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += part[k];
      atomicAdd(&norms[w - wlo], s);
    }
    __syncthreads();
  }
}

// Row pass, forward: split one number into digits, real FFT over the limb
// axis (N_z = 2M real points), write the M+1 non-redundant bins.
__global__ void __launch_bounds__(1024) k_rows_fwd(const uint64_t* __restrict__ in, int W, int P,
                                                   int w, int L, int count, int gather_n, int logM,
                                                   double2* __restrict__ out, int rows_alloc,
                                                   DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  const int r = blockIdx.x;
  if (r >= count) return;
  const int T = blockDim.x, t = threadIdx.x;
  const int M = 1 << logM;
  const int src = gather_row(r, gather_n);
  for (int q = t; q < W; q += T) wd[q] = in[(int64_t)src * W + q];
  __syncthreads();
  if (!number_in_range(wd, W, P) && t == 0) status_or(st, ST_RANGE);
  double* bd = reinterpret_cast<double*>(buf);
  for (int e = L + t; e < 2 * M; e += T) bd[e] = 0.0;
  split_balanced(wd, W, w, L, [&](int e, int d) { bd[e] = (double)d; }, red);
  __syncthreads();
  fft_lds(buf, logM, -1);
  // real-input packing: X[k] = 1/2 (Z[k] + conj Z[M-k]) - i/2 w^k (Z[k] - conj Z[M-k])
  const int rs = kRealTwN / (2 * M);
  for (int k = t; k <= M; k += T) {
    const double2 zk = buf[k & (M - 1)], zm = buf[(M - k) & (M - 1)];
    const double2 A = cadd(zk, conj2(zm)), B = csub(zk, conj2(zm));
    const double2 Q = cmul(g_rtw[k * rs], B);
    out[tile_index(k, r, rows_alloc)] = make_double2(0.5 * (A.x + Q.y), 0.5 * (A.y - Q.x));
  }
}

// Column pass of the plan: transform each limb-frequency column of h over the
// index axis and store it scaled by 2^-(log N_t + log N_z) (exact), so the
// matvec's unnormalised inverse transforms need no further scaling.
__global__ void __launch_bounds__(512) k_cols_plan(const double2* __restrict__ H1, int rows,
                                                   int C, int logNt, double scale,
                                                   double2* __restrict__ Hh) {
  extern __shared__ double2 buf[];
  const int c = xcd_column(blockIdx.x, gridDim.x);
  if (c >= C) return;
  const int T = blockDim.x, t = threadIdx.x, Nt = 1 << logNt;
  const double2* col = H1 + tile_index(c, 0, rows);
  for (int s = t; s < Nt; s += T) buf[s] = s < rows ? col[(int64_t)s * 8] : make_double2(0.0, 0.0);
  __syncthreads();
  fft_lds(buf, logNt, -1);
  double2* dst = Hh + (int64_t)c * Nt;
  for (int f = t; f < Nt; f += T) dst[f] = make_double2(buf[f].x * scale, buf[f].y * scale);
}

// Column pass of the matvec: x column reversed, forward FFT, times the
// resident spectrum of h, inverse FFT, keep rows n-1 .. 2n-2.
__global__ void __launch_bounds__(512) k_cols_pass(const double2* __restrict__ X1,
                                                   const double2* __restrict__ Hh, int n, int C,
                                                   int logNt, double2* __restrict__ Y1) {
  extern __shared__ double2 buf[];
  const int c = xcd_column(blockIdx.x, gridDim.x);
  if (c >= C) return;
  const int T = blockDim.x, t = threadIdx.x, Nt = 1 << logNt;
  const double2* xcol = X1 + tile_index(c, 0, n);
  for (int s = t; s < Nt; s += T)
    buf[s] = s < n ? xcol[(int64_t)(n - 1 - s) * 8] : make_double2(0.0, 0.0);
  __syncthreads();
  fft_lds(buf, logNt, -1);
  const double2* hc = Hh + (int64_t)c * Nt;
  for (int f = t; f < Nt; f += T) buf[f] = cmul(buf[f], hc[f]);
  __syncthreads();
  fft_lds(buf, logNt, +1);
  double2* ycol = Y1 + tile_index(c, 0, n);
  for (int i = t; i < n; i += T) ycol[(int64_t)i * 8] = buf[i + n - 1];
}

// Row pass, inverse: real inverse FFT over the limb axis, round every
// coefficient to its integer, exact carry / round-half-even / pack.
__global__ void __launch_bounds__(1024) k_rows_inv(const double2* __restrict__ Y1, int n, int logM,
                                                   int L, int w, int P, int W, int out_reverse,
                                                   uint64_t* __restrict__ y, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  const int i = blockIdx.x;
  if (i >= n) return;
  const int T = blockDim.x, t = threadIdx.x, M = 1 << logM;
  for (int k = t; k <= M; k += T) buf[k] = Y1[tile_index(k, i, n)];
  __syncthreads();
  // Z[k] = (Y[k] + conj Y[M-k]) + i w^-k (Y[k] - conj Y[M-k]),  k < M
  const int rs = kRealTwN / (2 * M);
  double2 z[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int k = t + a * T;
    if (k < M) {
      const double2 yk = buf[k], ym = buf[M - k];
      const double2 E = cadd(yk, conj2(ym)), D = csub(yk, conj2(ym));
      const double2 Q = cmul(D, conj2(g_rtw[k * rs]));
      z[a] = make_double2(E.x - Q.y, E.y + Q.x);
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int k = t + a * T;
    if (k < M) buf[k] = z[a];
  }
  __syncthreads();
  fft_lds(buf, logM, +1);
  // round to integers in place (double -> int64 in the same slot)
  const double* bd = reinterpret_cast<const double*>(buf);
  int64_t* coef = reinterpret_cast<int64_t*>(buf);
  const int NC = 2 * L - 1;
  double maxerr = 0.0;
  int bad = 0;
  for (int e = t; e < 2 * M; e += T) {
    const double v = bd[e];
    const double s = rint(v);
    maxerr = fmax(maxerr, fabs(v - s));
    const int64_t iv = (int64_t)s;
    if (e >= NC && iv != 0) bad = 1;
    coef[e] = iv;
  }
  for (int o = 32; o > 0; o >>= 1) maxerr = fmax(maxerr, __shfl_xor(maxerr, o, 64));
  if ((t & 63) == 0 && st)
    atomicMax(reinterpret_cast<unsigned long long*>(&st->max_err_bits),
              (unsigned long long)__double_as_longlong(maxerr));
  bad = __syncthreads_or(bad);
  if (bad && t == 0) status_or(st, ST_BOUND);
  uint64_t* sw = reinterpret_cast<uint64_t*>(buf + M + 1);
  const int NWS = carry_words(NC, w, P, W);
  const int row = out_reverse ? (n - 1 - i) : i;
  carry_round_pack(coef, NC, w, P, W, sw, NWS, y + (int64_t)row * W, red);
}

// ------------------------------------------------------------------ launchers
namespace {
int row_threads(int M, int P, int W, int L, int w) {
  int T = M / 16;
  if (T < 64) T = 64;
  const int NWS = carry_words(2 * L - 1, w, P, W);
  while (T < 1024 && (NWS + T - 1) / T > kCarryMaxPer) T += 64;
  return T;
}
int col_threads(int Nt) { return Nt / 16 < 64 ? 64 : Nt / 16; }

// Raise a kernel's dynamic-LDS limit once per (device, kernel, size) so that
// later launches (possibly under stream capture) make no attribute calls.
std::mutex g_lds_mu;
std::vector<std::pair<std::pair<int, const void*>, size_t>> g_lds_set;

hipError_t set_lds(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_lds_mu);
  for (auto& kv : g_lds_set)
    if (kv.first.first == dev && kv.first.second == fn) {
      if (kv.second >= bytes) return hipSuccess;
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e == hipSuccess) kv.second = bytes;
      return e;
    }
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) g_lds_set.push_back({{dev, fn}, bytes});
  return e;
}
}  // namespace

hipError_t launch_h_norms(const uint64_t* h, int W, int P, int rows, int gather_n, int wlo,
                          int whi, unsigned long long* norms, DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_h_norms, dim3(rows), dim3(256), 0, s, h, W, P, rows, gather_n, wlo, whi,
                     norms, st);
  return hipGetLastError();
}

hipError_t launch_rows_fwd(const uint64_t* in, int W, int P, int w, int L, int count,
                           int gather_n, int logM, double2* out, int rows_alloc, DevStatus* st,
                           hipStream_t s) {
  const int M = 1 << logM;
  const int T = row_threads(M, P, W, L, w);
  const size_t lds = sizeof(double2) * (size_t)M;
  hipError_t e = set_lds((const void*)k_rows_fwd, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rows_fwd, dim3(count), dim3(T), lds, s, in, W, P, w, L, count, gather_n,
                     logM, out, rows_alloc, st);
  return hipGetLastError();
}

hipError_t launch_cols_plan(const double2* H1, int rows, int C, int logNt, double scale,
                            double2* Hh, hipStream_t s) {
  const int Nt = 1 << logNt;
  const size_t lds = sizeof(double2) * (size_t)Nt;
  hipError_t e = set_lds((const void*)k_cols_plan, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8;
  hipLaunchKernelGGL(k_cols_plan, dim3(grid), dim3(col_threads(Nt)), lds, s, H1, rows, C, logNt,
                     scale, Hh);
  return hipGetLastError();
}

hipError_t launch_cols_pass(const double2* X1, const double2* Hh, int n, int C, int logNt,
                            double2* Y1, hipStream_t s) {
  const int Nt = 1 << logNt;
  const size_t lds = sizeof(double2) * (size_t)Nt;
  hipError_t e = set_lds((const void*)k_cols_pass, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8;
  hipLaunchKernelGGL(k_cols_pass, dim3(grid), dim3(col_threads(Nt)), lds, s, X1, Hh, n, C, logNt,
                     Y1);
  return hipGetLastError();
}

hipError_t launch_rows_inv(const double2* Y1, int n, int logM, int L, int w, int P, int W,
                           int out_reverse, uint64_t* y, DevStatus* st, hipStream_t s) {
  const int M = 1 << logM;
  const int T = row_threads(M, P, W, L, w);
  const int NWS = carry_words(2 * L - 1, w, P, W);
  const size_t lds = sizeof(double2) * (size_t)(M + 1) + 8 * (size_t)NWS;
  hipError_t e = set_lds((const void*)k_rows_inv, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rows_inv, dim3(n), dim3(T), lds, s, Y1, n, logM, L, w, P, W, out_reverse,
                     y, st);
  return hipGetLastError();
}

}  // namespace hmv
