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
__device__ __forceinline__ int xcd_slot(int b, int grid) {
  // work-groups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous run of indices so neighbours share its L2
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
__global__ void __launch_bounds__(256, 2) k_rows_fwd(const uint64_t* __restrict__ in, int W, int P,
                                                     int w, int L, int count, int gather_n,
                                                     int logM, double2* __restrict__ out,
                                                     int rows_alloc, DevStatus* st) {
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
  // digit e is the real (e even) or imaginary (e odd) part of element e/2
  double* bd = reinterpret_cast<double*>(buf);
  for (int e = L + t; e < 2 * M; e += T) bd[2 * swz(e >> 1) + (e & 1)] = 0.0;
  split_balanced(wd, W, w, L, [&](int e, int d) { bd[2 * swz(e >> 1) + (e & 1)] = (double)d; }, red);
  __syncthreads();
  fft_lds(buf, logM, -1);
  // real-input packing: X[k] = 1/2 (Z[k] + conj Z[M-k]) - i/2 w^k (Z[k] - conj Z[M-k])
  const int rs = kRealTwN / (2 * M);
  for (int k = t; k <= M; k += T) {
    const double2 zk = buf[swz(k & (M - 1))], zm = buf[swz((M - k) & (M - 1))];
    const double2 A = cadd(zk, conj2(zm)), B = csub(zk, conj2(zm));
    const double2 Q = cmul(g_rtw[k * rs], B);
    out[tile_index(k, r, rows_alloc)] = make_double2(0.5 * (A.x + Q.y), 0.5 * (A.y - Q.x));
  }
}

// The index-axis transforms of N_t = 2 Nh points are split by one radix-2
// decimation-in-frequency step into two Nh-point transforms: the even
// frequencies are the transform of a[s] = u[s] + u[s+Nh], the odd ones the
// transform of b[s] = (u[s] - u[s+Nh]) w^s (w = exp(-2 pi i / N_t)).  A
// column of the resident spectrum stores the Nh even bins, then the Nh odd
// bins.  The inverse of the product recombines as
//   y[s] = e[s] + w^-s o[s],   y[s+Nh] = e[s] - w^-s o[s]
// with e, o the two unnormalised Nh-point inverses (one radix-2
// decimation-in-time step).  Each half needs Nh points of LDS, so the
// headline shape (N_t = 8192) runs two work-groups per CU.

// Column pass of the plan: transform each limb-frequency column of h over the
// index axis and store it scaled by 2^-(log N_t + log N_z) (exact), so the
// matvec's unnormalised inverse transforms need no further scaling.
template <int LOGNH>
__global__ void __launch_bounds__(512) k_cols_plan(const double2* __restrict__ H1, int rows,
                                                   int C, double scale,
                                                   double2* __restrict__ Hh) {
  extern __shared__ double2 buf[];
  const int c = xcd_slot(blockIdx.x, gridDim.x);
  if (c >= C) return;
  constexpr int logNt = LOGNH + 1, Nh = 1 << LOGNH;
  constexpr int Ta = Nh >= 16 ? Nh >> 4 : 1, per = Nh >= 16 ? 16 : Nh;
  constexpr int rs = kRealTwN >> logNt;
  const int t = threadIdx.x;
  const bool act = t < Ta;
  const double2* col = H1 + tile_index(c, 0, rows);
  double2* he = Hh + (int64_t)c * (2 * Nh);
  double2* ho = he + Nh;
  double2 v[16];
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (act && j < per) {
        const int s = t + Ta * j;
        const double2 lo = s < rows ? col[(int64_t)s * 8] : make_double2(0.0, 0.0);
        const double2 hi = s + Nh < rows ? col[(int64_t)(s + Nh) * 8] : make_double2(0.0, 0.0);
        v[j] = half == 0 ? cadd(lo, hi) : cmul(csub(lo, hi), g_rtw[s * rs]);
      }
    }
    fft_regs<LOGNH>(v, buf, -1);
    double2* dst = half == 0 ? he : ho;
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (act && j < per) {
        const int f = t + Ta * j;
        dst[f] = make_double2(v[j].x * scale, v[j].y * scale);
      }
  }
}

// Column pass of the matvec: x column reversed (x_hat[s] = x[n-1-s], zero for
// s >= n; n <= Nh so the high half is zero), forward transform, times the
// resident spectrum of h, inverse transform, keep rows n-1 .. 2n-2.
template <int LOGNH>
__global__ void __launch_bounds__(512) k_cols_pass(const double2* __restrict__ X1,
                                                   const double2* __restrict__ Hh, int n, int C,
                                                   double2* __restrict__ Y1) {
  extern __shared__ double2 buf[];
  const int c = xcd_slot(blockIdx.x, gridDim.x);
  if (c >= C) return;
  constexpr int logNt = LOGNH + 1, Nh = 1 << LOGNH;
  constexpr int Ta = Nh >= 16 ? Nh >> 4 : 1, per = Nh >= 16 ? 16 : Nh;
  constexpr int rs = kRealTwN >> logNt;
  const int t = threadIdx.x;
  const bool act = t < Ta;
  const double2* xcol = X1 + tile_index(c, 0, n);
  const double2* he = Hh + (int64_t)c * (2 * Nh);
  const double2* ho = he + Nh;
  double2* ycol = Y1 + tile_index(c, 0, n);
  double2 v[16], e[16];
  // even frequencies
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) {
      const int s = t + Ta * j;
      v[j] = s < n ? xcol[(int64_t)(n - 1 - s) * 8] : make_double2(0.0, 0.0);
    }
  fft_regs<LOGNH>(v, buf, -1);
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) v[j] = cmul(v[j], he[t + Ta * j]);
  fft_regs<LOGNH>(v, buf, +1);
#pragma unroll
  for (int j = 0; j < 16; ++j) e[j] = v[j];
  // odd frequencies
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) {
      const int s = t + Ta * j;
      const double2 xv = s < n ? xcol[(int64_t)(n - 1 - s) * 8] : make_double2(0.0, 0.0);
      v[j] = cmul(xv, g_rtw[s * rs]);
    }
  fft_regs<LOGNH>(v, buf, -1);
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) v[j] = cmul(v[j], ho[t + Ta * j]);
  fft_regs<LOGNH>(v, buf, +1);
  // recombine and keep the window
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) {
      const int s = t + Ta * j;
      const double2 q = cmul(v[j], conj2(g_rtw[s * rs]));
      const int ra = s - (n - 1), rb = s + Nh - (n - 1);
      if (ra >= 0 && ra < n) ycol[(int64_t)ra * 8] = cadd(e[j], q);
      if (rb >= 0 && rb < n) ycol[(int64_t)rb * 8] = csub(e[j], q);
    }
}

// Row pass, inverse: real inverse FFT over the limb axis, round every
// coefficient to its integer, exact carry / round-half-even / pack.  The
// last FFT pass leaves the coefficients in registers, where they are rounded
// and then stored compactly (coefficient e in int64 slot e) at the start of
// the FFT buffer; the carry scratch follows at carry_off.
template <int LOGM>
__global__ void __launch_bounds__(256, 2) k_rows_inv(const double2* __restrict__ Y1, int n, int L,
                                                     int w, int P, int W, int out_reverse,
                                                     int carry_off, uint64_t* __restrict__ y,
                                                     DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  __shared__ double2 ytop;                 // Y[M]
  const int i = blockIdx.x;
  if (i >= n) return;
  constexpr int M = 1 << LOGM;
  constexpr int Ta = M >= 16 ? M >> 4 : 1, per = M >= 16 ? 16 : M;
  constexpr int rs = kRealTwN / (2 * M);
  const int T = blockDim.x, t = threadIdx.x;
  const bool act = t < Ta;
  // packing roots first: independent of the data
  double2 wk[16];
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) wk[j] = conj2(g_rtw[(t + Ta * j) * rs]);
  for (int k = t; k < M; k += T) buf[swz(k)] = Y1[tile_index(k, i, n)];
  if (t == 0) ytop = Y1[tile_index(M, i, n)];
  __syncthreads();
  // Z[k] = (Y[k] + conj Y[M-k]) + i w^-k (Y[k] - conj Y[M-k]),  k < M
  double2 v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) {
      const int k = t + Ta * j;
      const double2 yk = buf[swz(k)];
      const double2 ym = k == 0 ? ytop : buf[swz(M - k)];
      const double2 E = cadd(yk, conj2(ym)), D = csub(yk, conj2(ym));
      const double2 Q = cmul(D, wk[j]);
      v[j] = make_double2(E.x - Q.y, E.y + Q.x);
    }
  __syncthreads();
  fft_regs<LOGM>(v, buf, +1);
  // element m = t + Ta j holds coefficients 2m (real part) and 2m+1 (imaginary)
  int64_t* coef = reinterpret_cast<int64_t*>(buf);
  const int NC = 2 * L - 1;
  double maxerr = 0.0;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (act && j < per) {
      const int m = t + Ta * j;
      const double s0 = rint(v[j].x), s1 = rint(v[j].y);
      maxerr = fmax(maxerr, fmax(fabs(v[j].x - s0), fabs(v[j].y - s1)));
      const int64_t i0 = (int64_t)s0, i1 = (int64_t)s1;
      if (2 * m < NC) coef[2 * m] = i0;
      else if (i0 != 0) bad = 1;
      if (2 * m + 1 < NC) coef[2 * m + 1] = i1;
      else if (i1 != 0) bad = 1;
    }
  for (int o = 32; o > 0; o >>= 1) maxerr = fmax(maxerr, __shfl_xor(maxerr, o, 64));
  if ((t & 63) == 0 && st)
    atomicMax(reinterpret_cast<unsigned long long*>(&st->max_err_bits),
              (unsigned long long)__double_as_longlong(maxerr));
  bad = __syncthreads_or(bad);
  if (bad && t == 0) status_or(st, ST_BOUND);
  uint64_t* sw = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(buf) + carry_off);
  const int NWS = carry_words(NC, w, P, W);
  const int row = out_reverse ? (n - 1 - i) : i;
  carry_round_pack(coef, NC, w, P, W, sw, NWS, y + (int64_t)row * W, red);
}

// ------------------------------------------------------------------ launchers
namespace {
// Row kernels run M/16 threads (at least 64, at most 256: M <= 4096); the
// carry step needs at most kCarryMaxPer words per thread, which holds for
// every admissible (P, w) because the digit count L <= M.
int row_threads(int M, int P, int W, int L, int w) {
  int T = M / 16;
  if (T < 64) T = 64;
  const int NWS = carry_words(2 * L - 1, w, P, W);
  while (T < 256 && (NWS + T - 1) / T > kCarryMaxPer) T += 64;
  return T;
}
int col_threads(int Nt) { return Nt / 32 < 64 ? 64 : Nt / 32; }

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

template <int LOGNH>
hipError_t cols_plan_t(const double2* H1, int rows, int C, double scale, double2* Hh,
                       hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)(1 << LOGNH);
  hipError_t e = set_lds((const void*)k_cols_plan<LOGNH>, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8;
  hipLaunchKernelGGL(k_cols_plan<LOGNH>, dim3(grid), dim3(col_threads(2 << LOGNH)), lds, s, H1,
                     rows, C, scale, Hh);
  return hipGetLastError();
}

template <int LOGNH>
hipError_t cols_pass_t(const double2* X1, const double2* Hh, int n, int C, double2* Y1,
                       hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)(1 << LOGNH);
  hipError_t e = set_lds((const void*)k_cols_pass<LOGNH>, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8;
  hipLaunchKernelGGL(k_cols_pass<LOGNH>, dim3(grid), dim3(col_threads(2 << LOGNH)), lds, s, X1,
                     Hh, n, C, Y1);
  return hipGetLastError();
}

#define HMV_NT_DISPATCH(FN, ...)                  \
  switch (logNt - 1) {                            \
    case 1: return FN<1>(__VA_ARGS__);            \
    case 2: return FN<2>(__VA_ARGS__);            \
    case 3: return FN<3>(__VA_ARGS__);            \
    case 4: return FN<4>(__VA_ARGS__);            \
    case 5: return FN<5>(__VA_ARGS__);            \
    case 6: return FN<6>(__VA_ARGS__);            \
    case 7: return FN<7>(__VA_ARGS__);            \
    case 8: return FN<8>(__VA_ARGS__);            \
    case 9: return FN<9>(__VA_ARGS__);            \
    case 10: return FN<10>(__VA_ARGS__);          \
    case 11: return FN<11>(__VA_ARGS__);          \
    case 12: return FN<12>(__VA_ARGS__);          \
    case 13: return FN<13>(__VA_ARGS__);          \
    default: return hipErrorInvalidValue;         \
  }

hipError_t launch_cols_plan(const double2* H1, int rows, int C, int logNt, double scale,
                            double2* Hh, hipStream_t s) {
  HMV_NT_DISPATCH(cols_plan_t, H1, rows, C, scale, Hh, s)
}

hipError_t launch_cols_pass(const double2* X1, const double2* Hh, int n, int C, int logNt,
                            double2* Y1, hipStream_t s) {
  HMV_NT_DISPATCH(cols_pass_t, X1, Hh, n, C, Y1, s)
}

template <int LOGM>
hipError_t rows_inv_t(const double2* Y1, int n, int L, int w, int P, int W, int out_reverse,
                      uint64_t* y, DevStatus* st, hipStream_t s) {
  constexpr int M = 1 << LOGM;
  const int T = row_threads(M, P, W, L, w);
  const int NC = 2 * L - 1;
  // FFT points during the transform; afterwards NC int64 coefficients then
  // the carry scratch
  const size_t fft_part = sizeof(double2) * (size_t)M;
  const size_t carry_off = ((size_t)NC * 8 + 15) / 16 * 16;
  const size_t carry_part = carry_off + (size_t)carry_lds_bytes(NC, w, P, W);
  const size_t lds = fft_part > carry_part ? fft_part : carry_part;
  hipError_t e = set_lds((const void*)k_rows_inv<LOGM>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rows_inv<LOGM>, dim3(n), dim3(T), lds, s, Y1, n, L, w, P, W, out_reverse,
                     (int)carry_off, y, st);
  return hipGetLastError();
}

hipError_t launch_rows_inv(const double2* Y1, int n, int logM, int L, int w, int P, int W,
                           int out_reverse, uint64_t* y, DevStatus* st, hipStream_t s) {
  switch (logM) {
#define HMV_RI(k) \
  case k: return rows_inv_t<k>(Y1, n, L, w, P, W, out_reverse, y, st, s);
    HMV_RI(1) HMV_RI(2) HMV_RI(3) HMV_RI(4) HMV_RI(5) HMV_RI(6) HMV_RI(7) HMV_RI(8) HMV_RI(9)
    HMV_RI(10) HMV_RI(11) HMV_RI(12)
#undef HMV_RI
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hmv
