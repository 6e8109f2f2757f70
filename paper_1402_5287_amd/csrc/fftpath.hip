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
// Spectra between passes live in HBM in column tiles of TW complex values:
// element (row, k) of a [rows][C] half-plane sits at ((k/TW) rows + row) TW +
// k%TW (a row pass writes or reads 16 TW contiguous bytes of a row per tile, a
// column pass reads one 16-byte slot of them while the TW - 1 neighbouring
// columns of the tile run on the same XCD, column order being remapped per
// XCD, and hit in its L2).  TW = 2^lt is a run-time choice per plan, picked
// for the spectra of x and of y separately by the planner's timing runs.
#include <hip/hip_cooperative_groups.h>

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
std::vector<double> g_tw_host, g_rtw_host, g_rtw2_host, g_r3_host;

void ensure_host_tables() {
  if (g_beta < 0.0) {
    g_tw_host.assign(2 * kTwEntries, 0.0);
    g_rtw_host.assign(2 * kRealTwEntries, 0.0);
    g_r3_host.assign(2 * kR3Entries, 0.0);
    g_beta = gen_fft_tables(g_tw_host.data(), g_rtw_host.data(), g_r3_host.data());
    g_rtw2_host.assign(2 * kRealTwEntries2, 0.0);
    for (int64_t k = 0; k < kRealTwEntries2; ++k) {
      g_rtw2_host[2 * k] = g_rtw_host[4 * k];
      g_rtw2_host[2 * k + 1] = g_rtw_host[4 * k + 1];
    }
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
  e = hipMemcpyToSymbol(HIP_SYMBOL(g_rtw2), g_rtw2_host.data(),
                        sizeof(double) * g_rtw2_host.size());
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(g_r3tw), g_r3_host.data(), sizeof(double) * g_r3_host.size());
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

// Spectra of rows are stored in tiles of TW = 2^lt bins: bin k of row `row`
// at ((k / TW) rows + row) TW + k % TW.  The row passes touch TW contiguous
// bins per row, the index-axis pass reads a bin column at stride TW.
__device__ __forceinline__ int64_t tidx(int k, int row, int rows, int lt) {
  return ((((int64_t)(k >> lt)) * rows + row) << lt) + (k & ((1 << lt) - 1));
}
__device__ __forceinline__ int64_t tile_index(int k, int row, int rows) {
  return ((int64_t)(k >> 3) * rows + row) * 8 + (k & 7);
}

// Output row of spectrum row i: with rev_block = 0 the same row, otherwise
// reversed within its block of rev_block rows (the Toeplitz and circulant
// outputs of one vector are its Hankel rows in reverse order; a block of
// vectors stacks them).
__device__ __forceinline__ int out_row(int i, int rev_block) {
  if (rev_block <= 0) return i;
  const int q = i / rev_block;
  return q * rev_block + (rev_block - 1 - (i - q * rev_block));
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
  load_words(h + (int64_t)src * W, W, wd);
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

// Real-input packing of the M-point transform Z held in buf (the limb
// sequence as M complex points) into the M + 1 bins of the real transform,
//   X[k] = 1/2 (Z[k] + conj Z[M-k]) - i/2 w^k (Z[k] - conj Z[M-k]),
// stored to row r of the tiled spectrum.  A thread's root loads are issued
// eight at a time so that they are in flight together.
// Stored in tiles of 2^lt bins (tidx).
// PACK0: bins 0 and M, both real, share column 0 as X[0] + i X[M] (columns
// 0 .. M-1 are written); otherwise bins 0 .. M go to columns 0 .. M.
template <bool PACK0 = false>
__device__ inline void pack_real_row(const double2* buf, int M, double2* __restrict__ out, int r,
                                     int rows_alloc, int lt) {
  const int T = blockDim.x, t = threadIdx.x;
  const int rs = kRealTwN / (2 * M);
  for (int k0 = t; k0 <= M; k0 += 8 * T) {
    double2 wv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u * T;
      wv[u] = real_root(k <= M ? k : M, rs);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u * T;
      if (k <= M) {
        const double2 zk = buf[lds_slot(k & (M - 1))], zm = buf[lds_slot((M - k) & (M - 1))];
        const double2 A = cadd(zk, conj2(zm)), B = csub(zk, conj2(zm));
        const double2 Q = cmul(wv[u], B);
        const int64_t o = tidx(k, r, rows_alloc, lt);
        if constexpr (PACK0) {
          // X[0] = Z[0].re + Z[0].im, X[M] = Z[0].re - Z[0].im
          if (k == 0) out[o] = make_double2(zk.x + zk.y, zk.x - zk.y);
          else if (k < M) out[o] = make_double2(0.5 * (A.x + Q.y), 0.5 * (A.y - Q.x));
        } else {
          out[o] = make_double2(0.5 * (A.x + Q.y), 0.5 * (A.y - Q.x));
        }
      }
    }
  }
}

// Row pass, forward: split one number into digits, real FFT over the limb
// axis (N_z = 2M real points), write the M+1 non-redundant bins.
template <int LOGM>
__global__ void __launch_bounds__(256, 2) k_rows_fwd(const uint64_t* __restrict__ in, int W, int P,
                                                     int w, int L, int count, int gather_n,
                                                     double2* __restrict__ out, int rows_alloc,
                                                     int pack, int lt, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  // rows grouped per XCD: the rows that share the lines of a bin column are
  // written through one L2
  const int r = xcd_slot(blockIdx.x, gridDim.x);
  if (r >= count) return;
  const int T = blockDim.x, t = threadIdx.x;
  constexpr int M = 1 << LOGM;
  // digit e is the real (e even) or imaginary (e odd) part of element e/2;
  // the elements past the digits are zero (and the imaginary half of the
  // last one when L is odd), written while the words are in flight
  double* bd = reinterpret_cast<double*>(buf);
  __shared__ uint32_t rf[2];
  range_flags_init(rf);
  load_words_then(in + (int64_t)gather_row(r, gather_n) * W, W, wd, [&] {
    for (int k = (L + 1) / 2 + t; k < M; k += T) buf[lds_slot(k)] = make_double2(0.0, 0.0);
    if ((L & 1) && t == 0) bd[2 * lds_slot(L >> 1) + 1] = 0.0;
  });
  __syncthreads();
  // range check by every wave, read back after the split's barriers
  range_check_block(wd, W, P, rf);
  split_balanced(wd, W, w, L, [&](int e, int d) { bd[2 * lds_slot(e >> 1) + (e & 1)] = (double)d; }, red);
  __syncthreads();
  if (t == 0 && !range_flags_ok(rf)) status_or(st, ST_RANGE);
  fft_lds_t<LOGM>(buf, -1);
  if (pack) pack_real_row<true>(buf, M, out, r, rows_alloc, lt);
  else pack_real_row<false>(buf, M, out, r, rows_alloc, lt);
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

// Column 0 of the row spectra packs the two real bins of the limb axis (bin 0
// and the last bin of the Hermitian half), c = a + i b with a, b real
// columns.  Its index-axis transform U = A + i B gives the two spectra back
// through the partner bin U*[k] = conj U[N_t - k]:
//   A = (U + U*) / 2,   i B = (U - U*) / 2,
// and the product the matvec needs, A Ha + i (B Hb), keeps its two parts
// apart (the inverse of each is real):
//   V = (U + U*) Ha' + (U - U*) Hb',   Ha' = Ha / 2,  Hb' = Hb / 2,
// with Ha' in the resident column 0 and Hb' in the extra column C.  Partner
// bins inside the even / odd halves: k <-> (Nh - k) mod Nh (even),
// k <-> Nh - 1 - k (odd).  The real bins of the power-of-two form and of the
// 3K form are both packed this way when the plan's error bound allows it
// (pack = 1): a spectrum then has N_z / 2 columns, otherwise N_z / 2 + 1.

// Column pass of the plan: transform each limb-frequency column of h over the
// index axis and store it scaled by 1 / (N_t N_z) (exact for a power-of-two
// N_z, one rounding of 1/3 otherwise), so the matvec's unnormalised inverse
// transforms need no further scaling.  Packed: column 0 stores Ha' and Hb'
// (above).
template <int LOGNH>
__global__ void __launch_bounds__(512) k_cols_plan(const double2* __restrict__ H1, int rows,
                                                   int C, double scale, int pack, int lt,
                                                   double2* __restrict__ Hh) {
  extern __shared__ double2 buf[];
  const int c = xcd_slot(blockIdx.x, gridDim.x);
  if (c >= C) return;
  constexpr int logNt = LOGNH + 1, Nh = 1 << LOGNH;
  constexpr int Ta = Nh >= 16 ? Nh >> 4 : 1, per = Nh >= 16 ? 16 : Nh;
  constexpr int rs = kRealTwN >> logNt;
  const int t = threadIdx.x;
  const bool act = t < Ta;
  const double2* col = H1 + tidx(c, 0, rows, lt);       // bin column, stride 2^lt
  double2* he = Hh + (int64_t)c * (2 * Nh);
  double2* ho = he + Nh;
  double2 v[16];
  for (int half = 0; half < 2; ++half) {
    // one guarded block per loop (not one per element), with clamped
    // in-bounds addresses, so that all loads are in flight together
    if (act) {
#pragma unroll
      for (int j = 0; j < per; ++j) {
        const int s = t + Ta * j;
        const double2 lo = col[(int64_t)(s < rows ? s : 0) << lt];
        const double2 hi = col[(int64_t)(s + Nh < rows ? s + Nh : 0) << lt];
        const double2 l = s < rows ? lo : make_double2(0.0, 0.0);
        const double2 u = s + Nh < rows ? hi : make_double2(0.0, 0.0);
        v[j] = half == 0 ? cadd(l, u) : cmul(csub(l, u), real_root(s, rs));
      }
    }
    fft_regs<LOGNH>(v, buf, -1);
    double2* dst = half == 0 ? he : ho;
    if (pack && c == 0) {
      // Ha = (Hc + Hc*) / 2, Hb = -i (Hc - Hc*) / 2; stored halved and scaled
      if (act) {
#pragma unroll
        for (int j = 0; j < per; ++j) buf[lds_slot(t + Ta * j)] = v[j];
      }
      __syncthreads();
      double2* dstb = Hh + (int64_t)C * (2 * Nh) + (half == 0 ? 0 : Nh);
      const double q = 0.25 * scale;
      if (act) {
#pragma unroll
        for (int j = 0; j < per; ++j) {
          const int k = t + Ta * j;
          const int kp = half == 0 ? (Nh - k) & (Nh - 1) : Nh - 1 - k;
          const double2 pc = conj2(buf[lds_slot(kp)]);
          const double2 sa = cadd(v[j], pc), sb = csub(v[j], pc);
          dst[k] = make_double2(sa.x * q, sa.y * q);
          dstb[k] = make_double2(sb.y * q, -sb.x * q);
        }
      }
      __syncthreads();
    } else if (act) {
#pragma unroll
      for (int j = 0; j < per; ++j)
        dst[t + Ta * j] = make_double2(v[j].x * scale, v[j].y * scale);
    }
  }
}

// The product of the packed column 0 in one half (odd = 0 even bins, 1 odd
// bins): v[j] = (U + U*) Ha' + (U - U*) Hb' at bin k = t + Ta j, the partner
// bins exchanged through LDS.  Every thread of the block calls it.
template <int R>
__device__ __forceinline__ void packed_product(double2* v, double2* buf, const double2* ha,
                                               const double2* hb, int Nh, int odd, int Ta,
                                               int per) {
  const int t = threadIdx.x;
  const bool act = t < Ta;
  if (act) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (j < per) buf[lds_slot(t + Ta * j)] = v[j];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j < per) {
        const int k = t + Ta * j;
        const int kp = odd ? Nh - 1 - k : (Nh - k) & (Nh - 1);
        const double2 pc = conj2(buf[lds_slot(kp)]);
        v[j] = cadd(cmul(cadd(v[j], pc), ha[k]), cmul(csub(v[j], pc), hb[k]));
      }
    }
  }
  __syncthreads();
}

// Column pass of the matvec: x column reversed (x_hat[s] = x[n-1-s], zero for
// s >= n; n <= Nh so the high half is zero), forward transform, times the
// resident spectrum of h, inverse transform, keep rows n-1 .. 2n-2.
// Variants (picked per shape by the planner's tuning runs): R = elements per
// thread of the register-resident transforms (16, or 8 with twice the
// threads and at most 128 VGPRs so that four waves fit per SIMD; the radix-8
// form reloads the column for the odd half instead of keeping it), and the
// column order (XCD-grouped or linear).
//
// A block of kvec vectors (spectrum rows v n .. v n + n - 1 of X1 and Y1 for
// vector v) runs as kvec work-groups per column.  The kvec work-groups of a
// column take consecutive dispatch slots of one XCD, so they run side by
// side and read the same resident column through one L2: the spectrum of h
// crosses HBM about once per column instead of once per vector.
template <int LOGNH, int R>
__global__ void __launch_bounds__(512, (R == 8 ? 4 : 2)) k_cols_pass(
    const double2* __restrict__ X1, const double2* __restrict__ Hh, int n, int C, int linear,
    int pack, int kvec, int ltx, int lty, double2* __restrict__ Y1) {
  extern __shared__ double2 buf[];
  // block b: vector (b / 8) mod kvec, column slot 8 ((b / 8) / kvec) + b mod 8
  const int bq = (int)blockIdx.x >> 3;
  const int vec = bq % kvec;
  const int bc = ((bq / kvec) << 3) | ((int)blockIdx.x & 7);
  const int c = linear ? bc : xcd_slot(bc, (int)gridDim.x / kvec);
  if (c >= C) return;
  constexpr int logNt = LOGNH + 1, Nh = 1 << LOGNH;
  constexpr int Ta = Nh >= R ? Nh / R : 1, per = Nh >= R ? R : Nh;
  constexpr int rs = kRealTwN >> logNt;
  const int t = threadIdx.x;
  const bool act = t < Ta;
  const int rows = kvec * n;
  const bool packed = pack && c == 0;                // uniform
  // bin column of x, stride 2^ltx
  const double2* xcol = X1 + tidx(c, vec * n, rows, ltx);
  const double2* he = Hh + (int64_t)c * (2 * Nh);
  const double2* ho = he + Nh;
  double2* ycol = Y1 + tidx(c, vec * n, rows, lty);
  // Every per-element loop sits in one guarded block with in-bounds
  // (clamped) addresses, so its loads are issued together rather than one
  // round trip per element.  With R = 16 the column is read from HBM once:
  // v carries the even half, o keeps the input for the odd half (its
  // registers are live in the odd half anyway).
  double2 v[R], o[R];
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int s = t + Ta * j;
      const double2 xv = xcol[(int64_t)(s < n ? n - 1 - s : 0) << ltx];
      v[j] = s < n ? xv : make_double2(0.0, 0.0);
      if constexpr (R == 16) o[j] = v[j];
    }
  }
  // even frequencies
  fft_regs_r<LOGNH, R>(v, buf, -1);
  if (packed) {
    packed_product<R>(v, buf, he, Hh + (int64_t)C * (2 * Nh), Nh, 0, Ta, per);
  } else if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) v[j] = cmul(v[j], he[t + Ta * j]);
  }
  fft_regs_r<LOGNH, R>(v, buf, +1);
  // odd frequencies
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int s = t + Ta * j;
      if constexpr (R != 16) {
        const double2 xv = xcol[(int64_t)(s < n ? n - 1 - s : 0) << ltx];
        o[j] = s < n ? xv : make_double2(0.0, 0.0);
      }
      o[j] = cmul(o[j], real_root(s, rs));
    }
  }
  fft_regs_r<LOGNH, R>(o, buf, -1);
  if (packed) {
    packed_product<R>(o, buf, ho, Hh + (int64_t)C * (2 * Nh) + Nh, Nh, 1, Ta, per);
  } else if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) o[j] = cmul(o[j], ho[t + Ta * j]);
  }
  fft_regs_r<LOGNH, R>(o, buf, +1);
  // recombine and keep the window
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int s = t + Ta * j;
      const double2 q = cmul(o[j], conj2(real_root(s, rs)));
      const int ra = s - (n - 1), rb = s + Nh - (n - 1);
      if (ra >= 0 && ra < n) ycol[(int64_t)ra << lty] = cadd(v[j], q);
      if (rb >= 0 && rb < n) ycol[(int64_t)rb << lty] = csub(v[j], q);
    }
  }
}

// Row pass, inverse: real inverse FFT over the limb axis, round every
// coefficient to its integer, exact carry / round-half-even / pack.  The
// last FFT pass leaves the coefficients in registers, where they are rounded
// and then stored compactly (coefficient e in int64 slot e) at the start of
// the FFT buffer; the carry scratch follows at carry_off.
// R = elements per thread of the inverse transform (16, or 8 with twice the
// threads at four waves per SIMD), picked per shape by the tuning runs.
template <int LOGM, int R>
__global__ void __launch_bounds__(512, (R == 8 ? 4 : 2)) k_rows_inv(
    const double2* __restrict__ Y1, int n, int L, int w, int P, int W, int out_reverse,
    int carry_off, int pack, int lt, uint64_t* __restrict__ y, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  __shared__ RowStatus rst;
  __shared__ double2 ytop;                 // Y[M] (packed: the imaginary part of column 0)
  // rows grouped per XCD: consecutive rows share the lines of a Y1 tile
  const int i = xcd_slot(blockIdx.x, gridDim.x);
  if (i >= n) return;
  row_status_init(&rst);
  constexpr int M = 1 << LOGM;
  constexpr int Ta = M >= R ? M / R : 1, per = M >= R ? R : M;
  constexpr int rs = kRealTwN / (2 * M);
  const int t = threadIdx.x;
  const bool act = t < Ta;
  // the row and the packing roots, all loads in flight together (one
  // guarded block; element k = t + Ta j covers every k < M)
  double2 wk[R], v[R];
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int k = t + Ta * j;
      v[j] = Y1[tidx(k, i, n, lt)];
      wk[j] = conj2(real_root(k, rs));
    }
    // packed: column 0 holds Y[0] + i Y[M] (both real); otherwise Y[M] is
    // column M
    if (t == 0) {
      if (pack) {
        ytop = make_double2(v[0].y, 0.0);
        v[0] = make_double2(v[0].x, 0.0);
      } else {
        ytop = Y1[tidx(M, i, n, lt)];
      }
    }
#pragma unroll
    for (int j = 0; j < per; ++j) buf[lds_slot(t + Ta * j)] = v[j];
  }
  __syncthreads();
  // Z[k] = (Y[k] + conj Y[M-k]) + i w^-k (Y[k] - conj Y[M-k]),  k < M
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int k = t + Ta * j;
      const double2 yk = v[j];
      const double2 ym = k == 0 ? ytop : buf[lds_slot(M - k)];
      const double2 E = cadd(yk, conj2(ym)), D = csub(yk, conj2(ym));
      const double2 Q = cmul(D, wk[j]);
      v[j] = make_double2(E.x - Q.y, E.y + Q.x);
    }
  }
  __syncthreads();
  fft_regs_r<LOGM, R>(v, buf, +1);
  // element m = t + Ta j holds coefficients 2m (real part) and 2m+1 (imaginary)
  int64_t* coef = reinterpret_cast<int64_t*>(buf);
  const int NC = 2 * L - 1;
  double maxerr = 0.0;
  int bad = 0;
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int m = t + Ta * j;
      double r0, r1;
      const int64_t i0 = round_to_int(v[j].x, &r0), i1 = round_to_int(v[j].y, &r1);
      maxerr = fmax(maxerr, fmax(fabs(v[j].x - r0), fabs(v[j].y - r1)));
      // every true coefficient is below 2^50 in magnitude (plan constraint)
      if (fabs(v[j].x) >= kCoefLimit || fabs(v[j].y) >= kCoefLimit) bad = 1;
      // one 16-byte store per pair; for odd NC the pair's second slot at NC
      // lies in the padding before the carry scratch
      if (2 * m < NC) *reinterpret_cast<longlong2*>(coef + 2 * m) = make_longlong2(i0, i1);
      else if (i0 != 0) bad = 1;
      if (2 * m + 1 >= NC && i1 != 0) bad = 1;
    }
  }
  row_status_publish(&rst, maxerr, bad, st);
  int64_t* cs = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(buf) + carry_off);
  const int row = out_row(i, out_reverse);
  carry_round_pack_fit(coef, NC, w, P, W, cs, y + (int64_t)row * W, red);
}

// ------------------------------------------------------------------ 3K-point limb transforms
// Limb transforms of N_z = 3K real points (K = 2^LOGK) where 3K is the
// smallest admissible size (2L - 1 <= 3K < 2^ceil(log2(2L - 1))).  One
// radix-3 decimation-in-frequency step splits the transform of x (x[e] = 0
// for e >= L) into two K-point transforms, with w = exp(-2 pi i / 3K) and
// r = exp(-2 pi i / 3):
//   bin 3m   = sum_s w^(3ms) u0[s],  u0[s] = x[s] + x[s+K] + x[s+2K]      (real)
//   bin 3m+1 = sum_s w^(3ms) u1[s],  u1[s] = w^s (x[s] + r x[s+K] + r^2 x[s+2K])
// and bin 3m+2 = conj(bin 3(K-1-m)+1) for real x.  A row stores the K/2 + 1
// bins 3m (m <= K/2, the Hermitian half of the real K-point transform) and
// then the K bins 3m+1: N_z/2 + 1 columns, or N_z/2 when the real bins 0 and
// 3(K/2) share column 0 (pack), as for a power-of-two N_z.  Each limb
// frequency is one column of the 2-D transform.
// The inverse, with z0, z1 the unnormalised inverse K-point transforms of the
// bins 3m and 3m+1 and v[s] = w^-s z1[s]:
//   N_z x[s + jK] = z0[s] + 2 Re(r^-j v[s]),   j = 0, 1, 2
// i.e. z0 + 2 v.re,  z0 - v.re - sqrt3 v.im,  z0 - v.re + sqrt3 v.im.
// The real K-point transform runs as a K/2-point complex one plus the packing
// step; the K/2- and K-point transforms run together (fft_pair_lds).
__host__ __device__ constexpr int rows3_threads(int K) { return K / 8 < 64 ? 64 : K / 8; }

// One row of the forward pass (row r of `in`, spectrum row r of `out` in
// tiles of 2^lt columns); blockDim.x = rows3_threads(K).
template <int LOGK>
__device__ __forceinline__ void row_fwd3(const uint64_t* __restrict__ in, int W, int P, int w,
                                         int L, int gather_n, double2* __restrict__ out,
                                         int rows_alloc, int r, int pack, int lt, double2* buf,
                                         uint32_t* red, DevStatus* st) {
  constexpr int K = 1 << LOGK, KA = K / 2, T = rows3_threads(K), S = K / T;
  const int t = threadIdx.x;
  // the L digits (digit e in double 2 lds_slot(e/2) + e%2, the padded
  // layout), then the W words, share the transform buffer (L <= (3K+1)/2 and
  // W < L / 3 + 2: at most about 17 K of its 25.5 K bytes), which keeps the
  // work-group's LDS small enough for three per CU
  double* dig = reinterpret_cast<double*>(buf);
  uint64_t* wd = reinterpret_cast<uint64_t*>(buf + lds_points((L + 1) / 2));
  double2* bufA = buf;                              // K/2 points
  double2* bufB = buf + lds_points(KA);             // K points
  __shared__ uint32_t rf[2];
  range_flags_init(rf);
  load_words(in + (int64_t)gather_row(r, gather_n) * W, W, wd);
  __syncthreads();
  // range check by every wave, read back after the split's barriers
  range_check_block(wd, W, P, rf);
  split_balanced(wd, W, w, L, [&](int e, int d) { dig[2 * lds_slot(e >> 1) + (e & 1)] = (double)d; },
                 red);
  __syncthreads();
  if (t == 0 && !range_flags_ok(rf)) status_or(st, ST_RANGE);
  // radix-3 step: u0 exact (digit sums), u1 with one constant and one
  // tabulated root
  double u0[S];
  double2 u1[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int s = t + T * j;
    auto digit = [&](int e) { return e < L ? dig[2 * lds_slot(e >> 1) + (e & 1)] : 0.0; };
    const double a = digit(s), b = digit(s + K), c = digit(s + 2 * K);
    u0[j] = a + b + c;
    u1[j] = cmul(make_double2(a - 0.5 * (b + c), kSqrt3h * (c - b)), r3_root<LOGK>(s));
  }
  __syncthreads();
  double* bdA = reinterpret_cast<double*>(bufA);
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int s = t + T * j;
    bdA[2 * lds_slot(s >> 1) + (s & 1)] = u0[j];
    bufB[lds_slot(s)] = u1[j];
  }
  __syncthreads();
  fft_pair_lds<LOGK - 1, LOGK, T>(bufA, bufB, -1);
  if (pack) pack_real_row<true>(bufA, KA, out, r, rows_alloc, lt);
  else pack_real_row<false>(bufA, KA, out, r, rows_alloc, lt);
  const int b0 = pack ? KA : KA + 1;           // first column of the bins 3m+1
  for (int m = t; m < K; m += T) out[tidx(b0 + m, r, rows_alloc, lt)] = bufB[lds_slot(m)];
}

template <int LOGK>
__global__ void __launch_bounds__(256) k_rows_fwd3(const uint64_t* __restrict__ in, int W, int P,
                                                   int w, int L, int count, int gather_n,
                                                   double2* __restrict__ out, int rows_alloc,
                                                   int pack, int lt, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  const int r = xcd_slot(blockIdx.x, gridDim.x);
  if (r >= count) return;
  row_fwd3<LOGK>(in, W, P, w, L, gather_n, out, rows_alloc, r, pack, lt, buf, red, st);
}

// One row of the inverse pass (spectrum row i of the n rows of Y1 in tiles
// of 2^lt columns; output row out_row(i, out_reverse)); blockDim.x =
// rows3_threads(K).
template <int LOGK>
__device__ __forceinline__ void row_inv3(const double2* __restrict__ Y1, int n, int L, int w,
                                         int P, int W, int out_reverse, int carry_off, int pack,
                                         int lt, uint64_t* __restrict__ y, int i, double2* buf,
                                         uint32_t* red, DevStatus* st) {
  __shared__ RowStatus rst;
  __shared__ double2 ytop;                 // bin 3(K/2) (packed: the imaginary part of column 0)
  row_status_init(&rst);
  constexpr int K = 1 << LOGK, KA = K / 2, T = rows3_threads(K), S = K / T;
  constexpr int SA = KA >= T ? KA / T : 1;
  constexpr int rs = kRealTwN / K;         // packing roots of order K
  const int t = threadIdx.x;
  double2* bufA = buf;
  double2* bufB = buf + lds_points(KA);
  // the row: bins 3m in columns 0 .. K/2-1 (packed: column 0 = bin 0 + i
  // bin 3(K/2); otherwise bin 3(K/2) in column K/2), then the bins 3m+1, all
  // loads in flight together
  {
    const int b0 = pack ? KA : KA + 1;
    double2 va[SA], vb[S];
#pragma unroll
    for (int j = 0; j < SA; ++j) {
      const int k = t + T * j;
      va[j] = Y1[tidx(k < KA ? k : 0, i, n, lt)];
    }
#pragma unroll
    for (int j = 0; j < S; ++j) vb[j] = Y1[tidx(b0 + t + T * j, i, n, lt)];
    if (t == 0) {
      if (pack) {
        ytop = make_double2(va[0].y, 0.0);
        va[0] = make_double2(va[0].x, 0.0);
      } else {
        ytop = Y1[tidx(KA, i, n, lt)];
      }
    }
#pragma unroll
    for (int j = 0; j < SA; ++j) {
      const int k = t + T * j;
      if (k < KA) bufA[lds_slot(k)] = va[j];
    }
#pragma unroll
    for (int j = 0; j < S; ++j) bufB[lds_slot(t + T * j)] = vb[j];
  }
  __syncthreads();
  // unpacking step of the real K-point inverse:
  // Z[k] = (Y[k] + conj Y[K/2-k]) + i w_K^-k (Y[k] - conj Y[K/2-k]),  k < K/2
  {
    double2 za[SA];
#pragma unroll
    for (int j = 0; j < SA; ++j) {
      const int k = t + T * j;
      if (k < KA) {
        const double2 yk = bufA[lds_slot(k)];
        const double2 ym = k == 0 ? ytop : bufA[lds_slot(KA - k)];
        const double2 E = cadd(yk, conj2(ym)), D = csub(yk, conj2(ym));
        const double2 Q = cmul(D, conj2(real_root(k, rs)));
        za[j] = make_double2(E.x - Q.y, E.y + Q.x);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SA; ++j) {
      const int k = t + T * j;
      if (k < KA) bufA[lds_slot(k)] = za[j];
    }
  }
  __syncthreads();
  fft_pair_lds<LOGK - 1, LOGK, T>(bufA, bufB, +1);
  // recombine, round every coefficient to its integer
  const int NC = 2 * L - 1;
  const double* bdA = reinterpret_cast<const double*>(bufA);
  int64_t iv[S][3];
  double maxerr = 0.0;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int s = t + T * j;
    const double z0 = bdA[2 * lds_slot(s >> 1) + (s & 1)];
    const double2 v = cmul(bufB[lds_slot(s)], conj2(r3_root<LOGK>(s)));
    const double c[3] = {z0 + 2.0 * v.x, (z0 - v.x) - kSqrt3 * v.y, (z0 - v.x) + kSqrt3 * v.y};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double rr;
      iv[j][q] = round_to_int(c[q], &rr);
      maxerr = fmax(maxerr, fabs(c[q] - rr));
      // every true coefficient is below 2^50 in magnitude (plan constraint)
      if (fabs(c[q]) >= kCoefLimit) bad = 1;
    }
  }
  __syncthreads();
  int64_t* coef = reinterpret_cast<int64_t*>(buf);
#pragma unroll
  for (int j = 0; j < S; ++j) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int e = t + T * j + q * K;
      if (e < NC) coef[e] = iv[j][q];
      else if (iv[j][q] != 0) bad = 1;
    }
  }
  row_status_publish(&rst, maxerr, bad, st);
  int64_t* cs = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(buf) + carry_off);
  const int row = out_row(i, out_reverse);
  carry_round_pack_fit(coef, NC, w, P, W, cs, y + (int64_t)row * W, red);
}

template <int LOGK>
__global__ void __launch_bounds__(256) k_rows_inv3(const double2* __restrict__ Y1, int n, int L,
                                                   int w, int P, int W, int out_reverse,
                                                   int carry_off, int pack, int lt,
                                                   uint64_t* __restrict__ y, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  const int i = xcd_slot(blockIdx.x, gridDim.x);
  if (i >= n) return;
  row_inv3<LOGK>(Y1, n, L, w, P, W, out_reverse, carry_off, pack, lt, y, i, buf, red, st);
}

// ------------------------------------------------------------------ launchers
namespace {
// Work-group size of an N-point transform with R elements per thread: N/R
// threads, at least 64.
int fft_threads(int N, int R) { return N / R < 64 ? 64 : N / R; }
// The radix-8 variants exist for 8^k points.
constexpr bool has_radix8(int logn) { return logn == 6 || logn == 9 || logn == 12; }

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

template <int LOGM>
hipError_t rows_fwd_t(const uint64_t* in, int W, int P, int w, int L, int count, int gather_n,
                      double2* out, int rows_alloc, int pack, int lt, DevStatus* st,
                      hipStream_t s) {
  constexpr int M = 1 << LOGM;
  const int T = fft_threads(M, 16);           // the LDS transform needs N/16 threads
  const size_t lds = sizeof(double2) * (size_t)lds_points(M);
  hipError_t e = set_lds((const void*)k_rows_fwd<LOGM>, lds);
  if (e != hipSuccess) return e;
  const int grid = (count + 7) / 8 * 8;         // xcd_slot needs a multiple of 8
  hipLaunchKernelGGL(k_rows_fwd<LOGM>, dim3(grid), dim3(T), lds, s, in, W, P, w, L, count,
                     gather_n, out, rows_alloc, pack, lt, st);
  return hipGetLastError();
}

hipError_t launch_rows_fwd(const uint64_t* in, int W, int P, int w, int L, int count,
                           int gather_n, int logM, double2* out, int rows_alloc, int pack, int lt,
                           DevStatus* st, hipStream_t s) {
  switch (logM) {
#define HMV_RF(k) \
  case k:         \
    return rows_fwd_t<k>(in, W, P, w, L, count, gather_n, out, rows_alloc, pack, lt, st, s);
    HMV_RF(1) HMV_RF(2) HMV_RF(3) HMV_RF(4) HMV_RF(5) HMV_RF(6) HMV_RF(7) HMV_RF(8) HMV_RF(9)
    HMV_RF(10) HMV_RF(11) HMV_RF(12)
#undef HMV_RF
    default: return hipErrorInvalidValue;
  }
}

template <int LOGK>
hipError_t rows_fwd3_t(const uint64_t* in, int W, int P, int w, int L, int count, int gather_n,
                       double2* out, int rows_alloc, int pack, int lt, DevStatus* st,
                       hipStream_t s) {
  constexpr int K = 1 << LOGK;
  const size_t lds = sizeof(double2) * (size_t)(lds_points(K / 2) + lds_points(K));
  hipError_t e = set_lds((const void*)k_rows_fwd3<LOGK>, lds);
  if (e != hipSuccess) return e;
  const int grid = (count + 7) / 8 * 8;         // xcd_slot needs a multiple of 8
  hipLaunchKernelGGL(k_rows_fwd3<LOGK>, dim3(grid), dim3(rows3_threads(K)), lds, s, in, W, P, w,
                     L, count, gather_n, out, rows_alloc, pack, lt, st);
  return hipGetLastError();
}

hipError_t launch_rows_fwd3(const uint64_t* in, int W, int P, int w, int L, int count,
                            int gather_n, int logK, double2* out, int rows_alloc, int pack, int lt,
                            DevStatus* st, hipStream_t s) {
  switch (logK) {
#define HMV_RF3(k) \
  case k:          \
    return rows_fwd3_t<k>(in, W, P, w, L, count, gather_n, out, rows_alloc, pack, lt, st, s);
    HMV_RF3(6) HMV_RF3(7) HMV_RF3(8) HMV_RF3(9) HMV_RF3(10) HMV_RF3(11)
#undef HMV_RF3
    default: return hipErrorInvalidValue;
  }
}

template <int LOGNH>
hipError_t cols_plan_t(const double2* H1, int rows, int C, double scale, int pack, int lt,
                       double2* Hh, hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)lds_points(1 << LOGNH);
  hipError_t e = set_lds((const void*)k_cols_plan<LOGNH>, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8;
  hipLaunchKernelGGL(k_cols_plan<LOGNH>, dim3(grid), dim3(fft_threads(1 << LOGNH, 16)), lds, s, H1,
                     rows, C, scale, pack, lt, Hh);
  return hipGetLastError();
}

template <int LOGNH, int R>
hipError_t cols_pass_r(const double2* X1, const double2* Hh, int n, int C, int linear, int pack,
                       int kvec, int ltx, int lty, double2* Y1, hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)lds_points(1 << LOGNH);
  hipError_t e = set_lds((const void*)k_cols_pass<LOGNH, R>, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8 * kvec;    // xcd_slot needs a multiple of 8 per vector
  hipLaunchKernelGGL((k_cols_pass<LOGNH, R>), dim3(grid), dim3(fft_threads(1 << LOGNH, R)), lds,
                     s, X1, Hh, n, C, linear, pack, kvec, ltx, lty, Y1);
  return hipGetLastError();
}

// variant: bit 0 = radix-8 transforms (where they exist), bit 1 = linear
// column order
template <int LOGNH>
hipError_t cols_pass_t(const double2* X1, const double2* Hh, int n, int C, int variant, int pack,
                       int kvec, int ltx, int lty, double2* Y1, hipStream_t s) {
  const int linear = (variant >> 1) & 1;
  if constexpr (has_radix8(LOGNH)) {
    if (variant & 1)
      return cols_pass_r<LOGNH, 8>(X1, Hh, n, C, linear, pack, kvec, ltx, lty, Y1, s);
  }
  return cols_pass_r<LOGNH, 16>(X1, Hh, n, C, linear, pack, kvec, ltx, lty, Y1, s);
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
                            int pack, int lt, double2* Hh, hipStream_t s) {
  HMV_NT_DISPATCH(cols_plan_t, H1, rows, C, scale, pack, lt, Hh, s)
}

hipError_t launch_cols_pass(const double2* X1, const double2* Hh, int n, int C, int logNt,
                            int pack, double2* Y1, int variant, int ltx, int lty, hipStream_t s,
                            int kvec) {
  if (kvec < 1 || ltx < 0 || ltx > kMaxTileLog || lty < 0 || lty > kMaxTileLog)
    return hipErrorInvalidValue;
  HMV_NT_DISPATCH(cols_pass_t, X1, Hh, n, C, variant, pack, kvec, ltx, lty, Y1, s)
}

template <int LOGM, int R>
hipError_t rows_inv_r(const double2* Y1, int n, int L, int w, int P, int W, int out_reverse,
                      int pack, int lt, uint64_t* y, DevStatus* st, hipStream_t s) {
  constexpr int M = 1 << LOGM;
  const int T = fft_threads(M, R);
  const int NC = 2 * L - 1;
  // FFT points during the transform; afterwards NC int64 coefficients then
  // the carry scratch
  const size_t fft_part = sizeof(double2) * (size_t)lds_points(M);
  const size_t carry_off = ((size_t)NC * 8 + 15) / 16 * 16;
  const size_t carry_part = carry_off + (size_t)carry_lds_bytes(T);
  const size_t lds = fft_part > carry_part ? fft_part : carry_part;
  hipError_t e = set_lds((const void*)k_rows_inv<LOGM, R>, lds);
  if (e != hipSuccess) return e;
  const int grid = (n + 7) / 8 * 8;             // xcd_slot needs a multiple of 8
  hipLaunchKernelGGL((k_rows_inv<LOGM, R>), dim3(grid), dim3(T), lds, s, Y1, n, L, w, P, W,
                     out_reverse, (int)carry_off, pack, lt, y, st);
  return hipGetLastError();
}

// variant: bit 0 = radix-8 transform (where it exists)
template <int LOGM>
hipError_t rows_inv_t(const double2* Y1, int n, int L, int w, int P, int W, int out_reverse,
                      int pack, int lt, uint64_t* y, DevStatus* st, int variant, hipStream_t s) {
  if constexpr (has_radix8(LOGM)) {
    if (variant & 1)
      return rows_inv_r<LOGM, 8>(Y1, n, L, w, P, W, out_reverse, pack, lt, y, st, s);
  }
  return rows_inv_r<LOGM, 16>(Y1, n, L, w, P, W, out_reverse, pack, lt, y, st, s);
}

hipError_t launch_rows_inv(const double2* Y1, int n, int logM, int L, int w, int P, int W,
                           int out_reverse, int pack, int lt, uint64_t* y, DevStatus* st,
                           int variant, hipStream_t s) {
  switch (logM) {
#define HMV_RI(k) \
  case k: return rows_inv_t<k>(Y1, n, L, w, P, W, out_reverse, pack, lt, y, st, variant, s);
    HMV_RI(1) HMV_RI(2) HMV_RI(3) HMV_RI(4) HMV_RI(5) HMV_RI(6) HMV_RI(7) HMV_RI(8) HMV_RI(9)
    HMV_RI(10) HMV_RI(11) HMV_RI(12)
#undef HMV_RI
    default: return hipErrorInvalidValue;
  }
}

template <int LOGK>
hipError_t rows_inv3_t(const double2* Y1, int n, int L, int w, int P, int W, int out_reverse,
                       int pack, int lt, uint64_t* y, DevStatus* st, hipStream_t s) {
  constexpr int K = 1 << LOGK;
  const int T = rows3_threads(K);
  const int NC = 2 * L - 1;
  // transform points first; afterwards NC int64 coefficients then the carry
  // scratch
  const size_t fft_part = sizeof(double2) * (size_t)(lds_points(K / 2) + lds_points(K));
  const size_t carry_off = ((size_t)NC * 8 + 15) / 16 * 16;
  const size_t carry_part = carry_off + (size_t)carry_lds_bytes(T);
  const size_t lds = fft_part > carry_part ? fft_part : carry_part;
  hipError_t e = set_lds((const void*)k_rows_inv3<LOGK>, lds);
  if (e != hipSuccess) return e;
  const int grid = (n + 7) / 8 * 8;             // xcd_slot needs a multiple of 8
  hipLaunchKernelGGL(k_rows_inv3<LOGK>, dim3(grid), dim3(T), lds, s, Y1, n, L, w, P, W,
                     out_reverse, (int)carry_off, pack, lt, y, st);
  return hipGetLastError();
}

hipError_t launch_rows_inv3(const double2* Y1, int n, int logK, int L, int w, int P, int W,
                            int out_reverse, int pack, int lt, uint64_t* y, DevStatus* st,
                            hipStream_t s) {
  switch (logK) {
#define HMV_RI3(k) \
  case k: return rows_inv3_t<k>(Y1, n, L, w, P, W, out_reverse, pack, lt, y, st, s);
    HMV_RI3(6) HMV_RI3(7) HMV_RI3(8) HMV_RI3(9) HMV_RI3(10) HMV_RI3(11)
#undef HMV_RI3
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hmv

// ==================================================================== batch
// Many independent products.  Every instance runs
// the split-FFT path unplanned (its spectrum of h is built in the batch
// workspace).  Work items, in phase order over all instances:
//   phase 0  forward row transform of one h row (-> H1) or one x row (-> X1)
//   phase 1  index-axis transform of one limb column of H1 (-> resident Hh)
//   phase 2  index-axis pass of one limb column of X1 against Hh (-> Y1)
//   phase 3  inverse row transform + exact carry of one output row (-> y)
// Two drivers share the item code: a phase-synchronous one (one launch per
// pass and transform size, the one in use) and a single persistent launch in
// which work-groups take items from a global counter and wait on
// per-instance completion counters (bounded: past the spin limit it flags
// ST_SPIN and moves on).  The persistent driver is switched off and
// unreachable: its launch did not finish on either of two runs (the second
// after its counters and fences were moved to system scope), and the cause
// of that has not been established.
namespace hmv {

// Counters and the hand-off of results use system-scope atomics and
// fences: the workspace is ordinary (coarse-grained) device memory, whose
// lines may sit in the L2 of one XCD, and system scope forces the counter
// updates to memory and writes back / invalidates the L2s around them.
// A wait that exceeds the spin limit raises ST_SPIN; once that flag is up,
// every later wait gives up at once, so the whole launch stays bounded.
__device__ __forceinline__ bool batch_wait(const int* ctr, int target, int spin_limit,
                                           DevStatus* st) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    int spins = 0;
    ok = 1;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) < target) {
      const uint32_t fl =
          __hip_atomic_load(&st->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      if ((fl & ST_SPIN) || ++spins > spin_limit) {
        ok = 0;
        __hip_atomic_fetch_or(&st->flags, (uint32_t)ST_SPIN, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM);
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
  }
  __syncthreads();
  __threadfence_system();   // acquire for every wave: see the producers' data
  const bool r = ok != 0;
  __syncthreads();
  return r;
}

__device__ __forceinline__ void batch_done(int* ctr) {
  __threadfence_system();   // release: this work-group's results reach memory
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// forward row transform (the body of k_rows_fwd for one row)
__device__ __forceinline__ void b_row_fwd(const uint64_t* in, int W, int P, int w, int L, int gather_n, int logM,
                          double2* out, int rows_alloc, int r, double2* buf, uint64_t* wd,
                          uint32_t* red, DevStatus* st) {
  const int T = blockDim.x, t = threadIdx.x;
  const int M = 1 << logM;
  double* bd = reinterpret_cast<double*>(buf);
  __shared__ uint32_t rf[2];
  range_flags_init(rf);
  load_words_then(in + (int64_t)gather_row(r, gather_n) * W, W, wd, [&] {
    for (int k = (L + 1) / 2 + t; k < M; k += T) buf[lds_slot(k)] = make_double2(0.0, 0.0);
    if ((L & 1) && t == 0) bd[2 * lds_slot(L >> 1) + 1] = 0.0;
  });
  __syncthreads();
  range_check_block(wd, W, P, rf);
  split_balanced(wd, W, w, L, [&](int e, int d) { bd[2 * lds_slot(e >> 1) + (e & 1)] = (double)d; }, red);
  __syncthreads();
  if (t == 0 && !range_flags_ok(rf)) status_or(st, ST_RANGE);
  fft_lds(buf, logM, -1);
  pack_real_row<false>(buf, M, out, r, rows_alloc, 3);
  __syncthreads();
}

// index-axis transform of one column of H1 (even / odd halves, LDS FFT)
__device__ __forceinline__ void b_col_plan(const double2* H1, int rows, int logNt, double scale, double2* Hh,
                           int c, double2* buf) {
  const int T = blockDim.x, t = threadIdx.x;
  const int logNh = logNt - 1, Nh = 1 << logNh;
  const int rs = kRealTwN >> logNt;
  const double2* col = H1 + tile_index(c, 0, rows);
  double2* he = Hh + (int64_t)c * (2 * Nh);
  for (int half = 0; half < 2; ++half) {
    // four elements per thread at a time, loads first (clamped addresses)
    for (int s0 = t; s0 < Nh; s0 += 4 * T) {
      double2 lo[4], hi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = s0 + u * T;
        lo[u] = col[(int64_t)(s < rows ? s : 0) * 8];
        hi[u] = col[(int64_t)(s + Nh < rows ? s + Nh : 0) * 8];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = s0 + u * T;
        if (s < Nh) {
          const double2 l = s < rows ? lo[u] : make_double2(0.0, 0.0);
          const double2 h = s + Nh < rows ? hi[u] : make_double2(0.0, 0.0);
          buf[lds_slot(s)] = half == 0 ? cadd(l, h) : cmul(csub(l, h), real_root(s, rs));
        }
      }
    }
    __syncthreads();
    fft_lds(buf, logNh, -1);
    double2* dst = he + half * Nh;
    for (int f = t; f < Nh; f += T) {
      const double2 v = buf[lds_slot(f)];
      dst[f] = make_double2(v.x * scale, v.y * scale);
    }
    __syncthreads();
  }
}

// index-axis pass of one column: even half in the first lds_points(Nh)
// slots of buf, odd half in the next
__device__ __forceinline__ void b_col_pass(const double2* X1, const double2* Hh, int n, int logNt, double2* Y1,
                           int c, double2* buf) {
  const int T = blockDim.x, t = threadIdx.x;
  const int logNh = logNt - 1, Nh = 1 << logNh;
  const int rs = kRealTwN >> logNt;
  const double2* xcol = X1 + tile_index(c, 0, n);
  const double2* he = Hh + (int64_t)c * (2 * Nh);
  double2* be = buf;
  double2* bo = buf + lds_points(Nh);
  for (int s0 = t; s0 < Nh; s0 += 4 * T) {
    double2 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + u * T;
      xv[u] = xcol[(int64_t)(s < n ? n - 1 - s : 0) * 8];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + u * T;
      if (s < Nh) {
        const double2 v = s < n ? xv[u] : make_double2(0.0, 0.0);
        be[lds_slot(s)] = v;
        bo[lds_slot(s)] = cmul(v, real_root(s, rs));
      }
    }
  }
  __syncthreads();
  fft_lds(be, logNh, -1);
  fft_lds(bo, logNh, -1);
  for (int f0 = t; f0 < Nh; f0 += 4 * T) {
    double2 he4[4], ho4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = f0 + u * T < Nh ? f0 + u * T : 0;
      he4[u] = he[f];
      ho4[u] = he[Nh + f];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = f0 + u * T;
      if (f < Nh) {
        be[lds_slot(f)] = cmul(be[lds_slot(f)], he4[u]);
        bo[lds_slot(f)] = cmul(bo[lds_slot(f)], ho4[u]);
      }
    }
  }
  __syncthreads();
  fft_lds(be, logNh, +1);
  fft_lds(bo, logNh, +1);
  double2* ycol = Y1 + tile_index(c, 0, n);
  for (int s = t; s < Nh; s += T) {
    const double2 e = be[lds_slot(s)];
    const double2 q = cmul(bo[lds_slot(s)], conj2(real_root(s, rs)));
    const int ra = s - (n - 1), rb = s + Nh - (n - 1);
    if (ra >= 0 && ra < n) ycol[(int64_t)ra * 8] = cadd(e, q);
    if (rb >= 0 && rb < n) ycol[(int64_t)rb * 8] = csub(e, q);
  }
  __syncthreads();
}

// inverse row transform, rounding and carry of one output row
__device__ __forceinline__ void b_row_inv(const double2* Y1, int n, int logM, int L, int w, int P, int W,
                          int out_reverse, uint64_t* y, int i, double2* buf, uint32_t* red,
                          DevStatus* st) {
  __shared__ RowStatus rst;
  const int T = blockDim.x, t = threadIdx.x;
  const int M = 1 << logM;
  const int rs = kRealTwN / (2 * M);
  __shared__ double2 ytop;
  row_status_init(&rst);
  // loads four at a time per thread (clamped addresses), then LDS stores
  for (int k0 = t; k0 < M; k0 += 4 * T) {
    double2 ld[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * T;
      ld[u] = Y1[tile_index(k < M ? k : 0, i, n)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * T;
      if (k < M) buf[lds_slot(k)] = ld[u];
    }
  }
  if (t == 0) ytop = Y1[tile_index(M, i, n)];
  __syncthreads();
  double2 z[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int k = t + a * T;
    if (k < M) {
      const double2 yk = buf[lds_slot(k)];
      const double2 ym = k == 0 ? ytop : buf[lds_slot(M - k)];
      const double2 E = cadd(yk, conj2(ym)), D = csub(yk, conj2(ym));
      const double2 Q = cmul(D, conj2(real_root(k, rs)));
      z[a] = make_double2(E.x - Q.y, E.y + Q.x);
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int k = t + a * T;
    if (k < M) buf[lds_slot(k)] = z[a];
  }
  __syncthreads();
  fft_lds(buf, logM, +1);
  const int NC = 2 * L - 1;
  double maxerr = 0.0;
  int bad = 0;
  double2 v[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int m = t + a * T;
    if (m < M) v[a] = buf[lds_slot(m)];
  }
  __syncthreads();
  int64_t* coef = reinterpret_cast<int64_t*>(buf);
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int m = t + a * T;
    if (m < M) {
      double r0, r1;
      const int64_t i0 = round_to_int(v[a].x, &r0), i1 = round_to_int(v[a].y, &r1);
      maxerr = fmax(maxerr, fmax(fabs(v[a].x - r0), fabs(v[a].y - r1)));
      if (fabs(v[a].x) >= kCoefLimit || fabs(v[a].y) >= kCoefLimit) bad = 1;
      if (2 * m < NC) coef[2 * m] = i0;
      else if (i0 != 0) bad = 1;
      if (2 * m + 1 < NC) coef[2 * m + 1] = i1;
      else if (i1 != 0) bad = 1;
    }
  }
  row_status_publish(&rst, maxerr, bad, st);
  const int carry_off = (NC * 8 + 15) / 16 * 16;
  int64_t* cs = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(buf) + carry_off);
  const int row = out_reverse ? (n - 1 - i) : i;
  carry_round_pack_fit(coef, NC, w, P, W, cs, y + (int64_t)row * W, red);
}

__global__ void __launch_bounds__(256) k_batch(const BatchInst* __restrict__ inst,
                                               const int4* __restrict__ items, int nitems,
                                               int* __restrict__ head, int* __restrict__ ctr,
                                               int spin_limit, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  __shared__ int cur;
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(head, 1);
    __syncthreads();
    const int it = cur;
    __syncthreads();
    if (it >= nitems) break;
    const int4 d = items[it];
    const BatchInst I = inst[d.x];
    int* c = ctr + 4 * d.x;           // h rows, x rows, plan columns, pass columns
    const int rows_h = 2 * I.n - 1;
    if (d.y == 0) {
      if (d.z < rows_h) {
        b_row_fwd(I.h, I.W, I.P, I.w, I.L, I.gather, I.logM, I.H1, rows_h, d.z, buf, wd, red, st);
        batch_done(c + 0);
      } else {
        b_row_fwd(I.x, I.W, I.P, I.w, I.L, 0, I.logM, I.X1, I.n, d.z - rows_h, buf, wd, red, st);
        batch_done(c + 1);
      }
    } else if (d.y == 1) {
      batch_wait(c + 0, rows_h, spin_limit, st);
      b_col_plan(I.H1, rows_h, I.logNt, I.scale, I.Hh, d.z, buf);
      batch_done(c + 2);
    } else if (d.y == 2) {
      batch_wait(c + 1, I.n, spin_limit, st);
      batch_wait(c + 2, I.C, spin_limit, st);
      b_col_pass(I.X1, I.Hh, I.n, I.logNt, I.Y1, d.z, buf);
      batch_done(c + 3);
    } else {
      batch_wait(c + 3, I.C, spin_limit, st);
      b_row_inv(I.Y1, I.n, I.logM, I.L, I.w, I.P, I.W, I.reverse, I.y, d.z, buf, red, st);
    }
  }
}

// Phase-synchronous batch: one launch per pass and transform size, over the
// items of that pass of every instance (one item per work-group); kernel
// boundaries order the passes, so no work-group waits on another.  Each pass
// has its own kernel, so each gets the registers it needs, and each launch
// gets the LDS and the threads of its transform size.
__global__ void __launch_bounds__(256, 2) k_batch_rows_fwd(const BatchInst* __restrict__ inst,
                                                        const int4* __restrict__ items,
                                                        int nitems, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 d = items[it];
  const BatchInst I = inst[d.x];
  const int rows_h = 2 * I.n - 1;
  if (d.z < rows_h)
    b_row_fwd(I.h, I.W, I.P, I.w, I.L, I.gather, I.logM, I.H1, rows_h, d.z, buf, wd, red, st);
  else
    b_row_fwd(I.x, I.W, I.P, I.w, I.L, 0, I.logM, I.X1, I.n, d.z - rows_h, buf, wd, red, st);
}

__global__ void __launch_bounds__(256, 2) k_batch_cols_plan(const BatchInst* __restrict__ inst,
                                                         const int4* __restrict__ items,
                                                         int nitems, DevStatus*) {
  extern __shared__ double2 buf[];
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 d = items[it];
  const BatchInst I = inst[d.x];
  b_col_plan(I.H1, 2 * I.n - 1, I.logNt, I.scale, I.Hh, d.z, buf);
}

__global__ void __launch_bounds__(256, 2) k_batch_cols_pass(const BatchInst* __restrict__ inst,
                                                         const int4* __restrict__ items,
                                                         int nitems, DevStatus*) {
  extern __shared__ double2 buf[];
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 d = items[it];
  const BatchInst I = inst[d.x];
  b_col_pass(I.X1, I.Hh, I.n, I.logNt, I.Y1, d.z, buf);
}

__global__ void __launch_bounds__(256, 2) k_batch_rows_inv(const BatchInst* __restrict__ inst,
                                                        const int4* __restrict__ items,
                                                        int nitems, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 d = items[it];
  const BatchInst I = inst[d.x];
  b_row_inv(I.Y1, I.n, I.logM, I.L, I.w, I.P, I.W, I.reverse, I.y, d.z, buf, red, st);
}

// The row passes of instances whose limb transform has 3K = 3 * 2^LOGK
// points (the planned path's row bodies, with the batch's tiles of 8 columns
// and no shared column for the real bins).
template <int LOGK>
__global__ void __launch_bounds__(256) k_batch_rows_fwd3(const BatchInst* __restrict__ inst,
                                                         const int4* __restrict__ items,
                                                         int nitems, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 d = items[it];
  const BatchInst I = inst[d.x];
  const int rows_h = 2 * I.n - 1;
  if (d.z < rows_h)
    row_fwd3<LOGK>(I.h, I.W, I.P, I.w, I.L, I.gather, I.H1, rows_h, d.z, 0, 3, buf, red, st);
  else
    row_fwd3<LOGK>(I.x, I.W, I.P, I.w, I.L, 0, I.X1, I.n, d.z - rows_h, 0, 3, buf, red, st);
}

template <int LOGK>
__global__ void __launch_bounds__(256) k_batch_rows_inv3(const BatchInst* __restrict__ inst,
                                                         const int4* __restrict__ items,
                                                         int nitems, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint32_t red[32];
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 d = items[it];
  const BatchInst I = inst[d.x];
  // the coefficients (2L - 1 <= 3K int64) fit in the transform buffer; the
  // carry scratch follows it
  constexpr int K = 1 << LOGK;
  const int carry_off = (int)sizeof(double2) * (lds_points(K / 2) + lds_points(K));
  row_inv3<LOGK>(I.Y1, I.n, I.L, I.w, I.P, I.W, I.reverse, carry_off, 0, 3, I.y, d.z, buf, red,
                 st);
}

template <int LOGK>
hipError_t batch_rows3_t(int phase, const BatchInst* inst, const int4* items, int nitems,
                         DevStatus* st, hipStream_t s) {
  constexpr int K = 1 << LOGK;
  const int T = rows3_threads(K);
  size_t lds = sizeof(double2) * (size_t)(lds_points(K / 2) + lds_points(K));
  if (phase == 3) lds += (size_t)carry_lds_bytes(T) + 16;
  const void* fn = phase == 0 ? (const void*)k_batch_rows_fwd3<LOGK> : (const void*)k_batch_rows_inv3<LOGK>;
  hipError_t e = set_lds(fn, lds);
  if (e != hipSuccess) return e;
  if (phase == 0)
    hipLaunchKernelGGL(k_batch_rows_fwd3<LOGK>, dim3(nitems), dim3(T), lds, s, inst, items, nitems, st);
  else
    hipLaunchKernelGGL(k_batch_rows_inv3<LOGK>, dim3(nitems), dim3(T), lds, s, inst, items, nitems, st);
  return hipGetLastError();
}

// Items of one pass whose transforms have 2^logn points (the limb transform
// for passes 0 and 3, the index-axis half for passes 1 and 2).
hipError_t launch_batch_phase(int phase, int logn, const BatchInst* inst, const int4* items,
                              int nitems, DevStatus* st, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipError_t e = fft_tables_init();
  if (e != hipSuccess) return e;
  if ((phase == 0 || phase == 3) && logn >= kBatchLog3) {
    switch (logn - kBatchLog3) {
#define HMV_BR3(k) \
  case k: return batch_rows3_t<k>(phase, inst, items, nitems, st, s);
      HMV_BR3(6) HMV_BR3(7) HMV_BR3(8) HMV_BR3(9) HMV_BR3(10) HMV_BR3(11)
#undef HMV_BR3
      default: return hipErrorInvalidValue;
    }
  }
  const int N = 1 << logn;
  const int T = fft_threads(N, 16);
  const void* fn = phase == 0   ? (const void*)k_batch_rows_fwd
                   : phase == 1 ? (const void*)k_batch_cols_plan
                   : phase == 2 ? (const void*)k_batch_cols_pass
                                : (const void*)k_batch_rows_inv;
  size_t lds = sizeof(double2) * (size_t)lds_points(N);
  if (phase == 2) lds *= 2;                                  // both halves
  if (phase == 3) lds += (size_t)carry_lds_bytes(T) + 16;   // coefficients + carry scratch
  e = set_lds(fn, lds);
  if (e != hipSuccess) return e;
  if (phase == 0)
    hipLaunchKernelGGL(k_batch_rows_fwd, dim3(nitems), dim3(T), lds, s, inst, items, nitems, st);
  else if (phase == 1)
    hipLaunchKernelGGL(k_batch_cols_plan, dim3(nitems), dim3(T), lds, s, inst, items, nitems, st);
  else if (phase == 2)
    hipLaunchKernelGGL(k_batch_cols_pass, dim3(nitems), dim3(T), lds, s, inst, items, nitems, st);
  else
    hipLaunchKernelGGL(k_batch_rows_inv, dim3(nitems), dim3(T), lds, s, inst, items, nitems, st);
  return hipGetLastError();
}

// Single cooperative launch of a whole batch: every work-group stays
// resident (the launch is refused otherwise), takes the items of pass 0 in a
// grid-stride loop, waits at a grid-wide barrier, then takes those of pass
// 1, and so on.  The passes' items are independent within a pass and the
// barriers order the passes, so no work-group waits on another's progress
// except at the three barriers, which every work-group reaches.  One
// work-group shape serves every item: 256 threads, power-of-two limb
// transforms (the pass bodies of the persistent form).
__global__ void __launch_bounds__(256) k_batch_coop(const BatchInst* __restrict__ inst,
                                                    const int4* __restrict__ items, int4 starts,
                                                    int nitems, DevStatus* st) {
  extern __shared__ double2 buf[];
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  for (int ph = 0; ph < 4; ++ph) {
    const int lo = ph == 0 ? starts.x : ph == 1 ? starts.y : ph == 2 ? starts.z : starts.w;
    const int hi = ph == 0 ? starts.y : ph == 1 ? starts.z : ph == 2 ? starts.w : nitems;
    for (int it = lo + (int)blockIdx.x; it < hi; it += (int)gridDim.x) {
      const int4 d = items[it];
      const BatchInst I = inst[d.x];
      const int rows_h = 2 * I.n - 1;
      if (ph == 0) {
        if (d.z < rows_h)
          b_row_fwd(I.h, I.W, I.P, I.w, I.L, I.gather, I.logM, I.H1, rows_h, d.z, buf, wd, red,
                    st);
        else
          b_row_fwd(I.x, I.W, I.P, I.w, I.L, 0, I.logM, I.X1, I.n, d.z - rows_h, buf, wd, red,
                    st);
      } else if (ph == 1) {
        b_col_plan(I.H1, rows_h, I.logNt, I.scale, I.Hh, d.z, buf);
      } else if (ph == 2) {
        b_col_pass(I.X1, I.Hh, I.n, I.logNt, I.Y1, d.z, buf);
      } else {
        b_row_inv(I.Y1, I.n, I.logM, I.L, I.w, I.P, I.W, I.reverse, I.y, d.z, buf, red, st);
      }
      __syncthreads();
    }
    if (ph < 3) grid.sync();
  }
}

hipError_t launch_batch_coop(const BatchInst* inst, const int4* items, const int* starts,
                             int nitems, DevStatus* st, int* grid_used, hipStream_t s) {
  hipError_t e = fft_tables_init();
  if (e != hipSuccess) return e;
  const size_t lds = kBatchDynLds;
  e = set_lds((const void*)k_batch_coop, lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch_coop,
                                                     kBatchThreads, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int grid = per_cu * cus;
  if (grid_used) *grid_used = grid;
  int4 st4 = make_int4(starts[0], starts[1], starts[2], starts[3]);
  void* args[] = {(void*)&inst, (void*)&items, (void*)&st4, (void*)&nitems, (void*)&st};
  e = hipLaunchCooperativeKernel((const void*)k_batch_coop, dim3(grid), dim3(kBatchThreads), args,
                                 lds, s);
  return e;
}

__global__ void k_zero_ints(int* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}


hipError_t launch_batch(const BatchInst* inst, const int4* items, int nitems, int* head, int* ctr,
                        int nctr, int grid, int spin_limit, DevStatus* st, hipStream_t s) {
  hipError_t e = fft_tables_init();
  if (e != hipSuccess) return e;
  const int nz = nctr + 1;
  hipLaunchKernelGGL(k_zero_ints, dim3((nz + 255) / 256), dim3(256), 0, s, head, nz);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = kBatchDynLds;
  e = set_lds((const void*)k_batch, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBatchThreads), lds, s, inst, items, nitems, head, ctr,
                     spin_limit, st);
  return hipGetLastError();
}

}  // namespace hmv
