// Exact transform paths modulo p = 2^64 - 2^32 + 1.
//
// NTT path: the same decomposition as the split-FFT path (limb polynomials,
// bivariate index-by-limb correlation) with number-theoretic transforms, so
// every coefficient comes out exactly mod p.  The limb width keeps every
// true coefficient below p/2 in magnitude (n L 4^(w-1) < 2^62), so the
// centred residue is the coefficient itself.  The limb axis has no
// conjugate symmetry mod p: all N_z columns are kept.
//
// Karatsuba path (Section 4, Algorithm 1): the index-axis Hankel product
// of every limb-frequency column is computed by the recursive half-size
// scheme instead of a transform.  The recursion is linear, so its sums and
// differences act elementwise on whole rows of limb spectra: the host lays
// the recursion tree out breadth-first as lists of row operations, the
// leaves are small Hankel products done directly, and the results combine
// bottom-up.
//
// Arrays of limb spectra ([rows][N_z] residues) use tiles of T columns:
// element (row, k) at ((k/T) rows + row) T + k%T.  T = 16 (128 bytes) for the
// NTT path, whose column pass reads columns; T = N_z (plain row-major) for
// the Karatsuba path, whose kernels all work on whole rows.
#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "ntt.h"
#include "tables.h"

namespace hmv {

namespace {
std::mutex g_ntab_mu;
bool g_ntab_ready[64] = {};
}  // namespace

hipError_t ntt_tables_init() {
  std::lock_guard<std::mutex> lk(g_ntab_mu);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (g_ntab_ready[dev]) return hipSuccess;
  std::vector<uint64_t> tw(2 * kNttTwEntries), r16(32), split(2 * kNttSplitEntries);
  gen_ntt_tables(tw.data(), r16.data(), split.data());
  // the device applies the radix-16 internal roots as powers of two
  for (int m = 0; m < 16; ++m)
    if (r16[m] != gold_pow(2, (uint64_t)r16_exp<0>(m)) ||
        r16[16 + m] != gold_pow(2, (uint64_t)r16_exp<1>(m)))
      return hipErrorInvalidValue;
  e = hipMemcpyToSymbol(HIP_SYMBOL(g_ntw), tw.data(), 8 * tw.size());
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_nsplit), split.data(), 8 * split.size());
  if (e != hipSuccess) return e;
  g_ntab_ready[dev] = true;
  return hipSuccess;
}

__device__ __forceinline__ int64_t ntile(int k, int row, int rows, int logT) {
  return (((int64_t)(k >> logT) * rows + row) << logT) + (k & ((1 << logT) - 1));
}

__device__ __forceinline__ int n_gather_row(int r, int gather_n) {
  if (gather_n <= 0) return r;
  int s = (gather_n - 1 - r) % gather_n;
  return s < 0 ? s + gather_n : s;
}

__device__ __forceinline__ int n_xcd_slot(int b, int grid) {
  const int q = grid >> 3;
  return (b & 7) * q + (b >> 3);
}

// ------------------------------------------------------------------ rows
// Forward row transform: split a number into balanced digits (as residues)
// and transform the N_z-point limb sequence.
__global__ void __launch_bounds__(512) k_ntt_rows_fwd(const uint64_t* __restrict__ in, int W, int P,
                                                      int w, int L, int count, int gather_n,
                                                      int logN, uint64_t* __restrict__ out,
                                                      int rows_alloc, int logT, DevStatus* st) {
  extern __shared__ uint64_t nbuf[];
  __shared__ uint64_t wd[kMaxWords];
  __shared__ uint32_t red[32];
  // rows grouped per XCD, so that the rows sharing the lines of a tile
  // column are written through one L2
  const int r = n_xcd_slot(blockIdx.x, gridDim.x);
  if (r >= count) return;
  const int T = blockDim.x, t = threadIdx.x, N = 1 << logN;
  // the residues past the digits are zeroed while the words are in flight;
  // every wave checks part of the range, read back after the split's barriers
  __shared__ uint32_t rf[2];
  range_flags_init(rf);
  load_words_then(in + (int64_t)n_gather_row(r, gather_n) * W, W, wd, [&] {
    for (int e = L + t; e < N; e += T) nbuf[nswz(e)] = 0;
  });
  __syncthreads();
  range_check_block(wd, W, P, rf);
  split_balanced(wd, W, w, L, [&](int e, int d) { nbuf[nswz(e)] = gl_from_int(d); }, red);
  __syncthreads();
  if (t == 0 && !range_flags_ok(rf)) status_or(st, ST_RANGE);
  ntt_lds<0>(nbuf, logN);
  for (int k = t; k < N; k += T) out[ntile(k, r, rows_alloc, logT)] = nbuf[nswz(k)];
}

// Inverse row transform, centring and exact carry / round / pack.  The
// scale 1 / (N_t N_z) (or 1 / N_z) is already folded into the data.
__global__ void __launch_bounds__(512) k_ntt_rows_inv(const uint64_t* __restrict__ Y, int n,
                                                      int logN, int L, int w, int P, int W,
                                                      int out_reverse, int logT, int carry_off,
                                                      uint64_t* __restrict__ y, DevStatus* st) {
  extern __shared__ uint64_t nbuf[];
  __shared__ uint32_t red[32];
  const int i = blockIdx.x;
  if (i >= n) return;
  const int T = blockDim.x, t = threadIdx.x, N = 1 << logN;
  {
    // element k = t + T a; the loads of a thread are issued together
    uint64_t ld[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int k = t + a * T;
      ld[a] = Y[ntile(k < N ? k : 0, i, n, logT)];
    }
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int k = t + a * T;
      if (k < N) nbuf[nswz(k)] = ld[a];
    }
  }
  __syncthreads();
  ntt_lds<1>(nbuf, logN);
  const int NC = 2 * L - 1;
  int bad = 0;
  // centre every residue; coefficients past NC must vanish
  int64_t vals[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int e = t + a * T;
    if (e < N) {
      const int64_t c = gl_centre(nbuf[nswz(e)]);
      vals[a] = c;
      if (e >= NC && c != 0) bad = 1;
    }
  }
  __syncthreads();
  int64_t* coef = reinterpret_cast<int64_t*>(nbuf);
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int e = t + a * T;
    if (e < NC) coef[e] = vals[a];
  }
  bad = __syncthreads_or(bad);
  if (bad && t == 0) status_or(st, ST_BOUND);
  int64_t* cs = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(nbuf) + carry_off);
  const int row = out_reverse ? (n - 1 - i) : i;
  carry_round_pack_fit(coef, NC, w, P, W, cs, y + (int64_t)row * W, red);
}

// ------------------------------------------------------------------ columns
// The index axis of N_t = 2 Nh points is split into two Nh-point transforms
// exactly as on the binary64 path (even frequencies from u[s] + u[s+Nh], odd
// ones from (u[s] - u[s+Nh]) w^s); a spectrum column holds Nh even bins,
// then Nh odd bins.
template <int LOGNH>
__global__ void __launch_bounds__(512) k_ntt_cols_plan(const uint64_t* __restrict__ H1, int rows,
                                                       int C, uint64_t scale,
                                                       uint64_t* __restrict__ Hh) {
  extern __shared__ uint64_t nbuf[];
  const int c = n_xcd_slot(blockIdx.x, gridDim.x);
  if (c >= C) return;
  constexpr int logNt = LOGNH + 1, Nh = 1 << LOGNH;
  constexpr int Ta = Nh >= 16 ? Nh >> 4 : 1, per = Nh >= 16 ? 16 : Nh;
  constexpr int ss = kNttSplitN >> logNt;
  const int t = threadIdx.x;
  const bool act = t < Ta;
  uint64_t* he = Hh + (int64_t)c * (2 * Nh);
  uint64_t v[16];
  for (int half = 0; half < 2; ++half) {
    // one guarded block per loop with clamped addresses: loads in flight together
    if (act) {
#pragma unroll
      for (int j = 0; j < per; ++j) {
        const int s = t + Ta * j;
        const uint64_t l = H1[ntile(c, s < rows ? s : 0, rows, kNttXLogT)];
        const uint64_t u = H1[ntile(c, s + Nh < rows ? s + Nh : 0, rows, kNttXLogT)];
        const uint64_t lo = s < rows ? l : 0, hi = s + Nh < rows ? u : 0;
        v[j] = half == 0 ? gl_add(lo, hi) : gl_mul(gl_sub(lo, hi), g_nsplit[s * ss]);
      }
    }
    ntt_regs<LOGNH, 0>(v, nbuf);
    uint64_t* dst = he + half * Nh;
    if (act) {
#pragma unroll
      for (int j = 0; j < per; ++j) dst[t + Ta * j] = gl_mul(v[j], scale);
    }
  }
}

template <int LOGNH>
__global__ void __launch_bounds__(512) k_ntt_cols_pass(const uint64_t* __restrict__ X1,
                                                       const uint64_t* __restrict__ Hh, int n,
                                                       int C, uint64_t* __restrict__ Y1) {
  extern __shared__ uint64_t nbuf[];
  const int c = n_xcd_slot(blockIdx.x, gridDim.x);
  if (c >= C) return;
  constexpr int logNt = LOGNH + 1, Nh = 1 << LOGNH;
  constexpr int Ta = Nh >= 16 ? Nh >> 4 : 1, per = Nh >= 16 ? 16 : Nh;
  constexpr int ss = kNttSplitN >> logNt;
  const int t = threadIdx.x;
  const bool act = t < Ta;
  const uint64_t* he = Hh + (int64_t)c * (2 * Nh);
  const uint64_t* ho = he + Nh;
  // The column is read once (o keeps it for the odd half); every
  // per-element loop is one guarded block with clamped addresses, so its
  // loads are in flight together.
  uint64_t v[16], o[16];
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int s = t + Ta * j;
      const uint64_t xv = X1[ntile(c, s < n ? n - 1 - s : 0, n, kNttXLogT)];
      v[j] = s < n ? xv : 0;
      o[j] = v[j];
    }
  }
  __syncthreads();
  ntt_regs<LOGNH, 0>(v, nbuf);
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) v[j] = gl_mul(v[j], he[t + Ta * j]);
  }
  ntt_regs<LOGNH, 1>(v, nbuf);
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) o[j] = gl_mul(o[j], g_nsplit[(t + Ta * j) * ss]);
  }
  ntt_regs<LOGNH, 0>(o, nbuf);
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) o[j] = gl_mul(o[j], ho[t + Ta * j]);
  }
  ntt_regs<LOGNH, 1>(o, nbuf);
  if (act) {
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int s = t + Ta * j;
      const uint64_t q = gl_mul(o[j], g_nsplit[kNttSplitEntries + s * ss]);
      const int ra = s - (n - 1), rb = s + Nh - (n - 1);
      if (ra >= 0 && ra < n) Y1[ntile(c, ra, n, kNttYLogT)] = gl_add(v[j], q);
      if (rb >= 0 && rb < n) Y1[ntile(c, rb, n, kNttYLogT)] = gl_sub(v[j], q);
    }
  }
}

// ------------------------------------------------------------------ Karatsuba
// Row operations dst[o] = src[a] + sign * src[b] over whole rows of N_z
// residues (row-major); a or b < 0 reads as zero.  One op per entry of ops
// (int4: out row, a, b, sign).
__global__ void __launch_bounds__(256) k_kara_rowops(const int4* __restrict__ ops, int nops,
                                                     const uint64_t* __restrict__ src,
                                                     uint64_t* __restrict__ dst, int Nz) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nops * Nz;
  if (gid >= total) return;
  const int o = (int)(gid / Nz), k = (int)(gid % Nz);
  const int4 op = ops[o];
  const uint64_t a = op.y >= 0 ? src[(int64_t)op.y * Nz + k] : 0;
  const uint64_t b = op.z >= 0 ? src[(int64_t)op.z * Nz + k] : 0;
  dst[(int64_t)op.x * Nz + k] = op.w > 0 ? gl_add(a, b) : gl_sub(a, b);
}

// Leaf products: for a leaf (a, x, y, m), the plain Hankel product
//   Y[y + i] = sum_{j < m} A[a + i + j] X[x + j],  i < m,
// per column k (the limb-NTT domain is pointwise).  One thread per (leaf,
// column) keeps a window of kKaraWindow A values and m accumulators in
// registers: step j multiplies X[x + j] into every accumulator, then slides
// the window by one row, so each A and X value is read once.  The products
// are summed unreduced as 128-bit values with a count of the carries out of
// bit 127 (m <= 32 products stay below 2^133), and reduced once per output:
// 2^64 = 2^32 - 1 and 2^128 = -2^32 (mod p).
__global__ void __launch_bounds__(256) k_kara_leaves(const int4* __restrict__ leaves, int nleaves,
                                                     const uint64_t* __restrict__ A,
                                                     const uint64_t* __restrict__ X,
                                                     uint64_t* __restrict__ Yo, int Nz) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nleaves * Nz;
  if (gid >= total) return;
  const int o = (int)(gid / Nz), k = (int)(gid % Nz);
  const int4 lf = leaves[o];
  const int a = lf.x, x = lf.y, yr = lf.z, m = lf.w;
  constexpr int Wn = kKaraWindow;
  uint64_t win[Wn], lo[Wn], hi[Wn];
  uint32_t top[Wn];
#pragma unroll
  for (int i = 0; i < Wn; ++i) {
    win[i] = i < 2 * m - 1 ? A[(int64_t)(a + i) * Nz + k] : 0;
    lo[i] = hi[i] = 0;
    top[i] = 0;
  }
  for (int j = 0; j < m; ++j) {
    const uint64_t xj = X[(int64_t)(x + j) * Nz + k];
    const uint64_t nxt = j + Wn <= 2 * m - 2 ? A[(int64_t)(a + j + Wn) * Nz + k] : 0;
#pragma unroll
    for (int i = 0; i < Wn; ++i) {
      if (i < m) {
        const uint64_t pl = win[i] * xj, ph = __umul64hi(win[i], xj);
        const uint64_t l2 = lo[i] + pl;
        const uint64_t h1 = hi[i] + ph;
        const uint64_t h2 = h1 + (l2 < pl ? 1ull : 0ull);
        top[i] += (h1 < ph ? 1u : 0u) + (h2 < h1 ? 1u : 0u);
        lo[i] = l2;
        hi[i] = h2;
      }
    }
#pragma unroll
    for (int i = 0; i + 1 < Wn; ++i) win[i] = win[i + 1];
    win[Wn - 1] = nxt;
  }
#pragma unroll
  for (int i = 0; i < Wn; ++i)
    if (i < m) {
      // lo + hi 2^64 + top 2^128 = fold(lo, hi) - top 2^32  (mod p)
      const uint64_t f = gl_fold(lo[i], hi[i]);
      Yo[(int64_t)(yr + i) * Nz + k] = gl_sub(f, (uint64_t)top[i] << 32);
    }
}

// Scale whole rows by a residue (the 1 / N_z of the inverse limb transform).
__global__ void __launch_bounds__(256) k_ntt_scale(uint64_t* __restrict__ a, int64_t count,
                                                   uint64_t scale) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < count) a[gid] = gl_mul(a[gid], scale);
}

// ------------------------------------------------------------------ launchers
namespace {
std::mutex g_nlds_mu;
std::vector<std::pair<std::pair<int, const void*>, size_t>> g_nlds_set;

hipError_t nset_lds(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_nlds_mu);
  for (auto& kv : g_nlds_set)
    if (kv.first.first == dev && kv.first.second == fn) {
      if (kv.second >= bytes) return hipSuccess;
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e == hipSuccess) kv.second = bytes;
      return e;
    }
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) g_nlds_set.push_back({{dev, fn}, bytes});
  return e;
}

// Row kernels run N/16 threads, at least 64 (the inverse kernel holds 16
// residues per thread).
int nrow_threads(int N) { return N / 16 < 64 ? 64 : N / 16; }
}  // namespace

hipError_t launch_ntt_rows_fwd(const uint64_t* in, int W, int P, int w, int L, int count,
                               int gather_n, int logN, uint64_t* out, int rows_alloc, int logT,
                               DevStatus* st, hipStream_t s) {
  const int N = 1 << logN;
  const int T = nrow_threads(N);
  const size_t lds = 8 * (size_t)N;
  hipError_t e = nset_lds((const void*)k_ntt_rows_fwd, lds);
  if (e != hipSuccess) return e;
  const int grid = (count + 7) / 8 * 8;         // n_xcd_slot needs a multiple of 8
  hipLaunchKernelGGL(k_ntt_rows_fwd, dim3(grid), dim3(T), lds, s, in, W, P, w, L, count,
                     gather_n, logN, out, rows_alloc, logT, st);
  return hipGetLastError();
}

hipError_t launch_ntt_rows_inv(const uint64_t* Y, int n, int logN, int L, int w, int P, int W,
                               int out_reverse, int logT, uint64_t* y, DevStatus* st,
                               hipStream_t s) {
  const int N = 1 << logN;
  const int T = nrow_threads(N);
  const int NC = 2 * L - 1;
  const size_t carry_off = ((size_t)NC * 8 + 15) / 16 * 16;
  size_t lds = carry_off + (size_t)carry_lds_bytes(T);
  if (lds < 8 * (size_t)N) lds = 8 * (size_t)N;
  hipError_t e = nset_lds((const void*)k_ntt_rows_inv, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ntt_rows_inv, dim3(n), dim3(T), lds, s, Y, n, logN, L, w, P, W,
                     out_reverse, logT, (int)carry_off, y, st);
  return hipGetLastError();
}

template <int LOGNH>
hipError_t ntt_cols_plan_t(const uint64_t* H1, int rows, int C, uint64_t scale, uint64_t* Hh,
                           hipStream_t s) {
  const size_t lds = 8 * (size_t)(1 << LOGNH);
  hipError_t e = nset_lds((const void*)k_ntt_cols_plan<LOGNH>, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8;
  const int T = (1 << LOGNH) / 16 < 64 ? 64 : (1 << LOGNH) / 16;
  hipLaunchKernelGGL(k_ntt_cols_plan<LOGNH>, dim3(grid), dim3(T), lds, s, H1, rows, C, scale, Hh);
  return hipGetLastError();
}

template <int LOGNH>
hipError_t ntt_cols_pass_t(const uint64_t* X1, const uint64_t* Hh, int n, int C, uint64_t* Y1,
                           hipStream_t s) {
  const size_t lds = 8 * (size_t)(1 << LOGNH);
  hipError_t e = nset_lds((const void*)k_ntt_cols_pass<LOGNH>, lds);
  if (e != hipSuccess) return e;
  const int grid = (C + 7) / 8 * 8;
  const int T = (1 << LOGNH) / 16 < 64 ? 64 : (1 << LOGNH) / 16;
  hipLaunchKernelGGL(k_ntt_cols_pass<LOGNH>, dim3(grid), dim3(T), lds, s, X1, Hh, n, C, Y1);
  return hipGetLastError();
}

#define HMV_NNT_DISPATCH(FN, ...)                 \
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

hipError_t launch_ntt_cols_plan(const uint64_t* H1, int rows, int C, int logNt, uint64_t scale,
                                uint64_t* Hh, hipStream_t s) {
  HMV_NNT_DISPATCH(ntt_cols_plan_t, H1, rows, C, scale, Hh, s)
}

hipError_t launch_ntt_cols_pass(const uint64_t* X1, const uint64_t* Hh, int n, int C, int logNt,
                                uint64_t* Y1, hipStream_t s) {
  HMV_NNT_DISPATCH(ntt_cols_pass_t, X1, Hh, n, C, Y1, s)
}

hipError_t launch_kara_rowops(const int4* ops, int nops, const uint64_t* src, uint64_t* dst,
                              int Nz, hipStream_t s) {
  if (nops <= 0) return hipSuccess;
  const int64_t total = (int64_t)nops * Nz;
  const int grid = (int)((total + 255) / 256);
  hipLaunchKernelGGL(k_kara_rowops, dim3(grid), dim3(256), 0, s, ops, nops, src, dst, Nz);
  return hipGetLastError();
}

hipError_t launch_kara_leaves(const int4* leaves, int nleaves, const uint64_t* A,
                              const uint64_t* X, uint64_t* Y, int Nz, hipStream_t s) {
  if (nleaves <= 0) return hipSuccess;
  const int64_t total = (int64_t)nleaves * Nz;
  const int grid = (int)((total + 255) / 256);
  hipLaunchKernelGGL(k_kara_leaves, dim3(grid), dim3(256), 0, s, leaves, nleaves, A, X, Y, Nz);
  return hipGetLastError();
}

hipError_t launch_ntt_scale(uint64_t* a, int64_t count, uint64_t scale, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = (int)((count + 255) / 256);
  hipLaunchKernelGGL(k_ntt_scale, dim3(grid), dim3(256), 0, s, a, count, scale);
  return hipGetLastError();
}

}  // namespace hmv
