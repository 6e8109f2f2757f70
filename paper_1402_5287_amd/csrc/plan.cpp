// Plans: the transform of h kept resident (the Lanczos use of Section 1
// multiplies one fixed matrix by many vectors), limb-width selection by the
// proven error bound, and the planned matvec launches.
#include "plan.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "common.h"
#include "fft_layout.h"
#include "hmv.h"
#include "kernels.h"
#include "tables.h"

using namespace hmv;

namespace hmv {

int g_force_w = 0;

int ilog2_ceil(int64_t v) {
  int k = 0;
  while ((int64_t(1) << k) < v) ++k;
  return k;
}

bool fft_sizes(int64_t n, int32_t P, int w, FftSizes* z, bool planned) {
  const int L = limbs_of(P, w);
  int logNz = ilog2_ceil(2 * int64_t(L) - 1);
  if (logNz < 2) logNz = 2;
  int logNt = ilog2_ceil(2 * n - 1);
  if (logNt < 2) logNt = 2;
  if (logNz > kFftMaxLogNz || logNt > kFftMaxLogNt) return false;
  z->w = w;
  z->L = L;
  z->logM = logNz - 1;
  z->logNt = logNt;
  z->Nz = int64_t(1) << logNz;
  z->z3 = 0;
  // 3K points (K = 2^logK) when 2L - 1 <= 3K < 2^logNz
  const int logK = ilog2_ceil((2 * int64_t(L) - 1 + 2) / 3);
  if (planned && logK >= 6 && logK <= kR3MaxLogK && 3 * (int64_t(1) << logK) < z->Nz) {
    z->z3 = 1;
    z->logM = logK;
    z->Nz = 3 * (int64_t(1) << logK);
  }
  z->Nt = int64_t(1) << logNt;
  z->C = (int)(z->Nz / 2 + 1);
  z->tiles = (z->C + 7) / 8;
  z->plan_bytes = align_up(16 * int64_t(z->C) * z->Nt);
  // plan scratch: limb-norm counters + the row spectra of h; the tuning runs
  // reuse it as row spectra of x and of y (n rows each)
  const int64_t h_rows = align_up(16 * 8 * int64_t(z->tiles) * (2 * n - 1));
  const int64_t xy_rows = 2 * align_up(16 * 8 * int64_t(z->tiles) * n);
  z->plan_scratch = align_up(kNormSlots * 8) + (h_rows > xy_rows ? h_rows : xy_rows);
  // matvec scratch: row spectra of x and of y
  z->mv_scratch = 2 * align_up(16 * 8 * int64_t(z->tiles) * n);
  return true;
}

// largest admissible plan over the candidate widths (smallest width = most
// limbs) and both limb transform forms
bool fft_worst_sizes(int64_t n, int32_t P, FftSizes* z) {
  bool any = false;
  for (int w = kFftWMax; w >= kFftWMin; --w)
    for (int planned = 0; planned < 2; ++planned) {
      FftSizes c;
      if (!fft_sizes(n, P, w, &c, planned == 1)) continue;
      if (!any) *z = c;
      if (c.plan_bytes > z->plan_bytes) z->plan_bytes = c.plan_bytes;
      if (c.plan_scratch > z->plan_scratch) z->plan_scratch = c.plan_scratch;
      if (c.mv_scratch > z->mv_scratch) z->mv_scratch = c.mv_scratch;
      any = true;
    }
  return any;
}

double fft_bound_for(const FftSizes& z, int64_t n, double norm_h, int pack) {
  // worst-case x: every digit at magnitude 2^(w-1)
  const double norm_x = std::ldexp(1.0, z.w - 1) * std::sqrt((double)n * (double)z.L);
  // stages: log2(N_t) + log2(N_z) butterfly stages, plus the real-input
  // packing / unpacking step counted as two more.  For N_z = 3K the radix-3
  // step (one tabulated root and one constant multiplication along each data
  // path, sums that grow the norm by sqrt 3 < 2) counts as two binary stages,
  // and the inexact 1/3 of the scaling of the resident spectrum as one more.
  // The packed column of the two real bins adds one rounded sum or
  // difference with the partner bin on the x side, one on the h side and one
  // sum of two products: one more stage.
  const int k = (z.z3 ? z.logNt + z.logM + 2 + 1 + 2 : z.logNt + (z.logM + 1) + 2) + pack;
  return fft_conv_bound(norm_h, norm_x, k, fft_twiddle_beta());
}

}  // namespace hmv

// ------------------------------------------------------------------ split-FFT
namespace {

// Launch tuning.  For each shape the planner times, on the plan's own data,
// every combination of the spectrum tile widths (2, 4 or 8 bins for the
// spectra of x and of y) and the launch variants of the column pass and of
// the inverse row pass (kernels.h) over one whole matvec pipeline; the four
// fastest and the untuned default are timed again in interleaved rounds, and
// a choice replaces the default only if it is more than 1 % faster.  Results
// are cached per (device, n, P, w), so later plans of a shape (and one-shot
// calls) reuse them.
struct TuneChoice {
  int cols_variant, rows_inv_variant, ltx, lty;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int32_t, int>, TuneChoice> g_tune_cache;
int g_autotune = 1;
int g_force_cols = -1, g_force_rinv = -1;       // tests: fixed variants (-1 = tune)
int g_force_z3 = -1, g_force_pack = -1;         // tests: fixed spectrum layout (-1 = auto)
int g_force_ltx = -1, g_force_lty = -1;         // tests: fixed tile widths (-1 = tune)
constexpr int kDefaultTileLog = 2;              // 4 bins per tile when not tuned

bool radix8_ok(int logn) { return logn == 6 || logn == 9 || logn == 12; }

// Average time of `reps` launches after one warm-up, in milliseconds.
template <class F>
hipError_t time_launches(F launch, int reps, hipEvent_t a, hipEvent_t b, hipStream_t s,
                         float* ms) {
  hipError_t e = launch();
  if (e == hipSuccess) e = hipEventRecord(a, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  if (e == hipSuccess) *ms /= (float)reps;
  return e;
}

void apply_forced(hmv_plan* p) {
  if (g_force_cols >= 0) p->cols_variant = g_force_cols;
  if (g_force_rinv >= 0) p->rows_inv_variant = p->z3 ? 0 : g_force_rinv;
  if (g_force_ltx >= 0) p->ltx = g_force_ltx;
  if (g_force_lty >= 0) p->lty = g_force_lty;
}

// The first n rows of h stand in for x (valid inputs of the same shape); the
// outputs are discarded and the status block is cleared afterwards.
// Without may_run (one-shot calls) a shape that has not been tuned keeps
// the first variants and the default tile widths.
int fft_tune(hmv_plan* p, const uint64_t* h, DevStatus* st, char* scratch, bool may_run,
             hipStream_t s) {
  p->cols_variant = 0;
  p->rows_inv_variant = 0;
  p->ltx = p->lty = kDefaultTileLog;
  if (!g_autotune) {
    apply_forced(p);
    return HMV_OK;
  }
  const std::tuple<int, int64_t, int32_t, int> key{p->device, p->n, p->P, p->w};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      p->cols_variant = it->second.cols_variant;
      p->rows_inv_variant = it->second.rows_inv_variant;
      p->ltx = it->second.ltx;
      p->lty = it->second.lty;
      apply_forced(p);
      return HMV_OK;
    }
  }
  if (!may_run) {
    apply_forced(p);
    return HMV_OK;
  }
  const int n = (int)p->n, W = (int)words_of(p->P);
  double2* X1 = reinterpret_cast<double2*>(scratch + align_up(kNormSlots * 8));
  double2* Y1 = X1 + align_up(16 * 8 * int64_t(p->tiles) * n) / 16;
  uint64_t* yt = reinterpret_cast<uint64_t*>(X1);      // x's spectra are no longer needed then
  auto fwd = [&](int ltx) {
    return p->z3 ? launch_rows_fwd3(h, W, p->P, p->w, p->L, n, 0, p->logM, X1, n, p->pack, ltx,
                                    st, s)
                 : launch_rows_fwd(h, W, p->P, p->w, p->L, n, 0, p->logM, X1, n, p->pack, ltx,
                                   st, s);
  };
  auto inv = [&](int lty, int v) {
    return p->z3 ? launch_rows_inv3(Y1, n, p->logM, p->L, p->w, p->P, W, 0, p->pack, lty, yt, st,
                                    s)
                 : launch_rows_inv(Y1, n, p->logM, p->L, p->w, p->P, W, 0, p->pack, lty, yt, st,
                                   v, s);
  };
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  // every choice, timed over a whole matvec pipeline (forward rows, column
  // pass, inverse rows)
  std::vector<TuneChoice> cand;
  for (int lx = 1; lx <= kMaxTileLog; ++lx)
    for (int ly = 1; ly <= kMaxTileLog; ++ly)
      for (int cv = 0; cv < kColsVariants; ++cv) {
        if ((cv & 1) && !radix8_ok(p->logNt - 1)) continue;
        for (int rv = 0; rv < kRowsInvVariants; ++rv) {
          if ((rv & 1) && (p->z3 || !radix8_ok(p->logM))) continue;
          cand.push_back({cv, rv, lx, ly});
        }
      }
  auto pipeline = [&](const TuneChoice& c) {
    hipError_t r = fwd(c.ltx);
    if (r == hipSuccess)
      r = launch_cols_pass(X1, p->Hh, n, p->C, p->logNt, p->pack, Y1, c.cols_variant, c.ltx,
                           c.lty, s);
    if (r == hipSuccess) r = inv(c.lty, c.rows_inv_variant);
    return r;
  };
  std::vector<float> t1(cand.size(), 0.0f);
  for (size_t k = 0; k < cand.size() && e == hipSuccess; ++k)
    e = time_launches([&] { return pipeline(cand[k]); }, 2, a, b, s, &t1[k]);
  // the four fastest and the untuned default, re-timed in interleaved rounds
  std::vector<size_t> order(cand.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](size_t u, size_t v) { return t1[u] < t1[v]; });
  std::vector<TuneChoice> fin;
  fin.push_back({0, 0, kDefaultTileLog, kDefaultTileLog});
  for (size_t k = 0; k < order.size() && fin.size() < 5; ++k) {
    const TuneChoice& c = cand[order[k]];
    if (c.cols_variant == 0 && c.rows_inv_variant == 0 && c.ltx == kDefaultTileLog &&
        c.lty == kDefaultTileLog)
      continue;
    fin.push_back(c);
  }
  std::vector<float> t2(fin.size(), 0.0f);
  for (int round = 0; round < 3 && e == hipSuccess; ++round)
    for (size_t k = 0; k < fin.size() && e == hipSuccess; ++k) {
      float ms = 0.0f;
      e = time_launches([&] { return pipeline(fin[k]); }, 3, a, b, s, &ms);
      t2[k] += ms;
    }
  // the default unless a choice beats it by more than 1 %
  size_t best = 0;
  for (size_t k = 1; k < fin.size(); ++k)
    if (t2[k] < t2[best] && t2[k] < 0.99f * t2[0]) best = k;
  const int bc = fin[best].cols_variant, br = fin[best].rows_inv_variant;
  const int bx = fin[best].ltx, by = fin[best].lty;
  if (e == hipSuccess) e = launch_clear_status(st, s);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return status_from_hip(e, "tuning runs");
  p->cols_variant = bc;
  p->rows_inv_variant = br;
  p->ltx = bx;
  p->lty = by;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {bc, br, bx, by};
  }
  apply_forced(p);
  return HMV_OK;
}

int fft_plan_build(hmv_plan* p, const uint64_t* h, DevStatus* st, char* scratch,
                   int64_t scratch_bytes, char* plan_mem, int64_t plan_bytes, int force_w,
                   bool may_tune, hipStream_t s) {
  const int64_t n = p->n;
  const int32_t P = p->P;
  const int W = (int)words_of(P);
  FftSizes worst;
  if (!fft_worst_sizes(n, P, &worst)) return HMV_EUNSUPPORTED;
  if (scratch_bytes < worst.plan_scratch) return HMV_ENOMEM;
  hipError_t e = fft_tables_init();
  if (e != hipSuccess) return status_from_hip(e, "fft tables");
  const int gather = (p->kind == HMV_CIRCULANT) ? (int)n : 0;
  const int rows = (int)(2 * n - 1);
  // 1. limb norms of h for every candidate width
  unsigned long long* norms = reinterpret_cast<unsigned long long*>(scratch);
  char* h1mem = scratch + align_up(kNormSlots * 8);
  const bool allow3 = g_force_z3 != 0;
  int wlo = kFftWMax, whi = kFftWMin;
  for (int w = kFftWMin; w <= kFftWMax; ++w) {
    FftSizes c;
    if (fft_sizes(n, P, w, &c, allow3)) {
      if (w < wlo) wlo = w;
      if (w > whi) whi = w;
    }
  }
  if (force_w > 0) wlo = whi = force_w;
  e = hipMemsetAsync(norms, 0, kNormSlots * 8, s);
  if (e != hipSuccess) return status_from_hip(e, "memset norms");
  e = launch_h_norms(h, W, P, rows, gather, wlo, whi, norms, st, s);
  if (e != hipSuccess) return status_from_hip(e, "h norms");
  unsigned long long hn[kNormSlots];
  DevStatus hs;
  e = hipMemcpyAsync(hn, norms, sizeof(hn), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return status_from_hip(e, "read norms");
  if (hs.flags & ST_RANGE) return HMV_ERANGE;
  // 2. largest width whose proven bound is below 1/2
  FftSizes z;
  bool found = false;
  int pack = 0;
  for (int w = whi; w >= wlo && !found; --w) {
    FftSizes c;
    if (!fft_sizes(n, P, w, &c, allow3)) continue;
    const double nh = std::sqrt((double)hn[w - wlo]);
    // every true coefficient is an integer of magnitude <= n L 4^(w-1) < 2^50
    // (the rounding step converts with a 1.5 * 2^52 offset, exact below 2^51)
    const double cmax = (double)n * c.L * std::ldexp(1.0, 2 * (w - 1));
    if (cmax >= std::ldexp(1.0, 50)) continue;
    // the packed column where its bound allows it, else the plain layout
    for (int pk = 1; pk >= 0 && !found; --pk) {
      if (g_force_pack >= 0 && pk != g_force_pack) continue;
      const double b = fft_bound_for(c, n, nh, pk);
      if (b < 0.5) {
        z = c;
        pack = pk;
        p->bound = b;
        p->norm_h = nh;
        found = true;
      }
    }
  }
  if (!found) return HMV_EBOUND;
  if (plan_bytes < z.plan_bytes) return HMV_ENOMEM;
  p->w = z.w;
  p->L = z.L;
  p->logM = z.logM;
  p->z3 = z.z3;
  p->pack = pack;
  p->logNt = z.logNt;
  p->Nt = z.Nt;
  p->Nz = z.Nz;
  p->C = z.C - pack;
  p->tiles = z.tiles;
  p->beta = fft_twiddle_beta();
  p->plan_bytes_used = z.plan_bytes;
  p->mv_scratch = z.mv_scratch;
  p->Hh = reinterpret_cast<double2*>(plan_mem);
  // 3. forward 2-D transform of h, kept in the plan
  double2* H1 = reinterpret_cast<double2*>(h1mem);
  e = z.z3 ? launch_rows_fwd3(h, W, P, z.w, z.L, rows, gather, z.logM, H1, rows, pack,
                              kDefaultTileLog, st, s)
           : launch_rows_fwd(h, W, P, z.w, z.L, rows, gather, z.logM, H1, rows, pack,
                             kDefaultTileLog, st, s);
  if (e != hipSuccess) return status_from_hip(e, "rows fwd (h)");
  // 1 / (N_t N_z): a power of two, or for N_z = 3K one rounding of 1/3
  const double scale = z.z3 ? std::ldexp(1.0 / 3.0, -(z.logNt + z.logM))
                            : std::ldexp(1.0, -(z.logNt + z.logM + 1));
  e = launch_cols_plan(H1, rows, p->C, z.logNt, scale, pack, kDefaultTileLog, p->Hh, s);
  if (e != hipSuccess) return status_from_hip(e, "cols plan");
  // 4. tile widths and launch variants for this shape (h's first n rows
  //    stand in for x)
  return fft_tune(p, h, st, scratch, may_tune, s);
}

hipError_t mark(void* const* ev, int k, hipStream_t s) {
  if (!ev || !ev[k]) return hipSuccess;
  return hipEventRecord(static_cast<hipEvent_t>(ev[k]), s);
}

// Workspace after the status block for a block of kvec vectors: the row
// spectra of x and of y, kvec n rows each.
int64_t fft_mv_scratch(const hmv_plan* p, int kvec) {
  return 2 * align_up(16 * 8 * int64_t(p->tiles) * p->n * kvec);
}

// kvec vectors at once (x and y hold kvec n numbers, vector after vector):
// each row pass covers all kvec n rows in one launch, and the index-axis
// pass reads each resident column once for the kvec vectors (its kvec
// work-groups of a column share one L2).
// exact_words > 0: each output is the exact sum S_i, unrounded, in
// exact_words words (the carry step with P = 0) instead of y_i.
int fft_plan_matvec(const hmv_plan* p, const uint64_t* x, uint64_t* y, DevStatus* st,
                    char* scratch, int64_t scratch_bytes, hipStream_t s, void* const* ev,
                    int kvec = 1, int exact_words = 0) {
  const int64_t need = fft_mv_scratch(p, kvec);
  if (scratch_bytes < need) return HMV_ENOMEM;
  const int n = (int)p->n, rows = (int)(p->n * kvec);
  const int W = (int)words_of(p->P);
  const int Pout = exact_words > 0 ? 0 : p->P, Wout = exact_words > 0 ? exact_words : W;
  double2* X1 = reinterpret_cast<double2*>(scratch);
  double2* Y1 = reinterpret_cast<double2*>(scratch + need / 2);
  hipError_t e = mark(ev, 0, s);
  if (e == hipSuccess)
    e = p->z3
            ? launch_rows_fwd3(x, W, p->P, p->w, p->L, rows, 0, p->logM, X1, rows, p->pack,
                               p->ltx, st, s)
            : launch_rows_fwd(x, W, p->P, p->w, p->L, rows, 0, p->logM, X1, rows, p->pack,
                              p->ltx, st, s);
  if (e != hipSuccess) return status_from_hip(e, "rows fwd (x)");
  e = mark(ev, 1, s);
  if (e == hipSuccess)
    e = launch_cols_pass(X1, p->Hh, n, p->C, p->logNt, p->pack, Y1, p->cols_variant, p->ltx,
                         p->lty, s, kvec);
  if (e != hipSuccess) return status_from_hip(e, "cols pass");
  // Toeplitz and circulant outputs: each vector's rows reversed
  const int rev = (p->kind == HMV_HANKEL) ? 0 : n;
  e = mark(ev, 2, s);
  if (e == hipSuccess)
    e = p->z3 ? launch_rows_inv3(Y1, rows, p->logM, p->L, p->w, Pout, Wout, rev, p->pack, p->lty,
                                 y, st, s)
              : launch_rows_inv(Y1, rows, p->logM, p->L, p->w, Pout, Wout, rev, p->pack, p->lty,
                                y, st, p->rows_inv_variant, s);
  if (e == hipSuccess) e = mark(ev, 3, s);
  return status_from_hip(e, "rows inv");
}

// ------------------------------------------------------------------ exact paths
// Largest limb width whose worst-case coefficient n L 4^(w-1) stays below
// 2^62 (so the centred residue mod p is the coefficient) and whose sizes fit.
bool ntt_sizes_w(int64_t n, int32_t P, int w, NttSizes* z) {
  const int L = limbs_of(P, w);
  const long double cmax = (long double)n * L * std::ldexp(1.0L, 2 * (w - 1));
  if (cmax >= std::ldexp(1.0L, 62)) return false;
  int logNz = ilog2_ceil(2 * int64_t(L) - 1);
  if (logNz < 2) logNz = 2;
  int logNt = ilog2_ceil(2 * n - 1);
  if (logNt < 2) logNt = 2;
  if (logNz > kNttMaxLogNz || logNt > kNttMaxLogNt) return false;
  z->w = w;
  z->L = L;
  z->logNz = logNz;
  z->logNt = logNt;
  z->Nz = int64_t(1) << logNz;
  z->Nt = int64_t(1) << logNt;
  z->cols_padded = (z->Nz + 15) / 16 * 16;
  z->plan_bytes = align_up(8 * z->Nz * z->Nt);
  z->plan_scratch = align_up(8 * z->cols_padded * (2 * n - 1));
  z->mv_scratch = 2 * align_up(8 * z->cols_padded * n);
  return true;
}

bool ntt_sizes(int64_t n, int32_t P, NttSizes* z) {
  for (int w = 30; w >= 2; --w)
    if (ntt_sizes_w(n, P, w, z)) return true;
  return false;
}

int ntt_plan_build(hmv_plan* p, const uint64_t* h, DevStatus* st, char* scratch,
                   int64_t scratch_bytes, char* plan_mem, int64_t plan_bytes, hipStream_t s) {
  NttSizes z;
  if (!ntt_sizes(p->n, p->P, &z)) return HMV_EUNSUPPORTED;
  if (scratch_bytes < z.plan_scratch) return HMV_ENOMEM;
  if (plan_bytes < z.plan_bytes) return HMV_ENOMEM;
  hipError_t e = ntt_tables_init();
  if (e != hipSuccess) return status_from_hip(e, "ntt tables");
  const int n = (int)p->n, W = (int)words_of(p->P), rows = 2 * n - 1;
  const int gather = (p->kind == HMV_CIRCULANT) ? n : 0;
  p->w = z.w;
  p->L = z.L;
  p->logNz = z.logNz;
  p->logNt = z.logNt;
  p->Nt = z.Nt;
  p->Nz = z.Nz;
  p->cols_padded = z.cols_padded;
  p->plan_bytes_used = z.plan_bytes;
  p->mv_scratch = z.mv_scratch;
  p->Hn = reinterpret_cast<uint64_t*>(plan_mem);
  uint64_t* H1 = reinterpret_cast<uint64_t*>(scratch);
  e = launch_ntt_rows_fwd(h, W, p->P, z.w, z.L, rows, gather, z.logNz, H1, rows, kNttXLogT, st,
                          s);
  if (e != hipSuccess) return status_from_hip(e, "ntt rows fwd (h)");
  const uint64_t scale = gold_inv(gold_mul((uint64_t)z.Nt, (uint64_t)z.Nz));
  e = launch_ntt_cols_plan(H1, rows, (int)z.Nz, z.logNt, scale, p->Hn, s);
  return status_from_hip(e, "ntt cols plan");
}

int ntt_plan_matvec(const hmv_plan* p, const uint64_t* x, uint64_t* y, DevStatus* st,
                    char* scratch, int64_t scratch_bytes, hipStream_t s, void* const* ev,
                    int exact_words = 0) {
  if (scratch_bytes < p->mv_scratch) return HMV_ENOMEM;
  const int n = (int)p->n, W = (int)words_of(p->P);
  const int Pout = exact_words > 0 ? 0 : p->P, Wout = exact_words > 0 ? exact_words : W;
  uint64_t* X1 = reinterpret_cast<uint64_t*>(scratch);
  uint64_t* Y1 = reinterpret_cast<uint64_t*>(scratch + p->mv_scratch / 2);
  hipError_t e = mark(ev, 0, s);
  if (e == hipSuccess)
    e = launch_ntt_rows_fwd(x, W, p->P, p->w, p->L, n, 0, p->logNz, X1, n, kNttXLogT, st, s);
  if (e != hipSuccess) return status_from_hip(e, "ntt rows fwd (x)");
  e = mark(ev, 1, s);
  if (e == hipSuccess) e = launch_ntt_cols_pass(X1, p->Hn, n, (int)p->Nz, p->logNt, Y1, s);
  if (e != hipSuccess) return status_from_hip(e, "ntt cols pass");
  const int rev = (p->kind == HMV_HANKEL) ? 0 : 1;
  e = mark(ev, 2, s);
  if (e == hipSuccess)
    e = launch_ntt_rows_inv(Y1, n, p->logNz, p->L, p->w, Pout, Wout, rev, kNttYLogT, y, st, s);
  if (e == hipSuccess) e = mark(ev, 3, s);
  return status_from_hip(e, "ntt rows inv");
}

// ---- Karatsuba (Section 4, Algorithm 1) over the index axis
static_assert(kKaraLeaf <= kKaraWindow, "a leaf must fit the leaf kernel's window");
struct KaraTree {
  int depth = 0;
  int64_t rowsA = 0, rowsX = 0, rowsY = 0;
  std::vector<std::vector<int4>> aops, xops, cops;   // per level (split l -> l+1, combine l+1 -> l)
  std::vector<int4> leaf;
  int64_t mults = 0;
};

// Breadth-first layout of the recursion of Algorithm 1 (0-based form):
//   h_i = x_{2i}, f_i = x_{2i} - x_{2i+1}           (i < m,  x_n = 0)
//   c_i = a_{2i} + a_{2i+1}, d_i = a_{2i+1}          (i < 2m-1, a_{2n-1} = 0)
//   g_i = x_{2i-1} - x_{2i}                         (i < m1, x_{-1} = x_n = 0)
//   e_i = a_{2i}                                    (i < 2m1-1, a_{2n-1} = a_{2n} = 0)
//   p = C h, q = D f, r = E g;  y_{2i} = p_i - q_i, y_{2i+1} = p_i + r_i
// with m = floor((n+1)/2), m1 = ceil((n+1)/2); sizes <= leaf use the plain
// sum.  Rows of A (matrix vectors), X (vectors), Y (products) are numbered
// globally; every op is (out row, in row a or -1, in row b or -1, sign).
KaraTree kara_build(int64_t n, int leaf_max) {
  struct Node { int64_t m, a, x, y; };
  KaraTree T;
  std::vector<Node> level = {{n, 0, 0, 0}};
  T.rowsA = 2 * n - 1;
  T.rowsX = n;
  T.rowsY = n;
  while (!level.empty()) {
    std::vector<Node> next;
    std::vector<int4> aops, xops, cops;
    for (const Node& nd : level) {
      const int64_t m = nd.m;
      if (m <= leaf_max) {
        T.leaf.push_back(make_int4((int)nd.a, (int)nd.x, (int)nd.y, (int)m));
        T.mults += m * m;
        continue;
      }
      const int64_t mc = (m + 1) / 2, m1 = (m + 2) / 2;
      auto arow = [&](int64_t r) { return (r >= 0 && r <= 2 * m - 2) ? (int)(nd.a + r) : -1; };
      auto xrow = [&](int64_t r) { return (r >= 0 && r < m) ? (int)(nd.x + r) : -1; };
      Node C{mc, T.rowsA, T.rowsX, T.rowsY};
      T.rowsA += 2 * mc - 1; T.rowsX += mc; T.rowsY += mc;
      Node D{mc, T.rowsA, T.rowsX, T.rowsY};
      T.rowsA += 2 * mc - 1; T.rowsX += mc; T.rowsY += mc;
      Node E{m1, T.rowsA, T.rowsX, T.rowsY};
      T.rowsA += 2 * m1 - 1; T.rowsX += m1; T.rowsY += m1;
      for (int64_t i = 0; i < 2 * mc - 1; ++i) {
        aops.push_back(make_int4((int)(C.a + i), arow(2 * i), arow(2 * i + 1), 1));
        aops.push_back(make_int4((int)(D.a + i), -1, arow(2 * i + 1), 1));
      }
      for (int64_t i = 0; i < 2 * m1 - 1; ++i)
        aops.push_back(make_int4((int)(E.a + i), arow(2 * i), -1, 1));
      for (int64_t i = 0; i < mc; ++i) {
        xops.push_back(make_int4((int)(C.x + i), xrow(2 * i), -1, 1));
        xops.push_back(make_int4((int)(D.x + i), xrow(2 * i), xrow(2 * i + 1), -1));
      }
      for (int64_t i = 0; i < m1; ++i)
        xops.push_back(make_int4((int)(E.x + i), xrow(2 * i - 1), xrow(2 * i), -1));
      for (int64_t i = 0; i < mc; ++i) {
        cops.push_back(make_int4((int)(nd.y + 2 * i), (int)(C.y + i), (int)(D.y + i), -1));
        if (2 * i + 1 < m)
          cops.push_back(make_int4((int)(nd.y + 2 * i + 1), (int)(C.y + i), (int)(E.y + i), 1));
      }
      next.push_back(C);
      next.push_back(D);
      next.push_back(E);
    }
    if (!next.empty()) {
      T.aops.push_back(std::move(aops));
      T.xops.push_back(std::move(xops));
      T.cops.push_back(std::move(cops));
    }
    level.swap(next);
  }
  T.depth = (int)T.xops.size();
  return T;
}

struct KaraSizes {
  NttSizes z;
  int64_t rowsA, rowsX, rowsY, nx, nc, nl, na;
  int64_t plan_bytes, plan_scratch, mv_scratch;
};

bool kara_sizes(int64_t n, int32_t P, KaraSizes* k, KaraTree* tree_out) {
  if (!ntt_sizes(n, P, &k->z)) return false;
  KaraTree T = kara_build(n, kKaraLeaf);
  if (T.rowsA > INT32_MAX / 2) return false;
  k->rowsA = T.rowsA;
  k->rowsX = T.rowsX;
  k->rowsY = T.rowsY;
  k->nx = k->nc = k->na = 0;
  for (auto& v : T.xops) k->nx += (int64_t)v.size();
  for (auto& v : T.cops) k->nc += (int64_t)v.size();
  for (auto& v : T.aops) k->na += (int64_t)v.size();
  k->nl = (int64_t)T.leaf.size();
  const int64_t Nz = k->z.Nz;
  k->plan_bytes = align_up(8 * Nz * T.rowsA) + align_up(16 * k->nx) + align_up(16 * k->nc) +
                  align_up(16 * k->nl);
  k->plan_scratch = align_up(16 * (k->na > 0 ? k->na : 1));
  k->mv_scratch = align_up(8 * Nz * T.rowsX) + align_up(8 * Nz * T.rowsY);
  if (tree_out) *tree_out = std::move(T);
  return true;
}

int kara_plan_build(hmv_plan* p, const uint64_t* h, DevStatus* st, char* scratch,
                    int64_t scratch_bytes, char* plan_mem, int64_t plan_bytes, hipStream_t s) {
  KaraSizes k;
  KaraTree T;
  if (!kara_sizes(p->n, p->P, &k, &T)) return HMV_EUNSUPPORTED;
  if (scratch_bytes < k.plan_scratch || plan_bytes < k.plan_bytes) return HMV_ENOMEM;
  hipError_t e = ntt_tables_init();
  if (e != hipSuccess) return status_from_hip(e, "ntt tables");
  const int n = (int)p->n, W = (int)words_of(p->P), rows = 2 * n - 1;
  const NttSizes& z = k.z;
  const int64_t Nz = z.Nz;
  p->w = z.w;
  p->L = z.L;
  p->logNz = z.logNz;
  p->Nz = Nz;
  p->Nt = 0;
  p->rowsA = k.rowsA;
  p->rowsX = k.rowsX;
  p->rowsY = k.rowsY;
  p->depth = T.depth;
  p->leaves_mults = T.mults;
  p->plan_bytes_used = k.plan_bytes;
  p->mv_scratch = k.mv_scratch;
  char* q = plan_mem;
  p->Hn = reinterpret_cast<uint64_t*>(q);
  q += align_up(8 * Nz * k.rowsA);
  int4* d_x = reinterpret_cast<int4*>(q);
  q += align_up(16 * k.nx);
  int4* d_c = reinterpret_cast<int4*>(q);
  q += align_up(16 * k.nc);
  int4* d_l = reinterpret_cast<int4*>(q);
  p->d_xops = d_x;
  p->d_cops = d_c;
  p->d_leaf = d_l;
  p->nleaf = (int)k.nl;
  // flatten the per-level op lists
  std::vector<int4> xs, cs, as;
  std::vector<int> aoff, acnt;
  p->xops_off.clear();
  p->xops_cnt.clear();
  p->cops_off.clear();
  p->cops_cnt.clear();
  for (int l = 0; l < T.depth; ++l) {
    p->xops_off.push_back((int)xs.size());
    p->xops_cnt.push_back((int)T.xops[l].size());
    xs.insert(xs.end(), T.xops[l].begin(), T.xops[l].end());
    p->cops_off.push_back((int)cs.size());
    p->cops_cnt.push_back((int)T.cops[l].size());
    cs.insert(cs.end(), T.cops[l].begin(), T.cops[l].end());
    aoff.push_back((int)as.size());
    acnt.push_back((int)T.aops[l].size());
    as.insert(as.end(), T.aops[l].begin(), T.aops[l].end());
  }
  int4* d_a = reinterpret_cast<int4*>(scratch);
  if (!xs.empty()) e = hipMemcpyAsync(d_x, xs.data(), 16 * xs.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !cs.empty())
    e = hipMemcpyAsync(d_c, cs.data(), 16 * cs.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !T.leaf.empty())
    e = hipMemcpyAsync(d_l, T.leaf.data(), 16 * T.leaf.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !as.empty())
    e = hipMemcpyAsync(d_a, as.data(), 16 * as.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return status_from_hip(e, "karatsuba op lists");
  // limb spectra of h (row-major), scaled by 1/N_z for the inverse transform
  const int gather = (p->kind == HMV_CIRCULANT) ? n : 0;
  e = launch_ntt_rows_fwd(h, W, p->P, z.w, z.L, rows, gather, z.logNz, p->Hn, rows, z.logNz, st, s);
  if (e == hipSuccess) e = launch_ntt_scale(p->Hn, (int64_t)rows * Nz, gold_inv((uint64_t)Nz), s);
  for (int l = 0; l < T.depth && e == hipSuccess; ++l)
    e = launch_kara_rowops(d_a + aoff[l], acnt[l], p->Hn, p->Hn, (int)Nz, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // host op lists must outlive the copies
  return status_from_hip(e, "karatsuba plan");
}

int kara_plan_matvec(const hmv_plan* p, const uint64_t* x, uint64_t* y, DevStatus* st,
                     char* scratch, int64_t scratch_bytes, hipStream_t s, void* const* ev) {
  if (scratch_bytes < p->mv_scratch) return HMV_ENOMEM;
  const int n = (int)p->n, W = (int)words_of(p->P);
  const int Nz = (int)p->Nz;
  uint64_t* X = reinterpret_cast<uint64_t*>(scratch);
  uint64_t* Y = reinterpret_cast<uint64_t*>(scratch + align_up(8 * p->Nz * p->rowsX));
  hipError_t e = mark(ev, 0, s);
  if (e == hipSuccess)
    e = launch_ntt_rows_fwd(x, W, p->P, p->w, p->L, n, 0, p->logNz, X, n, p->logNz, st, s);
  for (int l = 0; l < p->depth && e == hipSuccess; ++l)
    e = launch_kara_rowops(p->d_xops + p->xops_off[l], p->xops_cnt[l], X, X, Nz, s);
  if (e == hipSuccess) e = mark(ev, 1, s);
  if (e == hipSuccess) e = launch_kara_leaves(p->d_leaf, p->nleaf, p->Hn, X, Y, Nz, s);
  for (int l = p->depth - 1; l >= 0 && e == hipSuccess; --l)
    e = launch_kara_rowops(p->d_cops + p->cops_off[l], p->cops_cnt[l], Y, Y, Nz, s);
  if (e == hipSuccess) e = mark(ev, 2, s);
  const int rev = (p->kind == HMV_HANKEL) ? 0 : 1;
  if (e == hipSuccess)
    e = launch_ntt_rows_inv(Y, n, p->logNz, p->L, p->w, p->P, W, rev, p->logNz, y, st, s);
  if (e == hipSuccess) e = mark(ev, 3, s);
  return status_from_hip(e, "karatsuba matvec");
}

bool planned_sizes(int kind, int64_t n, int32_t P, int algo, int64_t* plan_b, int64_t* ws_b) {
  (void)kind;
  int64_t pb = 0, sb = 0;
  bool ok = false;
  if (algo == HMV_SPLIT_FFT || algo == HMV_AUTO) {
    FftSizes z;
    if (fft_worst_sizes(n, P, &z)) {
      pb = std::max(pb, z.plan_bytes);
      sb = std::max(sb, std::max(z.plan_scratch, z.mv_scratch));
      ok = true;
    }
  }
  if (algo == HMV_NTT || algo == HMV_AUTO) {
    NttSizes z;
    if (ntt_sizes(n, P, &z)) {
      pb = std::max(pb, z.plan_bytes);
      sb = std::max(sb, std::max(z.plan_scratch, z.mv_scratch));
      ok = true;
    }
  }
  if (algo == HMV_KARATSUBA) {
    KaraSizes k;
    if (kara_sizes(n, P, &k, nullptr)) {
      pb = k.plan_bytes;
      sb = std::max(k.plan_scratch, k.mv_scratch);
      ok = true;
    }
  }
  if (!ok) return false;
  *plan_b = pb;
  *ws_b = kStatusBytes + sb;
  return true;
}

bool args_ok(int kind, int64_t n, int32_t P) {
  return valid_kind(kind) && n >= 1 && n <= HMV_MAX_N && P >= 1 && P <= HMV_MAX_P;
}

}  // namespace

namespace hmv {

int64_t oneshot_planned_bytes(int kind, int64_t n, int32_t P, int algo) {
  int64_t pb, wb;
  if (!planned_sizes(kind, n, P, algo, &pb, &wb)) return HMV_EUNSUPPORTED;
  return align_up(wb) + pb;
}

int oneshot_planned(int kind, const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n,
                    int32_t P, int algo, void* ws, int64_t ws_bytes, hipStream_t s) {
  int64_t pb, wb;
  if (!planned_sizes(kind, n, P, algo, &pb, &wb)) return HMV_EUNSUPPORTED;
  if (!ws || ws_bytes < align_up(wb) + pb) return HMV_ENOMEM;
  char* base = static_cast<char*>(ws);
  hmv_plan* p = nullptr;
  // one-shot calls reuse tuned launch variants but run no tuning of their own
  int rc = plan_h_impl(&p, kind, h, n, P, algo, base + align_up(wb), pb, base, wb, s, false);
  if (rc != HMV_OK) return rc;
  // the status block keeps what the transform of h flagged (the NTT and
  // Karatsuba plans do not read it back); the matvec adds its own flags
  rc = plan_matvec_impl(p, x, y, base, wb, s, nullptr, false);
  hmv_plan_destroy(p);
  return rc;
}

}  // namespace hmv

extern "C" {

int64_t hmv_plan_bytes(int kind, int64_t n, int32_t P, int algo) {
  if (!args_ok(kind, n, P)) return HMV_EINVAL;
  int64_t pb, wb;
  if (!planned_sizes(kind, n, P, algo, &pb, &wb)) return HMV_EUNSUPPORTED;
  return pb;
}

int64_t hmv_workspace_bytes(int kind, int64_t n, int32_t P, int algo) {
  if (!args_ok(kind, n, P)) return HMV_EINVAL;
  int64_t pb, wb;
  if (!planned_sizes(kind, n, P, algo, &pb, &wb)) return HMV_EUNSUPPORTED;
  return wb;
}

int hmv_plan_h(hmv_plan** out, int kind, const uint64_t* h, int64_t n, int32_t P, int algo,
               void* plan_mem, int64_t plan_bytes, void* ws, int64_t ws_bytes, void* stream) {
  return plan_h_impl(out, kind, h, n, P, algo, plan_mem, plan_bytes, ws, ws_bytes, stream, true);
}

}  // extern "C"

namespace hmv {

int plan_h_impl(hmv_plan** out, int kind, const uint64_t* h, int64_t n, int32_t P, int algo,
                void* plan_mem, int64_t plan_bytes, void* ws, int64_t ws_bytes, void* stream,
                bool may_tune) {
  if (!out || !h || !plan_mem || !ws) return HMV_EINVAL;
  if (!args_ok(kind, n, P)) return HMV_EINVAL;
  *out = nullptr;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (algo < HMV_AUTO || algo > HMV_KARATSUBA) return HMV_EINVAL;
  if (ws_bytes < kStatusBytes) return HMV_ENOMEM;
  const int a = algo;
  hmv_plan* p = new (std::nothrow) hmv_plan();
  if (!p) return HMV_ENOMEM;
  p->kind = kind;
  p->n = n;
  p->P = P;
  p->algo = a;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return HMV_EDEVICE;
  }
  DevStatus* st = static_cast<DevStatus*>(ws);
  hipError_t e = launch_clear_status(st, s);
  if (e != hipSuccess) {
    delete p;
    return status_from_hip(e, "clear status");
  }
  char* scratch = static_cast<char*>(ws) + kStatusBytes;
  const int64_t scratch_bytes = ws_bytes - kStatusBytes;
  int rc = HMV_EUNSUPPORTED;
  char* pm = static_cast<char*>(plan_mem);
  if (a == HMV_SPLIT_FFT || a == HMV_AUTO) {
    p->algo = HMV_SPLIT_FFT;
    rc = fft_plan_build(p, h, st, scratch, scratch_bytes, pm, plan_bytes, g_force_w, may_tune, s);
    if (a == HMV_AUTO && (rc == HMV_EBOUND || rc == HMV_EUNSUPPORTED)) {
      // no binary64 width passes the bound: fall back to the exact NTT path
      p->algo = HMV_NTT;
      e = launch_clear_status(st, s);
      if (e != hipSuccess) rc = status_from_hip(e, "clear status");
      else rc = ntt_plan_build(p, h, st, scratch, scratch_bytes, pm, plan_bytes, s);
    }
  } else if (a == HMV_NTT) {
    rc = ntt_plan_build(p, h, st, scratch, scratch_bytes, pm, plan_bytes, s);
  } else if (a == HMV_KARATSUBA) {
    rc = kara_plan_build(p, h, st, scratch, scratch_bytes, pm, plan_bytes, s);
  }
  if (rc != HMV_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return HMV_OK;
}

}  // namespace hmv

extern "C" {

int hmv_plan_matvec(const hmv_plan* p, const uint64_t* x, uint64_t* y, void* ws, int64_t ws_bytes,
                    void* stream) {
  return hmv_plan_matvec_events(p, x, y, ws, ws_bytes, stream, nullptr);
}

int hmv_plan_matvec_events(const hmv_plan* p, const uint64_t* x, uint64_t* y, void* ws,
                           int64_t ws_bytes, void* stream, void* const* events) {
  return hmv::plan_matvec_impl(p, x, y, ws, ws_bytes, static_cast<hipStream_t>(stream), events,
                               true);
}

}  // extern "C"

namespace hmv {

int plan_matvec_impl(const ::hmv_plan* p, const uint64_t* x, uint64_t* y, void* ws,
                     int64_t ws_bytes, hipStream_t s, void* const* events, bool clear) {
  if (!p || !x || !y || !ws) return HMV_EINVAL;
  if (ws_bytes < kStatusBytes) return HMV_ENOMEM;
  return plan_matvec_parts(p, x, y, static_cast<DevStatus*>(ws),
                           static_cast<char*>(ws) + kStatusBytes, ws_bytes - kStatusBytes, s,
                           events, clear);
}

int plan_matvec_parts(const ::hmv_plan* p, const uint64_t* x, uint64_t* y, DevStatus* st,
                      char* scratch, int64_t scratch_bytes, hipStream_t s, void* const* events,
                      bool clear, int exact_words) {
  if (!p || !x || !y || !st || !scratch) return HMV_EINVAL;
  clear_stale_error();
  if (clear) {
    hipError_t e = launch_clear_status(st, s);
    if (e != hipSuccess) return status_from_hip(e, "clear status");
  }
  if (p->algo == HMV_SPLIT_FFT)
    return fft_plan_matvec(p, x, y, st, scratch, scratch_bytes, s, events, 1, exact_words);
  if (p->algo == HMV_NTT)
    return ntt_plan_matvec(p, x, y, st, scratch, scratch_bytes, s, events, exact_words);
  if (exact_words > 0) return HMV_EUNSUPPORTED;
  if (p->algo == HMV_KARATSUBA)
    return kara_plan_matvec(p, x, y, st, scratch, scratch_bytes, s, events);
  return HMV_EUNSUPPORTED;
}

int plan_matvec_multi_impl(const ::hmv_plan* p, int32_t k, const uint64_t* x, uint64_t* y,
                           void* ws, int64_t ws_bytes, hipStream_t s, void* const* events) {
  if (!p || !x || !y || !ws) return HMV_EINVAL;
  if (k < 1 || k > HMV_MAX_VECTORS) return HMV_EINVAL;
  if (ws_bytes < kStatusBytes) return HMV_ENOMEM;
  clear_stale_error();
  DevStatus* st = static_cast<DevStatus*>(ws);
  char* scratch = static_cast<char*>(ws) + kStatusBytes;
  const int64_t scratch_bytes = ws_bytes - kStatusBytes;
  if (p->algo == HMV_SPLIT_FFT) {
    if (scratch_bytes < fft_mv_scratch(p, k)) return HMV_ENOMEM;
    hipError_t e = launch_clear_status(st, s);
    if (e != hipSuccess) return status_from_hip(e, "clear status");
    return fft_plan_matvec(p, x, y, st, scratch, scratch_bytes, s, events, k);
  }
  // the exact paths: one product after another on the same workspace
  if (scratch_bytes < p->mv_scratch) return HMV_ENOMEM;
  const int64_t stride = p->n * words_of(p->P);
  for (int32_t v = 0; v < k; ++v) {
    const int rc = plan_matvec_parts(p, x + v * stride, y + v * stride, st, scratch,
                                     scratch_bytes, s, v == 0 ? events : nullptr, v == 0);
    if (rc != HMV_OK) return rc;
  }
  return HMV_OK;
}

}  // namespace hmv

extern "C" {

int64_t hmv_plan_multi_workspace_bytes(const hmv_plan* p, int32_t k) {
  if (!p || k < 1 || k > HMV_MAX_VECTORS) return HMV_EINVAL;
  if (p->algo == HMV_SPLIT_FFT) return kStatusBytes + fft_mv_scratch(p, k);
  return kStatusBytes + p->mv_scratch;
}

int hmv_plan_matvec_multi(const hmv_plan* p, int32_t k, const uint64_t* x, uint64_t* y,
                          void* ws, int64_t ws_bytes, void* stream, void* const* events) {
  return hmv::plan_matvec_multi_impl(p, k, x, y, ws, ws_bytes, static_cast<hipStream_t>(stream),
                                     events);
}

int64_t hmv_plan_workspace_bytes(const hmv_plan* p) {
  if (!p) return HMV_EINVAL;
  return kStatusBytes + p->mv_scratch;
}

int hmv_plan_info(const hmv_plan* p, hmv_plan_info_t* info) {
  if (!p || !info) return HMV_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->kind = p->kind;
  info->algo = p->algo;
  info->n = p->n;
  info->P = p->P;
  info->w = p->w;
  info->L = p->L;
  info->Nt = p->Nt;
  info->Nz = p->Nz;
  info->bound = p->bound;
  info->beta = p->beta;
  info->norm_h = p->norm_h;
  info->plan_bytes = p->plan_bytes_used;
  info->matvec_workspace_bytes = kStatusBytes + p->mv_scratch;
  info->cols_variant = p->cols_variant;
  info->rows_inv_variant = p->rows_inv_variant;
  info->spectrum_cols = p->C;
  if (p->algo == HMV_SPLIT_FFT) {
    info->x_tile = 1 << p->ltx;
    info->y_tile = 1 << p->lty;
  }
  return HMV_OK;
}

int hmv_debug_force_variants(int32_t cols_variant, int32_t rows_inv_variant) {
  if (cols_variant < -1 || cols_variant >= kColsVariants || rows_inv_variant < -1 ||
      rows_inv_variant >= kRowsInvVariants)
    return HMV_EINVAL;
  g_force_cols = cols_variant;
  g_force_rinv = rows_inv_variant;
  return HMV_OK;
}

int hmv_debug_force_tiles(int32_t x_tile, int32_t y_tile) {
  auto lg = [](int32_t t) { return t == 2 ? 1 : t == 4 ? 2 : t == 8 ? 3 : -2; };
  const int lx = x_tile == -1 ? -1 : lg(x_tile), ly = y_tile == -1 ? -1 : lg(y_tile);
  if (lx == -2 || ly == -2) return HMV_EINVAL;
  g_force_ltx = lx;
  g_force_lty = ly;
  return HMV_OK;
}

int hmv_debug_force_layout(int32_t z3, int32_t pack) {
  if (z3 < -1 || z3 > 1 || pack < -1 || pack > 1) return HMV_EINVAL;
  g_force_z3 = z3;
  g_force_pack = pack;
  return HMV_OK;
}

int hmv_autotune(int32_t on) {
  if (on != 0 && on != 1) return HMV_EINVAL;
  g_autotune = on;
  return HMV_OK;
}

int hmv_plan_destroy(hmv_plan* p) {
  delete p;
  return HMV_OK;
}

double hmv_fft_error_bound(double norm_h, double norm_x, int32_t log2_points, double beta) {
  return fft_conv_bound(norm_h, norm_x, log2_points, beta);
}

double hmv_twiddle_beta(void) { return fft_twiddle_beta(); }

int hmv_debug_force_width(int32_t w) {
  if (w != 0 && (w < 2 || w > 30)) return HMV_EINVAL;
  g_force_w = w;
  return HMV_OK;
}

}  // extern "C"
