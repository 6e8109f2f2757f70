// Plans: the transform of h kept resident (the Lanczos use of Section 1
// multiplies one fixed matrix by many vectors), limb-width selection by the
// proven error bound, and the planned matvec launches.
#include "plan.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "common.h"
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

bool fft_sizes(int64_t n, int32_t P, int w, FftSizes* z) {
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
  z->Nt = int64_t(1) << logNt;
  z->C = (int)(z->Nz / 2 + 1);
  z->tiles = (z->C + 7) / 8;
  z->plan_bytes = align_up(16 * int64_t(z->C) * z->Nt);
  // plan scratch: limb-norm counters + the row spectra of h
  z->plan_scratch = align_up(kNormSlots * 8) + align_up(16 * 8 * int64_t(z->tiles) * (2 * n - 1));
  // matvec scratch: row spectra of x and of y
  z->mv_scratch = 2 * align_up(16 * 8 * int64_t(z->tiles) * n);
  return true;
}

// largest admissible plan over the candidate widths (smallest width = most limbs)
bool fft_worst_sizes(int64_t n, int32_t P, FftSizes* z) {
  bool any = false;
  for (int w = kFftWMax; w >= kFftWMin; --w) {
    FftSizes c;
    if (!fft_sizes(n, P, w, &c)) continue;
    if (!any) *z = c;
    if (c.plan_bytes > z->plan_bytes) z->plan_bytes = c.plan_bytes;
    if (c.plan_scratch > z->plan_scratch) z->plan_scratch = c.plan_scratch;
    if (c.mv_scratch > z->mv_scratch) z->mv_scratch = c.mv_scratch;
    any = true;
  }
  return any;
}

double fft_bound_for(const FftSizes& z, int64_t n, double norm_h) {
  // worst-case x: every digit at magnitude 2^(w-1)
  const double norm_x = std::ldexp(1.0, z.w - 1) * std::sqrt((double)n * (double)z.L);
  // stages: log2(N_t) + log2(N_z) butterfly stages, plus the real-input
  // packing / unpacking step counted as two more
  const int k = z.logNt + (z.logM + 1) + 2;
  return fft_conv_bound(norm_h, norm_x, k, fft_twiddle_beta());
}

}  // namespace hmv

// ------------------------------------------------------------------ split-FFT
namespace {

int fft_plan_build(hmv_plan* p, const uint64_t* h, DevStatus* st, char* scratch,
                   int64_t scratch_bytes, char* plan_mem, int64_t plan_bytes, int force_w,
                   hipStream_t s) {
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
  int wlo = kFftWMax, whi = kFftWMin;
  for (int w = kFftWMin; w <= kFftWMax; ++w) {
    FftSizes c;
    if (fft_sizes(n, P, w, &c)) {
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
  for (int w = whi; w >= wlo; --w) {
    FftSizes c;
    if (!fft_sizes(n, P, w, &c)) continue;
    const double nh = std::sqrt((double)hn[w - wlo]);
    const double b = fft_bound_for(c, n, nh);
    // every true coefficient is an integer of magnitude <= n L 4^(w-1) < 2^52
    const double cmax = (double)n * c.L * std::ldexp(1.0, 2 * (w - 1));
    if (b < 0.5 && cmax < std::ldexp(1.0, 52)) {
      z = c;
      p->bound = b;
      p->norm_h = nh;
      found = true;
      break;
    }
  }
  if (!found) return HMV_EBOUND;
  if (plan_bytes < z.plan_bytes) return HMV_ENOMEM;
  p->w = z.w;
  p->L = z.L;
  p->logM = z.logM;
  p->logNt = z.logNt;
  p->Nt = z.Nt;
  p->Nz = z.Nz;
  p->C = z.C;
  p->tiles = z.tiles;
  p->beta = fft_twiddle_beta();
  p->plan_bytes_used = z.plan_bytes;
  p->mv_scratch = z.mv_scratch;
  p->Hh = reinterpret_cast<double2*>(plan_mem);
  // 3. forward 2-D transform of h, kept in the plan
  double2* H1 = reinterpret_cast<double2*>(h1mem);
  e = launch_rows_fwd(h, W, P, z.w, z.L, rows, gather, z.logM, H1, rows, st, s);
  if (e != hipSuccess) return status_from_hip(e, "rows fwd (h)");
  const double scale = std::ldexp(1.0, -(z.logNt + z.logM + 1));
  e = launch_cols_plan(H1, rows, z.C, z.logNt, scale, p->Hh, s);
  if (e != hipSuccess) return status_from_hip(e, "cols plan");
  return HMV_OK;
}

hipError_t mark(void* const* ev, int k, hipStream_t s) {
  if (!ev || !ev[k]) return hipSuccess;
  return hipEventRecord(static_cast<hipEvent_t>(ev[k]), s);
}

int fft_plan_matvec(const hmv_plan* p, const uint64_t* x, uint64_t* y, DevStatus* st,
                    char* scratch, int64_t scratch_bytes, hipStream_t s, void* const* ev) {
  if (scratch_bytes < p->mv_scratch) return HMV_ENOMEM;
  const int n = (int)p->n;
  const int W = (int)words_of(p->P);
  double2* X1 = reinterpret_cast<double2*>(scratch);
  double2* Y1 = reinterpret_cast<double2*>(scratch + p->mv_scratch / 2);
  hipError_t e = mark(ev, 0, s);
  if (e == hipSuccess) e = launch_rows_fwd(x, W, p->P, p->w, p->L, n, 0, p->logM, X1, n, st, s);
  if (e != hipSuccess) return status_from_hip(e, "rows fwd (x)");
  e = mark(ev, 1, s);
  if (e == hipSuccess) e = launch_cols_pass(X1, p->Hh, n, p->C, p->logNt, Y1, s);
  if (e != hipSuccess) return status_from_hip(e, "cols pass");
  const int rev = (p->kind == HMV_HANKEL) ? 0 : 1;
  e = mark(ev, 2, s);
  if (e == hipSuccess) e = launch_rows_inv(Y1, n, p->logM, p->L, p->w, p->P, W, rev, y, st, s);
  if (e == hipSuccess) e = mark(ev, 3, s);
  return status_from_hip(e, "rows inv");
}

int resolve_algo(int algo) {
  if (algo == HMV_AUTO) return HMV_SPLIT_FFT;
  return algo;
}

bool planned_sizes(int kind, int64_t n, int32_t P, int algo, int64_t* plan_b, int64_t* ws_b) {
  (void)kind;
  algo = resolve_algo(algo);
  if (algo == HMV_SPLIT_FFT) {
    FftSizes z;
    if (!fft_worst_sizes(n, P, &z)) return false;
    *plan_b = z.plan_bytes;
    *ws_b = kStatusBytes + (z.plan_scratch > z.mv_scratch ? z.plan_scratch : z.mv_scratch);
    return true;
  }
  return false;
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
  int rc = hmv_plan_h(&p, kind, h, n, P, algo, base + align_up(wb), pb, base, wb, s);
  if (rc != HMV_OK) return rc;
  rc = hmv_plan_matvec(p, x, y, base, wb, s);
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
  if (!out || !h || !plan_mem || !ws) return HMV_EINVAL;
  if (!args_ok(kind, n, P)) return HMV_EINVAL;
  *out = nullptr;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int a = resolve_algo(algo);
  if (ws_bytes < kStatusBytes) return HMV_ENOMEM;
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
  int rc;
  if (a == HMV_SPLIT_FFT) {
    rc = fft_plan_build(p, h, st, scratch, scratch_bytes, static_cast<char*>(plan_mem),
                        plan_bytes, g_force_w, s);
  } else {
    rc = HMV_EUNSUPPORTED;
  }
  if (rc != HMV_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return HMV_OK;
}

int hmv_plan_matvec(const hmv_plan* p, const uint64_t* x, uint64_t* y, void* ws, int64_t ws_bytes,
                    void* stream) {
  return hmv_plan_matvec_events(p, x, y, ws, ws_bytes, stream, nullptr);
}

int hmv_plan_matvec_events(const hmv_plan* p, const uint64_t* x, uint64_t* y, void* ws,
                           int64_t ws_bytes, void* stream, void* const* events) {
  if (!p || !x || !y || !ws) return HMV_EINVAL;
  if (ws_bytes < kStatusBytes) return HMV_ENOMEM;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevStatus* st = static_cast<DevStatus*>(ws);
  hipError_t e = launch_clear_status(st, s);
  if (e != hipSuccess) return status_from_hip(e, "clear status");
  char* scratch = static_cast<char*>(ws) + kStatusBytes;
  const int64_t scratch_bytes = ws_bytes - kStatusBytes;
  if (p->algo == HMV_SPLIT_FFT)
    return fft_plan_matvec(p, x, y, st, scratch, scratch_bytes, s, events);
  return HMV_EUNSUPPORTED;
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
