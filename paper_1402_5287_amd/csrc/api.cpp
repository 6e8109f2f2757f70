// C-ABI layer of libhmv: argument checks, workspace carving, path selection
// and kernel launches.  No device memory is ever allocated here.
#include "hmv.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "common.h"
#include "kernels.h"
#include "plan.h"

using namespace hmv;

namespace hmv {

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

void* Carver::take(int64_t bytes) {
  const int64_t start = align_up(off);
  if (start + bytes > cap) {
    ok = false;
    return nullptr;
  }
  off = start + bytes;
  return base ? base + start : nullptr;
}

bool valid_kind(int kind) { return kind == HMV_HANKEL || kind == HMV_TOEPLITZ || kind == HMV_CIRCULANT; }

int64_t words_of(int32_t P) { return (int64_t(P) + 127) / 64; }

int limbs_of(int32_t P, int w) { return (P + 2 + w - 1) / w; }

int school_width(int64_t n, int32_t P) {
  // largest w <= 16 with n * L * 4^(w-1) < 2^53: every product and partial
  // sum of the binary64 accumulation is then an exact integer.
  for (int w = 16; w >= 2; --w) {
    const int L = limbs_of(P, w);
    if (2 * L - 1 > kSchoolMaxK * 512) continue;
    if (55 - 2 * w < 0) continue;
    if ((unsigned __int128)n * (unsigned)L < ((unsigned __int128)1 << (55 - 2 * w))) return w;
  }
  return -1;
}

thread_local char g_last_error[256] = "";

int status_from_hip(hipError_t e, const char* where) {
  if (e == hipSuccess) return HMV_OK;
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where ? where : "hip",
                hipGetErrorString(e));
  return HMV_EDEVICE;
}

void clear_stale_error() { (void)hipGetLastError(); }

int fail_with(int code, const char* msg) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg ? msg : "");
  return code;
}

}  // namespace hmv

namespace {

int check_common(int kind, int64_t n, int32_t P, const void* h, const void* x, const void* y) {
  if (!valid_kind(kind)) return HMV_EINVAL;
  if (n < 1 || n > HMV_MAX_N) return HMV_EINVAL;
  if (P < 1 || P > HMV_MAX_P) return HMV_EINVAL;
  if (!h || !x || !y) return HMV_EINVAL;
  return HMV_OK;
}

// ---------------------------------------------------------------- schoolbook
struct SchoolLayout {
  int w, L, ld;
  int64_t bytes;
  int64_t off_hd, off_xd;
};

bool school_layout(int kind, int64_t n, int32_t P, SchoolLayout* lay) {
  const int w = school_width(n, P);
  if (w < 0) return false;
  lay->w = w;
  lay->L = limbs_of(P, w);
  lay->ld = (lay->L + kSchoolMaxK + 1) & ~1;   // zero digits past L for the widened steps
  Carver c{nullptr, 0, INT64_MAX, true};
  c.take(kStatusBytes);
  lay->off_hd = align_up(c.off);
  c.take((2 * n - 1) * int64_t(lay->ld) * 8);
  lay->off_xd = align_up(c.off);
  c.take(n * int64_t(lay->ld) * 8);
  lay->bytes = c.off;
  (void)kind;
  return true;
}

// MFMA form of the schoolbook: 8-bit digits; Lp limbs (a multiple of the
// 256-limb tile), the index axis padded to n64; h's limb-major rows hold R2
// >= n + n64 + 8 bytes (every stage load stays inside, zeros past 2n - 1),
// in 16 copies, copy s shifted by s rows.
struct SchoolMfmaLayout {
  int L, Lp, R2, n64;
  int64_t bytes;
  int64_t off_hd, off_ht, off_xd, off_xt;
};

bool school_mfma_layout(int64_t n, int32_t P, SchoolMfmaLayout* m) {
  m->L = limbs_of(P, 8);
  m->Lp = (m->L + 255) / 256 * 256;
  m->n64 = (int)((n + 63) / 64 * 64);
  m->R2 = (int)((n + m->n64 + 8 + 63) / 64 * 64);
  if (school_mfma_lds_bytes(m->Lp) > (size_t)kSchoolMfmaMaxLds) return false;
  if ((int64_t)m->n64 * 16384 >= (int64_t(1) << 31)) return false;   // int32 sums stay exact
  Carver c{nullptr, 0, INT64_MAX, true};
  c.take(kStatusBytes);
  m->off_hd = align_up(c.off);
  c.take((2 * n - 1) * (int64_t)m->Lp);
  m->off_ht = align_up(c.off);
  c.take(16 * (int64_t)m->Lp * m->R2);
  m->off_xd = align_up(c.off);
  c.take(n * (int64_t)m->Lp);
  m->off_xt = align_up(c.off);
  c.take((int64_t)m->Lp * m->n64);
  m->bytes = c.off;
  return true;
}

int g_school_form = -1;   // -1: the MFMA form where it applies; 0: binary64 VALU; 1: MFMA

int school_mfma_oneshot(int kind, const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n,
                        int32_t P, const SchoolMfmaLayout& m, char* base, hipStream_t s) {
  DevStatus* st = reinterpret_cast<DevStatus*>(base);
  int8_t* hd = reinterpret_cast<int8_t*>(base + m.off_hd);
  int8_t* ht = reinterpret_cast<int8_t*>(base + m.off_ht);
  int8_t* xd = reinterpret_cast<int8_t*>(base + m.off_xd);
  int8_t* xt = reinterpret_cast<int8_t*>(base + m.off_xt);
  const int W = (int)words_of(P);
  hipError_t e = launch_clear_status(st, s);
  if (e != hipSuccess) return status_from_hip(e, "clear_status");
  const int gather = (kind == HMV_CIRCULANT) ? (int)n : 0;
  e = launch_split_digits_i8(h, W, P, m.L, m.Lp, (int)(2 * n - 1), gather, hd, st, s);
  if (e == hipSuccess) e = launch_split_digits_i8(x, W, P, m.L, m.Lp, (int)n, 0, xd, st, s);
  for (int sft = 0; sft < 16 && e == hipSuccess; ++sft)
    e = launch_transpose_i8(hd + (int64_t)sft * m.Lp, (int)(2 * n - 1) - sft, m.Lp,
                            ht + (int64_t)sft * m.Lp * m.R2, m.R2, s);
  if (e == hipSuccess) e = launch_transpose_i8(xd, (int)n, m.Lp, xt, m.n64, s);
  if (e != hipSuccess) return status_from_hip(e, "school digits");
  const int rev = (kind == HMV_HANKEL) ? 0 : 1;
  e = launch_school_mfma(ht, xt, (int)n, m.L, m.Lp, m.R2, m.n64, P, W, rev, y, s);
  return status_from_hip(e, "school mfma");
}

int school_oneshot(int kind, const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n,
                   int32_t P, void* ws, int64_t ws_bytes, hipStream_t s) {
  SchoolMfmaLayout m;
  const bool mfma_ok = school_mfma_layout(n, P, &m);
  if (g_school_form != 0 && mfma_ok) {
    if (!ws || ws_bytes < m.bytes) return HMV_ENOMEM;
    return school_mfma_oneshot(kind, h, x, y, n, P, m, static_cast<char*>(ws), s);
  }
  if (g_school_form == 1) return HMV_EUNSUPPORTED;
  SchoolLayout lay;
  if (!school_layout(kind, n, P, &lay)) return HMV_EUNSUPPORTED;
  if (!ws || ws_bytes < lay.bytes) return HMV_ENOMEM;
  char* base = static_cast<char*>(ws);
  DevStatus* st = reinterpret_cast<DevStatus*>(base);
  double* hd = reinterpret_cast<double*>(base + lay.off_hd);
  double* xd = reinterpret_cast<double*>(base + lay.off_xd);
  const int W = (int)words_of(P);
  hipError_t e = launch_clear_status(st, s);
  if (e != hipSuccess) return status_from_hip(e, "clear_status");
  // The circulant is the Toeplitz matrix of the extended vector
  // c_ext[t] = c[(n-1-t) mod n], t = 0..2n-2 (gathered while splitting).
  const int gather = (kind == HMV_CIRCULANT) ? (int)n : 0;
  e = launch_split_digits_f64(h, W, P, lay.w, lay.L, (int)(2 * n - 1), gather, hd, lay.ld, st, s);
  if (e != hipSuccess) return status_from_hip(e, "split h");
  e = launch_split_digits_f64(x, W, P, lay.w, lay.L, (int)n, 0, xd, lay.ld, st, s);
  if (e != hipSuccess) return status_from_hip(e, "split x");
  const int rev = (kind == HMV_HANKEL) ? 0 : 1;
  e = launch_school_rows(hd, xd, (int)n, lay.L, lay.ld, lay.w, P, W, rev, y, s);
  return status_from_hip(e, "school rows");
}

int oneshot(int kind, const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n, int32_t P,
            int algo, void* ws, int64_t ws_bytes, void* stream) {
  int rc = check_common(kind, n, P, h, x, y);
  if (rc != HMV_OK) return rc;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (algo) {
    case HMV_SCHOOLBOOK:
      return school_oneshot(kind, h, x, y, n, P, ws, ws_bytes, s);
    case HMV_AUTO:
    case HMV_SPLIT_FFT:
    case HMV_NTT:
    case HMV_KARATSUBA:
      return oneshot_planned(kind, h, x, y, n, P, algo, ws, ws_bytes, s);
    default:
      return HMV_EINVAL;
  }
}

}  // namespace

extern "C" {

int64_t hmv_words(int32_t P) {
  if (P < 1 || P > HMV_MAX_P) return HMV_EINVAL;
  return words_of(P);
}

const char* hmv_strerror(int code) {
  switch (code) {
    case HMV_OK: return "ok";
    case HMV_EINVAL: return "invalid argument";
    case HMV_ERANGE: return "input magnitude exceeds 1";
    case HMV_ENOMEM: return "buffer too small";
    case HMV_EDEVICE: return "HIP runtime error";
    case HMV_EBOUND: return "no exact path: FP64 error bound fails and NTT is excluded";
    case HMV_EUNSUPPORTED: return "size not supported by the selected algorithm";
    default: return "unknown status";
  }
}

const char* hmv_last_error(void) { return g_last_error; }

int hmv_debug_force_school(int32_t form) {
  if (form < -1 || form > 1) return HMV_EINVAL;
  g_school_form = form;
  return HMV_OK;
}

int64_t hmv_oneshot_workspace_bytes(int kind, int64_t n, int32_t P, int algo) {
  if (!valid_kind(kind) || n < 1 || n > HMV_MAX_N || P < 1 || P > HMV_MAX_P) return HMV_EINVAL;
  if (algo == HMV_SCHOOLBOOK) {
    // enough for either form
    SchoolLayout lay;
    SchoolMfmaLayout m;
    const bool v = school_layout(kind, n, P, &lay), q = school_mfma_layout(n, P, &m);
    if (!v && !q) return HMV_EUNSUPPORTED;
    return std::max(v ? lay.bytes : 0, q ? m.bytes : 0);
  }
  return oneshot_planned_bytes(kind, n, P, algo);
}

int hmv_hankel_matvec(const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n, int32_t P,
                      int algo, void* ws, int64_t ws_bytes, void* stream) {
  return oneshot(HMV_HANKEL, h, x, y, n, P, algo, ws, ws_bytes, stream);
}

int hmv_toeplitz_matvec(const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n, int32_t P,
                        int algo, void* ws, int64_t ws_bytes, void* stream) {
  return oneshot(HMV_TOEPLITZ, h, x, y, n, P, algo, ws, ws_bytes, stream);
}

int hmv_circulant_matvec(const uint64_t* c, const uint64_t* x, uint64_t* y, int64_t n,
                         int32_t P, int algo, void* ws, int64_t ws_bytes, void* stream) {
  return oneshot(HMV_CIRCULANT, c, x, y, n, P, algo, ws, ws_bytes, stream);
}

int hmv_read_status(const void* ws, void* stream, int32_t* flags, double* max_round_err) {
  if (!ws) return HMV_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevStatus host;
  clear_stale_error();
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return status_from_hip(e, "stream sync");
  e = hipMemcpy(&host, ws, sizeof(host), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return status_from_hip(e, "status copy");
  if (flags) *flags = (int32_t)host.flags;
  if (max_round_err) {
    double d;
    std::memcpy(&d, &host.max_err_bits, sizeof(d));
    *max_round_err = d;
  }
  if (host.flags & ST_RANGE) return HMV_ERANGE;
  if (host.flags & (ST_BOUND | ST_OVERFLOW)) return HMV_EBOUND;
  if (host.flags & ST_SPIN) return HMV_EDEVICE;
  return HMV_OK;
}

}  // extern "C"
