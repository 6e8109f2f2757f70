// Host-side helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "hmv.h"

namespace hmv {

constexpr int64_t kAlign = 256;
constexpr int64_t kStatusBytes = 256;

int64_t align_up(int64_t v);

// Sequential carving of a caller-owned buffer.  With base == nullptr it only
// measures.
struct Carver {
  char* base;
  int64_t off;
  int64_t cap;
  bool ok;
  void* take(int64_t bytes);
};

bool valid_kind(int kind);
int64_t words_of(int32_t P);
int limbs_of(int32_t P, int w);
int school_width(int64_t n, int32_t P);
int status_from_hip(hipError_t e, const char* where);
void clear_stale_error();

// ------------------------------------------------------------------ plans
constexpr int kFftWMin = 8;        // candidate limb widths of the binary64 path
constexpr int kFftWMax = 20;
constexpr int kFftMaxLogNz = 13;   // limb-axis real FFT up to 8192 points (LDS)
constexpr int kFftMaxLogNt = 14;   // index-axis FFT up to 16384 points (two 8192-point halves)
constexpr int kNormSlots = 32;

extern int g_force_w;              // tests: restrict the width candidates to one value

// Limb transforms: N_z = 2^(logM+1) real points, or with z3 = 1 N_z = 3 * 2^logM
// (a radix-3 step over two power-of-two transforms), where that is smaller
// and still holds the 2L - 1 coefficients.
struct FftSizes {
  int w, L, logM, logNt, C, tiles, z3;
  int64_t Nt, Nz;
  int64_t plan_bytes, plan_scratch, mv_scratch;
};

// exact paths modulo 2^64 - 2^32 + 1
constexpr int kNttMaxLogNz = 13;   // limb-axis transform up to 8192 residues (LDS)
constexpr int kNttMaxLogNt = 14;
constexpr int kKaraLeaf = 32;      // Algorithm 1 leaves: sizes <= 32 use the plain sum

struct NttSizes {
  int w, L, logNz, logNt;
  int64_t Nt, Nz, cols_padded;
  int64_t plan_bytes, plan_scratch, mv_scratch;
};

int ilog2_ceil(int64_t v);
// planned: sizes for the planned kernels, which also take the 3 * 2^k limb
// transform sizes (the batch kernels take powers of two).  C = N_z/2 + 1
// columns are allocated; a plan that packs the two real limb bins into one
// column processes C - 1 of them.
bool fft_sizes(int64_t n, int32_t P, int w, FftSizes* z, bool planned = false);
bool fft_worst_sizes(int64_t n, int32_t P, FftSizes* z);

// planned paths (split-FFT, NTT, Karatsuba) used by the one-shot entry points
int64_t oneshot_planned_bytes(int kind, int64_t n, int32_t P, int algo);
// hmv_plan_h with control over the launch tuning runs (one-shot calls pass
// false: they use tuned variants only when the shape was tuned before)
int plan_h_impl(::hmv_plan** out, int kind, const uint64_t* h, int64_t n, int32_t P, int algo,
                void* plan_mem, int64_t plan_bytes, void* ws, int64_t ws_bytes, void* stream,
                bool may_tune);
int oneshot_planned(int kind, const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n,
                    int32_t P, int algo, void* ws, int64_t ws_bytes, hipStream_t s);
// hmv_plan_matvec_events; clear = false keeps the flags already in the
// status block (a one-shot call's planning flags)
int plan_matvec_impl(const ::hmv_plan* p, const uint64_t* x, uint64_t* y, void* ws,
                     int64_t ws_bytes, hipStream_t s, void* const* events, bool clear);
// the same with the status block and the scratch given apart (the status
// block of a call need not precede its scratch)
struct DevStatus;
// exact_words > 0 (split-FFT and NTT plans): y receives the exact sums S_i,
// unrounded, exact_words words each, instead of the rounded y_i
int plan_matvec_parts(const ::hmv_plan* p, const uint64_t* x, uint64_t* y, DevStatus* st,
                      char* scratch, int64_t scratch_bytes, hipStream_t s, void* const* events,
                      bool clear, int exact_words = 0);
// records a message for hmv_last_error and returns code
int fail_with(int code, const char* msg);

}  // namespace hmv

// opaque plan handle of the C ABI (host memory only)
struct hmv_plan {
  int kind = 0, algo = 0;
  int64_t n = 0;
  int32_t P = 0;
  int device = 0;
  int w = 0, L = 0, logM = 0, logNt = 0, C = 0, tiles = 0, z3 = 0;
  int pack = 0;                    // 1: the two real limb bins share column 0 (C = N_z/2)
  int64_t Nt = 0, Nz = 0;
  double bound = 0.0, beta = 0.0, norm_h = 0.0;
  int64_t plan_bytes_used = 0, mv_scratch = 0;
  double2* Hh = nullptr;           // resident spectrum of h (in caller plan memory)
  int cols_variant = 0, rows_inv_variant = 0;   // launch variants picked by the tuning runs
  int ltx = 2, lty = 2;            // log2 tile widths of the spectra of x and of y
  // exact paths
  int logNz = 0;
  int64_t cols_padded = 0;
  uint64_t* Hn = nullptr;          // NTT: resident spectrum; Karatsuba: limb spectra of the tree
  // Karatsuba: breadth-first recursion tree as row-operation lists
  int depth = 0;
  int64_t rowsA = 0, rowsX = 0, rowsY = 0;
  const int4* d_xops = nullptr;     // x-side splits, all levels
  const int4* d_cops = nullptr;     // combines, all levels
  const int4* d_leaf = nullptr;     // leaves (A row, X row, Y row, size)
  std::vector<int> xops_off, xops_cnt, cops_off, cops_cnt;
  int nleaf = 0;
  int64_t leaves_mults = 0;         // scalar products per limb column (Algorithm 1 count)
};
