// Internal launcher declarations shared by the HIP translation units and the
// C-ABI layer.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hmv {

struct DevStatus;

constexpr int kMaxWords = 648;      // W for P up to 40960 is 641
constexpr int kSchoolMaxK = 16;      // outputs per thread of the schoolbook kernel, at most
constexpr int kSchoolThreads = 512;  // work-group size of the schoolbook kernel
constexpr int kBatchThreads = 256;   // work-group size of the single-launch batch kernels

// status block
hipError_t launch_clear_status(DevStatus* st, hipStream_t s);

// schoolbook path
size_t school_lds_bytes(int L, int w, int P, int W);
hipError_t launch_split_digits_f64(const uint64_t* in, int W, int P, int w, int L, int count,
                                   int gather_n, double* out, int ld, DevStatus* st,
                                   hipStream_t s);
// schoolbook, MFMA form: 8-bit digits (int8), limb-major operands; Hs holds
// 16 copies of h's, copy s shifted by s rows
constexpr int kSchoolMfmaMaxLds = 160 * 1024;
size_t school_mfma_lds_bytes(int Lp);
hipError_t launch_split_digits_i8(const uint64_t* in, int W, int P, int L, int Lp, int count,
                                  int gather_n, int8_t* out, DevStatus* st, hipStream_t s);
hipError_t launch_transpose_i8(const int8_t* src, int R, int Lp, int8_t* dst, int Rp,
                               hipStream_t s);
hipError_t launch_school_mfma(const int8_t* Hs, const int8_t* Xt, int n, int L, int Lp, int R2,
                              int n64, int P, int W, int out_reverse, uint64_t* y, hipStream_t s);
hipError_t launch_school_rows(const double* hd, const double* xd, int n, int L, int ld, int w,
                              int P, int W, int out_reverse, uint64_t* y, hipStream_t s);

}  // namespace hmv

namespace hmv {

// split-FFT path
double fft_twiddle_beta();
hipError_t fft_tables_init();
hipError_t launch_h_norms(const uint64_t* h, int W, int P, int rows, int gather_n, int wlo,
                          int whi, unsigned long long* norms, DevStatus* st, hipStream_t s);
// pack = 1: the two real limb bins share spectrum column 0 (C = N_z/2
// columns, the resident spectrum one more); pack = 0: C = N_z/2 + 1.
// lt, ltx, lty: log2 of the tile width of a row spectrum (tidx), 0..kMaxTileLog
constexpr int kMaxTileLog = 3;
hipError_t launch_rows_fwd(const uint64_t* in, int W, int P, int w, int L, int count,
                           int gather_n, int logM, double2* out, int rows_alloc, int pack, int lt,
                           DevStatus* st, hipStream_t s);
hipError_t launch_cols_plan(const double2* H1, int rows, int C, int logNt, double scale,
                            int pack, int lt, double2* Hh, hipStream_t s);
// variant bit 0: radix-8 register transforms (where they exist, 8^k points);
// bit 1 (column pass only): linear instead of XCD-grouped column order.
constexpr int kColsVariants = 4, kRowsInvVariants = 2;
// kvec vectors: X1 and Y1 hold kvec n rows, vector v in rows v n .. v n + n - 1
hipError_t launch_cols_pass(const double2* X1, const double2* Hh, int n, int C, int logNt,
                            int pack, double2* Y1, int variant, int ltx, int lty, hipStream_t s,
                            int kvec = 1);
// inverse row passes: n rows of Y1; out_reverse = 0 writes spectrum row i to
// output row i, out_reverse = m > 0 reverses the rows within each block of m
hipError_t launch_rows_inv(const double2* Y1, int n, int logM, int L, int w, int P, int W,
                           int out_reverse, int pack, int lt, uint64_t* y, DevStatus* st,
                           int variant, hipStream_t s);
// limb transforms of 3K = 3 * 2^logK points, 6 <= logK <= kR3MaxLogK (one
// launch variant each)
hipError_t launch_rows_fwd3(const uint64_t* in, int W, int P, int w, int L, int count,
                            int gather_n, int logK, double2* out, int rows_alloc, int pack, int lt,
                            DevStatus* st, hipStream_t s);
hipError_t launch_rows_inv3(const double2* Y1, int n, int logK, int L, int w, int P, int W,
                            int out_reverse, int pack, int lt, uint64_t* y, DevStatus* st,
                            hipStream_t s);

}  // namespace hmv

namespace hmv {

// exact paths modulo 2^64 - 2^32 + 1 (NTT and Karatsuba)
// Tiles of the NTT path's row spectra (log2 residues per tile): x's and h's
// spectra in tiles of 4 (32 bytes per row, read as strided columns by the
// index-axis pass), y's in tiles of 16 (full lines for the inverse row pass)
constexpr int kNttXLogT = 2, kNttYLogT = 4;
hipError_t ntt_tables_init();
hipError_t launch_ntt_rows_fwd(const uint64_t* in, int W, int P, int w, int L, int count,
                               int gather_n, int logN, uint64_t* out, int rows_alloc, int logT,
                               DevStatus* st, hipStream_t s);
hipError_t launch_ntt_rows_inv(const uint64_t* Y, int n, int logN, int L, int w, int P, int W,
                               int out_reverse, int logT, uint64_t* y, DevStatus* st,
                               hipStream_t s);
hipError_t launch_ntt_cols_plan(const uint64_t* H1, int rows, int C, int logNt, uint64_t scale,
                                uint64_t* Hh, hipStream_t s);
hipError_t launch_ntt_cols_pass(const uint64_t* X1, const uint64_t* Hh, int n, int C, int logNt,
                                uint64_t* Y1, hipStream_t s);
hipError_t launch_kara_rowops(const int4* ops, int nops, const uint64_t* src, uint64_t* dst,
                              int Nz, hipStream_t s);
// leaves: (first A row, first X row, first Y row, size m <= kKaraWindow)
constexpr int kKaraWindow = 32;
hipError_t launch_kara_leaves(const int4* leaves, int nleaves, const uint64_t* A,
                              const uint64_t* X, uint64_t* Y, int Nz, hipStream_t s);
hipError_t launch_ntt_scale(uint64_t* a, int64_t count, uint64_t scale, hipStream_t s);

}  // namespace hmv

namespace hmv {

// one instance of a batched launch (device-side descriptor)
struct BatchInst {
  const uint64_t* h;
  const uint64_t* x;
  uint64_t* y;
  double2* H1;
  double2* Hh;
  double2* X1;
  double2* Y1;
  int n, P, W, w, L, logM, logNt, C, gather, reverse;
  double scale;
};

constexpr size_t kBatchDynLds = 72 * 1024;   // dynamic LDS of the batch kernel
// the whole batch in one cooperative launch (power-of-two limb transforms);
// starts[p] = first item of pass p (items are pass-major); grid_used gets the
// number of work-groups
hipError_t launch_batch_coop(const BatchInst* inst, const int4* items, const int* starts,
                             int nitems, DevStatus* st, int* grid_used, hipStream_t s);
hipError_t launch_batch(const BatchInst* inst, const int4* items, int nitems, int* head, int* ctr,
                        int nctr, int grid, int spin_limit, DevStatus* st, hipStream_t s);
// one pass (0 forward rows, 1 plan columns, 2 matvec columns, 3 inverse rows)
// over items whose transforms have 2^logn points; for the row passes,
// logn = kBatchLog3 + k stands for limb transforms of 3 * 2^k points
constexpr int kBatchLog3 = 16;
hipError_t launch_batch_phase(int phase, int logn, const BatchInst* inst, const int4* items,
                              int nitems, DevStatus* st, hipStream_t s);

}  // namespace hmv
