/* hmv.h -- exact multiprecision Hankel / Toeplitz / circulant matrix-vector
 * products on AMD MI355X (gfx950).  C ABI of libhmv.so.
 *
 * Problem statement (Beliakov, "On fast matrix-vector multiplication with a
 * Hankel matrix in multiprecision arithmetics", Section 4, Algorithm 1 input
 * and output): given n, a vector a of 2n-1 entries that defines the Hankel
 * matrix A_H[i][j] = a_{i+j-1} (Section 2, eq. (1)) and x of n entries,
 * compute y = A_H x.  The Toeplitz matrix of eq. (2), A_T[i][j] = a_{n-i+j},
 * uses the same 2n-1 entries; the circulant of eq. (3) is given by its first
 * column of n entries, A_C[i][j] = c_{((i-j) mod n)+1}.
 *
 * NUMBER FORMAT.  Every number is fixed point with P fractional bits: value
 * X * 2^-P, X an integer.  It is stored as W = hmv_words(P) = ceil((P+64)/64)
 * little-endian uint64 words holding X in two's complement; an array of
 * numbers is row-major [count][W].  Inputs must satisfy |value| <= 1
 * (|X| <= 2^P).  Each output y_i is the exact sum rounded once to the nearest
 * multiple of 2^-P, ties to even; |y_i| <= n fits in W words.  The result is
 * unique, so every algorithm below returns identical words.
 *
 * MEMORY.  Every array argument (h, x, y, workspaces, plan memory) is a
 * DEVICE pointer owned by the caller; the library never allocates device
 * memory (hmv_plan_matvec_noalloc takes its workspace from a fixed array
 * inside the library instead).  Sizes come from the *_bytes queries.  y
 * must not alias h, x or a workspace.  Work is enqueued on `stream` (a
 * hipStream_t; NULL = the null stream); outputs are valid once the stream
 * has synchronised.
 *
 * ERRORS.  Calls return an hmv_status code and never throw.  Argument errors
 * (n < 1, P outside [1, HMV_MAX_P], null pointers, short buffers, unknown
 * kind or algorithm) are reported synchronously as HMV_EINVAL.  Inputs with
 * |value| > 1 are detected on the device: the call still completes (with
 * unspecified y) and hmv_read_status() on its workspace returns HMV_ERANGE.
 */
#ifndef HMV_H
#define HMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HMV_MAX_P 40960
#define HMV_MAX_N 16384

typedef enum {
  HMV_OK = 0,
  HMV_EINVAL = -1,       /* bad argument                                        */
  HMV_ERANGE = -2,       /* an input had |value| > 1 (device-detected)          */
  HMV_ENOMEM = -3,       /* a caller buffer is too small                        */
  HMV_EDEVICE = -4,      /* a HIP runtime call failed                           */
  HMV_EBOUND = -5,       /* no exact path: the FP64 bound fails and NTT is off  */
  HMV_EUNSUPPORTED = -6  /* size outside what the chosen algorithm handles      */
} hmv_status;

typedef enum { HMV_HANKEL = 0, HMV_TOEPLITZ = 1, HMV_CIRCULANT = 2 } hmv_kind;

typedef enum {
  HMV_AUTO = 0,        /* split-FFT when its proven bound holds, else NTT          */
  HMV_SPLIT_FFT = 1,   /* limbs + 2-D binary64 FFT correlation (Section 3)         */
  HMV_NTT = 2,         /* limbs + 2-D number-theoretic transform mod 2^64-2^32+1   */
  HMV_KARATSUBA = 3,   /* Algorithm 1 of Section 4 over the index axis             */
  HMV_SCHOOLBOOK = 4   /* the plain O(n^2) sum of Section 2, exact on limbs        */
} hmv_algo;

/* Words per number: ceil((P+64)/64), or HMV_EINVAL if P is out of range. */
int64_t hmv_words(int32_t P);

/* Text for a status code (static storage). */
const char* hmv_strerror(int code);

/* Name and text of the last HIP runtime error seen by this thread (behind an
 * HMV_EDEVICE return); empty if none.  Thread-local static storage. */
const char* hmv_last_error(void);

/* ---------------------------------------------------------------- one-shot
 * y = A x for one matrix, with no state kept between calls.  h has 2n-1
 * numbers (Hankel, Toeplitz) or n numbers (circulant); x and y have n.
 * ws must hold hmv_oneshot_workspace_bytes(kind, n, P, algo) bytes; its
 * first 256 bytes receive the device status of this call (hmv_read_status).
 * With algo SPLIT_FFT or AUTO the call synchronises `stream` once, to read
 * the limb norms that fix the limb width (the error bound needs them).     */
int64_t hmv_oneshot_workspace_bytes(int kind, int64_t n, int32_t P, int algo);
int hmv_hankel_matvec(const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n, int32_t P,
                      int algo, void* ws, int64_t ws_bytes, void* stream);
int hmv_toeplitz_matvec(const uint64_t* h, const uint64_t* x, uint64_t* y, int64_t n, int32_t P,
                        int algo, void* ws, int64_t ws_bytes, void* stream);
int hmv_circulant_matvec(const uint64_t* c, const uint64_t* x, uint64_t* y, int64_t n,
                         int32_t P, int algo, void* ws, int64_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- plans
 * plan_h keeps the 2-D transform of h resident in caller memory so that a
 * session of matvecs with one fixed matrix (the repeated products of a
 * Lanczos iteration, Section 1) pays for it once.
 *
 * hmv_plan_bytes / hmv_workspace_bytes give sizes that hold for every limb
 * width and spectrum layout the planner may pick (the width depends on the
 * data of h through the error bound; the layout, limb transforms of a power
 * of two or of 3 * 2^k points, on the width); hmv_plan_info reports the
 * bytes the plan actually uses.  plan_mem must stay valid and unmodified while the plan
 * is used; ws is scratch for plan_h and for each plan_matvec, and its first
 * 256 bytes receive the device status of that call.  hmv_plan_h synchronises
 * `stream` once (limb norms); hmv_plan_matvec is fully asynchronous.  A plan
 * is immutable: several streams may use it at once, each with its own ws.
 * The handle is host memory; hmv_plan_destroy frees only the handle.      */
typedef struct hmv_plan hmv_plan;

typedef struct {
  int32_t kind, algo;     /* algo actually used                                 */
  int64_t n;
  int32_t P, w, L;        /* limb width and limbs per number                     */
  int64_t Nt, Nz;         /* FFT / NTT sizes on the index and limb axes          */
  double bound;           /* proven bound on |coefficient error| (FP64 path)     */
  double beta;            /* bound on the error of the tabulated roots           */
  double norm_h;          /* Euclidean norm of the limb digits of h              */
  int64_t plan_bytes;     /* plan memory actually used                           */
  int64_t matvec_workspace_bytes;
  int32_t cols_variant;   /* split-FFT launch variants (see hmv_autotune)        */
  int32_t rows_inv_variant;
  int32_t spectrum_cols;  /* split-FFT: limb-frequency columns of the spectra of
                             x and y, Nz/2 when the two real limb bins share one
                             column (the error bound allows it), else Nz/2 + 1;
                             0 for the other paths                             */
  int32_t reserved;
  int32_t x_tile, y_tile; /* split-FFT: bins per tile of the stored spectra of x
                             and of y (2, 4 or 8; picked by the tuning runs) */
} hmv_plan_info_t;

int64_t hmv_plan_bytes(int kind, int64_t n, int32_t P, int algo);
int64_t hmv_workspace_bytes(int kind, int64_t n, int32_t P, int algo);
int hmv_plan_h(hmv_plan** out, int kind, const uint64_t* h, int64_t n, int32_t P, int algo,
               void* plan_mem, int64_t plan_bytes, void* ws, int64_t ws_bytes, void* stream);
int hmv_plan_matvec(const hmv_plan* plan, const uint64_t* x, uint64_t* y, void* ws,
                    int64_t ws_bytes, void* stream);
/* Same as hmv_plan_matvec, and records caller-created HIP events (hipEvent_t,
 * NULL entries skipped) on `stream` around the path's kernels, for per-kernel
 * timing.  Split-FFT and NTT: events[0] before the limb-axis forward pass,
 * [1] before the index-axis pass, [2] before the limb-axis inverse / carry
 * pass, [3] after it.  Karatsuba: [0] before the limb transforms of x, [1]
 * before the leaf products (after the splitting levels), [2] before the
 * inverse / carry pass (after the combining levels), [3] after it.          */
int hmv_plan_matvec_events(const hmv_plan* plan, const uint64_t* x, uint64_t* y, void* ws,
                           int64_t ws_bytes, void* stream, void* const* events);
int64_t hmv_plan_workspace_bytes(const hmv_plan* plan);
/* A block of k vectors with the same plan, Y = A [x_1 .. x_k] (the repeated
 * products with one fixed matrix of Section 1, several at a time: block
 * Lanczos, or independent sessions on one matrix).  x and y hold k n
 * numbers each, vector after vector ([k][n][W] words); 1 <= k <=
 * HMV_MAX_VECTORS.  ws must hold hmv_plan_multi_workspace_bytes(plan, k)
 * bytes (status block first).  Split-FFT plans run every pass once for the
 * whole block and read the resident transform of h about once per block
 * instead of once per vector; NTT and Karatsuba plans run the k products one
 * after another on one workspace.  Every output equals hmv_plan_matvec of
 * its vector.  events: NULL, or 4 events as in hmv_plan_matvec_events,
 * recorded around the block's passes (the first product's for the other
 * paths).  Asynchronous on `stream`.                                        */
#define HMV_MAX_VECTORS 64
int64_t hmv_plan_multi_workspace_bytes(const hmv_plan* plan, int32_t k);
int hmv_plan_matvec_multi(const hmv_plan* plan, int32_t k, const uint64_t* x, uint64_t* y,
                          void* ws, int64_t ws_bytes, void* stream, void* const* events);
/* Launch tuning of the split-FFT path (on by default).  When on, planning a
 * shape (n, P, limb width) for the first time in the process also times, on
 * the plan's own data (the first n rows of h standing in for x), every pair
 * of tile widths (2, 4 or 8 bins) of the stored spectra of x and of y over
 * a whole matvec, then at the chosen widths each launch variant of the
 * index-axis pass (radix-16 or radix-8 register transforms; XCD-grouped or
 * linear column order) and of the inverse limb pass (radix 16 or 8), and
 * keeps the fastest; later plans of that shape, and one-shot calls, reuse
 * the choice.  Every choice computes the same words.  Off: the first
 * variant of each and tiles of 4 bins.  Process-wide; returns HMV_EINVAL
 * for values other than 0 and 1.                                           */
int hmv_autotune(int32_t on);
int hmv_plan_info(const hmv_plan* plan, hmv_plan_info_t* info);
int hmv_plan_destroy(hmv_plan* plan);

/* ---------------------------------------------------------------- Lanczos
 * Lanczos tridiagonalisation over a Hankel plan (Section 1: repeated
 * products with one symmetric matrix reduce it to tridiagonal form, whose
 * eigenvalues QR iterations then find), in P-bit fixed point.  Every scalar
 * and entry is one rounding (nearest, ties to even, at 2^-P) of an exact
 * expression; from q_1 (|entries| <= 1, normally unit 2-norm), beta_1 = 0:
 *   w = A q_j (hmv_plan_matvec),  alpha_j = rne(q_j . w),
 *   r_i = rne(w_i - alpha_j q_j,i - beta_j q_j-1,i),  nu = rne(r . r),
 *   stop (beta_j+1 = 0) when nu < 2^-120, else rho = 1/sqrt(nu) by the
 *   fixed Newton iteration y <- y (3 - mu y^2) / 2 on mu = nu 4^-s in
 *   [1/4, 1) from y = 3/2, bitlen(P) + 6 steps, each product rounded, then
 *   rho = y 2^-s; beta_j+1 = rne(nu rho), q_j+1,i = rne(r_i rho) clamped to
 *   [-1, 1].
 * Runs `steps` steps asynchronously on `stream` with no host round trip.
 * alpha, beta: device arrays of `steps` numbers (hmv_words(P) words each):
 * alpha_1.., beta_2..; after a stop at step j, beta_j+1 = 0 and later
 * entries are left untouched.  *steps_done (device int32) receives the
 * number of alphas computed.  basis: NULL, or a device array of steps x n
 * numbers that receives q_1, q_2, ....  ws: hmv_lanczos_workspace_bytes
 * (status block first: matvec range errors show in hmv_read_status).
 * Hankel plans only (the matrix must be symmetric); any algorithm.        */
int64_t hmv_lanczos_workspace_bytes(const hmv_plan* plan);
int hmv_lanczos(const hmv_plan* plan, const uint64_t* q1, int32_t steps, uint64_t* alpha,
                uint64_t* beta, int32_t* steps_done, uint64_t* basis, void* ws, int64_t ws_bytes,
                void* stream);

/* ---------------------------------------------------------------- floating point
 * Multiprecision floating-point numbers (Section 2: a mantissa of b bits;
 * Section 3: a = B_0 sum_k B^k a_k, with a per-number factor B_0).  A number
 * is a significand M with |M| < 2^P, stored as hmv_words(P) words in two's
 * complement like the fixed-point numbers, and an int32 exponent e (a
 * separate device array): value M 2^(e-P).  y = A x is the exact sum
 * rounded once to P significant bits, to nearest with ties to even (as
 * MPFR's round-to-nearest); outputs are normalised, 2^(P-1) <= |M| < 2^P,
 * or zero with exponent 0.  Output exponents must fit in int32 (else the
 * overflow flag, HMV_EBOUND from hmv_read_status).
 *
 * `spread` is the widest exponent range the plan admits within h and within
 * each x (over nonzero entries): entries are aligned to their operand's
 * largest exponent as fixed-point integers of Q = P + spread fractional bits
 * (Q <= HMV_MAX_P), a fixed-point plan at Q holds the transform of h, and
 * its carry step keeps the exact sums, which are then rounded.  h wider
 * than spread, or a significand needing more than P bits, fails
 * hmv_fplan_h with HMV_ERANGE (it synchronises `stream` once, to read the
 * exponent range of h); such an x flags the range error on the device
 * (HMV_ERANGE from hmv_read_status on ws), and its y is unspecified.
 * Sizes: hmv_fplan_bytes (plan memory), hmv_fplan_workspace_bytes (ws of
 * both calls; its first 256 bytes receive the status).  x_exp, h_exp and
 * y_exp are device arrays of int32.  hmv_fplan_info reports the inner
 * fixed-point plan, Q and the largest exponent of h.                      */
typedef struct hmv_fplan hmv_fplan;
int64_t hmv_fplan_bytes(int kind, int64_t n, int32_t P, int32_t spread);
int64_t hmv_fplan_workspace_bytes(int kind, int64_t n, int32_t P, int32_t spread);
int hmv_fplan_h(hmv_fplan** out, int kind, const uint64_t* h_sig, const int32_t* h_exp,
                int64_t n, int32_t P, int32_t spread, void* plan_mem, int64_t plan_bytes,
                void* ws, int64_t ws_bytes, void* stream);
int hmv_fplan_matvec(const hmv_fplan* plan, const uint64_t* x_sig, const int32_t* x_exp,
                     uint64_t* y_sig, int32_t* y_exp, void* ws, int64_t ws_bytes, void* stream);
int hmv_fplan_info(const hmv_fplan* plan, hmv_plan_info_t* info, int32_t* Q, int32_t* Eh);
int hmv_fplan_destroy(hmv_fplan* plan);

/* ---------------------------------------------------------------- no allocation
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * result as hmv_plan_matvec, but the workspace is a fixed array of
 * HMV_NOALLOC_BYTES bytes inside the library (one per device, loaded on the
 * first call there and held until the process ends), so the caller passes
 * only the plan, x and y, plus an optional 256-byte device buffer `status`
 * that receives the device status of the call (read it with
 * hmv_read_status(status, ...)); with status == NULL the status block stays
 * in the fixed array.  The call allocates nothing and is asynchronous on
 * `stream`.  Returns HMV_ENOMEM (message in hmv_last_error) when the plan
 * needs more than HMV_NOALLOC_BYTES of workspace (hmv_plan_workspace_bytes:
 * n = 4096 at P = 33220 needs 385 MiB and fits), HMV_EINVAL when the plan
 * belongs to another device than the current one.  Every call on a device
 * shares that one array and leaves its contents behind (each call rewrites
 * all of what it reads): calls that overlap on one device -- on two streams,
 * or from two threads -- race and must be serialised by the caller.      */
#define HMV_NOALLOC_BYTES (448ll << 20)
int hmv_plan_matvec_noalloc(const hmv_plan* plan, const uint64_t* x, uint64_t* y, void* status,
                            void* stream);

/* ---------------------------------------------------------------- batches
 * Many independent products (any mix of kinds, n and P).  The work of all
 * instances is cut into items of four passes: forward limb transforms of
 * every h and x row; index-axis transforms of every h column; index-axis
 * passes of every x column; inverse limb transforms with carry of every
 * output row.  One launch covers the items of one pass whose transforms
 * have the same size (hmv_batch_launches counts them), one item per
 * work-group, with the LDS and threads of that size and no host round trip
 * in between.  Every instance runs the split-FFT path unplanned, with its
 * limb width taken from the worst-case bound (no data-dependent read back).
 * Limits: n <= 2048 per instance.  The descriptor array is host memory; h,
 * x, y are device pointers.  The call synchronises `stream` once, after
 * uploading its work list and before the launches; the products are ready
 * when the stream synchronises again.  ws (hmv_batch_workspace_bytes)
 * starts with the 256-byte status block.                                  */
typedef struct {
  int32_t kind;           /* HMV_HANKEL / HMV_TOEPLITZ / HMV_CIRCULANT                 */
  int32_t P;
  int64_t n;
  const uint64_t* h;      /* 2n-1 numbers (n for a circulant)                          */
  const uint64_t* x;      /* n numbers                                                 */
  uint64_t* y;            /* n numbers (output)                                        */
} hmv_problem;

int64_t hmv_batch_workspace_bytes(const hmv_problem* probs, int32_t count);
int hmv_batch_matvec(const hmv_problem* probs, int32_t count, void* ws, int64_t ws_bytes,
                     void* stream);
/* Number of kernel launches hmv_batch_matvec makes for these problems. */
int32_t hmv_batch_launches(const hmv_problem* probs, int32_t count);
/* The same products in ONE kernel launch (a cooperative launch: all its
 * work-groups are resident together; the runtime refuses it otherwise and
 * the call returns HMV_EDEVICE).  The work-groups take the items of each
 * pass in turn and meet at a grid-wide barrier between passes; every item
 * uses 256 threads and the limb transforms are of power-of-two size, so
 * the workspace is larger (hmv_batch_single_workspace_bytes) and the batch
 * slower than with hmv_batch_matvec.  Same arguments, limits, status block
 * and synchronisation as hmv_batch_matvec; the outputs are identical.
 * HMV_EINVAL for a batch with an instance whose power-of-two transforms do
 * not fit one work-group's LDS.                                           */
int64_t hmv_batch_single_workspace_bytes(const hmv_problem* probs, int32_t count);
int hmv_batch_matvec_single(const hmv_problem* probs, int32_t count, void* ws, int64_t ws_bytes,
                            void* stream);

/* ---------------------------------------------------------------- serving
 * A request scheduler for sessions of planned matvecs (continuous
 * batching).  The caller provides one device pool (pool_bytes) from which
 * the server carves each admitted request's workspace, and registers
 * resident plans.  A request (one matvec of a session) is admitted onto a
 * free stream slot as soon as the pool can hold its workspace; requests of
 * different sessions then overlap on the device, and requests submitted
 * while others run are admitted as slots and memory free up.  Requests of
 * one session run in submission order.  Admission is oldest-first with a
 * reservation for the oldest request that is waiting for memory.
 * hmv_server_submit enqueues and admits what fits (asynchronous);
 * hmv_server_poll retires finished requests (ids and their device status
 * flags, or a negative hmv_status) and admits waiting ones.  x and y must
 * stay valid until their request is retired.  The server creates its own
 * default-priority streams and events; destroy synchronises them.  One
 * thread at a time may call into a server.                                  */
typedef struct hmv_server hmv_server;

typedef struct {
  int64_t in_flight, waiting, admitted, completed, max_in_flight;
  int64_t pool_used, pool_peak, pool_bytes;
  int64_t large_in_flight, max_large_in_flight;   /* requests above large_bytes  */
  int64_t large_bytes, max_large;                 /* the admission policy        */
} hmv_server_stats_t;

int hmv_server_create(hmv_server** out, void* pool, int64_t pool_bytes, int32_t max_slots);
int hmv_server_add_plan(hmv_server* server, const hmv_plan* plan, int32_t* matrix_id);
/* Size-aware admission: a request whose workspace is above large_bytes is
 * large, and at most max_large (1 .. max_slots) large requests are in flight;
 * a large request held back by that cap lets younger, smaller requests
 * start.  Defaults: pool_bytes / 8 and max(1, max_slots / 4).  Takes effect
 * at the next admission; HMV_EINVAL for large_bytes < 0 or max_large out of
 * range.                                                                   */
int hmv_server_set_policy(hmv_server* server, int64_t large_bytes, int32_t max_large);
/* hmv_server_submit orders the request after all work enqueued on
 * `stream` (a hipStream_t, NULL = the null stream) before the call, as the
 * other entry points do: the server records an event there and the
 * request's kernels wait on it, so x may be written (and y last read) by
 * work still queued on that stream.                                        */
int hmv_server_submit(hmv_server* server, int32_t matrix_id, int64_t session, const uint64_t* x,
                      uint64_t* y, void* stream, int64_t* request_id);
int hmv_server_poll(hmv_server* server, int64_t* done_ids, int32_t* done_status, int32_t cap,
                    int32_t* n_done);
int hmv_server_stats(const hmv_server* server, hmv_server_stats_t* stats);
int hmv_server_destroy(hmv_server* server);

/* ---------------------------------------------------------------- diagnostics
 * Host-only helpers (no device access).
 * hmv_fft_error_bound: the bound used to pick the limb width of the binary64
 *   path, ||a||_2 ||b||_2 ((1+e)^(3k) (1+e sqrt5)^(3k+1) (1+beta)^(3k) - 1),
 *   e = 2^-53, k = log2_points (the form of Percival's bound for FFT
 *   multiplication, Math. Comp. 72 (2003)).
 * hmv_twiddle_beta: the beta of the library's root tables.
 * hmv_debug_force_width: tests only; restrict the binary64 limb width to w
 *   (0 restores the search).  The bound is still enforced.                  */
double hmv_fft_error_bound(double norm_h, double norm_x, int32_t log2_points, double beta);
double hmv_twiddle_beta(void);
int hmv_debug_force_width(int32_t w);
/* tests only: plan the split-FFT path with fixed launch variants (the
 * values of hmv_plan_info_t; a variant that does not exist for the shape
 * falls back to variant 0 of that bit); -1, -1 restores tuning.            */
int hmv_debug_force_variants(int32_t cols_variant, int32_t rows_inv_variant);
/* tests only: spectrum layout of later split-FFT plans.  z3 = 0 keeps the
 * limb transforms at powers of two (1 or -1: 3 * 2^k points where smaller);
 * pack = 0 or 1 fixes whether the two real limb bins share one column (-1:
 * packed where the error bound allows it).  The bound is still enforced.
 * Returns HMV_EINVAL for values outside -1..1.                             */
int hmv_debug_force_layout(int32_t z3, int32_t pack);
/* tests only: spectrum tile widths (2, 4 or 8 bins) of later split-FFT
 * plans for the spectra of x and of y; -1 keeps the tuned choice.
 * Returns HMV_EINVAL for other values.                                     */
int hmv_debug_force_tiles(int32_t x_tile, int32_t y_tile);
/* tests only: form of the schoolbook (HMV_SCHOOLBOOK): 0 = binary64 limb
 * sums on the vector units, 1 = int8 limb products on the matrix cores
 * (HMV_EUNSUPPORTED where its LDS row does not fit), -1 = the matrix-core
 * form wherever it applies (the default).  Both give the same words.      */
int hmv_debug_force_school(int32_t form);
/* tests only: spin limit of the dependency waits of the single-launch batch
 * driver (that driver is switched off; kept for its test); 0 = default.   */
int hmv_debug_batch_spin_limit(int32_t spins);

/* Device status of the last call that used workspace `ws`: synchronises
 * `stream`, stores the ST flags (bit 0 range, bit 1 bound, bit 2 spin limit,
 * bit 3 overflow) and, for the split-FFT path, the largest distance of an
 * FFT output coefficient from its nearest integer.  Either out pointer may
 * be NULL.  Returns, in this order of precedence:
 *   HMV_ERANGE  an input had |value| > 1 (y is unspecified);
 *   HMV_EBOUND  a transform output was not a trustworthy integer: a
 *               coefficient reached the planner's magnitude limit, a slot
 *               that must be zero was not, or a binary64 output lay more
 *               than 1/4 from its nearest integer (far outside the proven
 *               bound) -- y must not be used;
 *   HMV_EDEVICE a bounded device wait gave up (spin limit);
 *   HMV_OK      otherwise.                                                  */
int hmv_read_status(const void* ws, void* stream, int32_t* flags, double* max_round_err);

#ifdef __cplusplus
}
#endif
#endif /* HMV_H */
