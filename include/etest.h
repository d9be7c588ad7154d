/*
 * etest.h -- C ABI of the MI355X (gfx950) permutation two-sample test library.
 *
 * The library evaluates the efficient permutation test of Chaibub Neto,
 * "Computationally efficient permutation tests for the multivariate
 * two-sample problem based on energy distance or maximum mean discrepancy
 * statistics" (arXiv 2406.06488):
 *
 *   1. the three blocks D_XX, D_YY, D_XY (Euclidean distances, Alg. 3) or
 *      K_XX, K_YY, K_XY (Gaussian kernel, remark after Alg. 3) are computed
 *      once (Alg. 1, first three steps) -- never the pooled (nx+ny)^2 matrix
 *      of the pre-computation strategy (Alg. 5), and never D_YX (the
 *      memory-saving variant described after Alg. 1);
 *   2. the observed statistic is eq. (1) (energy distance, ED) or eq. (2)
 *      (biased MMD^2);
 *   3. B resampled statistics are evaluated from those blocks only, one per
 *      split of the pooled rows into x* (nx rows) and y* (ny rows) (Alg. 1
 *      loop, Alg. 2);
 *   4. the p-value is (1 + #{stat*_b >= threshold}) / (1 + B)
 *      (Section 3.1, unbiased estimator of Phipson and Smyth).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - X is nx-by-p and Y is ny-by-p, row-major and contiguous, one sample per
 *    row (Section 3, first paragraph).
 *  - Split b (0 <= b < B) is drawn from (seed, b) alone: Philox4x32-10 with
 *    key (seed mod 2^32, seed div 2^32) and counter (t div 2, b mod 2^32,
 *    b div 2^32, 0) gives a 64-bit uniform u_t for pooled item t (X rows
 *    first, then Y rows; even t takes words 0,1 and odd t words 2,3, low word
 *    first); item t joins x* when floor(u_t * (n - t) / 2^64) < need, where
 *    need starts at nx and drops by one at each member (selection sampling).
 *    So a run can be split into b-ranges and resumed bit-exactly.
 *  - The counting threshold is the identity split (x* = x, y* = y) evaluated
 *    by the same code that evaluates the B resampled splits; it equals the
 *    observed statistic up to rounding, and guarantees that a resampled split
 *    equal to the observed one is counted.
 *  - Gaussian kernel: k(x, y) = exp(-gamma * ||x - y||^2), gamma = 1/sigma^2.
 *  - Every function returns an etest_status.  On error nothing is written to
 *    the caller's outputs and etest_last_error() returns a message for the
 *    calling thread.  No C++ exception crosses this boundary.
 *  - Buffers are owned by the caller.  Host-buffer calls copy the inputs and
 *    keep no pointer after they return.  Device-buffer calls require the
 *    buffers to stay valid until the call returns (synchronous calls) or the
 *    stream reaches the work (the *_async calls).
 *  - There is no CPU fallback: every numerical step runs in the library's HIP
 *    kernels on the current HIP device.
 *  - Results depend only on (X, Y, p, B, seed, kind, prec, gamma), never on
 *    what else is in the same batch or server.
 */
#ifndef ETEST_H
#define ETEST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ETEST_OK = 0,
  ETEST_EINVAL = 1,      /* nx < 1, ny < 1, p < 1, B < 0 or B >= 2^31 - 1, NULL pointer, gamma <= 0 or
                            non-finite, nx + ny > 2^31 - 1, bad request field; a pooled
                            tile grid ceil(nx/128) + ceil(ny/128) above 46340 tiles; a
                            stage launch past one dispatch (2^31 workgroups or 2^32
                            work-items, e.g. one workgroup per stored 128 x 128 block
                            tile: nt (nt + 1) / 2 < 2^24), checked before any device work */
  ETEST_ENONFINITE = 2,  /* X or Y holds a NaN or an Inf                                 */
  ETEST_ENOMEM = 3,      /* device memory, or the server's memory budget, exhausted      */
  ETEST_EDEVICE = 4,     /* a HIP runtime call failed                                    */
  ETEST_EBUSY = 5,       /* server request not finished yet / server queue full         */
  ETEST_ENOTFOUND = 6    /* unknown server request id                                    */
} etest_status;

typedef enum {
  ETEST_PREC_F64 = 0,         /* FP64 inputs, FP64 blocks, FP64 reductions                */
  ETEST_PREC_F32 = 1,         /* FP32 inputs; Gram of FP32 accuracy on fp16 MFMA: each     */
                              /* centred value as two fp16 (22 bits), three exact products */
                              /* per term, FP32 accumulation; FP32 blocks, FP64 sums       */
  ETEST_PREC_BF16_REFINED = 2 /* FP32 inputs, BF16 Gram on MFMA with FP32 accumulation,   */
                              /* pairs with d^2 < 1e-3 (|x|^2 + |y|^2) recomputed as a    */
                              /* direct FP32 difference, FP64 sums                        */
} etest_prec;

typedef enum {
  ETEST_ED = 0, /* energy distance, eq. (1)             */
  ETEST_MMD = 1 /* biased MMD^2, Gaussian kernel, eq. (2) */
} etest_kind;

typedef struct {
  double statistic; /* observed statistic, eq. (1) or (2), from FP64 block sums            */
  double threshold; /* identity split as evaluated by the resampling stage                 */
  double p_value;   /* (1 + count_ge) / (1 + B); 1 when B == 0                             */
  int64_t count_ge; /* #{b : stat*_b >= threshold}                                         */
  int64_t B;        /* number of resampled splits                                          */
  int64_t n_refined;/* pairs recomputed by direct difference (BF16 form; 0 otherwise)      */
} etest_result;

/* One test described by device pointers (used by etest_run, etest_batch and the server). */
typedef struct {
  int32_t kind;       /* etest_kind                                                        */
  int32_t prec;       /* etest_prec                                                        */
  int64_t nx, ny, p;  /* sample sizes and dimension                                        */
  int64_t B;          /* resampled splits, >= 0                                            */
  uint64_t seed;      /* split stream seed                                                 */
  double gamma;       /* MMD only: kernel exp(-gamma ||x-y||^2), gamma > 0                 */
  const void* X;      /* nx*p row-major: double for ETEST_PREC_F64, float otherwise        */
  const void* Y;      /* ny*p row-major, same type as X                                    */
  double* perm_stats; /* [B] resampled statistics, or NULL to skip                        */
} etest_request;

/* ---- Synchronous calls on host buffers (the whole test: Alg. 1 end to end) ---- */

/* Energy-distance permutation test on float32 host data.  prec is ETEST_PREC_F32 or
   ETEST_PREC_BF16_REFINED.  perm_stats: host array of B doubles, or NULL.
   out: host struct, required. */
etest_status ed_test(const float* X, int64_t nx, const float* Y, int64_t ny, int64_t p,
                     int64_t B, uint64_t seed, int32_t prec, double* perm_stats,
                     etest_result* out);

/* Gaussian-kernel MMD^2 permutation test on float32 host data (eq. 2). */
etest_status mmd_test(const float* X, int64_t nx, const float* Y, int64_t ny, int64_t p,
                      double gamma, int64_t B, uint64_t seed, int32_t prec,
                      double* perm_stats, etest_result* out);

/* Same as ed_test / mmd_test with float64 host data and ETEST_PREC_F64 throughout. */
etest_status ed_test_f64(const double* X, int64_t nx, const double* Y, int64_t ny, int64_t p,
                         int64_t B, uint64_t seed, double* perm_stats, etest_result* out);
etest_status mmd_test_f64(const double* X, int64_t nx, const double* Y, int64_t ny,
                          int64_t p, double gamma, int64_t B, uint64_t seed,
                          double* perm_stats, etest_result* out);

/* ---- Device buffers ---- */

/* Run one test described by device pointers on `stream` (a hipStream_t, NULL = default
   stream) and wait for it; fills the host struct `out`. */
etest_status etest_run(const etest_request* req, void* stream, etest_result* out);

/* Enqueue one test on `stream` and return without waiting.  d_out is a device pointer to
   one etest_result, written by the pass's last kernel; it must stay valid until the stream
   has reached the end of the work.  Scratch memory: one workspace per (device, stream),
   allocated on the first call and kept for the calls that follow on that stream (they run
   in stream order, so each reuses it without waiting for the previous one); a call that
   needs more replaces it, which waits for the device once.  The workspace is held until
   the process ends.  Under stream capture the call allocates and frees its own workspace
   in stream order instead. */
etest_status ed_test_async(const etest_request* req, etest_result* d_out, void* stream);
etest_status mmd_test_async(const etest_request* req, etest_result* d_out, void* stream);

/* For callers that cannot allocate (code under graph capture, tight serving loops,
   harnesses that forbid allocation): ed_test_async / mmd_test_async (either kind, from
   req->kind) with the whole workspace in a fixed 128 MiB device array that each GPU the
   library runs on holds until the process ends.  Allocates nothing (no device, pinned or
   stream-ordered memory), creates no stream or event, and runs every stage on `stream`;
   same kernels and results, bit for bit, as the allocating calls.  req, d_out and stream
   as for ed_test_async; the caller owns X, Y, perm_stats and d_out.  Errors: EINVAL
   (arguments), ENOMEM when the test's workspace exceeds the array (e.g. 2000 + 2000 rows
   at p = 1000, B = 10^4 fit; 3000 + 3000 rows at p = 1000 do not) -- checked before any
   device work, outputs untouched; EDEVICE.  Calls on one GPU share the array: calls that
   overlap on that GPU (different streams or threads) race; the array keeps the last
   call's contents, which no call reads before writing. */
etest_status etest_run_async_noalloc(const etest_request* req, etest_result* d_out, void* stream);

/* ---- Cross tests (permutation-free; the paper's appendix on the cross-ED test) ---- */

typedef struct {
  double statistic; /* U = U_x - U_y: cross-MMD (Alg. 6) or cross-ED (Alg. 7) statistic       */
  double sigma;     /* studentising scale sqrt(s_x / nx1 + s_y / ny1)                          */
  double z;         /* U / sigma (+inf, -inf or 0 by the sign of U when sigma == 0)            */
  double p_value;   /* 1 - Phi(z)                                                              */
  int64_t n_refined;/* pairs recomputed by direct difference (BF16 form; 0 otherwise)          */
} etest_cross_result;

/* Cross-MMD / cross-ED test on device buffers, synchronous on `stream`.  x is cut into x1
   (its first floor(nx/2) rows) and x2 (the rest), y likewise; the four cross blocks
   K(x1,x2), K(y1,y2), K(x1,y2), K(y1,x2) (or distances) are computed on MFMA (FP32 / BF16
   forms, as for the blocks of a permutation test) or by direct FP64 differences, reduced
   to per-row means in FP64 and never stored.  req: kind, prec, nx, ny (both >= 2), p,
   gamma (MMD), X and Y as for etest_run; B, seed and perm_stats are ignored.  Errors:
   EINVAL (arguments), ENONFINITE (NaN / Inf input; out untouched), ENOMEM, EDEVICE. */
etest_status etest_cross(const etest_request* req, void* stream, etest_cross_result* out);

/* ---- Baselines: the standard and the pre-computation permutation tests ----
   Same request, splits (split b from (seed, b)), counting rule and result fields as
   etest_run, so that the three tests can be compared split by split; perm_stats is a device
   array of B doubles or NULL.  statistic and threshold are both the identity split as
   evaluated by the baseline's own code.  Synchronous on `stream`.  Errors: EINVAL
   (arguments), ENONFINITE (NaN / Inf input; perm_stats untouched), ENOMEM, EDEVICE. */

/* Standard permutation test (Alg. 4): for each of the B drawn splits and the identity
   split, X* and Y* are staged from the pooled rows in index order (x* items first) and the
   three blocks and the statistic, eq. (1) or (2), are recomputed from them.  The B + 1
   recomputations run as batched passes of up to 256 tests (each pass one launch per stage,
   within a 4 GiB workspace).  Cost: (B + 1) times the blocks of one test. */
etest_status etest_standard(const etest_request* req, void* stream, etest_result* out);

/* Pre-computation permutation test (Alg. 5): the distance (kernel) matrix of the pooled
   sample, D_WW, is computed once (as the stored upper tiles of the pooled tile grid: each
   unordered pair once), then for each split the sums of D_WW over x* x x*, y* x y* and
   x* x y* are taken entry by entry (each entry selected by the split's bits, FP64 sums) and
   combined into eq. (1) or (2).  Stage timing (etest_profile_enable): 0 staging, 1 blocks,
   2 split stream, 5 per-split sums, 6 statistics and p-value. */
etest_status etest_precomputed(const etest_request* req, void* stream, etest_result* out);

/* Pre-computation permutation test with D_WW as Alg. 5 prints it: the dense (nx + ny)^2
   pooled matrix, both orders of every pair (D_YX included), computed once by the pooled
   Gram over every tile of the (tx + ty)^2 tile grid; then for each split the sums over the
   X*X*, Y*Y* and X*Y* sub-blocks, read entry by entry (the Y*X* entries are skipped), in
   FP64 and combined into eq. (1) or (2).  Twice the Gram and twice the per-split reads of
   etest_precomputed; same splits, counting rule, results (up to FP64 summation order),
   stage timing and errors. */
etest_status etest_precomputed_dense(const etest_request* req, void* stream, etest_result* out);

/* ---- HSIC independence permutation test (the extension of the paper's discussion) ----
   Paired samples (x_i, y_i), i < n: X is n-by-p and Y n-by-q, row-major, device buffers
   (double for ETEST_PREC_F64, float otherwise).  The Gaussian kernel matrices K of x and
   L of y (exp(-gamma ||a - b||^2), gamma_x for x and gamma_y for y) are computed once, on
   the same staging and Gram kernels as the two-sample blocks; each permutation pi of the y
   sample then takes one pass over their n^2 entries.  With Kt = K - diag(K), Lt likewise,
   the statistic is the unbiased HSIC of Song et al. (2012):
     HSIC = [tr(Kt Lt_pi) + (1^T Kt 1)(1^T Lt 1) / ((n-1)(n-2)) - 2/(n-2) 1^T Kt Lt_pi 1]
            / (n (n-3)),   Lt_pi[i][j] = Lt[pi_i][pi_j].
   Permutation b orders the items 0..n-1 by a 64-bit Philox4x32-10 key (key (seed mod 2^32,
   seed div 2^32), counter (t div 2, b mod 2^32, b div 2^32, 1); even t takes words 0,1,
   odd t words 2,3, low word first), ties by index.  The identity permutation, evaluated by
   the same code, is both the reported statistic and the threshold; p = (1 + #{b :
   HSIC_b >= threshold}) / (1 + B).  4 <= n <= 4096.  prec: ETEST_PREC_F64 or ETEST_PREC_F32
   (the estimator is a small difference of three large terms -- on high-dimensional data
   about 1e-5 of the kernel entries under independence -- which the BF16 form's 8-bit
   coordinates cannot resolve; it is rejected with EINVAL). */
typedef struct {
  int32_t prec;          /* etest_prec                                                     */
  int32_t reserved;      /* must be 0                                                      */
  int64_t n, p, q;       /* pairs, dimension of x, dimension of y                          */
  int64_t B;             /* permutations, >= 0                                             */
  uint64_t seed;         /* permutation stream seed                                        */
  double gamma_x;        /* kernel on x: exp(-gamma_x ||a - b||^2), > 0                     */
  double gamma_y;        /* kernel on y, > 0                                               */
  const void* X;         /* n*p row-major                                                  */
  const void* Y;         /* n*q row-major                                                  */
  double* perm_stats;    /* [B] HSIC of each permutation (device), or NULL                 */
} etest_hsic_request;

/* The HSIC permutation test, synchronous on `stream`; out: host struct (n_refined counts
   the refined pairs of both Grams in the BF16 form).  Errors: EINVAL (arguments), ENONFINITE
   (NaN / Inf input; perm_stats untouched), ENOMEM, EDEVICE.  Stage timing: 0 staging,
   1 blocks, 2 permutations, 3 dense matrices and row sums, 5 per-permutation terms,
   6 statistics and p-value. */
etest_status etest_hsic(const etest_hsic_request* req, void* stream, etest_result* out);

/* Permutations b0 .. b0+count-1 of the HSIC test's stream: perms[(b - b0) * n + i] = the item
   at position i (device, count*n int32).  1 <= n <= 4096. */
etest_status etest_permutations(int64_t n, uint64_t seed, int64_t b0, int64_t count,
                                int32_t* perms, void* stream);

/* n independent tests in one batched pass: every stage is one launch covering all tests,
   and the launch sequence is captured once into a HIP graph and replayed while the same
   request shapes, the same stream and the same tuning rules come back; up to 4 graphs are
   kept (evicting one waits for the device), each holding its workspace until evicted.  With stage timing on (etest_profile_enable)
   the batch runs without a graph so that the stages can be timed.  outs: host array of n
   results.  Each test's result equals what etest_run gives for it alone. */
etest_status etest_batch(const etest_request* reqs, int64_t n, void* stream, etest_result* outs);

/* Asynchronous form of etest_batch: enqueue the n tests on `stream` and return without
   waiting.  The pass is etest_batch's cached graph, replayed (eager, on the stream's
   workspace as for ed_test_async, while stage timing is on or under stream capture).
   d_outs: device array of n etest_result; test t's result is written there by its last
   kernel, and the array must stay valid until the stream reaches the end of the work.
   Each result equals what etest_run gives for the test alone.  A test whose X or Y holds
   NaN or Inf gets NaN statistic and p-value in d_outs (the call has returned before the
   device sees the data).  The descriptor tables go up from one of a few pinned staging
   slots per host thread, each reused once its copy has run.  Under stream capture only
   n = 1 is accepted (its descriptor travels as kernel arguments).  Errors: EINVAL
   (arguments; n > 1 under capture), ENOMEM, EDEVICE. */
etest_status etest_batch_async(const etest_request* reqs, int64_t n, void* stream,
                               etest_result* d_outs);

/* ---- Stage-level calls (each step of the path, for parity checks) ---- */

/* Splits b0 .. b0+count-1 as membership bits: words[(b - b0) * W + t/32] bit (t % 32) is 1
   when pooled item t goes to x*; W = ceil((nx+ny)/32).  words: device, count*W uint32. */
etest_status etest_membership(int64_t nx, int64_t ny, uint64_t seed, int64_t b0,
                              int64_t count, uint32_t* words, void* stream);

/* The three blocks of Alg. 1, written as full row-major matrices into device buffers:
   dxx [nx*nx], dyy [ny*ny], dxy [nx*ny]; element type double for ETEST_PREC_F64 and
   float otherwise.  Diagonals of dxx / dyy are exactly 0 (ED) or 1 (MMD). */
etest_status etest_blocks(const etest_request* req, void* dxx, void* dyy, void* dxy,
                          void* stream);

/* Resampled statistics for caller-supplied splits: `words` (device, count*W uint32, same
   layout as etest_membership) each hold exactly nx members; stats (device, count doubles).
   Also returns the observed statistic and threshold in `out` (count_ge/p_value are over
   these splits).  Lets a caller evaluate the identity, complement or an enumeration. */
etest_status etest_perm_stats_from_membership(const etest_request* req, const uint32_t* words,
                                              int64_t count, double* stats, void* stream,
                                              etest_result* out);

/* ---- Continuous-batching server ---- */

typedef struct etest_server etest_server;

typedef struct {
  int64_t memory_budget_bytes; /* device bytes the server may hold for resident tests      */
  int32_t max_resident;        /* slots: tests resident at once                            */
  int32_t max_queue;           /* pending requests accepted before EBUSY                   */
  int64_t chunk_updates;       /* resampling work per scheduler step (block entries x
                                  splits summed over resident tests); <= 0 picks a default */
} etest_server_config;

/* Start a server with its own scheduler thread and HIP stream on the current device. */
etest_status etest_server_create(const etest_server_config* cfg, etest_server** out);

/* Queue a request.  X/Y/perm_stats are DEVICE pointers that must stay valid until the
   request completes.  Returns ENOMEM if the request alone exceeds the memory budget,
   EBUSY when the queue is full.  *id identifies the request. */
etest_status etest_server_submit(etest_server* s, const etest_request* req, uint64_t* id);

/* ETEST_OK and the result when finished (the id is then released), EBUSY while pending,
   ENOTFOUND for an unknown id, or the request's own error status. */
etest_status etest_server_poll(etest_server* s, uint64_t id, etest_result* out);

/* Block until the request finishes; same results as poll. */
etest_status etest_server_wait(etest_server* s, uint64_t id, etest_result* out);

/* Queue depth, resident tests, device bytes held and completed count. */
etest_status etest_server_stats(etest_server* s, int64_t* queued, int64_t* resident,
                                int64_t* bytes_held, int64_t* completed);

/* Finish outstanding work, join the scheduler thread and free everything. */
etest_status etest_server_destroy(etest_server* s);

/* ---- Diagnostics ---- */

/* Message for the calling thread's last error ("" when none).  Owned by the library. */
const char* etest_last_error(void);

/* Device bytes a single test needs (inputs excluded); used for server admission.  Pure
   host arithmetic: valid without a GPU. */
etest_status etest_footprint(const etest_request* req, int64_t* bytes);

/* Check a request's arguments without touching the device (same rules as every call). */
etest_status etest_validate(const etest_request* req);

/* Stage timing of the calling thread's etest_run / etest_batch / ed_test / mmd_test and
   ed_test_async / mmd_test_async calls: when on, HIP events on the call's stream bracket
   each stage (every pass has its own event set, so passes enqueued back to back are all
   timed) and their elapsed times accumulate when the host collects them.
   Stages: 0 staging (column means, cast, norms), 1 blocks (Gram + epilogue), 2 split stream,
   3 block sums + observed statistic, 4 centring, 5 resampling, 6 statistics + p-value.
   on = 0: off; 1: every stage; otherwise bits 1..7 of `on` select stages 0..6 (bit k+1 =
   stage k), so that only the kernels of interest are bracketed by events (each event adds
   a marker between launches).  Enabling also resets the totals. */
etest_status etest_profile_enable(int32_t on);

/* Accumulated milliseconds and launch counts per stage (arrays of n <= 7 entries).  Passes
   enqueued asynchronously and not yet collected are waited for and added first.  Changing
   the setting with etest_profile_enable drops the times of passes still pending. */
etest_status etest_profile_read(double* ms, int64_t* launches, int32_t n);

/* ---- Tuning of the resampling stage's work shape ---- */

/* Rule for tests of precision `prec` with n_lo <= nx + ny < n_hi: each resampling workgroup
   covers `kc` column tiles of 128 pooled items (1..256) and `cc` chunks of 256 splits
   (1..2 for the FP32 / BF16 forms, 1..8 for FP64).  Rules are matched in the order they
   were added; unmatched tests use the built-in default.  cc never changes results; kc
   regroups the FP32 partial sums of the resampling stage, so different kc values can
   differ at rounding level.  A test's results depend only on its own parameters and the
   rule that matches it, never on what it is batched with.  Process-wide. */
etest_status etest_tune_set(int32_t prec, int64_t n_lo, int64_t n_hi, int32_t kc, int32_t cc);

/* Remove every tuning rule. */
etest_status etest_tune_clear(void);

/* Gram workgroup shape for tests of precision prec (ETEST_PREC_F32 or _BF16_REFINED) with
   pooled size nx + ny in [n_lo, n_hi): 0 = one stored 128 x 128 block tile per workgroup,
   1 = one 256 x 256 super tile (2 x 2 stored tiles, one wave each) per workgroup, followed
   by a finishing pass over the stored tiles.  Without a rule: super tiles once there are
   512 or more of them (pooled size from about 8000 on), block tiles below.  Both shapes add
   each Gram entry's products in the same order and form every block value, sum and
   maximum the same way, so results are identical bit for bit; the shape changes speed
   only.  Process-wide; etest_tune_clear removes these rules too.
   Errors: EINVAL (prec, range or shape). */
etest_status etest_tune_set_gram(int32_t prec, int64_t n_lo, int64_t n_hi, int32_t shape);

#ifdef __cplusplus
}
#endif

#endif /* ETEST_H */
