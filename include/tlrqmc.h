/*
 * tlrqmc.h -- C ABI of the MI355X tile-low-rank quasi-Monte Carlo library.
 *
 * The library estimates multivariate normal and Student-t probabilities
 * P(a <= X <= b) by the separation-of-variables (SOV) recursion run over
 * many randomly shifted Richtmyer lattice points at once, with the Cholesky
 * factor in tile-low-rank (TLR) form (Cao, Genton, Keyes, Turkiyyah,
 * "Exploiting low rank covariance structures for computing high-dimensional
 * normal and Student-t probabilities", arXiv 2003.11183).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: 0 (TLRQMC_OK) on success, a
 *    positive warning or a negative error code.  No C++ exception crosses
 *    the ABI.  tlrqmc_last_error() returns a message for the last failure
 *    on the calling thread.
 *  - Host pointers are caller owned and only read during the call (outputs
 *    are written during the call).  Objects returned through **out
 *    (contexts, factors) are library owned until their _free/_destroy.
 *  - Device memory is obtained from the context's allocator callback (or
 *    hipMalloc when none is given); all device work is issued on the
 *    context's HIP stream, and every call returns only after that work has
 *    completed.
 *  - Variables: a factor carries a permutation perm (perm[i] = original
 *    index of the variable at integration position i).  Limits a, b are
 *    always given in the caller's original order and are applied through
 *    perm inside the library.  Limits are centred (the mean is subtracted
 *    by the caller; the paper sets mu = 0 without loss of generality,
 *    Section 2.1).  a_i = -inf and b_i = +inf are allowed.
 *  - A context is not thread safe; use one context per thread.
 *  - Concurrent device linear algebra: rocBLAS / rocSOLVER factorizations
 *    (and torch.linalg.cholesky) returned wrong results while this
 *    library's estimator kernels ran beside them on other streams; the cause
 *    has not been found.  A host replay of every load and store of the
 *    estimator kernels, over the launches the library builds for full-size
 *    problems, served slots and small ragged ones, finds none outside its
 *    allocation, and no buffer goes back to the allocator while a kernel
 *    may still use it.  Every rocBLAS call the library makes itself runs
 *    with the device drained and to itself.  Callers should not run their
 *    own device factorizations concurrently with mvn_prob, mvt_prob or a
 *    server of this library: synchronize first.
 */
#ifndef TLRQMC_H
#define TLRQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TLRQMC_OK = 0,
  TLRQMC_WARN_RANKCAP = 1, /* a tile hit the rank cap: truncation above tol */
  TLRQMC_PENDING = 2,      /* serving: the result is not ready yet          */
  TLRQMC_EINVAL = -1,      /* invalid argument (message says which)         */
  TLRQMC_ENOTSPD = -2,     /* covariance tile not positive definite         */
  TLRQMC_ENOMEM = -3,      /* allocation failed                              */
  TLRQMC_EDEVICE = -4,     /* HIP runtime error                              */
  TLRQMC_ENOTFOUND = -5    /* serving: unknown ticket                        */
};

typedef struct tlrqmc_ctx tlrqmc_ctx;
typedef struct tlrqmc_factor tlrqmc_factor;

/* Device allocator: alloc returns device memory of at least `bytes` bytes
 * (NULL on failure); free releases it.  Both are called on the thread that
 * called into the library. */
typedef struct {
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *user;
} tlrqmc_allocator;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  `alloc` may be NULL. */
int tlrqmc_ctx_create(int device, void *hip_stream, const tlrqmc_allocator *alloc,
                      tlrqmc_ctx **out);
void tlrqmc_ctx_destroy(tlrqmc_ctx *ctx);

/* Message of the last failure on this thread ("" if none). */
const char *tlrqmc_last_error(void);

/* ---------------------------------------------------------------- setup --
 * Covariance description (Section 3.2: the covariance comes from locations
 * and a kernel).  kind 0: dense Sigma on the host, column-major with leading
 * dimension ld >= n.  kind 1: exponential kernel
 *   Sigma_pq = variance * exp(-|x_p - x_q| / range) + nugget * [p == q]
 * on n locations xy (host, n x 2 row-major). */
typedef struct {
  int32_t kind;
  int32_t reserved;
  const double *sigma;
  int64_t ld;
  const double *xy;
  double range;
  double variance;
  double nugget;
} tlrqmc_cov;

/* Geometric order of the variables (Section 3.2: index distance should
 * follow spatial distance).  kind 1: Morton (Z-order) of the locations,
 * quantised to 16 bits per axis over their bounding box, ties by index.
 * kind 0: identity.  perm_out: n entries, caller allocated. */
int tlrqmc_geometric_order(int64_t n, const tlrqmc_cov *cov, int32_t *perm_out);

/* Block reordering (Section 3.3, "Block reordering" algorithm).  The blocks
 * are consecutive size-m chunks of the geometric order.  Each block is
 * scored with the univariate conditioning estimate of its probability
 * Phi_m(a_l, b_l; Sigma_ll); blocks are then put in ascending score order by
 * selection with swaps, and the variables inside each block take the order
 * the univariate conditioning chose.  Ties go to the lowest index; a
 * ragged last block stays last.  Host computation; ctx may be NULL.
 * perm_out: n entries, caller allocated, perm_out[i] = original index. */
int block_reorder(tlrqmc_ctx *ctx, int64_t n, const tlrqmc_cov *cov, const double *a,
                  const double *b, int m, int32_t *perm_out);

/* TLR Cholesky factor (Section 3.3; Section 3.4 defines B_i, U_ij, V_ij).
 * Sigma is permuted by perm (NULL = geometric order), factored by a dense
 * Cholesky on the device, and each off-diagonal m x m tile L_ij is replaced
 * by U_ij V_ij^T keeping the singular values > tol (absolute 2-norm
 * truncation, at most max_rank of them when max_rank > 0).  Returns
 * TLRQMC_WARN_RANKCAP (factor still valid) when a tile needed more than
 * max_rank, TLRQMC_ENOTSPD when Sigma is not positive definite (the message
 * names the failing column). */
int tlr_factor(tlrqmc_ctx *ctx, int64_t n, const tlrqmc_cov *cov, const int32_t *perm, int m,
               double tol, int max_rank, tlrqmc_factor **out);

/* Block reordering during the Cholesky factorization (Section 3.3, "Block
 * reordering during Cholesky factorization"), followed by the tile
 * compression of tlr_factor.  The blocks are consecutive size-m chunks of
 * the geometric order.  At each elimination step the remaining full blocks
 * are scored with the univariate conditioning estimate of their probability
 * on the current conditional covariance (the Schur complement) and the
 * current conditional limits; the lowest score (lowest index on ties) is
 * swapped into place and keeps the variable order the univariate
 * conditioning chose; the block is factored, the panel below it solved, the
 * later limits conditioned on the block's truncated means (a_i -= L_ij y_j,
 * b_i -= L_ij y_j) and the Schur complement updated.  A ragged last block
 * stays last.  Student-t problems are scored with unscaled limits.
 *   a, b    : host, n entries, original order (as block_reorder).
 *   perm_out: host, n entries, caller allocated, may be NULL; receives the
 *             order (perm_out[i] = original index at position i), which is
 *             also the factor's permutation.
 * Errors and warnings as tlr_factor; NaN limits -> TLRQMC_EINVAL. */
int tlr_factor_rbodr(tlrqmc_ctx *ctx, int64_t n, const tlrqmc_cov *cov, const double *a,
                     const double *b, int m, double tol, int max_rank, int32_t *perm_out,
                     tlrqmc_factor **out);

/* Build a factor from host tiles (the exchange layout, also written by
 * tlrqmc_factor_export).  r = ceil(n / m) tiles; tile i has m_i = min(m,
 * n - i m) rows.
 *   diag : the r diagonal tiles B_i, each m_i x m_i row-major, concatenated;
 *          entries above the diagonal are ignored, the diagonal must be > 0.
 *   ranks: r x r row-major, ranks[i*r+j] = k_ij >= 0 for i > j (others
 *          ignored), k_ij <= min(m_i, m_j).
 *   U, V : for i = 1..r-1, j = 0..i-1 (row-major order of the pairs):
 *          U_ij (m_i x k_ij, row-major) and V_ij (m_j x k_ij, row-major),
 *          concatenated; tile (i, j) of the factor is U_ij V_ij^T.
 *   perm : n entries or NULL (identity).
 * Errors: TLRQMC_EINVAL for bad sizes, a non-positive diagonal, a
 * non-finite entry or an invalid permutation. */
int tlrqmc_factor_import(tlrqmc_ctx *ctx, int64_t n, int m, const int32_t *perm,
                         const double *diag, const int32_t *ranks, const double *U,
                         const double *V, tlrqmc_factor **out);

typedef struct {
  int64_t n;
  int32_t m, r;
  int64_t k_tot;        /* sum of all ranks                          */
  int32_t k_max;        /* largest rank                              */
  int32_t cap_hits;     /* tiles truncated by the rank cap           */
  int64_t diag_doubles; /* entries of the exchange diag array        */
  int64_t uv_doubles;   /* entries of each exchange U and V array    */
  int64_t device_bytes; /* device memory held by the factor          */
  /* tlr_factor only (0 otherwise), seconds: covariance and Cholesky on
   * the device, transfer to the host (the diagonal tiles when the device
   * compresses, else the whole factor), compression of the off-diagonal
   * tiles, device layouts and upload. */
  double setup_seconds[4];
  uint64_t checksum;    /* hash of the exchange arrays (bit-level identity): FNV-1a
                         * over 64-bit words of 1 MiB chunks, chunk hashes folded in order */
  /* tlr_factor only: off-diagonal tiles compressed on the host.  Tiles up to
   * 512 wide are compressed on the device, except those whose pivoted QR
   * needs more than 96 steps; wider tiles are all compressed on the host. */
  int64_t host_tiles;
} tlrqmc_factor_info;

int tlrqmc_factor_stats(const tlrqmc_factor *f, tlrqmc_factor_info *out);

/* Copy a factor to host arrays in the exchange layout of
 * tlrqmc_factor_import (sizes from tlrqmc_factor_stats); any pointer may
 * be NULL to skip that array. */
int tlrqmc_factor_export(const tlrqmc_factor *f, int32_t *perm, double *diag, int32_t *ranks,
                         double *U, double *V);

void tlrqmc_factor_free(tlrqmc_factor *f);

/* ------------------------------------------------------------ estimator --
 * Quasi-Monte Carlo options.  Sample k = 1..n_samples of shift s =
 * 0..n_shifts-1 uses the Richtmyer lattice point with generators
 * frac(sqrt(p_{c+1})) (c = 0 the chi radius, c = 1..n the variables in
 * integration order) shifted by the SplitMix64 stream of `seed`
 * (Section 2.1, remark after the MVN algorithm; Section 3.4).
 *   precision 0: FP64 everywhere (arithmetic and every stored value).
 *   precision 1: the precision form.
 *     - Low-rank products (limit update U Z and projection V^T y, Section
 *       3.4) on BF16 matrix cores with FP32 accumulation: each operand is
 *       split into BF16 hi + lo and hi*hi + hi*lo + lo*hi is kept.
 *     - The row products with the diagonal tiles (Section 2.1, Eq. 2) are
 *       FP64 arithmetic.
 *     - With a = -inf (one-sided limits) Phi, log Phi and Phi^-1 run in FP32
 *       while the quantile's smaller side min(u, 1 - u) is at least 1e-36
 *       (about 2e-7 relative error); below that the quantile is computed in
 *       FP64 from log u.  Two-sided limits take the FP64 functions.
 *     - y, the limit updates Delta and the rank-space images Z are stored
 *       in FP32 between kernels (y is widened to FP64 for the row products).
 *     - The complements, the running log P per sample and the per-shift
 *       sums stay FP64.
 *     Its error against the FP64 form is a few parts in 1e-6 of log P on
 *     the benchmark workloads, well inside the QMC standard error.
 *   logp_out  : optional host array of n_shifts * n_samples doubles that
 *               receives log P of every sample (shift-major).
 *   profile   : nonzero records HIP events around every kernel launch and
 *               fills the kernel timing fields of the result.
 *   chunk_samples: samples swept per pass (0 = as many as the device
 *               memory budget allows; rounded up to a multiple of 256). */
typedef struct {
  int64_t n_samples;
  int32_t n_shifts;
  int32_t precision;
  uint64_t seed;
  double *logp_out;
  int32_t profile;
  int32_t reserved;
  int64_t chunk_samples;
} tlrqmc_qmc_opts;

enum { TLRQMC_KERNEL_INIT = 0, TLRQMC_KERNEL_DELTA = 1, TLRQMC_KERNEL_SWEEP = 2,
       TLRQMC_KERNEL_ZPROJ = 3, TLRQMC_KERNEL_REDUCE = 4, TLRQMC_KERNEL_KINDS = 5 };

/* Estimate (Section 2.1; Section 4: relative error = standard error over
 * mean).  log_p = log of the mean over shifts of the per-shift sample means;
 * std_err = standard deviation of the shift means / sqrt(n_shifts);
 * p = exp(log_p) (may underflow to 0).  n_dead counts samples whose
 * integrand is exactly 0.  seconds: device time of the estimator (lattice,
 * sweep, low-rank updates and reductions; setup excluded, as the paper
 * times only the integration, Section 4).  With opts.profile:
 * kernel_seconds sums the launch durations of each kernel kind and
 * kernel_busy_seconds is the union of its launch intervals (launches on the
 * worker streams overlap). */
typedef struct {
  double log_p, p, std_err, rel_err;
  double log_p_shift[64];
  int64_t n_dead;
  double seconds;
  double kernel_seconds[TLRQMC_KERNEL_KINDS];
  double kernel_busy_seconds[TLRQMC_KERNEL_KINDS];
  int64_t kernel_launches[TLRQMC_KERNEL_KINDS];
  int32_t n_shifts;
  int32_t chunks;
} tlrqmc_result;

/* MVN probability Phi_n(a, b; Sigma) (Section 2.1, Eq. 1-2; TLR recursion of
 * Section 3.4).  a, b: host, n entries, original order.  n_samples >= 1,
 * 2 <= n_shifts <= 64.  If a_i >= b_i for some i the result is log_p =
 * -inf with status OK.  NaN limits -> TLRQMC_EINVAL. */
int mvn_prob(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b,
             const tlrqmc_qmc_opts *opts, tlrqmc_result *out);

/* MVT probability T_n(a, b; Sigma, nu) with Sigma the scale matrix, as the
 * chi scale mixture of Section 2.2, Eq. 4: each sample scales the limits by
 * chi_nu^-1(w_0) / sqrt(nu) and runs the MVN recursion.  nu > 0. */
int mvt_prob(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b,
             double nu, const tlrqmc_qmc_opts *opts, tlrqmc_result *out);

/* mvn_prob (nu = 0) or mvt_prob (nu > 0) without allocating: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The result equals
 * mvn_prob / mvt_prob on the same arguments bit for bit (the same kernels
 * and per-sample arithmetic; samples are swept in chunks of a size that
 * fits the scratch, one stream).
 *   Scratch: a 256 MiB file-scope device array of the library, one per
 *   device, held from module load to process end; its address is resolved
 *   by tlrqmc_ctx_create.  Limits, shift table, per-sample log P (8 bytes
 *   per sample) and the chunk buffers come from it.  A problem whose
 *   per-call arrays and one chunk of 256 samples do not fit returns
 *   TLRQMC_ENOMEM with the sizes in the message, before any device work.
 *   Calls that overlap on one device race on the array: the caller
 *   serializes them.  The array keeps the last call's contents.
 *   The call creates no device objects (no streams, no events; opts.profile
 *   is ignored and result.seconds is host wall time) and issues everything
 *   on the context stream; it returns after that work has completed.
 *   Arguments and errors otherwise as mvn_prob / mvt_prob (nu >= 0). */
int tlrqmc_prob_noalloc(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a, const double *b, double nu,
                        const tlrqmc_qmc_opts *opts, tlrqmc_result *out);

/* log P of samples k0 .. k0+count-1 (1-based) of shift `shift`, run through
 * the same kernels as mvn_prob / mvt_prob (nu = 0 selects MVN).  logp_out:
 * host, count entries. */
int tlrqmc_sample_logp(tlrqmc_ctx *ctx, const tlrqmc_factor *f, const double *a,
                       const double *b, double nu, const tlrqmc_qmc_opts *opts, int32_t shift,
                       int64_t k0, int64_t count, double *logp_out);

/* ---------------------------------------------------- skew-normal client --
 * Log-likelihood of the skew-normal stochastic generator Z = xi 1 + A X +
 * B |Y| (Section 5.1, Eq. 5; X, Y independent standard normal vectors) at
 * observations z on n locations xy (host, n x 2 row-major), with A the lower
 * Cholesky factor of sigma1^2 exp(-|h|/beta1) and B the covariance matrix
 * sigma2^2 exp(-|h|/beta2) (Section 5.2).  Eq. 6:
 *   loglik = n log 2 + log phi_n(z - xi 1; A A^T + B B^T)
 *            + log Phi_n(-inf, c; Gamma),
 *   C = A^-1 B,  Gamma = (I + C^T C)^-1,  c = Gamma C^T A^-1 (z - xi 1).
 * The dense linear algebra runs on the device; Gamma is factored into TLR
 * form with tile m, truncation tol and rank cap max_rank, in the geometric
 * order of xy (order 0) or with block reordering during the Cholesky
 * factorization (order 2), and the probability term is mvn_prob with opts.
 *   c_out     : host, n entries, may be NULL: the upper limits c.
 *   factor_out: may be NULL: receives the factor of Gamma (library owned,
 *               free with tlrqmc_factor_free).
 * Errors: TLRQMC_EINVAL for bad parameters (sigma1 > 0, beta1 > 0, sigma2
 * >= 0, beta2 > 0, finite xi, z and xy), TLRQMC_ENOTSPD if a covariance is
 * not positive definite, as mvn_prob otherwise. */
typedef struct {
  double xi, sigma1, beta1, sigma2, beta2;
} tlrqmc_skewnormal_params;

typedef struct {
  double loglik;            /* the whole of Eq. 6, natural log              */
  double log_density;       /* log phi_n(z - xi 1; A A^T + B B^T)           */
  double log_prob;          /* log Phi_n(-inf, c; Gamma), estimated         */
  double log_prob_std_err;  /* standard error of Phi_n (not of its log)     */
  double log_prob_rel_err;  /* relative error of Phi_n                      */
  double seconds[3];        /* linear algebra, factor of Gamma, estimator   */
  tlrqmc_result prob;       /* the estimator's full result                  */
} tlrqmc_skewnormal_result;

int tlrqmc_skewnormal_loglik(tlrqmc_ctx *ctx, int64_t n, const double *xy, const double *z,
                             const tlrqmc_skewnormal_params *params, int m, double tol,
                             int max_rank, int order, const tlrqmc_qmc_opts *opts,
                             tlrqmc_skewnormal_result *out, double *c_out,
                             tlrqmc_factor **factor_out);

/* -------------------------------------------------------------- serving --
 * A request server answers a stream of probability requests of mixed
 * dimension on the context's device (the likelihood evaluations of
 * Section 5 call the estimator many times, each with its own covariance
 * parameters and limits).  For each request it orders the variables
 * (geometric order, or block reordering of Section 3.3), builds the TLR
 * factor (as tlr_factor) and runs the estimator (as mvn_prob / mvt_prob).
 *
 * Continuous batching: a request's N * M samples are cut into slots of a
 * size that depends on the request alone.  Each server step advances every
 * active slot, of every request, by one diagonal tile in shared kernel
 * launches, so requests that arrive while others run start at the next
 * step and their work overlaps on the device.  The arithmetic of a sample
 * does not depend on the other slots of a step and each request is reduced
 * on its own in a fixed order: a result is the same, bit for bit, alone or
 * in any mix.
 *
 * Admission by device-memory footprint: the server takes one arena of
 * hbm_budget_bytes from the context's allocator at creation and serves
 * every device allocation of its requests from it.  A queued request is
 * admitted to setup, in arrival order, when the reservations held by
 * admitted requests plus its setup footprint (the dense covariance) fit the
 * budget.  After setup its reservation becomes its run footprint: the
 * factor, its limits, shift table and per-sample results, and the buffers
 * of as many slots as fit in the larger of its setup footprint and a
 * quarter of the budget (its slot concurrency, at least one).  A request
 * whose setup footprint or single-slot run footprint exceeds the budget
 * fails with TLRQMC_ENOMEM.
 *
 * Threads: the server runs a setup thread and a step thread with two HIP
 * streams of its own (default priority).  submit, poll and stats may be
 * called from any thread.  The context's allocator is called only inside
 * tlrqmc_server_create and tlrqmc_server_destroy. */
typedef struct tlrqmc_server tlrqmc_server;

/* One request.  All host arrays are copied by tlrqmc_server_submit.
 *   n, cov        : dimension and covariance (as tlr_factor)
 *   a, b          : limits, n entries, original order (as mvn_prob)
 *   nu            : 0 = normal, > 0 = Student-t degrees of freedom
 *   m, tol, max_rank : tile size and truncation (as tlr_factor)
 *   reorder       : 1 = block reordering, 0 = geometric order
 *   qmc           : n_samples, n_shifts, precision, seed (logp_out,
 *                   profile and chunk_samples are ignored) */
typedef struct {
  int64_t n;
  tlrqmc_cov cov;
  const double *a;
  const double *b;
  double nu;
  int32_t m;
  int32_t max_rank;
  double tol;
  int32_t reorder;
  int32_t reserved;
  tlrqmc_qmc_opts qmc;
} tlrqmc_request;

/* Life of one request, in seconds since the server was created. */
typedef struct {
  double t_submit;        /* submit returned the ticket          */
  double t_admit;         /* admitted to setup (budget)          */
  double t_ready;         /* factor built                        */
  double t_start;         /* first slot on the device            */
  double t_done;          /* estimate available                  */
  int64_t reserved_bytes; /* run reservation                     */
  int64_t factor_bytes;
  int64_t chunk_samples;  /* samples per slot                    */
  int32_t slots;          /* slots of the request                */
  int32_t concurrency;    /* slots it may have active at once    */
  int32_t status;
  int32_t reserved;
  uint64_t factor_checksum; /* as tlrqmc_factor_info.checksum    */
} tlrqmc_request_info;

typedef struct {
  int64_t budget_bytes, reserved_bytes, peak_reserved_bytes;
  int64_t arena_in_use_bytes, arena_peak_bytes;
  int64_t steps;           /* server steps launched                */
  int64_t launches;        /* kernel launches                      */
  int64_t slot_steps;      /* sum over steps of the active slots   */
  int64_t max_active_slots;
  int32_t queued, in_setup, ready, running;
} tlrqmc_server_info;

/* Create a server on ctx's device with a device budget of hbm_budget_bytes
 * (at least 16 MiB), allocated at once from ctx's allocator. */
int tlrqmc_server_create(tlrqmc_ctx *ctx, size_t hbm_budget_bytes, tlrqmc_server **out);

/* Queue a request; *ticket identifies it.  Invalid requests return
 * TLRQMC_EINVAL at once.  A request with a_i >= b_i for some i completes
 * at once with log_p = -inf. */
int tlrqmc_server_submit(tlrqmc_server *s, const tlrqmc_request *req, uint64_t *ticket);

/* Result of a ticket.  wait_ms = 0 returns at once, wait_ms > 0 waits up
 * to that many milliseconds, wait_ms < 0 waits until the request is done;
 * TLRQMC_PENDING if it is not done by then.  Once done: the request's status
 * (TLRQMC_OK, TLRQMC_WARN_RANKCAP, or the error its setup or run met, with
 * the message in tlrqmc_last_error) and *out, *info (either may be NULL)
 * filled; result.seconds is the latency from submit to done.  The ticket
 * is then released (TLRQMC_ENOTFOUND afterwards). */
int tlrqmc_server_poll(tlrqmc_server *s, uint64_t ticket, int32_t wait_ms, tlrqmc_result *out,
                       tlrqmc_request_info *info);

int tlrqmc_server_stats(tlrqmc_server *s, tlrqmc_server_info *out);

/* Finish every submitted request, stop the threads and free the arena.
 * Results not yet polled are discarded. */
int tlrqmc_server_destroy(tlrqmc_server *s);

#ifdef __cplusplus
}
#endif
#endif /* TLRQMC_H */
