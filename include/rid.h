/*
 * rid.h -- C ABI of librid, a randomized interpolative decomposition (ID) of
 * complex matrices on AMD Instinct MI355X (gfx950).
 *
 * Method: Lucas, Stalzer & Feo, "Parallel implementation of fast randomized
 * algorithms for the decomposition of low rank matrices", arXiv 1205.3830.
 * Given A (m x n, approximate rank k), find k columns B = A(:, J) and a
 * k x n matrix P with A ~= B P (Sec. 2, problem statement).  The steps are
 *   1. randomization  Y = G A with an l x m complex Gaussian G, l >= k
 *      (Sec. 2 randomization step; the paper's own operator is a subsampled
 *      FFT, and Sec. 2 allows a faster randomization in its place);
 *   2. a QR factorization of Y with column pivoting, whose first k pivots
 *      are the skeleton J (Sec. 2, approximate QR and column permutation);
 *   3. P = [I T] with R2 = R1 T, written in the original column order
 *      (Sec. 2, interpolation matrix);
 *   4. the error ||A - A(:, J) P||_2 of Table 5, estimated by power iteration.
 *
 * Conventions for every entry point
 *  - Matrices are column-major with a leading dimension ld >= rows, complex
 *    stored as interleaved (re, im) pairs: complex128 = two doubles (the
 *    layout of std::complex<double> and torch.complex128).  Exception: the
 *    Gaussian operator G is stored by rows (entry (i, p) at G[i * ldg + p]).
 *  - Indices are 0-based int64.
 *  - Every data pointer is a DEVICE pointer owned by the caller, unless the
 *    argument's comment says "host".  The library never frees caller memory
 *    and never writes A.
 *  - Calls are asynchronous on `stream` unless their comment says they
 *    synchronise.  A handle serialises nothing by itself: calls on one handle
 *    must be ordered by their streams (the handle's workspace is shared).
 *  - Argument errors are reported synchronously, before anything is
 *    launched, as RID_ERR_INVALID_ARG.  A failed HIP call is reported as
 *    RID_ERR_HIP; rid_last_hip_error() returns the hipError_t.
 *  - Numerical rank failure (rank(Y) < k, Sec. 2) is recorded in a device
 *    status word of the handle by rid_pivqr; rid_query_status() reads it.
 *    rid_decompose() reads it itself and redraws G with the next seed, as
 *    Sec. 2 prescribes for this failure.
 *  - Arithmetic: `RID_FP64` runs every step in double precision, with the
 *    residual's sums over A compensated (double-double).  The QR, the
 *    triangular solve and the norms are double in every precision mode; a
 *    lower `rid_prec` changes the sketch product, and the residual's sums
 *    over A become plain double (rid_set_residual chooses otherwise).
 *  - Determinism: no floating-point atomics; a call repeated with the same
 *    inputs on the same device gives bit-identical outputs.
 */
#ifndef RID_H
#define RID_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rid_ctx *rid_handle;

typedef enum {
  RID_OK = 0,
  RID_ERR_INVALID_ARG = 1,
  RID_ERR_UNSUPPORTED = 2,
  RID_ERR_NOMEM = 3,
  RID_ERR_HIP = 4,
  RID_ERR_RANK = 5 /* rank(Y) < k at the QR step (Sec. 2 failure case) */
} rid_status;

/* Storage type of A. */
typedef enum { RID_C128 = 0, RID_C64 = 1 } rid_dtype;

/* Arithmetic of the sketch product Y = G A (Y itself is always complex128).
 *   RID_FP64   double products and accumulation (either storage type);
 *   RID_FP32   single-precision products, single accumulation;
 *   RID_BF16X2 each operand split into two bfloat16 terms (16 significant
 *              bits), the three leading bf16 products per real product on
 *              the bf16 matrix cores, single accumulation (error near
 *              2^-16 relative);
 *   RID_BF16X3 each operand split into three bfloat16 terms, the six
 *              leading bf16 products per real product, single accumulation
 *              (FP32-level error).
 * Single IDs and batches take all four.                                  */
typedef enum { RID_FP64 = 0, RID_FP32 = 1, RID_BF16X2 = 2, RID_BF16X3 = 3 } rid_prec;

/* ---------------------------------------------------------------- handle */

/* Create a handle bound to HIP device `device` (host out-pointer `h`).
 * Allocates a small device status word; workspace is allocated on first use
 * or by rid_reserve().  A call that needs more workspace allocates a larger
 * buffer (at least 1.5x) without waiting for the device; the superseded
 * buffers are kept until rid_destroy, as work in flight may still use them.
 * Errors: INVALID_ARG (null h, bad device), HIP.                          */
rid_status rid_create(rid_handle *h, int device);

/* Free the handle and its workspace.  The caller must make sure no work
 * that uses the handle is still running.  A null handle is a no-op.      */
rid_status rid_destroy(rid_handle h);

/* Static string naming a status code (never null). */
const char *rid_status_string(int status);

/* hipError_t of the last failed HIP call on this handle (0 if none). */
int rid_last_hip_error(rid_handle h);

/* Pre-size the workspace for every call with m <= max_m, n <= max_n,
 * l <= max_l, k <= max_k, so that later calls allocate nothing (needed
 * before capturing calls into a HIP graph).  Errors: INVALID_ARG
 * (negative sizes), NOMEM.                                               */
rid_status rid_reserve(rid_handle h, int64_t max_m, int64_t max_n, int64_t max_l,
                       int64_t max_k);

/* Method of the column-pivoted QR of rid_pivqr and rid_decompose (batches
 * always use Householder).  Both pivot on exact trailing norms, so they pick
 * the same J away from near-ties and give the same T = R1^-1 R2 up to
 * rounding.                                                              */
typedef enum {
  RID_QR_HOUSEHOLDER = 0, /* Householder reflections (default)                 */
  RID_QR_CGS2 = 1         /* Gram-Schmidt with reorthogonalisation (Sec. 3.2); k <= 1024 */
} rid_qr_kind;

/* Select the QR method of this handle's later calls.  Errors: INVALID_ARG. */
rid_status rid_set_qr(rid_handle h, int kind);

/* ---------------------------------------------------------------- step 1 */

/* The Gaussian sketch operator of the randomization step (Sec. 2), or any
 * block of the project's Gaussian stream: out (rows x cols complex128,
 * row-major, entry (i, j) at out[i * ld + j], ld >= cols) receives
 *   g(i, j) = sqrt(-ln u1) * exp(2 pi i u2),   Re, Im ~ N(0, 1/2),
 * where (u1, u2) are two 52-bit uniforms in (0, 1), u = (2x + 1) 2^-53 with x
 * the top 52 bits of a 64-bit word pair, taken from the Philox4x32-10 block
 * (Salmon et al., SC'11) with counter (j mod 2^32, j >> 32, i, stream_id) and
 * key (seed mod 2^32, seed >> 32): words (w0, w1) give u1 and (w2, w3) u2.
 * stream_id 0 is the sketch operator G (l x m), stream_id 1 the power-
 * iteration start vector (1 x n).
 * Errors: INVALID_ARG (rows or cols < 0, ld < cols, null out), HIP.      */
rid_status rid_gaussian(rid_handle h, hipStream_t stream, int64_t rows, int64_t cols,
                        uint64_t seed, uint32_t stream_id, void *out, int64_t ld);

/* Kind of random operator that rid_sketch and rid_decompose draw. */
typedef enum {
  RID_SKETCH_GAUSSIAN = 0, /* complex Gaussian G (rid_gaussian, stream 0); default */
  RID_SKETCH_SRFT = 1      /* the paper's S F D (rid_srft_operator)              */
} rid_sketch_kind;

/* Select the operator kind of this handle's later rid_sketch and
 * rid_decompose calls (Sec. 2 names S F D and allows a faster
 * randomization in its place).  With S F D and m a multiple of 8 the sketch
 * runs as a four-step DFT, in one pass over A when no residue group of the
 * sampled rows exceeds 32 rows, else in two; RID_SRFT_TWO_PASS=1 in the
 * environment forces the two-pass form (the results agree to rounding).
 * Errors: INVALID_ARG.                                                    */
rid_status rid_set_sketch(rid_handle h, int kind);

/* The paper's randomization operator (Sec. 2, eqs. (4)-(7)) written out as
 * rows x m complex128, row-major (entry (i, p) at out[i * ld + p], ld >= m):
 *   out(i, p) = exp(2 pi i (phi_p - (s_i p mod m) / m)),
 * i.e. row s_i of the unnormalised DFT F times D = diag(exp(2 pi i phi_p)).
 * phi_p = the first uniform (u1 of rid_gaussian's construction) of the
 * Philox block with counter (p, 0, 0, 5); s_i = floor(u1 m) of the block
 * with counter (i, 0, 0, 6) -- rows are drawn i.i.d. with replacement, as
 * eq. (5) specifies.  Applying it costs 8 rows m n flops like the Gaussian
 * operator; the FFT of eq. (6) is never formed.  Requires 1 <= m < 2^31.
 * Errors: INVALID_ARG, HIP.                                               */
rid_status rid_srft_operator(rid_handle h, hipStream_t stream, int64_t rows, int64_t m,
                             uint64_t seed, void *out, int64_t ld);

/* Randomization step (Sec. 2) with the operator of `seed` (the handle's
 * kind, Gaussian unless rid_set_sketch chose S F D):
 *   Y (l x n complex128, ldy >= l) = G(seed) (l x m) * A (m x n, lda >= m).
 * A is complex128 or complex64 per `dtype`; `prec` selects the product
 * arithmetic.  The operator is drawn into the handle's workspace (16 l m
 * bytes).
 * Requires 1 <= l, 0 <= m, 0 <= n; A 16-byte aligned for RID_C128 (8 for
 * RID_C64), Y 16-byte aligned.  Errors: INVALID_ARG, UNSUPPORTED (dtype/prec
 * pair not built), NOMEM, HIP.                                            */
rid_status rid_sketch(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                      int64_t m, int64_t n, int64_t l, const void *A, int64_t lda,
                      uint64_t seed, void *Y, int64_t ldy);

/* As rid_sketch, with a caller-supplied operator G (l x m complex128,
 * row-major, entry (i, p) at G[i * ldg + p], ldg >= m).                  */
rid_status rid_sketch_explicit(rid_handle h, hipStream_t stream, rid_dtype dtype,
                               rid_prec prec, int64_t m, int64_t n, int64_t l, const void *A,
                               int64_t lda, const void *G, int64_t ldg, void *Y, int64_t ldy);

/* ---------------------------------------------------------------- step 2 */

/* Column-pivoted QR of Y (Sec. 2 approximate QR with the column
 * permutation), k steps of Householder reflections with exact pivoting:
 * step t picks, among the columns not yet picked, the one whose rows t..l-1
 * (after the t earlier reflections) have the largest 2-norm, the lowest
 * column index winning an exact tie; those trailing norms are recomputed at
 * every step.  On return
 *   Y(0:k, :)  holds R = [R1 R2] in ORIGINAL column order: R(:, perm[t]) is
 *              column t of the upper-triangular R1 (zero below row t), the
 *              other columns are R2; rows k..l-1 of Y are left undefined;
 *   perm[0:k]  is the skeleton J in pivot order, perm[k:n] the remaining
 *              columns in increasing order;
 *   gaps[t]    (if gaps is not null) = (best - second best) / best trailing
 *              norm at step t (1 when one candidate is left).
 * If at some step the best trailing norm is <= rank_tol * (the best norm of
 * step 0), the handle's status word is set to RID_ERR_RANK and the outputs
 * are undefined (Sec. 2: rank(Y) < k).  Requires 1 <= k <= min(l, n),
 * ldy >= l.  For a Y of more than 512 MB the Householder steps keep up to 4
 * reflectors pending and write the trailing rows back every 4th step, still
 * pivoting on exact norms; RID_QR_PANEL=1 (=0) in the environment forces
 * (forbids) that form (the results agree to rounding).
 * Errors: INVALID_ARG, NOMEM, HIP.                                        */
rid_status rid_pivqr(rid_handle h, hipStream_t stream, int64_t l, int64_t n, int64_t k,
                     void *Y, int64_t ldy, int64_t *perm, double *gaps, double rank_tol);

/* Bytes of the device scratch array that rid_pivqr_static uses. */
#define RID_STATIC_SCRATCH_BYTES (32 << 20)

/* rid_pivqr without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results
 * (bit for bit) as rid_pivqr; the QR's scratch (per-workgroup pivot
 * candidates and column copies, per-column pivot steps, the panel
 * reflectors, and with RID_QR_CGS2 the Gram-Schmidt basis) lives in a
 * file-scope device array of RID_STATIC_SCRATCH_BYTES, one per device, held
 * until the process ends and located by rid_create.  The QR of an l x n Y
 * needs about 2 ceil(n / 64) (16 l + 24) + 4 n + 64 l bytes (plus
 * 16 (l k + k n) with RID_QR_CGS2): with Householder up to about 300000
 * columns at l = 208 and 33000 at l = 2000.  Larger problems return
 * RID_ERR_NOMEM before any launch.
 * Every call on a device shares that device's array, and the array keeps
 * what the last call left (every kernel initialises what it reads):
 * calls that overlap on one device -- on different streams or from
 * different threads or handles -- race and must be ordered by the caller.
 * Profiling (rid_profile) does not record these calls.
 * Errors: INVALID_ARG, UNSUPPORTED, NOMEM (problem beyond the array), HIP. */
rid_status rid_pivqr_static(rid_handle h, hipStream_t stream, int64_t l, int64_t n, int64_t k,
                            void *Y, int64_t ldy, int64_t *perm, double *gaps,
                            double rank_tol);

/* ---------------------------------------------------------------- step 3 */

/* Interpolation matrix (Sec. 2): with R1 = R(:, J) upper triangular and R2
 * the other columns of R (k x n complex128, ORIGINAL column order, ldr >= k,
 * as left by rid_pivqr), solve R1 T = R2 column by column by back
 * substitution and write P (k x n complex128, ldp >= k) in original column
 * order: P(:, J[t]) = e_t exactly, P(:, j) = R1^{-1} R(:, j) otherwise.
 * J: k distinct indices in [0, n) (device).  Requires 1 <= k <= n.
 * Errors: INVALID_ARG, HIP.                                               */
rid_status rid_interp(rid_handle h, hipStream_t stream, int64_t n, int64_t k, const void *R,
                      int64_t ldr, const int64_t *J, void *P, int64_t ldp);

/* ---------------------------------------------------------------- step 4 */

/* Accumulation of the residual's passes over A (rid_residual,
 * rid_decompose, batches).  The O(n k) side steps are compensated in every
 * kind; norms and the iteration vectors are double.                     */
typedef enum {
  RID_RESIDUAL_AUTO = 0, /* by the sketch arithmetic `prec` of the call: DOT2
                            for RID_FP64, FP64 for the reduced-precision
                            forms (default)                               */
  RID_RESIDUAL_DOT2 = 1, /* compensated sums (Ogita-Rump-Oishi Dot2), x~ and
                            u as double-double: agrees with an exact
                            iteration to ~1e-10 even where E = A - A(:,J) P
                            is 1e-10 of A                                  */
  RID_RESIDUAL_FP64 = 2, /* plain double FMA chains, x~ rounded to double:
                            relative error about u sqrt(m + n) ||A||_F /
                            sigma, far below the reduced-precision forms'
                            own error                                     */
  RID_RESIDUAL_FP32 = 3  /* single-precision products and sums within each
                            workgroup's slab, partials combined in double
                            (a reported variant: error about 2^-24 sqrt(slab)
                            ||A||_F / sigma)                               */
} rid_residual_kind;

/* Select the residual accumulation of this handle's later calls.
 * Errors: INVALID_ARG.                                                   */
rid_status rid_set_residual(rid_handle h, int kind);

/* Power-iteration estimate of ||E||_2, E = A - A(:, J) P (the error of
 * Table 5), without forming E: E x = A x~ with x~ = x - S_J (P x), and
 * E^H z = u - P^H u_J with u = A^H z.  Start vector x0 = rid_gaussian(seed,
 * stream_id 1) (1 x n), normalised.  Step t = 1..q: z = E x,
 * sigma_t = ||z||_2, and for t < q, x = E^H z / ||E^H z||; if E^H z = 0 the
 * iteration stops and later sigma_t repeat the last value.  The sums over
 * A take the handle's residual kind (rid_set_residual); by default they are
 * compensated (double-double) for prec = RID_FP64 and plain double for the
 * reduced-precision forms (RID_FP32, RID_BF16X2, RID_BF16X3), whose ID
 * error is far above plain double rounding.  Outputs: *sigma (device
 * double) = sigma_q; hist (device, q doubles, or null) = sigma_1..sigma_q.
 * A: m x n (lda >= m) of type `dtype`; P: k x n complex128 (ldp >= k);
 * J: k device indices.  Requires 0 <= k <= n, k <= 1024, q >= 1.
 * Errors: INVALID_ARG, UNSUPPORTED, NOMEM, HIP.                           */
rid_status rid_residual(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                        int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                        const int64_t *J, const void *P, int64_t ldp, int q, uint64_t seed,
                        double *sigma, double *hist);

/* ---------------------------------------------------------------- all steps */

/* The whole ID (Sec. 2): sketch with G(seed), pivoted QR, interpolation,
 * residual (q power steps, start vector of the same seed).  If the QR finds
 * rank(Y) < k, the draw is repeated with seed + 1, up to max_retries more
 * times (Sec. 2 failure remedy).  Outputs: J (k device int64, pivot order),
 * P (k x n complex128, ldp >= k), *sigma (device double), *seed_used (host,
 * may be null) = the seed of the successful draw.  Requires
 * 1 <= k <= min(l, n), l <= m, q >= 1, max_retries >= 0.  SYNCHRONISES the
 * stream (to read the rank status).  Errors: INVALID_ARG, UNSUPPORTED,
 * NOMEM, HIP, RANK (every draw failed).                                   */
rid_status rid_decompose(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                         int64_t m, int64_t n, int64_t k, int64_t l, const void *A,
                         int64_t lda, uint64_t seed, int q, int max_retries, double rank_tol,
                         int64_t *J, void *P, int64_t ldp, double *sigma,
                         uint64_t *seed_used);

/* As rid_decompose, with a caller-supplied operator G0 (l x m complex128,
 * row-major, entry (i, p) at G0[i * ldg + p], ldg >= m, 16-byte aligned) in
 * place of the first draw's: if G0 A has rank < k, the redraws use the
 * operators of seed + 1, seed + 2, ... (Sec. 2 failure remedy), so
 * *seed_used = seed + a for the a-th redraw; if the first draw succeeds,
 * *seed_used = seed and the start vector of the power iteration is that of
 * seed.  A test hook for the redraw path (G0 rank-deficient on purpose).
 * Errors: as rid_decompose; INVALID_ARG also for a null G0.              */
rid_status rid_decompose_explicit(rid_handle h, hipStream_t stream, rid_dtype dtype,
                                  rid_prec prec, int64_t m, int64_t n, int64_t k, int64_t l,
                                  const void *A, int64_t lda, const void *G0, int64_t ldg,
                                  uint64_t seed, int q, int max_retries, double rank_tol,
                                  int64_t *J, void *P, int64_t ldp, double *sigma,
                                  uint64_t *seed_used);

/* ---------------------------------------------------------------- SVD */

/* SVD built on the ID (Sec. 1 lists fast SVDs among the ID's uses): the
 * rank-k SVD of A(:, J) P,  A(:, J) P = U diag(S) V^H, computed without
 * forming A(:, J) P: B = A(:, J) = Q R_B and (R_B P)^H = Q_X R_X by shifted
 * CholeskyQR3, R_X Z = W diag(S) by one-sided Jacobi, U = Q Z, V = Q_X W.
 * A: m x n (lda >= m) of type `dtype`; J: k device indices in [0, n) (as
 * left by rid_decompose); P: k x n complex128 (ldp >= k).  Outputs (device,
 * caller-owned): U m x k complex128 (ldu >= m) with orthonormal columns,
 * S k doubles in descending order, V n x k complex128 (ldv >= n) with
 * orthonormal columns; the phase of each singular pair is arbitrary.
 * *sweeps (host, may be null) = Jacobi sweeps used (they stop when every
 * pair is orthogonal to sqrt(k) * 2^-52 relative, at most 60).  Requires
 * 1 <= k <= min(m, n), k <= 256 (else UNSUPPORTED), m <= 2^22, n < 2^31.
 * Returns RID_ERR_RANK when one of the two QRs breaks down (a Cholesky
 * pivot that is not positive, or a last Gram matrix far from I): exact
 * rank loss such as a zero column of A(:, J) (an index outside [0, n) is
 * read as one) or P = 0.  An input that is only numerically rank deficient
 * (a repeated index) still gives an SVD, whose trailing singular values
 * are at rounding level.  Workspace about (6 max(m, n) k) complex128.
 * SYNCHRONISES the stream.  Errors: INVALID_ARG, UNSUPPORTED, NOMEM, HIP,
 * RANK.                                                                   */
rid_status rid_svd(rid_handle h, hipStream_t stream, rid_dtype dtype, int64_t m, int64_t n,
                   int64_t k, const void *A, int64_t lda, const int64_t *J, const void *P,
                   int64_t ldp, void *U, int64_t ldu, double *S, void *V, int64_t ldv,
                   int *sweeps);

/* ---------------------------------------------------------------- profiling */

/* Kernel families timed by the profiling hook. */
typedef enum {
  RID_KERNEL_SKETCH = 0,  /* Y = G A product kernel (one launch per sketch)   */
  RID_KERNEL_AX = 1,      /* z = A x~ pass of the residual (one per step)      */
  RID_KERNEL_AHZ = 2,     /* u = A^H z pass of the residual (one per step < q) */
  RID_KERNEL_PIVQR = 3,   /* all launches of one pivoted QR, as one interval   */
  RID_KERNEL_INTERP = 4,  /* the back-substitution kernel                      */
  RID_KERNEL_COUNT = 5
} rid_kernel;

/* enable = 1: forget earlier records and, from now on, record a HIP event
 * pair on the launch stream around every launch of the kernel families
 * above (in a batch, one launch covers that step of every job); enable = 0:
 * stop recording (records are kept).  Recording adds two event records per
 * launch and nothing else, except that batches run while recording are
 * launched directly instead of through a captured graph.
 * Errors: INVALID_ARG.                                                    */
rid_status rid_profile(rid_handle h, int enable);

/* Total elapsed milliseconds and number of recorded launches of one kernel
 * family since rid_profile(h, 1) (host out-pointers; either may be null).
 * Synchronises on the recorded events.  Errors: INVALID_ARG, HIP.        */
rid_status rid_profile_read(rid_handle h, int kernel, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------- batches */

/* One ID of a batch.  A: m x n column-major of the batch's dtype (lda >= m,
 * device); J: k int64 (device, out); P: k x n complex128 column-major
 * (ldp >= k, device, out); sigma: one double (device, out). */
typedef struct {
  int64_t m, n, k, l;
  const void *A;
  int64_t lda;
  uint64_t seed;
  int64_t *J;
  void *P;
  int64_t ldp;
  double *sigma;
} rid_job;

/* Many independent IDs of uneven sizes (Sec. 2 for each), each with its own
 * seed: every step runs as one launch over all jobs (the pivoted QR as one
 * launch per pivot step, or with RID_BATCH_QR=jobs in the environment as one
 * launch with a workgroup per job for all its steps; the results agree bit
 * for bit), captured into a HIP graph and replayed on `stream` (set
 * RID_BATCH_GRAPH=0 in the environment to launch directly).  A job
 * whose sketch has rank < k is redrawn with seed + 1, up to max_retries
 * times.  Results per job are those of rid_decompose with the same inputs
 * and arguments, up to the split order of the sketch sums.
 * jobs: host array of `count`; job_status (host, count, or null) receives
 * RID_OK / RID_ERR_RANK per job; seed_used (host, count, or null) the seed
 * of each job's last draw.  Limits per job: 1 <= k <= l <= m, k <= n,
 * k <= 256, l <= 224, n < 2^31.  A job's results do not depend on the
 * other jobs of the batch (bitwise).  SYNCHRONISES the stream.  Errors:
 * INVALID_ARG, UNSUPPORTED, NOMEM, HIP, RANK (some job failed every draw;
 * the others hold their results).                                        */
rid_status rid_decompose_batched(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                                 const rid_job *jobs, int count, int q, int max_retries,
                                 double rank_tol, int *job_status, uint64_t *seed_used);

/* The plan of this handle's batches: rows of A per sketch K split
 * (multiple of 16, 16 .. 2^20; default 1024), bytes of A per workgroup of
 * the residual's A x pass (4 KiB .. 1 GiB; default 256 KiB) and columns per
 * wave of its A^H z pass (4 or 8; default 8).  Per-job results depend on the
 * plan only through summation order (within the FP64 tolerances of
 * rid_decompose).  Errors: INVALID_ARG.                                  */
rid_status rid_set_batch_plan(rid_handle h, int64_t sketch_rows, int64_t res_block_bytes,
                              int ahz_cols);

/* The current batch plan (host out-pointers; any may be null).            */
rid_status rid_get_batch_plan(rid_handle h, int64_t *sketch_rows, int64_t *res_block_bytes,
                              int *ahz_cols);

/* Autotuner of the batch plan on the caller's own batch: times the batch
 * (launched directly, HIP events around each kernel family) under six
 * candidate plans -- sketch split rows {128, 256, 512, 1024, 2048, 4096},
 * A-pass workgroup bytes {32, 64, 128, 256, 512, 1024} KiB and A^H z
 * columns per wave {8, 4, 8, 4, 8, 4}, the i-th of each together -- keeps
 * the fastest value of each parameter (each changes only its own kernel
 * family) in the handle and returns it (host out-pointers, may be null).
 * The jobs' outputs are overwritten (contents unspecified afterwards).
 * SYNCHRONISES the stream.  Errors: INVALID_ARG, UNSUPPORTED, NOMEM, HIP. */
rid_status rid_tune_batched(rid_handle h, hipStream_t stream, rid_dtype dtype, rid_prec prec,
                            const rid_job *jobs, int count, int q, int64_t *sketch_rows,
                            int64_t *res_block_bytes, int *ahz_cols);

/* ---------------------------------------------------------------- serving */

/* A request loop on one device with continuous batching: requests arrive at
 * any time (rid_server_submit); each is admitted as soon as its data and the
 * workspace its lane must add for it fit the memory budget beside the data
 * of the jobs already admitted and the workspaces the lanes hold (a lane
 * keeps its workspace between jobs; when a group cannot fit, idle lanes free
 * theirs), and admitted jobs run while others are still running.  Jobs whose A has fewer
 * than big_bytes bytes are grouped, per (dtype, prec, q, max_retries,
 * rank_tol), into batches of up to max_batch that run as one
 * rid_decompose_batched call (one job alone: rid_decompose); larger jobs run
 * one per big lane through rid_decompose.  Every lane owns a handle and a
 * non-blocking stream of default priority, so batches and big jobs overlap
 * on the device.  A job's results equal those of the same entry point
 * called alone (the batched path's per-job results do not depend on the
 * other jobs of its batch).                                               */
typedef struct rid_server_ctx *rid_server;

typedef struct {
  int64_t hbm_budget; /* device bytes that admitted jobs' data and the lanes'
                         workspaces may hold at once */
  int64_t big_bytes;  /* A of at least this many bytes: a big job */
  int big_lanes;      /* big jobs running at once (0: big jobs are batched too) */
  int batch_lanes;    /* batches running at once (>= 1) */
  int max_batch;      /* jobs per batch (>= 1) */
} rid_server_config;

typedef struct {
  int64_t m, n, k, l;
  rid_dtype dtype;
  rid_prec prec;
  uint64_t seed;
  int q, max_retries;
  double rank_tol;
  int64_t fill_bytes; /* transient device bytes the admit callback uses */
} rid_request;

/* Called on a lane thread once the request `ticket` is admitted: place A on
 * the device (enqueued on `stream`, or complete before returning) and set
 * job->A, lda, J, P, ldp and sigma (device memory the caller owns; m, n, k,
 * l and seed are already set).  Return 0, or non-zero to fail the job with
 * RID_ERR_INVALID_ARG.  Callbacks of different lanes may run at once.     */
typedef int (*rid_admit_fn)(void *ctx, uint64_t ticket, hipStream_t stream, rid_job *job);

/* Called on a lane thread when the job's results are final: status (RID_OK,
 * RID_ERR_RANK, ...), the seed of the last draw, and times[4] = seconds
 * since rid_server_create at arrival, admission, A in place, and done.    */
typedef void (*rid_done_fn)(void *ctx, uint64_t ticket, int status, uint64_t seed_used,
                            const double *times);

/* Start the lanes on `device`.  A job's data is bytes(A) + fill_bytes + its
 * outputs; its footprint is that + the workspace of rid_decompose for its
 * shape.  Errors: INVALID_ARG, HIP, NOMEM.                                */
rid_status rid_server_create(rid_server *s, int device, const rid_server_config *cfg,
                             rid_admit_fn admit, rid_done_fn done, void *ctx);

/* Queue one request; *ticket (host) receives its id (> 0).  Does not block.
 * Errors: INVALID_ARG (sizes as rid_decompose), UNSUPPORTED, NOMEM (the
 * footprint alone exceeds the budget).                                   */
rid_status rid_server_submit(rid_server s, const rid_request *req, uint64_t *ticket);

/* Block until every submitted job is done.                               */
rid_status rid_server_drain(rid_server s);

/* Peak of the counted bytes (admitted data, reserved workspace growth and
 * the workspaces the lanes hold), jobs completed, and batches run so far
 * (host out-pointers; any may be null).                                   */
rid_status rid_server_stats(rid_server s, int64_t *peak_bytes, int64_t *completed,
                            int64_t *batches);

/* Drain, stop the lanes and release everything the server holds.         */
rid_status rid_server_destroy(rid_server s);

/* Synchronise `stream` and return the handle's status word: RID_OK, or
 * RID_ERR_RANK if the last rid_pivqr on this handle met rank(Y) < k.
 * Errors: HIP.                                                            */
rid_status rid_query_status(rid_handle h, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RID_H */
