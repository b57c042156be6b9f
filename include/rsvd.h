/*
 * rsvd.h -- C ABI of librsvd.so: randomized range finder and truncated SVD
 * (PCA by SVD) of a tall-skinny, column-centred matrix on one AMD Instinct
 * MI355X (gfx950).
 *
 * The method is the one compared in "Tutorial: Complexity analysis of
 * Singular Value Decomposition and its variants" (Li, Wang, Cai; arXiv
 * 1906.12085):
 *   - Randomized PCA (Sec. 3.1.2): G standard normal (n x l), H = A G,
 *     power iterations H = A (A^T H), QR of H -> Q, T = A^T Q, SVD of T,
 *     U~ = Q W;
 *   - truncated SVD through A^T A (Sec. 2.3, Sec. 3.1.3): eig(A^T A) -> V,
 *     lambda; s_i = sqrt(lambda_i) (Eq. LambdaSigma); u_i = A v_i / s_i;
 *   - the number of principal components K from the cumulative explained
 *     variance threshold t (Sec. 2.4), with the denominator ||A||_F^2
 *     (Eq. sumeigen).
 *
 * Conventions for every entry point (Sec. 1 "Notations"/"Assumptions"):
 *   - A is m x n, real, m >= n, rows are examples, columns are features (the
 *     caller centres the columns; the library does not).
 *   - Matrices are ROW-MAJOR with an explicit leading dimension (elements
 *     between the starts of consecutive rows), ld >= number of columns.
 *   - Every matrix/vector pointer is a DEVICE pointer (hipMalloc'd or a
 *     torch tensor's storage) on the plan's device, unless stated otherwise.
 *     The caller owns all buffers it passes; the library never frees them.
 *   - Element type of A, U, V is the plan's dtype (double for RSVD_F64,
 *     float for RSVD_F32).  Singular values S and all FP64 buffers are double.
 *   - Singular values are returned in descending order.  Each pair (u_i, v_i)
 *     is signed so that the lowest-index entry of v_i whose magnitude is
 *     within 0.1% of the largest magnitude of v_i is positive.
 *   - Calls are stream-ordered on the plan's stream and asynchronous: results
 *     are valid after that stream has synchronised.  Argument errors are
 *     detected synchronously on the host before anything is launched.
 *     Numerical outcomes (breakdown, non-finite input, threshold not reached)
 *     are written to a device status word read by rsvd_plan_status().
 *   - A plan is not thread-safe: calls that use one plan must not overlap.
 */
#ifndef RSVD_H
#define RSVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsvd_plan_s* rsvd_plan_t;

typedef enum {
  RSVD_F64 = 0, /* A, U, V double; products on FP64 matrix cores */
  RSVD_F32 = 1, /* A, U, V float; products on FP32 matrix cores with FP32
                   accumulation inside a row block; Gram matrices, Cholesky
                   factors, the small SVD and the eigensolver in FP64 */
  RSVD_BF16 = 2, /* A stored as bfloat16 with optional FP32 column scales
                    (the matrix is Aq diag(s)); U, V float.  The passes over A
                    run on BF16 matrix cores with FP32 accumulation, their
                    right factors split into hi + lo bfloat16 pairs; the rest
                    as RSVD_F32.  Randomized PCA only (no A^T A route). */
  RSVD_FP8 = 3   /* as RSVD_BF16 with A stored as OCP FP8 E4M3 bytes (bias 7,
                    largest 448, S.1111.111 = NaN), widened exactly to
                    bfloat16 in registers */
} rsvd_dtype;

typedef enum {
  RSVD_OK = 0,
  RSVD_WARN_THRESHOLD = 1,   /* the k computed lambda_i capture < t ||A||_F^2: K = k */
  RSVD_WARN_ZERO_MATRIX = 2, /* ||A||_F = 0: K = 0, outputs are zero */
  RSVD_ERR_ARG = -1,         /* null pointer, bad k/p/q/t, bad leading dimension */
  RSVD_ERR_SHAPE = -2,       /* m < n, n < 1, or sizes above the plan's maxima */
  RSVD_ERR_NOMEM = -3,       /* device allocation failed */
  RSVD_ERR_DEVICE = -4,      /* a HIP runtime call or kernel launch failed */
  RSVD_ERR_BREAKDOWN = -5,   /* non-positive pivot in a Cholesky factorisation
                                (the sketch has numerical rank < l) */
  RSVD_ERR_NONFINITE = -6,   /* A contains NaN or Inf (||A||_F^2 not finite) */
  RSVD_ERR_NOCONV = -7       /* a Jacobi iteration hit its sweep limit */
} rsvd_status;

/* Human-readable name of a status code (static storage, never NULL). */
const char* rsvd_status_string(int32_t status);

/* ---------------------------------------------------------------- plans --
 * rsvd_plan_create: allocate the device workspace for problems up to
 * m_max x n_max with sketch width l = k + p <= l_max (Sec. 3.2.2 lists what a
 * Randomized PCA solve keeps: the l-column sketch and basis, the n x l
 * projection, the small SVD factors).  With want_gram != 0 the plan is also
 * sized for gram_eig_solve on n_max x n_max (Sec. 3.2.3: A^T A and V).
 *   plan      out: the new plan (NULL on failure)
 *   dtype     RSVD_F64 or RSVD_F32
 *   seed      seeds the Gaussian sketch G of rsvd_solve (Philox4x32-10 +
 *             Box-Muller, see rsvd_gaussian_fill)
 *   stream    hipStream_t to order all work on; NULL = the null stream
 * Limits: l_max <= 192 (the l x l Cholesky factor and its inverse share one
 * workgroup's registers); with want_gram, n_max <= 1024 (every workgroup of
 * the eigensolver is resident).  Sketches wider than 96 columns take their
 * small SVD on the cooperative block-Jacobi solver (one cooperative launch
 * per solve).
 * Also m_max <= 2^40 and n_max <= 2^20 (sizes stay within 64-bit arithmetic).
 * Errors: RSVD_ERR_ARG (plan NULL, bad dtype, l_max < 1), RSVD_ERR_SHAPE
 * (m_max < n_max, n_max < 1, or a limit above exceeded), RSVD_ERR_NOMEM,
 * RSVD_ERR_DEVICE. */
int32_t rsvd_plan_create(rsvd_plan_t* plan, int64_t m_max, int64_t n_max, int32_t l_max,
                         int32_t dtype, int32_t want_gram, uint64_t seed, void* stream);

/* Free the workspace (synchronises the plan's stream first). NULL is a no-op. */
int32_t rsvd_plan_destroy(rsvd_plan_t plan);

/* Synchronise the plan's stream and return the status word written by the
 * last solve's kernels (RSVD_OK, RSVD_WARN_*, RSVD_ERR_BREAKDOWN,
 * RSVD_ERR_NONFINITE, RSVD_ERR_NOCONV); resets it to RSVD_OK. */
int32_t rsvd_plan_status(rsvd_plan_t plan);

/* Synchronise and copy diagnostics of the last solve to host memory `out`
 * (up to `count` doubles): [0] ||A||_F^2, [1] captured fraction
 * sum_{i<=K} s_i^2 / ||A||_F^2, [2] Jacobi sweeps of the small SVD or of the
 * eigensolver, [3] largest off-diagonal measure left by that Jacobi, [4] K,
 * [5] 1 when the small SVD of a solve was repeated with its rotations
 * accumulated (its values spanning more than six decades), else 0.
 * Returns the number of values written. */
int32_t rsvd_plan_diag(rsvd_plan_t plan, double* out, int32_t count);

/* Per-kernel launch durations, measured with HIP events recorded on the
 * plan's stream immediately before and after each launch of the timed
 * kernels (no other work between them), for benchmarking against rooflines.
 * Returns, for each kind i < count (at most 5): ms[i] = mean duration in
 * milliseconds of the launches since the previous call, launches[i] = their
 * number (at most 256 per kind are kept); kinds: [0] symmetric eigensolver
 * of the A^T A route, [1] fp32 pass Y = A X with l <= 128 columns, [2] fp32
 * pass A^T Q with l <= 128 columns (without its partial-sum reduction),
 * [3] fp32 symmetric A^T A (without its reduction), [4] fp32 wide product
 * A X (more than 128 columns).  Then clears the records and turns timing on
 * (enable != 0) or off for later calls on this plan.  Synchronises the
 * plan's stream.  Returns the number of kinds written, RSVD_ERR_ARG (NULL
 * plan, count < 0, NULL arrays with count > 0), RSVD_ERR_NOMEM. */
int32_t rsvd_plan_kernel_times(rsvd_plan_t plan, int32_t enable, double* ms, int32_t* launches,
                               int32_t count);

/* ------------------------------------------------------------- solvers --
 * rsvd_solve: Randomized PCA (Sec. 3.1.2) of A (m x n, lda) with target rank
 * k, oversampling p (sketch width l = min(k + p, n)) and q power iterations;
 * each product with A or A^T is followed by an orthonormalisation
 * (CholeskyQR2 for the m x l basis), and K is chosen by threshold t in (0, 1]
 * over the k computed values (Sec. 2.4).
 *   A          element type of the plan: double (RSVD_F64), float
 *              (RSVD_F32), bfloat16 (RSVD_BF16) or FP8 E4M3 bytes
 *              (RSVD_FP8); for the last two the matrix is
 *              A diag(col_scale), as in rsvd_solve_bf16 / rsvd_solve_fp8
 *   col_scale  (n floats, device) column scales of bfloat16 / FP8 storage,
 *              NULL = all ones; must be NULL on RSVD_F64 / RSVD_F32 plans
 *   U  (m x k, ldu >= k)  left singular vectors U~ = Q W (first k columns)
 *   S  (k, double)        singular values, descending
 *   V  (n x k, ldv >= k)  right singular vectors (the principal axes)
 *   K  (1 int32, device)  number of components meeting t (K <= k)
 * The sketch G is drawn from the plan's seed: repeated calls on one plan use
 * the same G.  Errors (synchronous): RSVD_ERR_ARG (a NULL pointer, k < 1,
 * k > n, p < 0, q < 0, t outside (0, 1], lda < n, ldu < k, ldv < k,
 * col_scale given on an RSVD_F64 / RSVD_F32 plan, the storage conditions of
 * rsvd_solve_bf16 / rsvd_solve_fp8 on a low-precision plan), RSVD_ERR_SHAPE
 * (m < n, or m, n, l above the plan's maxima). */
int32_t rsvd_solve(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                   const float* col_scale, int32_t k, int32_t p, int32_t q, double t,
                   void* U, int64_t ldu, double* S, void* V, int64_t ldv, int32_t* K);

/* Same as rsvd_solve with the sketch G supplied: `omega` is a device FP64
 * row-major n x l matrix, l = min(k + p, n) (it is rounded to the plan's
 * dtype before use), or NULL for the plan's seeded sketch.  For parity tests
 * and for callers with their own G. */
int32_t rsvd_solve_omega(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                         const float* col_scale, int32_t k, int32_t p, int32_t q, double t,
                         const double* omega, void* U, int64_t ldu, double* S, void* V,
                         int64_t ldv, int32_t* K);

/* rsvd_solve_adaptive: Randomized PCA (Sec. 3.1.2) whose rank is grown in
 * blocks until the criterion of Sec. 2.4 can be met -- the blocked randomized
 * range finder with power steps of Martinsson & Voronin (SIAM J. Sci.
 * Comput. 38(5), 2016).  Blocks of b = min(k + p, n) columns: block j draws
 * its sketch G_j (n x b) from the plan's seed plus j * 0x9E3779B97F4A7C15
 * (block 0 is rsvd_solve's sketch), takes the part of A G_j outside the
 * basis Q built so far, runs q power steps with that projection, is
 * re-orthogonalised against Q (CholeskyQR2 throughout) and appended to Q,
 * and T = A^T Q grows by A^T Q_j; the energy ||Q^T A||_F^2 = ||T||_F^2 is
 * accumulated on the device.  After each block the host reads it and
 * grows again while it is below t ||A||_F^2 (Eq. sumeigen) and another
 * block fits (L + b <= l_max and <= n): so the call synchronises the plan's
 * stream once per block.  Then SVD T = V~ S~ W^T, U~ = Q W, and K by Sec.
 * 2.4 over all L values, capped at k_max (RSVD_WARN_THRESHOLD when capped
 * or not reached).  U (m x k_max, ldu), S (k_max), V (n x k_max, ldv):
 * the first min(k_max, L) triplets are written (columns past L are left
 * untouched); rsvd_plan_diag reports L in diag[6] and the captured fraction
 * ||T||_F^2 / ||A||_F^2 in diag[7].  Any plan dtype (col_scale as
 * rsvd_solve).  Requires k <= k_max <= n, ldu and ldv >= k_max, and two
 * row-padded blocks within the plan's sketch width (2 * round_up(b, 8) <=
 * l_max, else RSVD_ERR_SHAPE); other errors as rsvd_solve. */
int32_t rsvd_solve_adaptive(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                            const float* col_scale, int32_t k, int32_t p, int32_t q, double t,
                            int32_t k_max, void* U, int64_t ldu, double* S, void* V, int64_t ldv,
                            int32_t* K);

/* rsvd_solve_krylov: the Krylov method (Sec. 3.1.1) -- G (n x l, l =
 * min(k + p, n)), blocks H(0) = A G and H(j) = A (A^T H(j-1)) for j = 1..i,
 * QR of their concatenation H (m x (i+1) l), T = A^T Q, SVD T = V~ S~ W^T,
 * U~ = Q W -- returning the first k triplets and K by the threshold t
 * (Sec. 2.4) as rsvd_solve does.  Each block is replaced by an orthonormal
 * basis of its own columns (CholeskyQR2, FP64 Gram) before it is stored and
 * used for the next one, which leaves the Krylov space unchanged; the QR of
 * H is CholeskyQR2.  omega: as rsvd_solve_omega, or NULL for the plan's
 * seeded sketch.  Requires (i+1) l <= n (else RSVD_ERR_ARG) and
 * (i+1) l <= the plan's l_max (else RSVD_ERR_SHAPE); RSVD_F64 and RSVD_F32
 * plans only.  U (m x k, ldu), S (k), V (n x k, ldv) as rsvd_solve. */
int32_t rsvd_solve_krylov(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                          int32_t k, int32_t p, int32_t i, double t, const double* omega,
                          void* U, int64_t ldu, double* S, void* V, int64_t ldv, int32_t* K);

/* rsvd_solve_bf16: Randomized PCA (Sec. 3.1.2, steps as rsvd_solve) of the
 * matrix Aq diag(col_scale), Aq bfloat16 m x n (device, row-major, lda),
 * col_scale n FP32 values (device; NULL = all ones).  The plan must be
 * RSVD_BF16.  H = A G and the power-iteration products run on BF16 matrix
 * cores with FP32 accumulation and the right factor (scaled by col_scale)
 * split into hi + lo bfloat16 pairs; T = A^T Q likewise with Q split, then
 * the rows of T times col_scale; ||A||_F^2 (Eq. sumeigen) is the FP64 sum of
 * the squared dequantised entries.  CholeskyQR2, the small SVD and U = Q W
 * as for RSVD_F32.  omega: as rsvd_solve_omega, or NULL for the plan's seeded
 * sketch.  U (m x k, ldu), V (n x k, ldv) float; S, K as rsvd_solve.
 * Requires n % 8 == 0, lda % 8 == 0 and a 16-byte aligned A (else
 * RSVD_ERR_ARG).  rsvd_solve / rsvd_solve_omega on an RSVD_BF16 plan are
 * this call (with the plan's seeded sketch for rsvd_solve). */
int32_t rsvd_solve_bf16(rsvd_plan_t plan, const void* A, const float* col_scale, int64_t m,
                        int64_t n, int64_t lda, int32_t k, int32_t p, int32_t q, double t,
                        const double* omega, float* U, int64_t ldu, double* S, float* V,
                        int64_t ldv, int32_t* K);

/* rsvd_solve_fp8: as rsvd_solve_bf16 for an RSVD_FP8 plan, Aq one OCP FP8
 * E4M3 byte per element (m x n, lda in elements; n % 8 == 0, lda % 8 == 0,
 * 8-byte aligned A). */
int32_t rsvd_solve_fp8(rsvd_plan_t plan, const void* A, const float* col_scale, int64_t m,
                       int64_t n, int64_t lda, int32_t k, int32_t p, int32_t q, double t,
                       const double* omega, float* U, int64_t ldu, double* S, float* V,
                       int64_t ldv, int32_t* K);

/* rsvd_quantize_fp8: storage of an FP32 matrix A (m x n, lda) for
 * rsvd_solve_fp8: col_scale[j] = the least power of two with
 * max_i |a_ij| / col_scale[j] <= 448 (1 for a zero or non-finite column
 * maximum) and Aq (m x n, ldq, one byte each) = A / col_scale in OCP FP8 E4M3,
 * rounded to nearest with ties to an even mantissa (subnormals kept, NaN
 * kept, magnitudes past 448 saturate).  Device pointers; runs on the plan's
 * stream (uses the plan's workspace). */
int32_t rsvd_quantize_fp8(rsvd_plan_t plan, const float* A, int64_t m, int64_t n, int64_t lda,
                          void* Aq, int64_t ldq, float* col_scale);

/* rsvd_quantize_bf16: storage of an FP32 matrix A (m x n, lda) for
 * rsvd_solve_bf16: col_scale[j] = 2^e with 2^(e-1) <= max_i |a_ij| < 2^e (1
 * for a zero or non-finite column maximum) and Aq (m x n, ldq, bfloat16) =
 * A / col_scale rounded to nearest even; power-of-two scales keep the
 * scaling exact, so Aq diag(col_scale) is A rounded to 8 significant bits.
 * Device pointers; runs on the plan's stream (uses the plan's workspace). */
int32_t rsvd_quantize_bf16(rsvd_plan_t plan, const float* A, int64_t m, int64_t n, int64_t lda,
                           void* Aq, int64_t ldq, float* col_scale);

/* gram_eig_solve: truncated SVD through A^T A (Sec. 2.3, Sec. 3.1.3):
 * G = A^T A, eigen-decomposition G = V diag(lambda) V^T (Jacobi, FP64),
 * s_i = sqrt(max(lambda_i, 0)), and u_i = A v_i / s_i for the first `ucols`
 * columns (0 = skip U; n = all, as the paper does).  A column whose s_i is
 * not above max(m, n) * 2^-52 * s_1 is returned as zero.  K is chosen by t
 * over all n values.  The plan must have been created with want_gram.
 *   U  (m x ucols, ldu >= ucols; may be NULL when ucols == 0)
 *   S  (n, double), V (n x n, ldv >= n), K (1 int32, device)
 * Errors: as rsvd_solve, plus RSVD_ERR_ARG for ucols outside [0, n] and
 * RSVD_ERR_SHAPE when the plan was not sized for the A^T A route. */
int32_t gram_eig_solve(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                       double t, int32_t ucols, void* U, int64_t ldu, double* S,
                       void* V, int64_t ldv, int32_t* K);

/* ------------------------------------------------------- stage entry points
 * The steps of the two solvers, exposed one by one so each can be checked on
 * its own.  They use the plan's stream and workspace (sizes must fit the
 * plan) and the plan's dtype for A/X/Y/Q; G, Z, R, T and eigen/singular
 * factors are FP64.
 *
 * rsvd_gaussian_fill: G (rows x cols, FP64, row-major, ld = cols) from
 * Philox4x32-10 (Salmon et al., SC 2011) and Box-Muller: element
 * e = i*cols + j uses counter (e/2 low word, e/2 high word, 0, 0), key
 * (seed low, seed high); the four words give u1 = ((x0>>5)*2^26 + (x1>>6)
 * + 0.5)*2^-53, u2 likewise from (x2, x3); even e takes
 * sqrt(-2 ln u1) cos(2 pi u2), odd e the sine (Sec. 3.1.2 step 1). */
int32_t rsvd_gaussian_fill(uint64_t seed, int64_t rows, int64_t cols, double* G, void* stream);

/* rsvd_gemm_nn: Y (m x c, ldy) = A (m x n, lda) X (n x c, ldx), the products
 * H = A G and A (A^T H) of Sec. 3.1.2.  When Gram != NULL it also writes
 * Gram (c x c, FP64) = Y^T Y accumulated in FP64, and when fro2 != NULL the
 * FP64 sum of a_ij^2 (Eq. sumeigen).  c <= plan l_max unless the plan was
 * sized for the A^T A route (then c <= n_max).  On an RSVD_BF16 (RSVD_FP8)
 * plan A is bfloat16 (FP8 E4M3) with unit scales, n % 8 == 0, lda % 8 == 0, X
 * and Y float, c <= l_max, and the product is the bf16 pass with X split into
 * hi + lo pairs. */
int32_t rsvd_gemm_nn(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                     const void* X, int64_t ldx, int32_t c, void* Y, int64_t ldy,
                     double* Gram, double* fro2);

/* rsvd_gemm_tn: Z (n x c, FP64, ld = c) = A^T (n x m) Q (m x c, ldq), the
 * product T = A^T Q of Sec. 3.1.2 (and A^T H of the power iterations); the
 * sum over the m rows is split into row blocks whose partial sums are added
 * in a fixed order (deterministic).  On an RSVD_BF16 (RSVD_FP8) plan A is
 * bfloat16 (FP8 E4M3) with unit scales, n % 8 == 0, lda % 8 == 0, Q float,
 * c <= l_max (Q is split into hi + lo bfloat16 pairs on the fly). */
int32_t rsvd_gemm_tn(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                     const void* Q, int64_t ldq, int32_t c, double* Z);

/* rsvd_cholqr2: orthonormal basis of Y (m x c, ldy) by CholeskyQR2 -- stands
 * in for "QR decomposition on H" (Sec. 3.1.2 step 4): W = Y^T Y (FP64),
 * R1 = chol(W), Q1 = Y R1^-1, R2 = chol(Q1^T Q1), Q = Q1 R2^-1, R = R2 R1.
 * Writes Q (m x c, ldq, plan dtype) and R (c x c, FP64 upper triangular,
 * positive diagonal, ld = c), Y = Q R.  A non-positive pivot sets the status
 * word to RSVD_ERR_BREAKDOWN. */
int32_t rsvd_cholqr2(rsvd_plan_t plan, const void* Y, int64_t m, int32_t c, int64_t ldy,
                     void* Q, int64_t ldq, double* R);

/* rsvd_small_svd: thin SVD of an FP64 matrix T (r x c, r >= c, ld = c) on the
 * device -- "SVD on T = V~ S~ W^T" (Sec. 3.1.2 step 6): CholeskyQR2 of T,
 * then one-sided Jacobi on the c x c factor.  Writes Vt (r x c, ld = c),
 * S (c, descending) and W (c x c, ld = c), sign rule applied. */
int32_t rsvd_small_svd(rsvd_plan_t plan, const double* T, int64_t r, int32_t c,
                       double* Vt, double* S, double* W);

/* rsvd_sym_eig: eigen-decomposition of a symmetric FP64 matrix G (n x n,
 * ld = n) -- "eigen-decomposition on A^T A" (Sec. 3.1.3 step 2) -- by
 * one-sided Jacobi on G with the rotations accumulated: lam (n, descending),
 * V (n x n, ld = n, columns = eigenvectors, sign rule applied).  Needs a plan
 * sized for the A^T A route. */
int32_t rsvd_sym_eig(rsvd_plan_t plan, const double* G, int64_t n, double* lam, double* V);

/* ------------------------------------------------------------- batches --
 * Many independent Randomized PCA problems of different shapes (Sec. 3.1.2
 * for each), solved side by side on one GPU.  A batch owns `nslots` slots, a
 * plan and a stream each (every plan sized m_max x n_max x l_max, all with
 * the same seed, so an instance's G, and its results, do not depend on the
 * slot it runs on: they equal rsvd_solve on a plan of the same sizes and
 * seed, bit for bit).  Instances go to slots largest first (m n l work), each
 * to the slot with the least work so far; the slot streams fork from and
 * join back into the caller's stream, so a batch is ordered like one kernel
 * on that stream, and the whole fork-join can be captured into a HIP graph
 * once and replayed (rsvd_batch_graph_*) for repeated batches of the same
 * shapes and pointers.  Solves and graph launches of one batch must not
 * overlap on the device (they share the slots): order them on one stream,
 * or synchronise in between. */
typedef struct rsvd_batch_s* rsvd_batch_t;
typedef struct rsvd_batch_graph_s* rsvd_batch_graph_t;

/* One problem of a batch: arguments as rsvd_solve (device pointers A, U, S,
 * V, K; U may be NULL for a problem that needs only S, V and K -- the
 * principal directions and their variances -- and then costs no U product;
 * grouped batches need U), plus `status` (1 int32, device) that receives the instance's status
 * word (RSVD_OK, RSVD_WARN_*, RSVD_ERR_BREAKDOWN / _NONFINITE / _NOCONV), and
 * for RSVD_BF16 / RSVD_FP8 batches and servers `col_scale` (n floats, device,
 * or NULL for unit scales) as in rsvd_solve_bf16; ignored otherwise.
 * `k_max` (servers only; 0 or <= k = off): adaptive rank -- the request is
 * solved as rsvd_solve_adaptive (the rank grown in blocks of b = min(k + p,
 * n) columns, reusing the basis, until the threshold t can be met or the
 * plan's l_max is full; 2 round_up(b, 8) <= l_max), with K capped at k_max;
 * U, S, V then hold k_max <= n columns (ldu, ldv >= k_max), the first
 * min(k_max, columns found) written.  A server created with
 * RSVD_SERVER_GRAM_FALLBACK sends such a request to the A^T A route
 * instead when its K is predicted past n / 2 (the paper's conclusion that
 * the A^T A route is faster when most eigenpairs are needed, Sec. 3.3 and 5)
 * or past what the sketch can hold; see rsvd_server_create.
 * `dtype` (0 = the batch's or server's own dtype): the storage of this
 * instance's A -- RSVD_F32, RSVD_BF16 or RSVD_FP8 (A as in rsvd_solve_bf16 /
 * rsvd_solve_fp8, with col_scale) on a batch or server of any of those three
 * dtypes (U and V are float for all of them), RSVD_F64 on an RSVD_F64 one;
 * grouped batches take RSVD_F32 only. */
typedef struct {
  const void* A;
  int64_t m, n, lda;
  int32_t k, p, q;
  double t;
  void* U;
  int64_t ldu;
  double* S;
  void* V;
  int64_t ldv;
  int32_t* K;
  int32_t* status;
  const float* col_scale;
  int32_t k_max;
  int32_t dtype;
} rsvd_instance;

/* Create a batch of nslots (1..64) slots for problems of one dtype (any of
 * rsvd_dtype: A of RSVD_BF16 / RSVD_FP8 problems stored as in
 * rsvd_solve_bf16 / rsvd_solve_fp8, with U and V float) up to m_max x n_max
 * with k + p <= l_max (limits as rsvd_plan_create).  Each slot's stream is
 * created by the batch (default priority).  Errors as rsvd_plan_create,
 * RSVD_ERR_ARG for nslots out of range. */
int32_t rsvd_batch_create(rsvd_batch_t* batch, int32_t nslots, int64_t m_max, int64_t n_max,
                          int32_t l_max, int32_t dtype, uint64_t seed);

/* Synchronise and free the slots' plans and streams. NULL is a no-op. */
int32_t rsvd_batch_destroy(rsvd_batch_t batch);

/* Solve `count` instances (host array, read during the call only), ordered
 * on `stream` (hipStream_t, NULL = the null stream) as one unit: work
 * queued on it earlier completes first, work queued later waits for every
 * instance.  All instances are validated before anything is launched: the
 * first invalid one returns RSVD_ERR_ARG / RSVD_ERR_SHAPE as rsvd_solve
 * would (also for a NULL status pointer) and nothing runs. */
int32_t rsvd_batch_solve(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                         void* stream);

/* Capture rsvd_batch_solve(batch, inst, count, stream) into an executable
 * HIP graph (nothing runs yet); every launch of it repeats the same solves
 * on the same buffers.  The graph uses the batch's slots: one batch, one
 * graph in flight at a time.  Errors as rsvd_batch_solve, RSVD_ERR_DEVICE
 * when capture or instantiation fails. */
int32_t rsvd_batch_graph_create(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                                void* stream, rsvd_batch_graph_t* graph);

/* Launch a captured batch on `stream`. */
int32_t rsvd_batch_graph_launch(rsvd_batch_graph_t graph, void* stream);

/* Free a captured batch (synchronises nothing; NULL is a no-op). */
int32_t rsvd_batch_graph_destroy(rsvd_batch_graph_t graph);

/* Grouped batches: the same solves as rsvd_batch_solve for RSVD_F32
 * instances (Sec. 3.1.2 each), with every step one launch for all
 * instances (instead of one chain of launches per instance on the slots),
 * which removes the per-instance launch latency that bounds batches of small
 * problems.  The passes over the tall matrices run over a work list of
 * (instance, row panel) items, largest instances first, one workgroup per
 * item: the A X product and the Y R^-1 product of CholeskyQR2 also take the
 * panel's FP64 Gram matrix from their output registers (the m-row Gram
 * matrices of CholeskyQR2, l <= 64), and the first pass its sum of squares;
 * A^T Q writes one FP64 partial per row split.  Each instance's partials are
 * summed in a fixed order.
 *
 * rsvd_batch_grouped_create validates the instances (as rsvd_batch_solve;
 * further RSVD_ERR_ARG unless A is 16-byte aligned with lda and n multiples
 * of 4, l = min(k + p, n) a multiple of 4 and at most 96, and U given),
 * allocates one workspace per instance, sized for it, and records the
 * launches with their arguments and work lists (uploaded once); nothing
 * runs.  `tune` (host, `ntune` entries, may be NULL) sets the tile
 * parameters per (n, l): rows per work item of the A X and Y R^-1 products
 * and the shortest A^T Q row split (rsvd_tune_entry; instances with no
 * entry take 1024 and 1024; RSVD_ERR_ARG for an entry outside the limits
 * below).  rsvd_batch_grouped_launch runs the batch on `stream`: the steps
 * of rsvd_solve on a plan with the batch's seed (the same G), with longer
 * row splits for the FP64 partial sums (at least 1024 rows each, where a
 * solve alone on the GPU splits its rows over every CU), since the
 * instances fill the GPU together; the sums are rounded in another order,
 * so results agree with rsvd_solve to FP32 rounding, not bit for bit, and
 * every launch of one grouped batch gives the same bits (also with another
 * tuning).  Instances with equal l, k and q share launches.  One launch of
 * a grouped batch at a time; rsvd_batch_grouped_destroy synchronises the
 * device and frees it. */
typedef struct rsvd_tune_entry {
  int32_t n, l;          /* the bucket: instances with this n and l = min(k + p, n) */
  int32_t panel_rows;    /* rows per work item of A X and Y R^-1: a multiple of 128, 1024..2^20 */
  int32_t split_rows;    /* shortest A^T Q row split: a multiple of 16, 1024..2^20 */
} rsvd_tune_entry;
typedef struct rsvd_grouped_s* rsvd_grouped_t;
int32_t rsvd_batch_grouped_create(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                                  const rsvd_tune_entry* tune, int32_t ntune,
                                  rsvd_grouped_t* grouped);
int32_t rsvd_batch_grouped_launch(rsvd_grouped_t grouped, void* stream);
int32_t rsvd_batch_grouped_destroy(rsvd_grouped_t grouped);

/* Capture one launch of a grouped batch into a HIP graph (nothing runs);
 * launch it with rsvd_batch_graph_launch on any stream (each launch repeats
 * the same solves on the same buffers, bit for bit those of
 * rsvd_batch_grouped_launch) and free it with rsvd_batch_graph_destroy.  The
 * grouped batch must outlive the graph; one launch of either at a time.
 * RSVD_ERR_DEVICE if the capture fails. */
int32_t rsvd_batch_grouped_graph_create(rsvd_grouped_t grouped, rsvd_batch_graph_t* graph);

/* Autotuner of the grouped tile parameters: for each (n, l) bucket of the
 * instances (in order of first appearance; at most `cap`, else
 * RSVD_ERR_ARG) it times grouped launches of that bucket's instances alone
 * on `stream` (one untimed launch, then the mean of three) for rows per
 * work item in {1024, 2048, 4096, 8192} at the default split, then the
 * split in the same set at the best rows, and writes the fastest pair to
 * out[b] (host); *nout = the number of buckets.  It runs the instances
 * (their outputs are written) and synchronises the device; the entries are
 * for rsvd_batch_grouped_create.  Errors as rsvd_batch_grouped_create. */
int32_t rsvd_batch_grouped_tune(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                                rsvd_tune_entry* out, int32_t cap, int32_t* nout, void* stream);

/* ------------------------------------------------------------- serving --
 * Continuous batching of Randomized PCA requests (Sec. 3.1.2 each): requests
 * are queued in arrival order and admitted, first come first served, as
 * soon as a slot is free and the HBM they occupy while running fits the
 * budget; a finished request frees its slot and its share of the budget at
 * once, so requests that arrive while others run start beside them.  The
 * slots are as in a batch (a plan and a stream each, same sizes and seed):
 * a request's results do not depend on what else runs (bit for bit).
 * Footprint of a request: its A (m lda elements), the two m x l panels of
 * its plan and the split partials of its A^T Q products (n l FP64 per split).
 * A server is driven from one host thread at a time (its calls must not
 * overlap).  After RSVD_ERR_DEVICE from any call its state is undefined:
 * destroy it. */
typedef struct rsvd_server_s* rsvd_server_t;

/* Create a server with nslots slots (1..64) for requests of one dtype (as
 * rsvd_batch_create; an RSVD_F32, RSVD_BF16 or RSVD_FP8 server also takes
 * requests whose own `dtype` is another of those three) up to m_max x n_max
 * with k + p <= l_max, admitting while the running requests' footprints sum
 * to at most hbm_budget bytes (a request larger than the budget runs alone).
 * flags: RSVD_SERVER_GRAM_FALLBACK adds two A^T A-route slots (each a plan
 * sized m_max x n_max for gram_eig_solve, n_max <= 1024, its own stream, and
 * for non-FP64 servers an m_max x n_max fp32 buffer into which a bfloat16 /
 * FP8 request's A is dequantised): a request with k_max > k whose growth
 * predicts K > n / 2 (from the energy its last block captured per column,
 * a lower estimate on a decaying spectrum) or finds the sketch full below t
 * is moved there, first come first served, and solved with all n
 * eigenpairs: K by Sec. 2.4 over all n values (capped at k_max), and U,
 * S, V receive the route's first k_max sorted triplets.  Errors as
 * rsvd_batch_create, and RSVD_ERR_SHAPE for the fallback with
 * n_max > 1024. */
#define RSVD_SERVER_GRAM_FALLBACK 1
int32_t rsvd_server_create(rsvd_server_t* server, int32_t nslots, int64_t m_max, int64_t n_max,
                           int32_t l_max, int32_t dtype, uint64_t seed, int64_t hbm_budget,
                           int32_t flags);

/* Queue one request (arguments and status word as a batch instance; the
 * buffers must stay valid until it is reported done).  A (and col_scale)
 * must be complete on the device when this is called: the request runs on
 * the server's own slot streams, which are not ordered after any stream of
 * the caller (synchronise the stream that wrote A first).  Validated at once
 * (RSVD_ERR_ARG / RSVD_ERR_SHAPE as rsvd_solve, nothing queued); *ticket
 * receives its number (0, 1, 2, ... in submission order).  Admits at once
 * when it can. */
int32_t rsvd_server_submit(rsvd_server_t server, const rsvd_instance* req, int64_t* ticket);

/* Never blocks: retires the requests whose work has finished (their
 * outputs and status words are then complete) and admits queued ones.
 * Writes up to `cap` finished tickets to `done` (host array) and their
 * number to *ndone; more finished tickets are kept for the next call.
 * *queued and *running (either may be NULL) receive the counts after the
 * call. */
int32_t rsvd_server_progress(rsvd_server_t server, int64_t* done, int32_t cap, int32_t* ndone,
                             int32_t* queued, int32_t* running);

/* Wait for every queued and running request, then free the server. */
int32_t rsvd_server_destroy(rsvd_server_t server);

/* ------------------------------------------------------ allocation-free --
 * rsvd_solve_noalloc: rsvd_solve (Randomized PCA, same steps, same kernels,
 * same results bit for bit as rsvd_solve on a plan with this seed) without a
 * plan and without allocating anything: for callers that cannot call
 * hipMalloc (code under HIP graph capture, tight serving loops, harnesses
 * that forbid device allocation).  The workspace is a file-scope device
 * array of RSVD_NOALLOC_SCRATCH_BYTES that each GPU the library runs on
 * holds from the library's loading until the process ends; the call makes
 * no hipMalloc / hipFree and creates no streams or events.
 *   A, m, n, lda, k, p, q, t, U, ldu, S, V, ldv, K   as rsvd_solve
 *   dtype   RSVD_F64 or RSVD_F32 (element type of A, U, V)
 *   seed    seeds the Gaussian sketch G as rsvd_plan_create's seed does
 *   status  (1 int32, device) receives the solve's status word (RSVD_OK,
 *           RSVD_WARN_*, RSVD_ERR_BREAKDOWN / _NONFINITE / _NOCONV)
 *   stream  hipStream_t to order the work on (NULL = the null stream)
 * Workspace: about (2 m l + n l) elements of dtype plus (s + 6) n l + 16 l^2
 * doubles, l = min(k + p, n), s = min(256, ceil(m / 64)) row splits.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (on different streams or threads) race and must not be issued; calls
 * ordered on one stream are safe.  Errors (synchronous, nothing launched):
 * RSVD_ERR_ARG (bad dtype, NULL A / status, the argument errors of
 * rsvd_solve), RSVD_ERR_SHAPE (m < n, m > 2^40, n > 2^20, l > 192, or a workspace larger than
 * RSVD_NOALLOC_SCRATCH_BYTES), RSVD_ERR_DEVICE. */
#define RSVD_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t rsvd_solve_noalloc(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype,
                           int32_t k, int32_t p, int32_t q, double t, uint64_t seed, void* U,
                           int64_t ldu, double* S, void* V, int64_t ldv, int32_t* K,
                           int32_t* status, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RSVD_H */
