/*
 * oracle.c -- plain FP64 CPU reference for the PCA-by-SVD hot path of
 * "Tutorial: Complexity analysis of Singular Value Decomposition and its
 * variants" (Li, Wang, Cai; arXiv 1906.12085).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU library never
 * links, includes or calls it, and it shares no code with the GPU path.
 *
 * Conventions (paper, Sec. 1 "Notations"/"Assumptions" and Sec. 2.2):
 *   - A is m x n, real, m >= n, rows are examples, columns are features.
 *   - Every matrix here is double precision, row-major, with an explicit
 *     leading dimension (elements between consecutive rows).
 *   - Singular values / eigenvalues are returned in descending order.
 *
 * What each routine computes, and the passage it follows:
 *   orc_gemm_nn / orc_gemm_tn   dense products (Sec. 3.1, FLOP convention)
 *   orc_fro2                    sum of a_ij^2 (Eq. sumeigen)
 *   orc_qr_householder          thin QR, Householder reflections; stands in
 *                               for "QR decomposition on H" (Sec. 3.1.2 step 4)
 *   orc_svd_jacobi              one-sided (Hestenes) Jacobi SVD; A = U S V^T
 *                               with U^T U = V^T V = I (Sec. 2.1, Eq. AV)
 *   orc_svd_exact               QR of A, then one-sided Jacobi on R
 *   orc_eig_sym_jacobi          cyclic two-sided Jacobi eigensolver for a
 *                               symmetric matrix (eig of A^T A, Sec. 2.3)
 *   orc_select_k                cumulative explained variance criterion
 *                               (Sec. 2.4, Eq. sumeigen for the denominator)
 *   orc_sign_convention         output sign rule (not in the paper)
 *   orc_rsvd                    Randomized PCA (Sec. 3.1.2) with a QR after
 *                               every product with A or A^T
 *   orc_krylov                  Krylov method (Sec. 3.1.1), blocks kept
 *                               orthonormal (same Krylov space)
 *   orc_gram_eig                truncated SVD through A^T A (Sec. 2.3,
 *                               Sec. 3.1.3)
 *   orc_rsvd_blocked            Randomized PCA with the rank grown in blocks
 *                               until the criterion of Sec. 2.4 can be met
 *                               (Martinsson & Voronin 2016, blocked range
 *                               finder with power steps)
 *
 * Reductions are split into a fixed number of row chunks whose partial
 * results are added in chunk order, so results do not depend on the number
 * of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* status words shared with the Python wrapper (oracle/__init__.py) */
#define ORC_OK 0
#define ORC_WARN_THRESHOLD 1   /* sum of the k captured lambda_i < t ||A||_F^2 */
#define ORC_WARN_ZERO 2        /* ||A||_F == 0 */
#define ORC_ERR_ARG (-1)
#define ORC_ERR_NOMEM (-3)
#define ORC_ERR_NOCONV (-7)    /* Jacobi did not converge in the sweep limit */

#define ORC_CHUNKS 64          /* fixed reduction split, see header */
#define ORC_MAX_SWEEPS 80

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Dense products.  One multiply-add per term, the counting rule of Sec. 3.1. */

/* C (m x n) = A (m x k) * B (k x n). */
void orc_gemm_nn(int64_t m, int64_t k, int64_t n,
                 const double* A, int64_t lda, const double* B, int64_t ldb,
                 double* C, int64_t ldc) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    double* c = C + i * ldc;
    for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
    for (int64_t p = 0; p < k; ++p) {
      const double a = A[i * lda + p];
      const double* b = B + p * ldb;
      for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
    }
  }
}

/* C (k x n) = A^T B, A (m x k), B (m x n): the sum over the m rows is split
 * into ORC_CHUNKS fixed row chunks added in order. */
int orc_gemm_tn(int64_t m, int64_t k, int64_t n,
                const double* A, int64_t lda, const double* B, int64_t ldb,
                double* C, int64_t ldc) {
  const int64_t nch = m < ORC_CHUNKS ? (m > 0 ? m : 1) : ORC_CHUNKS;
  double* part = (double*)calloc((size_t)(nch * k * n), sizeof(double));
  if (!part) return ORC_ERR_NOMEM;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nch; ++c) {
    const int64_t r0 = m * c / nch, r1 = m * (c + 1) / nch;
    double* P = part + c * k * n;
    for (int64_t r = r0; r < r1; ++r) {
      const double* a = A + r * lda;
      const double* b = B + r * ldb;
      for (int64_t i = 0; i < k; ++i) {
        const double ai = a[i];
        double* p = P + i * n;
        for (int64_t j = 0; j < n; ++j) p[j] += ai * b[j];
      }
    }
  }
  for (int64_t i = 0; i < k; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t c = 0; c < nch; ++c) s += part[c * k * n + i * n + j];
      C[i * ldc + j] = s;
    }
  free(part);
  return ORC_OK;
}

/* Sum of a_ij^2 = ||A||_F^2 = tr(A^T A) = sum of all lambda_i (Eq. sumeigen). */
double orc_fro2(int64_t m, int64_t n, const double* A, int64_t lda) {
  const int64_t nch = m < ORC_CHUNKS ? (m > 0 ? m : 1) : ORC_CHUNKS;
  double part[ORC_CHUNKS];
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    double s = 0.0;
    for (int64_t r = m * c / nch; r < m * (c + 1) / nch; ++r)
      for (int64_t j = 0; j < n; ++j) s += A[r * lda + j] * A[r * lda + j];
    part[c] = s;
  }
  double s = 0.0;
  for (int64_t c = 0; c < nch; ++c) s += part[c];
  return s;
}

/* w[c] = sum_{i=r0}^{m-1} v[i*ldv] * X[i*ldx + c] for c in [c0, c1): the row
 * sum is split into ORC_CHUNKS fixed chunks added in chunk order. */
static int orc_weighted_colsum(int64_t r0, int64_t m, const double* v, int64_t ldv,
                               const double* X, int64_t ldx, int64_t c0, int64_t c1, double* w) {
  const int64_t rows = m - r0, width = c1 - c0;
  for (int64_t c = c0; c < c1; ++c) w[c] = 0.0;
  if (rows <= 0 || width <= 0) return ORC_OK;
  const int64_t nch = rows < ORC_CHUNKS ? rows : ORC_CHUNKS;
  double* part = (double*)calloc((size_t)(nch * width), sizeof(double));
  if (!part) return ORC_ERR_NOMEM;
#pragma omp parallel for schedule(static)
  for (int64_t ch = 0; ch < nch; ++ch) {
    double* P = part + ch * width;
    for (int64_t i = r0 + rows * ch / nch; i < r0 + rows * (ch + 1) / nch; ++i) {
      const double vi = v[i * ldv];
      for (int64_t c = c0; c < c1; ++c) P[c - c0] += vi * X[i * ldx + c];
    }
  }
  for (int64_t ch = 0; ch < nch; ++ch)
    for (int64_t c = c0; c < c1; ++c) w[c] += part[ch * width + c - c0];
  free(part);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Thin QR by Householder reflections (Golub & Van Loan, Matrix Computations,
 * 4th ed., Alg. 5.2.1 with backward accumulation of Q).  X (m x n, m >= n) is
 * not modified.  Q (m x n) has orthonormal columns, R (n x n) is upper
 * triangular with R_jj >= 0, and X = Q R.  This is the orthonormaliser the
 * paper calls "QR decomposition on H" (Sec. 3.1.2, step 4). */
int orc_qr_householder(int64_t m, int64_t n, const double* X, int64_t ldx,
                       double* Q, int64_t ldq, double* R, int64_t ldr) {
  if (m < n || n < 1) return ORC_ERR_ARG;
  double* W = (double*)malloc((size_t)(m * n) * sizeof(double)); /* working copy */
  double* vs = (double*)malloc((size_t)(m * n) * sizeof(double)); /* reflectors, v_j in column j, rows j.. */
  double* beta = (double*)malloc((size_t)n * sizeof(double));
  double* w = (double*)malloc((size_t)n * sizeof(double));
  if (!W || !vs || !beta || !w) { free(W); free(vs); free(beta); free(w); return ORC_ERR_NOMEM; }
  for (int64_t i = 0; i < m; ++i) memcpy(W + i * n, X + i * ldx, (size_t)n * sizeof(double));
  memset(vs, 0, (size_t)(m * n) * sizeof(double));

  for (int64_t j = 0; j < n; ++j) {
    /* reflector that maps x = W[j:, j] onto alpha e_1, alpha = -sign(x_0)||x|| */
    double nrm2 = 0.0;
    for (int64_t i = j; i < m; ++i) nrm2 += W[i * n + j] * W[i * n + j];
    const double x0 = W[j * n + j];
    const double nrm = sqrt(nrm2);
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    double vtv = 0.0;
    for (int64_t i = j; i < m; ++i) {
      const double v = (i == j) ? x0 - alpha : W[i * n + j];
      vs[i * n + j] = v;
      vtv += v * v;
    }
    beta[j] = vtv > 0.0 ? 2.0 / vtv : 0.0;
    if (beta[j] == 0.0) continue;  /* x already a multiple of e_1 (or zero) */
    /* W[j:, j:] -= beta v (v^T W[j:, j:]) ; two passes over the rows */
    if (orc_weighted_colsum(j, m, vs + j, n, W, n, j, n, w) != ORC_OK) {
      free(W); free(vs); free(beta); free(w); return ORC_ERR_NOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = j; i < m; ++i) {
      const double bv = beta[j] * vs[i * n + j];
      for (int64_t c = j; c < n; ++c) W[i * n + c] -= bv * w[c];
    }
  }
  /* Q = H_0 H_1 ... H_{n-1} [I_n; 0], applied from the last reflector back */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i)
    for (int64_t c = 0; c < n; ++c) Q[i * ldq + c] = (i == c) ? 1.0 : 0.0;
  for (int64_t j = n - 1; j >= 0; --j) {
    if (beta[j] == 0.0) continue;
    if (orc_weighted_colsum(j, m, vs + j, n, Q, ldq, 0, n, w) != ORC_OK) {
      free(W); free(vs); free(beta); free(w); return ORC_ERR_NOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = j; i < m; ++i) {
      const double bv = beta[j] * vs[i * n + j];
      for (int64_t c = 0; c < n; ++c) Q[i * ldq + c] -= bv * w[c];
    }
  }
  /* R = upper triangle of W; make its diagonal non-negative (unique QR) */
  for (int64_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < n; ++c) R[i * ldr + c] = (c >= i) ? W[i * n + c] : 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (R[j * ldr + j] < 0.0) {
      for (int64_t c = 0; c < n; ++c) R[j * ldr + c] = -R[j * ldr + c];
      for (int64_t i = 0; i < m; ++i) Q[i * ldq + j] = -Q[i * ldq + j];
    }
  }
  free(W); free(vs); free(beta); free(w);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sorting helper: permutation that orders key[] descending (stable). */
static void orc_order_desc(int64_t n, const double* key, int64_t* perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  for (int64_t i = 1; i < n; ++i) { /* insertion sort: n is small */
    const int64_t p = perm[i];
    int64_t j = i - 1;
    while (j >= 0 && key[perm[j]] < key[p]) { perm[j + 1] = perm[j]; --j; }
    perm[j + 1] = p;
  }
}

/* One-sided (Hestenes) Jacobi SVD of X (m x n, m >= n):  X = U S V^T with
 * U^T U = I_n, V^T V = V V^T = I_n, S descending (Sec. 2.1).  Column pairs
 * (p, q) are rotated until every pair is orthogonal to working precision;
 * V accumulates the rotations, so X V = U S, i.e. X v_i = s_i u_i (Eq. AV).
 * A column whose norm is exactly zero gives s_i = 0 and u_i = 0.
 * Returns the number of sweeps used, or ORC_ERR_NOCONV. */
int orc_svd_jacobi(int64_t m, int64_t n, const double* X, int64_t ldx,
                   double* U, int64_t ldu, double* S, double* V, int64_t ldv) {
  if (m < n || n < 1) return ORC_ERR_ARG;
  /* column-major working copies: column j of W is W + j*m */
  double* W = (double*)malloc((size_t)(m * n) * sizeof(double));
  double* J = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* nrm = (double*)malloc((size_t)n * sizeof(double));
  int64_t* perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!W || !J || !nrm || !perm) { free(W); free(J); free(nrm); free(perm); return ORC_ERR_NOMEM; }
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) W[j * m + i] = X[i * ldx + j];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) J[j * n + i] = (i == j) ? 1.0 : 0.0;

  const double tol = 2.220446049250313e-16 * sqrt((double)m);
  int sweep = 0, converged = 0;
  while (!converged && sweep < ORC_MAX_SWEEPS) {
    ++sweep;
    int64_t rotations = 0;
    for (int64_t p = 0; p < n - 1; ++p) {
      for (int64_t q = p + 1; q < n; ++q) {
        double* wp = W + p * m;
        double* wq = W + q * m;
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int64_t i = 0; i < m; ++i) {
          alpha += wp[i] * wp[i];
          beta += wq[i] * wq[i];
          gamma += wp[i] * wq[i];
        }
        if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
        ++rotations;
        /* rotation that makes the two columns orthogonal:
           zeta = (beta - alpha) / (2 gamma), t = sign(zeta)/(|zeta| + sqrt(1+zeta^2)) */
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
        for (int64_t i = 0; i < m; ++i) {
          const double xp = wp[i], xq = wq[i];
          wp[i] = c * xp - s * xq;
          wq[i] = s * xp + c * xq;
        }
        double* jp = J + p * n;
        double* jq = J + q * n;
        for (int64_t i = 0; i < n; ++i) {
          const double xp = jp[i], xq = jq[i];
          jp[i] = c * xp - s * xq;
          jq[i] = s * xp + c * xq;
        }
      }
    }
    converged = (rotations == 0);
  }
  /* singular values are the column norms; U = normalised columns */
  for (int64_t j = 0; j < n; ++j) {
    double s2 = 0.0;
    for (int64_t i = 0; i < m; ++i) s2 += W[j * m + i] * W[j * m + i];
    nrm[j] = sqrt(s2);
  }
  orc_order_desc(n, nrm, perm);
  for (int64_t jj = 0; jj < n; ++jj) {
    const int64_t j = perm[jj];
    S[jj] = nrm[j];
    const double inv = nrm[j] > 0.0 ? 1.0 / nrm[j] : 0.0;
    for (int64_t i = 0; i < m; ++i) U[i * ldu + jj] = W[j * m + i] * inv;
    for (int64_t i = 0; i < n; ++i) V[i * ldv + jj] = J[j * n + i];
  }
  free(W); free(J); free(nrm); free(perm);
  return converged ? sweep : ORC_ERR_NOCONV;
}

/* Exact thin SVD X = U S V^T (m >= n): Householder QR X = Q R, one-sided
 * Jacobi on R = U_R S V^T, U = Q U_R.  Returns sweeps or an error. */
int orc_svd_exact(int64_t m, int64_t n, const double* X, int64_t ldx,
                  double* U, int64_t ldu, double* S, double* V, int64_t ldv) {
  if (m < n || n < 1) return ORC_ERR_ARG;
  double* Q = (double*)malloc((size_t)(m * n) * sizeof(double));
  double* R = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* UR = (double*)malloc((size_t)(n * n) * sizeof(double));
  if (!Q || !R || !UR) { free(Q); free(R); free(UR); return ORC_ERR_NOMEM; }
  int rc = orc_qr_householder(m, n, X, ldx, Q, n, R, n);
  if (rc == ORC_OK) rc = orc_svd_jacobi(n, n, R, n, UR, n, S, V, ldv);
  if (rc >= 0) {
    /* U = Q U_R */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t p = 0; p < n; ++p) s += Q[i * n + p] * UR[p * n + j];
        U[i * ldu + j] = s;
      }
  }
  free(Q); free(R); free(UR);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Cyclic-by-row two-sided Jacobi for a symmetric n x n matrix G (Golub & Van
 * Loan, Alg. 8.5.2 / 8.5.3): G = V diag(lam) V^T, V^T V = I, lam descending.
 * This is the "eigen-decomposition on A^T A" of Sec. 2.3 / Sec. 3.1.3 step 2.
 * A pair is skipped when |g_pq| <= eps * sqrt(|g_pp g_qq|).
 * Returns the number of sweeps used, or an error. */
int orc_eig_sym_jacobi(int64_t n, const double* G, int64_t ldg,
                       double* lam, double* V, int64_t ldv) {
  if (n < 1) return ORC_ERR_ARG;
  double* M = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* Z = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* d = (double*)malloc((size_t)n * sizeof(double));
  int64_t* perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!M || !Z || !d || !perm) { free(M); free(Z); free(d); free(perm); return ORC_ERR_NOMEM; }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      M[i * n + j] = 0.5 * (G[i * ldg + j] + G[j * ldg + i]);
      Z[i * n + j] = (i == j) ? 1.0 : 0.0;
    }
  const double eps = 2.220446049250313e-16;
  int sweep = 0, converged = (n == 1);
  while (!converged && sweep < ORC_MAX_SWEEPS) {
    ++sweep;
    int64_t rotations = 0;
    for (int64_t p = 0; p < n - 1; ++p) {
      for (int64_t q = p + 1; q < n; ++q) {
        const double apq = M[p * n + q];
        const double app = M[p * n + p], aqq = M[q * n + q];
        if (apq == 0.0 || fabs(apq) <= eps * sqrt(fabs(app) * fabs(aqq))) continue;
        ++rotations;
        /* symmetric Schur decomposition of the 2x2 block (GVL Alg. 8.5.1):
           tau = (a_qq - a_pp)/(2 a_pq), t = sign(tau)/(|tau| + sqrt(1+tau^2)) */
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = t * c;
        /* M <- J^T M J with J = [[c, s], [-s, c]] in rows/cols (p, q) */
        for (int64_t k = 0; k < n; ++k) { /* columns p and q: M <- M J */
          const double mkp = M[k * n + p], mkq = M[k * n + q];
          M[k * n + p] = c * mkp - s * mkq;
          M[k * n + q] = s * mkp + c * mkq;
        }
        for (int64_t k = 0; k < n; ++k) { /* rows p and q: M <- J^T M */
          const double mpk = M[p * n + k], mqk = M[q * n + k];
          M[p * n + k] = c * mpk - s * mqk;
          M[q * n + k] = s * mpk + c * mqk;
        }
        M[p * n + q] = 0.0;
        M[q * n + p] = 0.0;
        for (int64_t k = 0; k < n; ++k) { /* Z <- Z J */
          const double zkp = Z[k * n + p], zkq = Z[k * n + q];
          Z[k * n + p] = c * zkp - s * zkq;
          Z[k * n + q] = s * zkp + c * zkq;
        }
      }
    }
    converged = (rotations == 0);
  }
  for (int64_t i = 0; i < n; ++i) d[i] = M[i * n + i];
  orc_order_desc(n, d, perm);
  for (int64_t jj = 0; jj < n; ++jj) {
    lam[jj] = d[perm[jj]];
    for (int64_t i = 0; i < n; ++i) V[i * ldv + jj] = Z[i * n + perm[jj]];
  }
  free(M); free(Z); free(d); free(perm);
  return converged ? sweep : ORC_ERR_NOCONV;
}

/* ------------------------------------------------------------------------ */
/* Cumulative explained variance criterion (Sec. 2.4): the minimal K with
 * (lambda_1 + ... + lambda_K) / (sum of all lambda_i) >= t, lambda_i = s_i^2
 * (Eq. LambdaSigma), and the denominator taken as ||A||_F^2 (Eq. sumeigen),
 * so a method that holds only k of the n singular values can still apply it.
 * The partial sums run in index order.  K is searched in 1..k; if even K = k
 * falls short, K = k and ORC_WARN_THRESHOLD is returned; fro2 == 0 gives
 * K = 0 and ORC_WARN_ZERO. */
int orc_select_k(int64_t k, const double* s, double fro2, double t, int64_t* K) {
  if (k < 1 || !(t > 0.0 && t <= 1.0) || !(fro2 >= 0.0)) return ORC_ERR_ARG;
  if (fro2 == 0.0) { *K = 0; return ORC_WARN_ZERO; }
  double cum = 0.0;
  for (int64_t i = 0; i < k; ++i) {
    cum += s[i] * s[i];
    if (cum >= t * fro2) { *K = i + 1; return ORC_OK; }
  }
  *K = k;
  return ORC_WARN_THRESHOLD;
}

/* Output sign rule (the paper fixes none; singular vector pairs are defined
 * up to a common sign): flip (u_i, v_i) so that the lowest-index entry of v_i
 * whose magnitude is within 0.1% of the largest magnitude is positive.  The
 * 0.1% band makes exact ties (e.g. +-1/sqrt2) independent of rounding. */
void orc_sign_convention(int64_t m, int64_t n, int64_t k,
                         double* U, int64_t ldu, double* V, int64_t ldv) {
  for (int64_t j = 0; j < k; ++j) {
    double vmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double a = fabs(V[i * ldv + j]);
      if (a > vmax) vmax = a;
    }
    int64_t best = 0;
    for (int64_t i = 0; i < n; ++i)
      if (fabs(V[i * ldv + j]) >= 0.999 * vmax) { best = i; break; }
    if (V[best * ldv + j] < 0.0) {
      for (int64_t i = 0; i < n; ++i) V[i * ldv + j] = -V[i * ldv + j];
      if (U)
        for (int64_t i = 0; i < m; ++i) U[i * ldu + j] = -U[i * ldu + j];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Randomized PCA (Sec. 3.1.2), in the paper's notation:
 *   1. G (n x l) standard normal           -- passed in as `G` (l = k + p,
 *                                              clamped to n)
 *   2. H = A G                             -- then QR: H = Q R
 *   3. i = 1..q power iterations H = A (A^T H); an orthonormalisation follows
 *      every product (A^T Q -> QR, A Q~ -> QR), as in the subspace iteration
 *      of Halko, Martinsson & Tropp (SIAM Review 2011, Alg. 4.4)
 *   4. QR of H -> Q (m x l)
 *   5. T = A^T Q (n x l)
 *   6. SVD T = V~ S~ W^T
 *   7. U~ = Q W
 * Outputs: U (m x k, ldu), S (k), V (n x k, ldv) = the first k columns of
 * U~, S~, V~ after the sign rule; K by the criterion of Sec. 2.4 over the k
 * values; fro2 = ||A||_F^2.  Returns ORC_OK / ORC_WARN_* or an error. */
int orc_rsvd(int64_t m, int64_t n, const double* A, int64_t lda,
             const double* G, int64_t k, int64_t p, int64_t q, double t,
             double* U, int64_t ldu, double* S, double* V, int64_t ldv,
             int64_t* K, double* fro2) {
  if (m < n || n < 1 || k < 1 || k > n || p < 0 || q < 0 || !(t > 0.0 && t <= 1.0))
    return ORC_ERR_ARG;
  const int64_t l = (k + p < n) ? k + p : n;
  double* H = (double*)malloc((size_t)(m * l) * sizeof(double));
  double* Q = (double*)malloc((size_t)(m * l) * sizeof(double));
  double* T = (double*)malloc((size_t)(n * l) * sizeof(double));
  double* Qt = (double*)malloc((size_t)(n * l) * sizeof(double));
  double* R = (double*)malloc((size_t)(l * l) * sizeof(double));
  double* Vt = (double*)malloc((size_t)(n * l) * sizeof(double));
  double* St = (double*)malloc((size_t)l * sizeof(double));
  double* W = (double*)malloc((size_t)(l * l) * sizeof(double));
  int rc = ORC_OK;
  if (!H || !Q || !T || !Qt || !R || !Vt || !St || !W) { rc = ORC_ERR_NOMEM; goto done; }

  *fro2 = orc_fro2(m, n, A, lda);                               /* Eq. sumeigen */
  orc_gemm_nn(m, n, l, A, lda, G, l, H, l);                    /* H = A G */
  if ((rc = orc_qr_householder(m, l, H, l, Q, l, R, l)) != ORC_OK) goto done;
  for (int64_t it = 0; it < q; ++it) {                          /* H = A (A^T H) */
    if ((rc = orc_gemm_tn(m, n, l, A, lda, Q, l, T, l)) != ORC_OK) goto done;
    if ((rc = orc_qr_householder(n, l, T, l, Qt, l, R, l)) != ORC_OK) goto done;
    orc_gemm_nn(m, n, l, A, lda, Qt, l, H, l);
    if ((rc = orc_qr_householder(m, l, H, l, Q, l, R, l)) != ORC_OK) goto done;
  }
  if ((rc = orc_gemm_tn(m, n, l, A, lda, Q, l, T, l)) != ORC_OK) goto done;  /* T = A^T Q */
  rc = orc_svd_exact(n, l, T, l, Vt, l, St, W, l);              /* T = V~ S~ W^T */
  if (rc < 0) goto done;
  /* U~ = Q W, first k columns */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < k; ++j) {
      double s = 0.0;
      for (int64_t r = 0; r < l; ++r) s += Q[i * l + r] * W[r * l + j];
      U[i * ldu + j] = s;
    }
  for (int64_t j = 0; j < k; ++j) S[j] = St[j];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < k; ++j) V[i * ldv + j] = Vt[i * l + j];
  orc_sign_convention(m, n, k, U, ldu, V, ldv);
  rc = orc_select_k(k, S, *fro2, t, K);
done:
  free(H); free(Q); free(T); free(Qt); free(R); free(Vt); free(St); free(W);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Krylov method (Sec. 3.1.1), the paper's steps in its order:
 *   1. G (n x l) given, l = min(k + p, n);   2. H(0) = A G;
 *   3. H(j) = A (A^T H(j-1)) for j = 1..i;
 *   4. H = [H(0) | ... | H(i)] (m x L, L = (i+1) l; requires L <= n);
 *   5. QR of H -> Q;   6. T = A^T Q (n x L);
 *   7. SVD T = V~ S~ W^T;   8. U~ = Q W, first k columns.
 * Reading: a block is replaced by an orthonormal basis of its own columns
 * (Householder QR) before it is stored in H and used for the next block, and
 * A^T H(j-1) likewise before the product with A; a block times an invertible
 * l x l matrix spans the same columns, so the Krylov space and Q's span are
 * the paper's.  K by the criterion of Sec. 2.4 over the first k values. */
int orc_krylov(int64_t m, int64_t n, const double* A, int64_t lda,
               const double* G, int64_t k, int64_t p, int64_t i, double t,
               double* U, int64_t ldu, double* S, double* V, int64_t ldv,
               int64_t* K, double* fro2) {
  if (m < n || n < 1 || k < 1 || k > n || p < 0 || i < 0 || !(t > 0.0 && t <= 1.0))
    return ORC_ERR_ARG;
  const int64_t l = (k + p < n) ? k + p : n;
  const int64_t L = (i + 1) * l;
  if (L > n) return ORC_ERR_ARG;
  double* B = (double*)malloc((size_t)(m * l) * sizeof(double));
  double* Qb = (double*)malloc((size_t)(m * l) * sizeof(double));
  double* Tl = (double*)malloc((size_t)(n * l) * sizeof(double));
  double* Qt = (double*)malloc((size_t)(n * l) * sizeof(double));
  double* Rl = (double*)malloc((size_t)(l * l) * sizeof(double));
  double* H = (double*)malloc((size_t)(m * L) * sizeof(double));
  double* Q = (double*)malloc((size_t)(m * L) * sizeof(double));
  double* R = (double*)malloc((size_t)(L * L) * sizeof(double));
  double* T = (double*)malloc((size_t)(n * L) * sizeof(double));
  double* Vt = (double*)malloc((size_t)(n * L) * sizeof(double));
  double* St = (double*)malloc((size_t)L * sizeof(double));
  double* W = (double*)malloc((size_t)(L * L) * sizeof(double));
  int rc = ORC_OK;
  if (!B || !Qb || !Tl || !Qt || !Rl || !H || !Q || !R || !T || !Vt || !St || !W) {
    rc = ORC_ERR_NOMEM;
    goto done;
  }
  *fro2 = orc_fro2(m, n, A, lda);                               /* Eq. sumeigen */
  orc_gemm_nn(m, n, l, A, lda, G, l, B, l);                    /* H(0) = A G */
  for (int64_t j = 0; j <= i; ++j) {
    if (j > 0) {                                                /* H(j) = A (A^T H(j-1)) */
      if ((rc = orc_gemm_tn(m, n, l, A, lda, Qb, l, Tl, l)) != ORC_OK) goto done;
      if ((rc = orc_qr_householder(n, l, Tl, l, Qt, l, Rl, l)) != ORC_OK) goto done;
      orc_gemm_nn(m, n, l, A, lda, Qt, l, B, l);
    }
    if ((rc = orc_qr_householder(m, l, B, l, Qb, l, Rl, l)) != ORC_OK) goto done;
    for (int64_t r = 0; r < m; ++r)                             /* block j of H */
      for (int64_t c = 0; c < l; ++c) H[r * L + j * l + c] = Qb[r * l + c];
  }
  if ((rc = orc_qr_householder(m, L, H, L, Q, L, R, L)) != ORC_OK) goto done;   /* QR of H */
  if ((rc = orc_gemm_tn(m, n, L, A, lda, Q, L, T, L)) != ORC_OK) goto done;    /* T = A^T Q */
  rc = orc_svd_exact(n, L, T, L, Vt, L, St, W, L);              /* T = V~ S~ W^T */
  if (rc < 0) goto done;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)                               /* U~ = Q W */
    for (int64_t c = 0; c < k; ++c) {
      double s = 0.0;
      for (int64_t e = 0; e < L; ++e) s += Q[r * L + e] * W[e * L + c];
      U[r * ldu + c] = s;
    }
  for (int64_t c = 0; c < k; ++c) S[c] = St[c];
  for (int64_t r = 0; r < n; ++r)
    for (int64_t c = 0; c < k; ++c) V[r * ldv + c] = Vt[r * L + c];
  orc_sign_convention(m, n, k, U, ldu, V, ldv);
  rc = orc_select_k(k, S, *fro2, t, K);
done:
  free(B); free(Qb); free(Tl); free(Qt); free(Rl); free(H); free(Q); free(R); free(T);
  free(Vt); free(St); free(W);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Truncated SVD through the n x n matrix A^T A (Sec. 2.3, Sec. 3.1.3):
 *   1. A^T A                      (Eq. AB: A^T A = V S^2 V^T)
 *   2. eigen-decomposition        lam_i, v_i   (orc_eig_sym_jacobi)
 *   3. s_i = sqrt(lam_i)          (Eq. LambdaSigma; a negative lam_i, which
 *                                  only rounding can produce, is taken as 0)
 *   4. u_i = A v_i / s_i          for i < ucols; a column whose s_i is not
 *                                  above max(m,n) * eps * s_1 is returned as
 *                                  zero (its direction is not determined)
 * S (n) and V (n x n) are always returned; U (m x ucols) only if ucols > 0.
 * K by the criterion of Sec. 2.4 over all n values, denominator ||A||_F^2. */
int orc_gram_eig(int64_t m, int64_t n, const double* A, int64_t lda, double t,
                 int64_t ucols, double* U, int64_t ldu, double* S,
                 double* V, int64_t ldv, int64_t* K, double* fro2) {
  if (m < n || n < 1 || ucols < 0 || ucols > n || !(t > 0.0 && t <= 1.0)) return ORC_ERR_ARG;
  double* Gm = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* lam = (double*)malloc((size_t)n * sizeof(double));
  int rc = ORC_OK;
  if (!Gm || !lam) { rc = ORC_ERR_NOMEM; goto done; }
  *fro2 = orc_fro2(m, n, A, lda);
  if ((rc = orc_gemm_tn(m, n, n, A, lda, A, lda, Gm, n)) != ORC_OK) goto done;
  rc = orc_eig_sym_jacobi(n, Gm, n, lam, V, ldv);
  if (rc < 0) goto done;
  for (int64_t i = 0; i < n; ++i) S[i] = lam[i] > 0.0 ? sqrt(lam[i]) : 0.0;
  orc_sign_convention(m, n, n, NULL, 0, V, ldv);
  if (ucols > 0) {
    const double floor_s = (double)(m > n ? m : n) * 2.220446049250313e-16 * S[0];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < ucols; ++j) {
        double s = 0.0;
        if (S[j] > floor_s) {
          for (int64_t r = 0; r < n; ++r) s += A[i * lda + r] * V[r * ldv + j];
          s /= S[j];
        }
        U[i * ldu + j] = s;
      }
  }
  rc = orc_select_k(n, S, *fro2, t, K);
done:
  free(Gm); free(lam);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Randomized PCA with the rank grown in blocks of b columns until the
 * criterion of Sec. 2.4 can be met: the blocked randomized range finder with
 * power steps of Martinsson & Voronin (SIAM J. Sci. Comput. 38(5), 2016,
 * randQB_b with power iterations), with B = Q^T A kept as T = B^T = A^T Q.
 *   for j = 0, 1, ... (block j of G: columns j b .. j b + b - 1):
 *     Y = A G_j - Q (T^T G_j)          the part of A G_j outside span(Q)
 *     Q_j = qr(Y)
 *     q times:  Z = qr(A^T Q_j);  Y = A Z - Q (T^T Z);  Q_j = qr(Y)
 *     Q_j = qr(Q_j - Q (Q^T Q_j))      re-orthogonalisation against Q
 *     T_j = A^T Q_j;  Q = [Q Q_j];  T = [T T_j];  L = L + b
 *     energy[j] = ||T||_F^2 = ||Q^T A||_F^2, the part of ||A||_F^2 (Eq.
 *     sumeigen) that span(Q) holds; stop when energy[j] >= t ||A||_F^2 or
 *     when another block would pass min(lmax, n) columns
 *   SVD T = V~ S~ W^T;  U~ = Q W;  K by Sec. 2.4 over all L values.
 * The first min(kcap, L) triplets are returned (sign rule applied); K is
 * capped at kcap, with ORC_WARN_THRESHOLD when capped or not reached.
 * Reading: Martinsson & Voronin also subtract B^T (Q^T Q_j) before the A^T
 * product of a power step; Q_j was projected off span(Q) just before, so
 * that term is rounding only, and the re-orthogonalisation that ends the
 * block restores Q_j's orthogonality to Q; it is left out. */
int orc_rsvd_blocked(int64_t m, int64_t n, const double* A, int64_t lda,
                     const double* G, int64_t ldg, int64_t b, int64_t q, double t,
                     int64_t lmax, int64_t kcap, double* U, int64_t ldu, double* S,
                     double* V, int64_t ldv, int64_t* K, int64_t* Lout, double* energy,
                     double* fro2) {
  const int64_t Lcap = (lmax < n) ? lmax : n;
  if (m < n || n < 1 || b < 1 || b > Lcap || q < 0 || kcap < 1 || kcap > n ||
      ldg < b || !(t > 0.0 && t <= 1.0))
    return ORC_ERR_ARG;
  double* Q = (double*)calloc((size_t)(m * Lcap), sizeof(double));
  double* T = (double*)calloc((size_t)(n * Lcap), sizeof(double));
  double* Y = (double*)malloc((size_t)(m * b) * sizeof(double));
  double* Qj = (double*)malloc((size_t)(m * b) * sizeof(double));
  double* Gj = (double*)malloc((size_t)(n * b) * sizeof(double));
  double* Z = (double*)malloc((size_t)(n * b) * sizeof(double));
  double* Zq = (double*)malloc((size_t)(n * b) * sizeof(double));
  double* C = (double*)malloc((size_t)(Lcap * b) * sizeof(double));
  double* Rb = (double*)malloc((size_t)(b * b) * sizeof(double));
  double* Tc = (double*)malloc((size_t)(n * Lcap) * sizeof(double));
  double* Vt = (double*)malloc((size_t)(n * Lcap) * sizeof(double));
  double* St = (double*)malloc((size_t)Lcap * sizeof(double));
  double* W = (double*)malloc((size_t)(Lcap * Lcap) * sizeof(double));
  int rc = ORC_OK;
  int64_t L = 0;
  if (!Q || !T || !Y || !Qj || !Gj || !Z || !Zq || !C || !Rb || !Tc || !Vt || !St || !W) {
    rc = ORC_ERR_NOMEM;
    goto done;
  }
  *fro2 = orc_fro2(m, n, A, lda);                               /* Eq. sumeigen */
  /* Y -= Q C (C = L x b) */
#define ORC_SUB_QC(Ymat)                                                      \
  do {                                                                        \
    _Pragma("omp parallel for schedule(static)")                              \
    for (int64_t r = 0; r < m; ++r)                                           \
      for (int64_t c = 0; c < b; ++c) {                                       \
        double s = 0.0;                                                       \
        for (int64_t e = 0; e < L; ++e) s += Q[r * Lcap + e] * C[e * b + c];  \
        (Ymat)[r * b + c] -= s;                                               \
      }                                                                       \
  } while (0)
  for (int64_t j = 0;; ++j) {
    for (int64_t r = 0; r < n; ++r)
      for (int64_t c = 0; c < b; ++c) Gj[r * b + c] = G[r * ldg + j * b + c];
    orc_gemm_nn(m, n, b, A, lda, Gj, b, Y, b);                 /* Y = A G_j */
    if (L > 0) {                                                /* - Q (T^T G_j) */
      if ((rc = orc_gemm_tn(n, L, b, T, Lcap, Gj, b, C, b)) != ORC_OK) goto done;
      ORC_SUB_QC(Y);
    }
    if ((rc = orc_qr_householder(m, b, Y, b, Qj, b, Rb, b)) != ORC_OK) goto done;
    for (int64_t it = 0; it < q; ++it) {
      if ((rc = orc_gemm_tn(m, n, b, A, lda, Qj, b, Z, b)) != ORC_OK) goto done;
      if ((rc = orc_qr_householder(n, b, Z, b, Zq, b, Rb, b)) != ORC_OK) goto done;
      orc_gemm_nn(m, n, b, A, lda, Zq, b, Y, b);               /* Y = A Z */
      if (L > 0) {                                              /* - Q (T^T Z) */
        if ((rc = orc_gemm_tn(n, L, b, T, Lcap, Zq, b, C, b)) != ORC_OK) goto done;
        ORC_SUB_QC(Y);
      }
      if ((rc = orc_qr_householder(m, b, Y, b, Qj, b, Rb, b)) != ORC_OK) goto done;
    }
    if (L > 0) {                                                /* Q_j - Q (Q^T Q_j) */
      if ((rc = orc_gemm_tn(m, L, b, Q, Lcap, Qj, b, C, b)) != ORC_OK) goto done;
      ORC_SUB_QC(Qj);
      memcpy(Y, Qj, (size_t)(m * b) * sizeof(double));
      if ((rc = orc_qr_householder(m, b, Y, b, Qj, b, Rb, b)) != ORC_OK) goto done;
    }
    if ((rc = orc_gemm_tn(m, n, b, A, lda, Qj, b, Z, b)) != ORC_OK) goto done;   /* T_j */
    for (int64_t r = 0; r < m; ++r)
      for (int64_t c = 0; c < b; ++c) Q[r * Lcap + L + c] = Qj[r * b + c];
    for (int64_t r = 0; r < n; ++r)
      for (int64_t c = 0; c < b; ++c) T[r * Lcap + L + c] = Z[r * b + c];
    L += b;
    double e2 = 0.0;                                            /* ||T||_F^2 */
    for (int64_t r = 0; r < n; ++r)
      for (int64_t c = 0; c < L; ++c) e2 += T[r * Lcap + c] * T[r * Lcap + c];
    energy[j] = e2;
    if (!(e2 < t * *fro2) || L + b > Lcap) break;
  }
#undef ORC_SUB_QC
  for (int64_t r = 0; r < n; ++r)
    for (int64_t c = 0; c < L; ++c) Tc[r * L + c] = T[r * Lcap + c];
  rc = orc_svd_exact(n, L, Tc, L, Vt, L, St, W, L);             /* T = V~ S~ W^T */
  if (rc < 0) goto done;
  {
    const int64_t kc = kcap < L ? kcap : L;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r)                             /* U~ = Q W */
      for (int64_t c = 0; c < kc; ++c) {
        double s = 0.0;
        for (int64_t e = 0; e < L; ++e) s += Q[r * Lcap + e] * W[e * L + c];
        U[r * ldu + c] = s;
      }
    for (int64_t c = 0; c < kc; ++c) S[c] = St[c];
    for (int64_t r = 0; r < n; ++r)
      for (int64_t c = 0; c < kc; ++c) V[r * ldv + c] = Vt[r * L + c];
    orc_sign_convention(m, n, kc, U, ldu, V, ldv);
    rc = orc_select_k(L, St, *fro2, t, K);
    if (rc >= 0 && *K > kcap) {
      *K = kcap;
      rc = ORC_WARN_THRESHOLD;
    }
  }
done:
  *Lout = L;
  free(Q); free(T); free(Y); free(Qj); free(Gj); free(Z); free(Zq); free(C); free(Rb);
  free(Tc); free(Vt); free(St); free(W);
  return rc;
}
