/* Host sanitizer driver for oracle/oracle.c (test infrastructure): calls
 * every exported routine on small seeded inputs, edge shapes and bad
 * arguments; built with -fsanitize=address,undefined by
 * tests/test_sanitizers.py, which fails on any report or a non-zero exit. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_num_threads(void);
void orc_gemm_nn(int64_t m, int64_t k, int64_t n, const double* A, int64_t lda, const double* B,
                 int64_t ldb, double* C, int64_t ldc);
int orc_gemm_tn(int64_t m, int64_t k, int64_t n, const double* A, int64_t lda, const double* B,
                int64_t ldb, double* C, int64_t ldc);
double orc_fro2(int64_t m, int64_t n, const double* A, int64_t lda);
int orc_qr_householder(int64_t m, int64_t n, const double* X, int64_t ldx, double* Q,
                       int64_t ldq, double* R, int64_t ldr);
int orc_svd_exact(int64_t m, int64_t n, const double* X, int64_t ldx, double* U, int64_t ldu,
                  double* S, double* V, int64_t ldv);
int orc_eig_sym_jacobi(int64_t n, const double* G, int64_t ldg, double* lam, double* V,
                       int64_t ldv);
int orc_select_k(int64_t k, const double* s, double fro2, double t, int64_t* K);
int orc_rsvd(int64_t m, int64_t n, const double* A, int64_t lda, const double* G, int64_t k,
             int64_t p, int64_t q, double t, double* U, int64_t ldu, double* S, double* V,
             int64_t ldv, int64_t* K, double* fro2);
int orc_krylov(int64_t m, int64_t n, const double* A, int64_t lda, const double* G, int64_t k,
               int64_t p, int64_t i, double t, double* U, int64_t ldu, double* S, double* V,
               int64_t ldv, int64_t* K, double* fro2);
int orc_gram_eig(int64_t m, int64_t n, const double* A, int64_t lda, double t, int64_t ucols,
                 double* U, int64_t ldu, double* S, double* V, int64_t ldv, int64_t* K,
                 double* fro2);

static uint64_t state = 88172645463325252ull;
static double urand(void) {   /* xorshift64: inputs only */
  state ^= state << 13; state ^= state >> 7; state ^= state << 17;
  return (double)(state >> 11) * 0x1p-53 - 0.5;
}
static double* filled(int64_t count) {
  double* p = (double*)malloc((size_t)count * sizeof(double));
  for (int64_t i = 0; i < count; ++i) p[i] = urand();
  return p;
}

static int fails = 0;
#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) { fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #cond); ++fails; } \
  } while (0)

static void solve_shapes(int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p, int64_t q) {
  const int64_t l = (k + p < n) ? k + p : n;
  double* A = filled(m * lda);
  double* G = filled(n * l);
  double* U = (double*)calloc((size_t)(m * k), sizeof(double));
  double* S = (double*)calloc((size_t)n, sizeof(double));
  double* V = (double*)calloc((size_t)(n * n), sizeof(double));
  double* Ug = (double*)calloc((size_t)(m * n), sizeof(double));
  int64_t K = -1;
  double f2 = 0.0;
  EXPECT(orc_rsvd(m, n, A, lda, G, k, p, q, 0.9, U, k, S, V, k, &K, &f2) >= 0);
  EXPECT(K >= 1 && K <= k && f2 > 0.0);
  if ((q + 1) * l <= n)
    EXPECT(orc_krylov(m, n, A, lda, G, k, p, q, 0.9, U, k, S, V, k, &K, &f2) >= 0);
  EXPECT(orc_gram_eig(m, n, A, lda, 0.9, n, Ug, n, S, V, n, &K, &f2) >= 0);
  EXPECT(orc_gram_eig(m, n, A, lda, 0.9, 0, NULL, 0, S, V, n, &K, &f2) >= 0);
  free(A); free(G); free(U); free(S); free(V); free(Ug);
}

int main(void) {
  EXPECT(orc_num_threads() >= 1);
  /* products, norms, QR, SVD, eigensolver on ragged shapes */
  {
    const int64_t m = 37, k = 11, n = 5;
    double *A = filled(m * (k + 3)), *B = filled(k * n), *C = filled(m * (n + 2));
    double *Bt = filled(m * n), *D = filled(k * n);
    orc_gemm_nn(m, k, n, A, k + 3, B, n, C, n + 2);
    EXPECT(orc_gemm_tn(m, k, n, A, k + 3, Bt, n, D, n) == 0);
    EXPECT(orc_fro2(m, k, A, k + 3) > 0.0);
    double *Q = filled(m * k), *R = filled(k * k);
    EXPECT(orc_qr_householder(m, k, A, k + 3, Q, k, R, k) == 0);
    double *Us = filled(m * k), *Ss = filled(k), *Vs = filled(k * k);
    EXPECT(orc_svd_exact(m, k, A, k + 3, Us, k, Ss, Vs, k) >= 0);
    double* Gm = filled(k * k);
    for (int64_t i = 0; i < k; ++i)
      for (int64_t j = 0; j < i; ++j) Gm[i * k + j] = Gm[j * k + i];
    double* lam = filled(k);
    EXPECT(orc_eig_sym_jacobi(k, Gm, k, lam, Vs, k) >= 0);
    int64_t K = -1;
    EXPECT(orc_select_k(k, Ss, orc_fro2(m, k, A, k + 3), 0.5, &K) >= 0 && K >= 1 && K <= k);
    free(A); free(B); free(C); free(Bt); free(D); free(Q); free(R); free(Us); free(Ss);
    free(Vs); free(Gm); free(lam);
  }
  /* whole solves: ragged m, padded lda, l clamped to n, p = 0, q = 0, square */
  solve_shapes(203, 17, 17, 5, 3, 2);
  solve_shapes(64, 20, 23, 8, 0, 0);
  solve_shapes(40, 12, 12, 10, 9, 1);
  solve_shapes(15, 15, 15, 1, 2, 3);
  /* zero matrix: K = 0 and the zero-matrix warning */
  {
    double* Z = (double*)calloc(50 * 6, sizeof(double));
    double *G = filled(6 * 4), *U = filled(50 * 3), *S = filled(6), *V = filled(36);
    int64_t K = -1;
    double f2 = 1.0;
    EXPECT(orc_rsvd(50, 6, Z, 6, G, 3, 1, 1, 0.9, U, 3, S, V, 3, &K, &f2) == 2 && K == 0);
    free(Z); free(G); free(U); free(S); free(V);
  }
  /* argument errors: nothing is read or written */
  {
    double x = 0.0;
    int64_t K = 0;
    EXPECT(orc_rsvd(5, 10, &x, 10, &x, 2, 1, 1, 0.9, &x, 2, &x, &x, 2, &K, &x) < 0);
    EXPECT(orc_rsvd(50, 10, &x, 10, &x, 11, 1, 1, 0.9, &x, 2, &x, &x, 2, &K, &x) < 0);
    EXPECT(orc_rsvd(50, 10, &x, 10, &x, 2, -1, 1, 0.9, &x, 2, &x, &x, 2, &K, &x) < 0);
    EXPECT(orc_rsvd(50, 10, &x, 10, &x, 2, 1, 1, 1.5, &x, 2, &x, &x, 2, &K, &x) < 0);
    EXPECT(orc_krylov(50, 10, &x, 10, &x, 4, 2, 1, 0.9, &x, 2, &x, &x, 2, &K, &x) < 0);
    EXPECT(orc_gram_eig(50, 10, &x, 10, 0.9, 11, &x, 2, &x, &x, 10, &K, &x) < 0);
    EXPECT(orc_select_k(3, &x, 1.0, 0.0, &K) < 0);
  }
  if (fails) fprintf(stderr, "%d checks failed\n", fails);
  else printf("oracle driver ok\n");
  return fails ? 1 : 0;
}
