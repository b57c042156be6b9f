// rsvd_internal.h -- shared declarations of the HIP kernels behind librsvd.so.
// Target: gfx950 (CDNA4), wave64.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rsvd.h"

namespace rsvd {

// Device memory through address-space-1 (global) pointers.  A pointer that
// reaches a kernel through an argument record is generic, and generic (flat)
// accesses may alias LDS: the compiler then orders them against the kernel's
// LDS accesses (a wait on both counters after each).  Only for pointers to
// device memory.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* to_global(T* p) {
  return (gmem<T>*)p;
}
template <typename T>
__device__ __forceinline__ const gmem<T>* to_global(const T* p) {
  return (const gmem<T>*)p;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// 16x16x4 matrix-core products.  For both, lane l supplies a = Aop[l%16][l/16]
// and b = Bop[l/16][l%16]; the 16x16 result is spread over the wave as four
// values per lane.  Row of value e held by lane l (column is always l%16):
//   fp32: 4*(l/16) + e        fp64: (l/16) + 4*e
template <typename C> struct Mfma;
template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};
template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};

// 32x32x2 fp32, the full-rate fp32 matrix-core shape on gfx950 (4096 flops
// in the issue time of 16x16x4's 2048 x 1.6): lane l supplies
// a = Aop[l%32][l/32], b = Bop[l/32][l%32]; value e of lane l is at row
// (e%4) + 8*(e/4) + 4*(l/32), column l%32.
typedef float f32x16 __attribute__((ext_vector_type(16)));
struct Mfma32f {
  typedef f32x16 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int e) {
    return (e & 3) + 8 * (e >> 2) + 4 * (lane >> 5);
  }
};

// ---------------------------------------------------------------------------
// Launchers (host functions; every one returns hipSuccess or the launch error).

// Y (m x c) = A (m x n) X (n x c), all row-major; T = float or double.
// fro2_part != nullptr: per-block partial sums of a_ij^2 (FP64), count
// returned through *nparts.
template <typename T>
hipError_t launch_gemm_nn(const T* A, int64_t m, int64_t n, int64_t lda, const T* X, int64_t ldx,
                          int c, T* Y, int64_t ldy, double* fro2_part, int* nparts,
                          hipStream_t s);

// Y (m x c) = A (m x n) Xt^T with Xt given transposed (c x n, row-major), for
// outputs wider than 128 columns (fp32; two-level tiled on 32x32x2).
hipError_t launch_gemm_nt_wide(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                               int64_t ldxt, int c, float* Y, int64_t ldy, hipStream_t s);

// Y (m x c) = A Xt^T for fp32 with c <= 192 (Xt is c x n), optional per-block
// FP64 partial sums of a_ij^2 (*nparts of them); requires nt_tall_applies.
bool nt_tall_applies(const float* A, int64_t n, int64_t lda, const float* Xt, int64_t ldxt, int c);
// Y (m x c) = A Xt^T for a lower-triangular Xt with exact zeros above its
// diagonal (the transposed inverse Cholesky factor of CholeskyQR): the
// products of its zero blocks are skipped.  Same requirements as
// launch_gemm_nt_tall.
hipError_t launch_gemm_nt_tri(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                              int64_t ldxt, int c, float* Y, int64_t ldy, hipStream_t s);
// Y (m x c) = A Xt^T on the narrow kernel (n <= 96, c <= 96) for a lower-
// triangular Xt (as launch_gemm_nt_tri) with the FP64 Gram matrix Y^T Y of
// the stored output as per-block c x c partials at gram_part (*nparts of
// them, at most max_parts), summed by launch_reduce_partials.
bool nt_narrow_gram_applies(const float* A, int64_t n, int64_t lda, const float* Xt, int64_t ldxt,
                            int c);
hipError_t launch_gemm_nt_narrow_gram(const float* A, int64_t m, int64_t n, int64_t lda,
                                      const float* Xt, int64_t ldxt, int c, float* Y, int64_t ldy,
                                      double* gram_part, int64_t max_parts, int* nparts,
                                      hipStream_t s);
hipError_t launch_gemm_nt_tall(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                               int64_t ldxt, int c, float* Y, int64_t ldy, double* fro2_part,
                               int* nparts, hipStream_t s);
// Partials P[s] (n x c, FP64) of A^T Q for fp32 with c <= 160 (16-byte rows);
// *nsplit returns their number.
bool tn_tall_applies(const float* A, int64_t lda, const float* Q, int64_t ldq, int c);
hipError_t launch_gemm_tn_tall(const float* A, int64_t m, int64_t n, int64_t lda, const float* Q,
                               int64_t ldq, int c, double* P, int64_t max_split, int* nsplit,
                               hipStream_t s);

// G (n x n, FP64, ld n) = A^T A for fp32 A with n > 128 (upper tile pairs,
// mirrored); P is scratch of p_cap doubles for the partial tiles.  ev0/ev1,
// when given, are recorded around the tile kernel (not the reduction).
hipError_t launch_syrk_f32(const float* A, int64_t m, int64_t n, int64_t lda, double* P,
                           int64_t p_cap, double* G, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
// Whether launch_syrk_f32 takes this operand (16-byte rows, n > 128).
bool syrk_f32_applies(const float* A, int64_t n, int64_t lda);

// Partials P[s] (n x c, FP64) of A^T Q over row splits; C = compute type of
// the matrix-core product (double gives an exact-product FP64 Gram for float
// data).  *nsplit returns the number of partial matrices written.
template <typename T, typename C>
hipError_t launch_gemm_tn_partial(const T* A, int64_t m, int64_t n, int64_t lda, const T* Q,
                                  int64_t ldq, int c, double* P, int64_t max_split, int* nsplit,
                                  hipStream_t s);

// Symmetric partial Gram matrices P[s] (c x c, FP64) of a tall m x c panel Y,
// one per row split, accumulated in FP64 from exact products (every wave of
// a split holds all upper tile pairs for c <= 96; above that, up to 192, the
// split's rows are staged in LDS and its waves share out the tile pairs).
template <typename T>
hipError_t launch_gram_f64(const T* Y, int64_t m, int c, int64_t ldy, double* P, int64_t max_split,
                           int* nsplit, hipStream_t s);

// W (c x c, FP64, ldw) = Y^T Y for a short panel (m <= kGramShortRows) in one
// launch: one workgroup per 16 x 16 tile pair, no partials.
constexpr int64_t kGramShortRows = 8192;
template <typename T>
hipError_t launch_gram_short(const T* Y, int64_t m, int c, int64_t ldy, double* W, int64_t ldw,
                             hipStream_t s);

// Z (rows x cols) = sum over s < nsplit of P[s] (each rows x cols), fixed order.
hipError_t launch_reduce_partials(const double* P, int nsplit, int64_t rows, int64_t cols,
                                  double* Z, int64_t ldz, hipStream_t s);
// out[0] = sum of parts[0..n) in order (single block).
hipError_t launch_reduce_scalar(const double* parts, int n, double* out, hipStream_t s);

// Largest number of row splits launch_gemm_tn_partial uses for (m, n, c).
int64_t tn_max_split(int64_t m, int64_t n, int c);

// ---- small FP64 kernels (small.hip) ----
hipError_t launch_gaussian_fill(uint64_t seed, int64_t rows, int64_t cols, double* G,
                                hipStream_t s);
// Casts between the FP64 staging copies and the working type (row-major);
// the _t variant writes dst (cols x rows, ld ldd) = src^T.
template <typename T>
hipError_t launch_cast_t_from_f64(const double* src, int64_t rows, int64_t cols, int64_t lds,
                                  T* dst, int64_t ldd, hipStream_t s);
template <typename T>
hipError_t launch_cast_from_f64(const double* src, int64_t rows, int64_t cols, int64_t lds,
                                T* dst, int64_t ldd, hipStream_t s);
template <typename T>
hipError_t launch_cast_to_f64(const T* src, int64_t rows, int64_t cols, int64_t lds,
                              double* dst, int64_t ldd, hipStream_t s);

// Cholesky of the symmetric c x c matrix W (ld = c, c <= chol_inv_max_c()):
// R upper with W = R^T R, Rinv = R^-1 (upper), both ld = c, each written
// only when not null.  Rinv also written, rounded, to RinvT
// (type T, ld = c) when RinvT != nullptr, transposed when trans != 0.
// Non-positive pivot -> status word = RSVD_ERR_BREAKDOWN, R = 0 and
// Rinv = identity (so later kernels stay finite).
template <typename T>
hipError_t launch_chol_inv(const double* W, int c, double* R, double* Rinv, T* RinvT,
                           int32_t* status, hipStream_t s, int trans = 0);
// Largest c launch_chol_inv takes (the grouped launcher: at most 96).
int chol_inv_max_c();

// C (r x c2) = A (r x c1) B (c1 x c2), FP64, all ld = their column counts.
// Optional rounded copy CT (type T): C itself (ld = c2), or C^T (ld = r)
// when trans != 0.
template <typename T>
hipError_t launch_small_gemm(const double* A, const double* B, int64_t r, int c1, int c2,
                             double* C, T* CT, hipStream_t s, int trans = 0);

// One-sided Jacobi SVD of a c x c FP64 matrix M (ld = c, c <= 96), in one
// workgroup, on M itself or (transpose != 0) on M^T =: N:  N J = Uo diag(S)
// with J orthogonal; writes Uo (c x c) and S (c), unsorted, and into J
// (c x c): J itself when acc_j != 0, else Uo diag(S)^-1 (zero columns where
// S = 0) from which the caller forms the columns of J it needs (N = R^T:
// J = R Uo diag(S)^-1, accurate for the leading values); sweeps used and the
// final off-diagonal measure to diag[2..3].  redo (device word, may be null):
// with acc_j = 0 it receives 1.0 when min S <= 1e-6 max S (J from Uo S^-1
// too inexact), else 0.0; with acc_j != 0 the launch does nothing unless
// *redo is nonzero (null: unconditional).
hipError_t launch_jacobi_svd_small(const double* M, int c, int transpose, double* Uo, double* S,
                                   double* J, int acc_j, double* diag, int32_t* status,
                                   double* redo, hipStream_t s);

// Eigen-decomposition of a symmetric n x n FP64 matrix by one-sided block
// Jacobi on its columns: on entry X = G and J = I (column j at X + j*n);
// X <- X R, J <- J R until the columns of X are orthogonal; then lambda_j =
// +-||x_j|| (sign of the Rayleigh quotient j_j^T x_j) and the eigenvectors
// are the columns of J (unsorted).  `flags` holds jacobi_eig_flag_words()
// int32 words and `scratch` jacobi_eig_scratch_doubles(n) doubles; sweeps
// used go to diag[2].  inner_sweeps < 0 selects the default; ev0/ev1, when
// given, are recorded around the solver kernel itself.
// svd != 0: the same iteration as a one-sided Jacobi SVD of any square X
// (X J = Uo diag(lam) with lam_j = ||x_j||, unsigned): pairs are rotated on
// the cosine test alone (no absolute floor, so small singular values keep
// their relative accuracy).
hipError_t launch_jacobi_eig(double* X, double* J, int64_t n, double* lam, double* diag,
                             int32_t* flags, double* scratch, int32_t* status, hipStream_t s,
                             int inner_sweeps = -1, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr, int svd = 0);
// Doubles of scratch launch_jacobi_eig needs for matrices up to n.
int64_t jacobi_eig_scratch_doubles(int64_t n);

// Sort (descending by key), apply the sign rule, and scatter the first kout
// singular triplets: S_out[i] = key-sorted S, Vout (r x kout, type T, ldv)
// and/or Vd_out (r x kout, FP64) from the columns of Vsrc (r x c, FP64),
// Wout (c x kout, FP64) from the columns of Wsrc (c x c, row-major), the
// vector pair flipped together.
// Element i of source column col is Vsrc[i * vrs + col * vcs].
template <typename T>
hipError_t launch_sort_sign_scatter(const double* S, int c, const double* Vsrc, int64_t r,
                                    int64_t vrs, int64_t vcs, const double* Wsrc, int kout,
                                    double* S_out, T* Vout, int64_t ldv, double* Vd_out,
                                    double* Wout, hipStream_t s);

// K by the explained-variance criterion over S[0..k), denominator *fro2;
// writes *K (device int32), diag[0] = fro2, diag[1] = captured fraction,
// diag[4] = K, and RSVD_WARN_* / RSVD_ERR_NONFINITE into *status.
hipError_t launch_select_k(const double* S, int k, const double* fro2, double t, int32_t* K,
                           double* diag, int32_t* status, hipStream_t s);

// Scale the columns of V (n x cols, FP64) by 1/S[j] into X (type T), with a
// zero column when S[j] <= floor_rel * S[0]; trans != 0 stores X^T (cols x n).
template <typename T>
hipError_t launch_scale_cols_inv(const double* V, int64_t n, int cols, int64_t ldv,
                                 const double* S, double floor_rel, T* X, int64_t ldx, int trans,
                                 hipStream_t s);
// Xt (cols x rows) = X^T for a row-major fp32 X.
hipError_t launch_transpose_f32(const float* X, int64_t rows, int64_t cols, int64_t ldx, float* Xt,
                                int64_t ldxt, hipStream_t s);

// ---- bfloat16 storage of A (lowp.hip) ----
// Aq (m x n, ldq) = bf16(A / s), s (n) = power-of-two column scales from the
// column maxima (cmax: n words of workspace).
hipError_t launch_quantize_bf16(const float* A, int64_t m, int64_t n, int64_t lda, __bf16* Aq,
                                int64_t ldq, float* scale, unsigned* cmax, hipStream_t s);
// Xhi + Xlo (c x n, ld ldx) = (diag(scale) X)^T split into bf16 pairs; X is
// n x c FP64 row-major (ld c); scale may be null (ones).
hipError_t launch_cast_hilo_t(const double* X, int64_t n, int c, const float* scale, __bf16* Xhi,
                              __bf16* Xlo, int64_t ldx, hipStream_t s);
// Z (n x c, ld c) rows times scale (no-op for a null scale).
hipError_t launch_scale_rows(double* Z, int64_t n, int c, const float* scale, hipStream_t s);
// FP8 E4M3 storage: Aq (m x n, ldq, one byte each) = E4M3(A / s), s the least
// powers of two with max |A_j| / s_j <= 448.
hipError_t launch_quantize_fp8(const float* A, int64_t m, int64_t n, int64_t lda, void* Aq,
                               int64_t ldq, float* scale, unsigned* cmax, hipStream_t s);
// Whether the low-precision passes take A of es bytes per element (2:
// bfloat16, 1: FP8 E4M3): n % 8 == 0, lda % 8 == 0, rows aligned to 8 es
// bytes, c <= 192.
bool bf16_pass_applies(const void* A, int es, int64_t n, int64_t lda, int c);
// Y (m x c, fp32) = Aq (Xhi + Xlo)^T on the bf16 matrix cores (FP8 widened to
// bf16 in registers); per-block FP64 sums of the squared dequantised entries
// into fro2_part (count in *nparts) when non-null.
hipError_t launch_gemm_nt_bf16(const void* A, int es, int64_t m, int64_t n, int64_t lda,
                               const __bf16* Xhi, const __bf16* Xlo, int64_t ldx, int c,
                               const float* scale, float* Y, int64_t ldy, double* fro2_part,
                               int* nparts, hipStream_t s);
// FP64 partials (nsplit x n x c) of Aq^T Q (unscaled), Q fp32 with ldq % 8 == 0
// and round_up(c, 8) readable columns per row.
hipError_t launch_gemm_tn_bf16(const void* A, int es, int64_t m, int64_t n, int64_t lda,
                               const float* Q, int64_t ldq, int c, double* P, int64_t max_split,
                               int* nsplit, hipStream_t s);

// A32 (m x n, ld lda32, fp32) = Aq diag(scale) for A stored in bfloat16
// (es = 2) or FP8 E4M3 (es = 1); scale may be null (ones).
hipError_t launch_dequantize(const void* Aq, int es, int64_t m, int64_t n, int64_t lda,
                             const float* scale, float* A32, int64_t lda32, hipStream_t s);

// Shifted CholeskyQR's diagonal shift on the c x c Gram W of an m x c matrix:
// W += 11 (m c + c (c+1)) 2^-53 trace(W) I (one block).
hipError_t launch_shift_diag(double* W, int c, int64_t m, hipStream_t s);
// S[i] = sqrt(max(lam[i], 0)).
hipError_t launch_sqrt_clamp(const double* lam, int n, double* S, hipStream_t s);
// p[0..n) = v (a kernel, so the fill can be captured in a graph).
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s);
// Number of int32 words launch_jacobi_eig needs in `flags`.
int jacobi_eig_flag_words();
// Largest n the Jacobi eigensolver supports (every workgroup resident).
int64_t jacobi_eig_max_n();


// ---------------------------------------------------------------------------
// Grouped launches: one launch runs one kernel for many problems.  Each
// kernel below takes, as its last argument, an optional array of per-problem
// arguments (nullptr for an ordinary launch); in a grouped launch blockIdx.y
// selects the problem, whose arguments replace the kernel's own, and blocks
// with blockIdx.x >= nblk (that problem's own grid) leave at once, so every
// problem runs exactly the blocks an ordinary launch would give it.
//
// The passes over tall matrices (the A X and Y R^-1 products, A^T Q) take a
// work list instead: a 1-D grid with one block per item {problem, item},
// ordered on the host (largest problems first).  For the two NT products an
// item is a row panel of `tpp` 128-row tiles that the block walks one tile
// after the other, writing one FP64 partial per panel: the sum of squares
// of A (fro2 != nullptr) and, with gram != nullptr, the Gram matrix Y^T Y of
// the panel's output rows, taken on the FP64 matrix cores straight from the
// FP32 accumulator registers (c x c, symmetric, at gram + item c^2).  For
// A^T Q an item is one block of the problem's ordinary grid.
struct GWork {
  int32_t inst, item;
};
struct GArgTall {   // k_gemm_nt_tall
  const float* A; int64_t m, n, lda; const float* Xt; int64_t ldxt; int c;
  float* Y; int64_t ldy; double* fro2; double* gram; int tpp;
};
struct GArgNarrow {   // k_gemm_nt_narrow
  const float* A; int64_t m, n, lda; const float* Xt; int64_t ldxt; int c;
  float* Y; int64_t ldy; double* gram; int tpp;
};
struct GArgTn {   // k_gemm_tn_tall, k_gemm_tn_narrow
  const float* A; int64_t m, n, lda; const float* Q; int64_t ldq; int c; int64_t rps;
  int ntile; double* P;
};
struct GArgGram {   // k_gram_f64
  const void* Y; int64_t m; int c; int64_t ldy; double* P; int64_t rpb; int nblk;
};
struct GArgRed {   // k_reduce_partials
  const double* P; int nsplit; int64_t rows, cols; double* Z; int64_t ldz; int nblk;
};
struct GArgRedS {   // k_reduce_scalar
  const double* parts; int n; double* out; int nblk;
};
struct GArgNn {   // k_gemm_nn
  const void* A; int64_t m, n, lda; const void* X; int64_t ldx; int c; void* Y; int64_t ldy;
  double* fro2; int ncol_tiles; int nblk;
};
struct GArgFill {   // k_gaussian_fill
  uint64_t seed; int64_t total; double* G; int nblk;
};
struct GArgCast {   // k_cast_t
  const double* src; int64_t rows, cols, lds; void* dst; int64_t ldd; int nblk;
};
struct GArgChol {   // k_chol_inv
  const double* W; int c; double* R; double* Rinv; void* RinvT; int trans; int32_t* status;
  int nblk;
};
struct GArgSg {   // k_small_gemm
  const double* A; const double* B; int64_t r; int c1, c2; double* C; void* CT; int trans;
  int nblk;
};
struct GArgJac {   // k_jacobi_svd_small
  const double* M; int c; int transpose; double* Uo; double* S; double* J; double* diag;
  int32_t* status; double* redo; int nblk;
};
struct GArgSort {   // k_sort_sign_scatter
  const double* S; int c; const double* Vsrc; int64_t r, vrs, vcs; const double* Wsrc; int kout;
  double* S_out; void* Vout; int64_t ldv; double* Vd_out; double* Wout; int nblk;
};
struct GArgSel {   // k_select_k
  const double* S; int k; const double* fro2; double t; int32_t* K; double* diag;
  int32_t* status; int nblk;
};
struct GArgStat {   // k_reset (src = nullptr: status = RSVD_OK, diag zeroed) and k_status_take
  const int32_t* src; int32_t* dst; double* diag; int nd; int nblk;
};

// Launch geometry shared by the ordinary and the grouped launchers.
// Row splits of the Gram and A^T Q partial sums: min_rows is the shortest
// split (the defaults suit a solve alone on the GPU; grouped batches take
// kGroupedSplitRows).
constexpr int64_t kGroupedSplitRows = 1024;
int64_t gram_blocks(int64_t m, int64_t max_split, int64_t* rows_per_block, int64_t min_rows = 256);
int64_t tn_tall_splits(int64_t m, int64_t n, int64_t max_split, int64_t* rows_per_split,
                       int* ntile, int64_t min_rows = 16);
int tn_col_waves(int64_t n);
int64_t narrow_blocks(int64_t m);
int64_t tall_blocks(int64_t m);
int nn_col_tiles(int c, int nt);
int64_t nn_row_blocks(int64_t m);

// Grouped launchers: `a` is a device array of `count` argument records,
// `maxblk` the largest nblk among them; the template choices (column tiles
// nt, k slabs ns, element type) are the same for every problem of a launch.
// The three work-list launchers take the item list `wl` (nwork items) and
// the records it indexes; gram selects the fused-Gram kernels (nt <= 4);
// tri: every Xt of the launch is lower triangular with exact zeros (an
// inverse Cholesky factor), and the products of its zero blocks are skipped.
constexpr int kGramFuseMaxNt = 4;
hipError_t launch_gemm_nt_tall_grouped(const GArgTall* a, const GWork* wl, int nwork, int nt,
                                       bool gram, hipStream_t s);
hipError_t launch_gemm_nt_narrow_grouped(const GArgNarrow* a, const GWork* wl, int nwork, int nt,
                                         int ns, bool gram, bool tri, hipStream_t s);
hipError_t launch_gemm_tn_tall_grouped(const GArgTn* a, const GWork* wl, int nwork, int nt,
                                       int cw, hipStream_t s);
template <typename T>
hipError_t launch_gram_f64_grouped(const GArgGram* a, int count, int maxblk, int nt, int cmax,
                                   hipStream_t s);
hipError_t launch_reduce_partials_grouped(const GArgRed* a, int count, int maxblk, hipStream_t s);
hipError_t launch_reduce_scalar_grouped(const GArgRedS* a, int count, hipStream_t s);
hipError_t launch_gemm_nn_f64_grouped(const GArgNn* a, int count, int maxblk, int nt,
                                      hipStream_t s);
hipError_t launch_gaussian_fill_grouped(const GArgFill* a, int count, int maxblk, hipStream_t s);
template <typename T>
hipError_t launch_cast_t_from_f64_grouped(const GArgCast* a, int count, int maxblk,
                                          hipStream_t s);
template <typename T>
hipError_t launch_chol_inv_grouped(const GArgChol* a, int count, int cmax, hipStream_t s);
template <typename T>
hipError_t launch_small_gemm_grouped(const GArgSg* a, int count, int maxblk, hipStream_t s);
hipError_t launch_jacobi_svd_small_grouped(const GArgJac* a, int count, int cmax, int acc_j,
                                           hipStream_t s);
template <typename T>
hipError_t launch_sort_sign_scatter_grouped(const GArgSort* a, int count, int maxblk, int cmax,
                                            hipStream_t s);
hipError_t launch_select_k_grouped(const GArgSel* a, int count, int kmax, hipStream_t s);

}  // namespace rsvd
