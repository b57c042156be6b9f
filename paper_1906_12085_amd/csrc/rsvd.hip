// rsvd.hip -- the C ABI of librsvd.so (declared in include/rsvd.h): plans,
// argument validation and the stream-ordered sequence of kernels for
// Randomized PCA (paper Sec. 3.1.2) and the truncated SVD through A^T A
// (Sec. 2.3 / 3.1.3).  No host synchronisation happens inside a solve.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <functional>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "rsvd_internal.h"

using namespace rsvd;

namespace {

// Largest sketch width l supported: the l x l Cholesky factor and its
// inverse share one workgroup's registers (192 columns at most).  Up to
// kSmallSvdMaxC columns the small SVD runs in one workgroup's LDS; wider
// factors go to the cooperative block-Jacobi solver, which is kept out of
// grouped batches and of captured batch graphs (both take l <= kSmallSvdMaxC).
constexpr int kMaxL = 192;
constexpr int kSmallSvdMaxC = 96;
// Dimension limits checked before any size arithmetic: with m <= 2^40 rows
// and n <= 2^20 columns every workspace size below stays far inside int64_t.
constexpr int64_t kMaxRows = (int64_t)1 << 40;
constexpr int64_t kMaxCols = (int64_t)1 << 20;
constexpr int kDiagWords = 8;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Per-kernel launch timing (off unless enabled by rsvd_plan_kernel_times):
// HIP event pairs recorded on the plan's stream around one kind of kernel.
enum KernelKind { KT_EIG = 0, KT_PASS_NN, KT_PASS_TN, KT_SYRK, KT_NT_WIDE, KT_COUNT };
constexpr int kTimerPairs = 256;
struct KernelTimer {
  hipEvent_t ev[kTimerPairs][2] = {};
  int used = 0;
};

struct rsvd_plan_s {
  bool timing = false;
  KernelTimer* kt = nullptr;   // KT_COUNT timers, allocated when timing is first enabled
  int device = 0;
  int dtype = RSVD_F64;
  int64_t m_max = 0, n_max = 0;
  int l_max = 0;
  bool gram = false;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  int64_t max_split = 1;

  char* base = nullptr;   // one device allocation, carved below
  size_t bytes = 0;

  // rSVD workspace
  double* omega = nullptr;   // n x l   FP64 sketch
  void* Xs = nullptr;        // n x cmax (T) right operand of A X
  void* Y = nullptr;         // m x l (T) sketch / power-iteration iterate
  void* Q1 = nullptr;        // m x l (T) first CholeskyQR factor (Q = Q1 R2^-1)
  double* part = nullptr;    // split-m partials
  double* fro2_part = nullptr;
  double* scal = nullptr;    // [0] = ||A||_F^2
  double *Wg = nullptr, *R1 = nullptr, *R1inv = nullptr, *R2 = nullptr, *R2inv = nullptr;
  void* RinvT = nullptr;     // l x l (T)
  double *R1s = nullptr, *R1invs = nullptr, *R2s = nullptr, *R2invs = nullptr;
  void* RinvTs = nullptr;    // l x l (T) of the FP64 n x l orthonormalisations
  double *Zd = nullptr, *Z2 = nullptr, *Z1 = nullptr, *Zq = nullptr;   // n x l
  double *Rt = nullptr, *Uo = nullptr, *Jm = nullptr, *Su = nullptr, *Vt = nullptr;
  double *Wk = nullptr, *Mk = nullptr;
  void* MkT = nullptr;       // l x l (T)
  double* EsS = nullptr;     // block-Jacobi scratch of the small SVD (l > kSmallSvdMaxC)
  double* Tp = nullptr;      // n x l_max (ld l_max) A^T Q of a basis grown in blocks
  int32_t* status = nullptr;
  double* diag = nullptr;
  int32_t* flags = nullptr;
  // A^T A route
  double *Gd = nullptr, *Xe = nullptr, *Je = nullptr, *Es = nullptr, *lam = nullptr, *Se = nullptr,
         *Vd = nullptr;
};

namespace {

#define RSVD_CHECK(expr)                                   \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return RSVD_ERR_DEVICE;          \
  } while (0)

// Working type of Y, Q, U, V: double for RSVD_F64, float otherwise (a BF16
// plan stores only A in bfloat16).
size_t elem_size(int dtype) { return dtype == RSVD_F64 ? sizeof(double) : sizeof(float); }
// Row stride of Q1: l rounded up to 8 (the bf16 projection reads whole
// 16-byte groups of Q's rows).
int64_t ldq1_of(int64_t l) { return (l + 7) / 8 * 8; }

// Carve the workspace; with base == nullptr it only counts bytes.
// The next event pair of timer `kind` (both null when timing is off or the
// pairs are used up).  The launcher records e0 on the plan's stream right
// before the timed kernel and e1 right after it.
struct KtPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
};
KtPair kt_reserve(rsvd_plan_s* p, int kind) {
  KtPair r;
  if (!p->timing || !p->kt) return r;
  KernelTimer& t = p->kt[kind];
  if (t.used >= kTimerPairs) return r;
  hipEvent_t* pr = t.ev[t.used];
  if (!pr[0] && (hipEventCreate(&pr[0]) != hipSuccess || hipEventCreate(&pr[1]) != hipSuccess))
    return r;
  ++t.used;
  r.e0 = pr[0];
  r.e1 = pr[1];
  return r;
}
// Times one single-kernel launch: records e0 now and e1 when it goes out of scope.
struct KtScope {
  hipStream_t s;
  KtPair pr;
  KtScope(rsvd_plan_s* p, int kind) : s(p->stream), pr(kt_reserve(p, kind)) {
    if (pr.e0) (void)hipEventRecord(pr.e0, s);
  }
  ~KtScope() {
    if (pr.e1) (void)hipEventRecord(pr.e1, s);
  }
};

int64_t p_cmax(const rsvd_plan_s* p) {
  return p->gram ? (p->n_max > p->l_max ? p->n_max : p->l_max) : p->l_max;
}

size_t carve(rsvd_plan_s* p, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* ptr = base ? base + off : nullptr;
    off += align_up(bytes > 0 ? bytes : 1);
    return ptr;
  };
  const size_t es = elem_size(p->dtype);
  const int64_t n = p->n_max, m = p->m_max, l = p->l_max;
  const int64_t cmax = p->gram ? (n > l ? n : l) : l;
  p->omega = (double*)take(n * l * 8);
  p->Xs = take(n * cmax * es);
  p->Y = take(m * l * es);
  p->Q1 = take(m * ldq1_of(l) * es);
  p->part = (double*)take(p->max_split * n * cmax * 8);
  p->fro2_part = (double*)take(((m + 127) / 128 + 1) * 8);
  p->scal = (double*)take(64);
  p->Wg = (double*)take(l * l * 8);
  p->R1 = (double*)take(l * l * 8);
  p->R1inv = (double*)take(l * l * 8);
  p->R2 = (double*)take(l * l * 8);
  p->R2inv = (double*)take(l * l * 8);
  p->RinvT = take(l * l * es);
  p->R1s = (double*)take(l * l * 8);
  p->R1invs = (double*)take(l * l * 8);
  p->R2s = (double*)take(l * l * 8);
  p->R2invs = (double*)take(l * l * 8);
  p->RinvTs = take(l * l * 8);
  p->Zd = (double*)take(n * l * 8);
  p->Z2 = (double*)take(n * l * 8);
  p->Z1 = (double*)take(n * l * 8);
  p->Zq = (double*)take(n * l * 8);
  p->Rt = (double*)take(l * l * 8);
  p->Uo = (double*)take(l * l * 8);
  p->Jm = (double*)take(l * l * 8);
  p->Su = (double*)take(l * 8);
  p->Vt = (double*)take(n * l * 8);
  p->Wk = (double*)take(l * l * 8);
  p->Mk = (double*)take(l * l * 8);
  p->MkT = take(l * l * es);
  if (l > kSmallSvdMaxC) p->EsS = (double*)take(jacobi_eig_scratch_doubles(l) * 8);
  p->Tp = (double*)take(n * l * 8);
  p->status = (int32_t*)take(64);
  p->diag = (double*)take(kDiagWords * 8);
  p->flags = (int32_t*)take(jacobi_eig_flag_words() * 4);
  if (p->gram) {
    p->Gd = (double*)take(n * n * 8);
    p->Xe = (double*)take(n * n * 8);
    p->Je = (double*)take(n * n * 8);
    p->lam = (double*)take(n * 8);
    p->Se = (double*)take(n * 8);
    p->Vd = (double*)take(n * n * 8);
    p->Es = (double*)take(jacobi_eig_scratch_doubles(n) * 8);
  }
  return off;
}

__global__ void k_reset(int32_t* status, double* diag, int nd) {
  if (threadIdx.x == 0) *status = RSVD_OK;
  if ((int)threadIdx.x < nd) diag[threadIdx.x] = 0.0;
}

__global__ void k_trace(const double* G, int64_t n, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += G[i * n + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// J = I (c x c).
__global__ void k_eye(double* J, int c) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c * c) return;
  J[idx] = (idx / c == idx % c) ? 1.0 : 0.0;
}

// From the block-Jacobi SVD of N (c x c; X = N J with orthogonal columns,
// column j at X + j c, and J column-major likewise): Uo (row-major) = the
// columns of X over S_j (a zero column where S_j = 0), Jm = J row-major.
__global__ void k_svd_finish(const double* __restrict__ X, const double* __restrict__ J,
                             const double* __restrict__ S, int c, double* __restrict__ Uo,
                             double* __restrict__ Jm) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c * c) return;
  const int i = idx / c, j = idx - i * c;
  const double s = S[j];
  Uo[idx] = s > 0.0 ? X[j * c + i] / s : 0.0;
  Jm[idx] = J[j * c + i];
}

// X = G (a symmetric matrix is its own column-major copy), J = I.
__global__ void k_init_eig(const double* G, int64_t n, double* X, double* J) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  X[idx] = 0.5 * (G[i * n + j] + G[j * n + i]);
  J[idx] = (i == j) ? 1.0 : 0.0;
}

hipError_t reset(rsvd_plan_s* p) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, p->stream, p->status, p->diag, kDiagWords);
  return hipGetLastError();
}

// A stored in bfloat16 (es = 2) or FP8 E4M3 (es = 1) with FP32 column
// scales (null: ones).
struct LowpA {
  const void* A;
  const float* scale;
  int es;
};
// Bytes per stored element of A for a low-precision plan (0 otherwise).
int lowp_es(int dtype) { return dtype == RSVD_BF16 ? 2 : (dtype == RSVD_FP8 ? 1 : 0); }

template <typename T>
struct Path {
  rsvd_plan_s* p;
  hipStream_t s;
  explicit Path(rsvd_plan_s* plan) : p(plan), s(plan->stream) {}

  // Z (n x c, FP64) = A^T Q for bfloat16 A: Aq^T Q on the bf16 matrix cores
  // (Q split into hi + lo), then the rows times the column scales.
  hipError_t tn_bf16(const LowpA& lp, int64_t m, int64_t n, int64_t lda, const float* Q,
                     int64_t ldq, int c, double* Z) {
    int ns = 0;
    hipError_t e;
    {
      KtScope ts(p, KT_PASS_TN);
      e = launch_gemm_tn_bf16(lp.A, lp.es, m, n, lda, Q, ldq, c, p->part, p->max_split, &ns, s);
    }
    if (e != hipSuccess) return e;
    if ((e = launch_reduce_partials(p->part, ns, n, c, Z, c, s)) != hipSuccess) return e;
    return launch_scale_rows(Z, n, c, lp.scale, s);
  }

  // Wout (c x c) = Y^T Y with exact FP64 products, fixed-order reduction.
  hipError_t gram(const T* Y, int64_t m, int c, int64_t ldy, double* Wout) {
    if (m <= kGramShortRows) return launch_gram_short<T>(Y, m, c, ldy, Wout, c, s);
    int ns = 0;
    hipError_t e = launch_gram_f64<T>(Y, m, c, ldy, p->part, p->max_split, &ns, s);
    if (e != hipSuccess) return e;
    return launch_reduce_partials(p->part, ns, c, c, Wout, c, s);
  }

  // Z (n x c, FP64) = A^T Q.
  hipError_t tn(const T* A, int64_t m, int64_t n, int64_t lda, const T* Q, int64_t ldq, int c,
                double* Z) {
    int ns = 0;
    hipError_t e;
    if (std::is_same<T, float>::value &&
        tn_tall_applies(reinterpret_cast<const float*>(A), lda, reinterpret_cast<const float*>(Q),
                        ldq, c))
    {
      KtScope ts(p, KT_PASS_TN);
      e = launch_gemm_tn_tall(reinterpret_cast<const float*>(A), m, n, lda,
                              reinterpret_cast<const float*>(Q), ldq, c, p->part, p->max_split,
                              &ns, s);
    }
    else
      e = launch_gemm_tn_partial<T, T>(A, m, n, lda, Q, ldq, c, p->part, p->max_split, &ns, s);
    if (e != hipSuccess) return e;
    return launch_reduce_partials(p->part, ns, n, c, Z, c, s);
  }

  // Y Rinv (m x c, type T) with Rinv held in RinvT (c x c; an inverse
  // Cholesky factor, upper triangular with exact zeros below its diagonal);
  // fp32 with a narrow right factor takes it transposed (row j = column j of
  // Rinv) and skips the products of its zero blocks.
  static bool times_rinv_tall(const T* Y, int c, int64_t ldy, const T* RinvT) {
    return std::is_same<T, float>::value &&
           nt_tall_applies(reinterpret_cast<const float*>(Y), c, ldy,
                           reinterpret_cast<const float*>(RinvT), c, c);
  }
  hipError_t times_rinv(const T* Y, int64_t m, int c, int64_t ldy, const T* RinvT, bool tall,
                        T* Out, int64_t ldo) {
    if (tall)
      return launch_gemm_nt_tri(reinterpret_cast<const float*>(Y), m, c, ldy,
                                reinterpret_cast<const float*>(RinvT), c, c,
                                reinterpret_cast<float*>(Out), ldo, s);
    if (std::is_same<T, double>::value && m <= kGramShortRows && ldy == c && ldo == c)
      return launch_small_gemm<double>(reinterpret_cast<const double*>(Y),
                                       reinterpret_cast<const double*>(RinvT), m, c, c,
                                       reinterpret_cast<double*>(Out), nullptr, s, 0);
    return launch_gemm_nn<T>(Y, m, c, ldy, RinvT, c, c, Out, ldo, nullptr, nullptr, s);
  }

  // CholeskyQR2 of Y (m x c): Q1 = Y R1^-1 (type T), R2 = chol(Q1^T Q1); the
  // orthonormal basis is Q = Q1 R2^-1 (kept implicit: R2inv).  R1^-1 passes
  // through RinvT; R2^-1 is written there as well when trans2 >= 0, in the
  // layout times_rinv takes for trans2 = 1.
  hipError_t cqr2(const T* Y, int64_t m, int c, int64_t ldy, T* Q1, int64_t ldq, double* R1,
                  double* R1inv, double* R2, double* R2inv, T* RinvT, int trans2 = -1) {
    hipError_t e;
    const bool tall = times_rinv_tall(Y, c, ldy, RinvT);
    if ((e = gram(Y, m, c, ldy, p->Wg)) != hipSuccess) return e;
    if ((e = launch_chol_inv<T>(p->Wg, c, R1, R1inv, RinvT, p->status, s, tall)) != hipSuccess)
      return e;
    if (tall && nt_narrow_gram_applies(reinterpret_cast<const float*>(Y), c, ldy,
                                       reinterpret_cast<const float*>(RinvT), c, c)) {
      // Q1 = Y R1^-1 with Q1^T Q1 summed from the product's accumulators
      int np = 0;
      const int64_t cap = p->max_split * p->n_max * p_cmax(p) / ((int64_t)c * c);
      if ((e = launch_gemm_nt_narrow_gram(reinterpret_cast<const float*>(Y), m, c, ldy,
                                          reinterpret_cast<const float*>(RinvT), c, c,
                                          reinterpret_cast<float*>(Q1), ldq, p->part, cap, &np,
                                          s)) != hipSuccess)
        return e;
      if ((e = launch_reduce_partials(p->part, np, c, c, p->Wg, c, s)) != hipSuccess) return e;
    } else {
      if ((e = times_rinv(Y, m, c, ldy, RinvT, tall, Q1, ldq)) != hipSuccess) return e;
      if ((e = gram(Q1, m, c, ldq, p->Wg)) != hipSuccess) return e;
    }
    return launch_chol_inv<T>(p->Wg, c, R2, R2inv, trans2 >= 0 ? RinvT : nullptr, p->status, s,
                              trans2 > 0);
  }

  // Shifted CholeskyQR (Fukaya et al., SIAM J. Sci. Comput. 2020): Q0 = Y R0^-1
  // with R0 = chol(Y^T Y + shift I); it brings a matrix whose condition number
  // is up to about 2^53 within CholeskyQR2's reach (followed by cqr2 of Q0).
  hipError_t cqr_shifted(const T* Y, int64_t m, int c, int64_t ldy, T* Q0, int64_t ldq,
                         double* R0, double* R0inv, T* RinvT) {
    hipError_t e;
    const bool tall = times_rinv_tall(Y, c, ldy, RinvT);
    if ((e = gram(Y, m, c, ldy, p->Wg)) != hipSuccess) return e;
    if ((e = launch_shift_diag(p->Wg, c, m, s)) != hipSuccess) return e;
    if ((e = launch_chol_inv<T>(p->Wg, c, R0, R0inv, RinvT, p->status, s, tall)) != hipSuccess)
      return e;
    return times_rinv(Y, m, c, ldy, RinvT, tall, Q0, ldq);
  }
};

// Orthonormalise an FP64 n x c matrix Zin: Zout = Q (explicit), and with
// keep_r R2s R1s = R (otherwise the factors are not stored).
hipError_t cqr2_small(rsvd_plan_s* p, const double* Zin, int64_t n, int c, double* Zout,
                      bool keep_r = false) {
  Path<double> d(p);
  hipError_t e = d.cqr2(Zin, n, c, c, p->Z1, c, keep_r ? p->R1s : nullptr, nullptr,
                        keep_r ? p->R2s : nullptr, nullptr, (double*)p->RinvTs, 0);
  if (e != hipSuccess) return e;
  if (n <= kGramShortRows)   // a short panel: the one-thread-per-output product
    return launch_small_gemm<double>(p->Z1, (const double*)p->RinvTs, n, c, c, Zout, nullptr,
                                     p->stream, 0);
  return launch_gemm_nn<double>(p->Z1, n, c, c, (const double*)p->RinvTs, c, c, Zout, c, nullptr,
                                nullptr, p->stream);
}

// Thin SVD of the FP64 matrix Tm (r x c): Tm = Qt R (CholeskyQR2), then
// one-sided Jacobi on R^T (QR-preconditioned Jacobi in the manner of Drmac &
// Veselic, SIAM J. Matrix Anal. Appl. 2008: the columns of R^T are already
// close to orthogonal, so few sweeps are needed): R^T J = Uo diag(Su), so
// R = J diag(Su) Uo^T and Tm = (Qt J) diag(Su) Uo^T: V~ = Qt J, W = Uo.  J is
// accumulated in the rotations when only leading columns are used
// (all_columns = false): it is then R Uo diag(Su)^-1, whose column for a
// value Su_j carries a rounding error of order eps Su_1 / Su_j -- small for
// the k largest values a solve keeps.  When the values span more than six
// decades the kernel flags it (diag[5] = 1) and a second, otherwise empty
// launch repeats the decomposition with J accumulated, replacing Uo, Su and
// J.  Leaves V~ unsorted in p->Vt, the values in p->Su and W in p->Uo.
hipError_t small_svd_unsorted(rsvd_plan_s* p, const double* Tm, int64_t r, int c,
                              bool all_columns = false) {
  hipError_t e;
  if ((e = cqr2_small(p, Tm, r, c, p->Zq, true)) != hipSuccess) return e;
  if ((e = launch_small_gemm<double>(p->R2s, p->R1s, c, c, c, p->Rt, nullptr, p->stream)) != hipSuccess)
    return e;
  if (c > kSmallSvdMaxC) {
    // the same one-sided Jacobi on R^T, as blocks of columns shared out over
    // workgroups (the column j of R^T is row j of Rt, so Rt is R^T stored
    // column by column); J accumulated, every column exact
    const unsigned nb = (unsigned)((c * c + 255) / 256);
    hipLaunchKernelGGL(k_eye, dim3(nb), dim3(256), 0, p->stream, p->Mk, c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_jacobi_eig(p->Rt, p->Mk, c, p->Su, p->diag, p->flags, p->EsS, p->status,
                               p->stream, -1, nullptr, nullptr, 1)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_svd_finish, dim3(nb), dim3(256), 0, p->stream, p->Rt, p->Mk, p->Su, c,
                       p->Uo, p->Jm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_small_gemm<double>(p->Zq, p->Jm, r, c, c, p->Vt, nullptr, p->stream);
  }
  if (all_columns) {
    if ((e = launch_jacobi_svd_small(p->Rt, c, 1, p->Uo, p->Su, p->Jm, 1, p->diag, p->status,
                                     nullptr, p->stream)) != hipSuccess)
      return e;
  } else {
    double* redo = p->diag + 5;
    if ((e = launch_jacobi_svd_small(p->Rt, c, 1, p->Uo, p->Su, p->Mk, 0, p->diag, p->status,
                                     redo, p->stream)) != hipSuccess)
      return e;
    if ((e = launch_small_gemm<double>(p->Rt, p->Mk, c, c, c, p->Jm, nullptr, p->stream)) !=
        hipSuccess)
      return e;
    if ((e = launch_jacobi_svd_small(p->Rt, c, 1, p->Uo, p->Su, p->Jm, 1, p->diag, p->status,
                                     redo, p->stream)) != hipSuccess)
      return e;
  }
  return launch_small_gemm<double>(p->Zq, p->Jm, r, c, c, p->Vt, nullptr, p->stream);
}

template <typename T>
int32_t rsvd_run(rsvd_plan_s* p, const T* A, int64_t m, int64_t n, int64_t lda, int k, int pov,
                 int q, double t, const double* omega, T* U, int64_t ldu, double* S, T* V,
                 int64_t ldv, int32_t* K, const LowpA* lp = nullptr) {
  const int l = (int)((k + pov < n) ? k + pov : n);
  hipStream_t s = p->stream;
  Path<T> P(p);
  T* Xs = (T*)p->Xs;
  T* Y = (T*)p->Y;
  T* Q1 = (T*)p->Q1;
  // Q1's row stride: l, or l rounded up to 8 for the bf16 projection
  const int64_t lq = lp ? ldq1_of(l) : l;
  RSVD_CHECK(reset(p));
  // step 1: the Gaussian sketch matrix G (n x l)
  if (!omega) {
    RSVD_CHECK(launch_gaussian_fill(p->seed, n, l, p->omega, s));
    omega = p->omega;
  }
  // fp32 passes with a narrow right factor take it transposed (l x n)
  const bool tall = std::is_same<T, float>::value &&
                    nt_tall_applies(reinterpret_cast<const float*>(A), n, lda,
                                    reinterpret_cast<const float*>(Xs), n, l);
  auto pass_nn = [&](const double* X64, double* fro2_part, int* np) -> hipError_t {
    hipError_t e;
    if (lp) {
      // bf16 A: (diag(s) X)^T as hi + lo bf16 pairs (l x n each) in Xs
      __bf16* Xhi = reinterpret_cast<__bf16*>(p->Xs);
      __bf16* Xlo = Xhi + (int64_t)l * n;
      if ((e = launch_cast_hilo_t(X64, n, l, lp->scale, Xhi, Xlo, n, s)) != hipSuccess) return e;
      KtScope ts(p, KT_PASS_NN);
      return launch_gemm_nt_bf16(lp->A, lp->es, m, n, lda, Xhi, Xlo, n, l, lp->scale,
                                 reinterpret_cast<float*>(Y), l, fro2_part, np, s);
    }
    if (tall) {
      if ((e = launch_cast_t_from_f64<T>(X64, n, l, l, Xs, n, s)) != hipSuccess) return e;
      KtScope ts(p, KT_PASS_NN);
      return launch_gemm_nt_tall(reinterpret_cast<const float*>(A), m, n, lda,
                                 reinterpret_cast<const float*>(Xs), n, l,
                                 reinterpret_cast<float*>(Y), l, fro2_part, np, s);
    }
    if ((e = launch_cast_from_f64<T>(X64, n, l, l, Xs, l, s)) != hipSuccess) return e;
    return launch_gemm_nn<T>(A, m, n, lda, Xs, l, l, Y, l, fro2_part, np, s);
  };
  // step 2: H = A G, with ||A||_F^2 (Eq. sumeigen) from the same pass
  int np = 0;
  RSVD_CHECK(pass_nn(omega, p->fro2_part, &np));
  RSVD_CHECK(launch_reduce_scalar(p->fro2_part, np, p->scal, s));
  // only R2^-1 (and R1^-1 through RinvT) of the CholeskyQR2 factors is used
  RSVD_CHECK(P.cqr2(Y, m, l, l, Q1, lq, nullptr, nullptr, nullptr, p->R2inv, (T*)p->RinvT));
  auto pass_tn = [&](double* Z) -> hipError_t {
    if (lp) return P.tn_bf16(*lp, m, n, lda, reinterpret_cast<const float*>(Q1), lq, l, Z);
    return P.tn(A, m, n, lda, Q1, lq, l, Z);
  };
  // step 3: power iterations H = A (A^T H), orthonormalised after each product
  for (int it = 0; it < q; ++it) {
    RSVD_CHECK(pass_tn(p->Zd));
    RSVD_CHECK(launch_small_gemm<T>(p->Zd, p->R2inv, n, l, l, p->Z2, nullptr, s));  // A^T Q
    RSVD_CHECK(cqr2_small(p, p->Z2, n, l, p->Zq));
    RSVD_CHECK(pass_nn(p->Zq, nullptr, nullptr));
    RSVD_CHECK(P.cqr2(Y, m, l, l, Q1, lq, nullptr, nullptr, nullptr, p->R2inv, (T*)p->RinvT));
  }
  // step 5: T = A^T Q
  RSVD_CHECK(pass_tn(p->Zd));
  RSVD_CHECK(launch_small_gemm<T>(p->Zd, p->R2inv, n, l, l, p->Z2, nullptr, s));
  // step 6: T = V~ S~ W^T
  RSVD_CHECK(small_svd_unsorted(p, p->Z2, n, l));
  RSVD_CHECK(launch_sort_sign_scatter<T>(p->Su, l, p->Vt, n, l, 1, p->Uo, k, S, V, ldv, nullptr,
                                         p->Wk, s));
  // step 7: U~ = Q W = Q1 (R2^-1 W), first k columns; fp32 takes the l x k
  // factor transposed into the tall kernel
  const bool tall_u = std::is_same<T, float>::value &&
                      nt_tall_applies(reinterpret_cast<const float*>(Q1), l, lq,
                                      reinterpret_cast<const float*>(p->MkT), l, k);
  if (U) {   // (batch instances and server requests may ask for S, V and K only)
    RSVD_CHECK(launch_small_gemm<T>(p->R2inv, p->Wk, l, l, k, nullptr, (T*)p->MkT, s, tall_u));
    if (tall_u)
      RSVD_CHECK(launch_gemm_nt_tall(reinterpret_cast<const float*>(Q1), m, l, lq,
                                     reinterpret_cast<const float*>(p->MkT), l, k,
                                     reinterpret_cast<float*>(U), ldu, nullptr, nullptr, s));
    else
      RSVD_CHECK(launch_gemm_nn<T>(Q1, m, l, lq, (const T*)p->MkT, k, k, U, ldu, nullptr, nullptr,
                                   s));
  }
  // K by the explained-variance criterion (Sec. 2.4)
  RSVD_CHECK(launch_select_k(S, k, p->scal, t, K, p->diag, p->status, s));
  return RSVD_OK;
}

// Krylov method (Sec. 3.1.1): blocks H(0) = A G and H(j) = A (A^T H(j-1)),
// j = 1..i, each turned into an orthonormal basis Q(j) of its own columns
// (CholeskyQR2 and the explicit product Q1 R2^-1; the same Krylov space) and
// stored side by side as the m x L panel H, L = (i+1) l; CholeskyQR2 of H
// gives Q = Q1 R2^-1, then T = A^T Q, the small SVD and U = Q W as for
// Randomized PCA.  The panel lives in the plan's Y buffer (row stride L),
// which needs L <= l_max.
template <typename T>
int32_t krylov_run(rsvd_plan_s* p, const T* A, int64_t m, int64_t n, int64_t lda, int k, int pov,
                   int iblk, double t, const double* omega, T* U, int64_t ldu, double* S, T* V,
                   int64_t ldv, int32_t* K) {
  const int l = (int)((k + pov < n) ? k + pov : n);
  const int L = (iblk + 1) * l;
  hipStream_t s = p->stream;
  Path<T> P(p);
  T* Xs = (T*)p->Xs;
  T* H = (T*)p->Y;
  T* Q1 = (T*)p->Q1;
  RSVD_CHECK(reset(p));
  // step 1: the Gaussian sketch matrix G (n x l)
  if (!omega) {
    RSVD_CHECK(launch_gaussian_fill(p->seed, n, l, p->omega, s));
    omega = p->omega;
  }
  const bool tall = std::is_same<T, float>::value &&
                    nt_tall_applies(reinterpret_cast<const float*>(A), n, lda,
                                    reinterpret_cast<const float*>(Xs), n, l);
  // A X (X n x l, FP64) into block j of the panel
  auto pass_nn = [&](const double* X64, int j, double* fro2_part, int* np) -> hipError_t {
    hipError_t e;
    T* Yj = H + (int64_t)j * l;
    if (tall) {
      if ((e = launch_cast_t_from_f64<T>(X64, n, l, l, Xs, n, s)) != hipSuccess) return e;
      KtScope ts(p, KT_PASS_NN);
      return launch_gemm_nt_tall(reinterpret_cast<const float*>(A), m, n, lda,
                                 reinterpret_cast<const float*>(Xs), n, l,
                                 reinterpret_cast<float*>(Yj), L, fro2_part, np, s);
    }
    if ((e = launch_cast_from_f64<T>(X64, n, l, l, Xs, l, s)) != hipSuccess) return e;
    return launch_gemm_nn<T>(A, m, n, lda, Xs, l, l, Yj, L, fro2_part, np, s);
  };
  // steps 2-4: the blocks, each replaced by its orthonormal basis in place
  int np = 0;
  for (int j = 0; j <= iblk; ++j) {
    if (j == 0) {
      RSVD_CHECK(pass_nn(omega, 0, p->fro2_part, &np));                    // H(0) = A G
      RSVD_CHECK(launch_reduce_scalar(p->fro2_part, np, p->scal, s));     // Eq. sumeigen
    } else {
      RSVD_CHECK(P.tn(A, m, n, lda, H + (int64_t)(j - 1) * l, L, l, p->Zd));  // A^T Q(j-1)
      RSVD_CHECK(cqr2_small(p, p->Zd, n, l, p->Zq));
      RSVD_CHECK(pass_nn(p->Zq, j, nullptr, nullptr));                    // H(j)
    }
    T* Yj = H + (int64_t)j * l;
    const bool tb = P.times_rinv_tall(Q1, l, l, (const T*)p->RinvT);
    RSVD_CHECK(P.cqr2(Yj, m, l, L, Q1, l, nullptr, nullptr, nullptr, p->R2inv, (T*)p->RinvT, tb));
    RSVD_CHECK(P.times_rinv(Q1, m, l, l, (const T*)p->RinvT, tb, Yj, L));   // Q(j) = Q1 R2^-1
  }
  // step 5: QR of the panel.  Its blocks overlap more as the Krylov space
  // converges (condition numbers of 1e4 .. 1e11 on decaying spectra), so a
  // shifted CholeskyQR pass (H -> Q1) precedes CholeskyQR2 (Q1 -> the panel's
  // own storage, no longer needed): Q = H R2^-1, kept implicit.
  RSVD_CHECK(P.cqr_shifted(H, m, L, L, Q1, L, nullptr, nullptr, (T*)p->RinvT));
  RSVD_CHECK(P.cqr2(Q1, m, L, L, H, L, nullptr, nullptr, nullptr, p->R2inv, (T*)p->RinvT));
  Q1 = H;
  // step 6: T = A^T Q = (A^T Q1) R2^-1
  RSVD_CHECK(P.tn(A, m, n, lda, Q1, L, L, p->Zd));
  RSVD_CHECK(launch_small_gemm<T>(p->Zd, p->R2inv, n, L, L, p->Z2, nullptr, s));
  // step 7: T = V~ S~ W^T
  RSVD_CHECK(small_svd_unsorted(p, p->Z2, n, L));
  RSVD_CHECK(launch_sort_sign_scatter<T>(p->Su, L, p->Vt, n, L, 1, p->Uo, k, S, V, ldv, nullptr,
                                         p->Wk, s));
  // step 8: U~ = Q W = Q1 (R2^-1 W), first k columns
  const bool tall_u = std::is_same<T, float>::value &&
                      nt_tall_applies(reinterpret_cast<const float*>(Q1), L, L,
                                      reinterpret_cast<const float*>(p->MkT), L, k);
  RSVD_CHECK(launch_small_gemm<T>(p->R2inv, p->Wk, L, L, k, nullptr, (T*)p->MkT, s, tall_u));
  if (tall_u)
    RSVD_CHECK(launch_gemm_nt_tall(reinterpret_cast<const float*>(Q1), m, L, L,
                                   reinterpret_cast<const float*>(p->MkT), L, k,
                                   reinterpret_cast<float*>(U), ldu, nullptr, nullptr, s));
  else
    RSVD_CHECK(launch_gemm_nn<T>(Q1, m, L, L, (const T*)p->MkT, k, k, U, ldu, nullptr, nullptr, s));
  RSVD_CHECK(launch_select_k(S, k, p->scal, t, K, p->diag, p->status, s));
  return RSVD_OK;
}

// ---------------------------------------------------------------------------
// Randomized PCA with the rank grown in blocks of b columns until the
// criterion of Sec. 2.4 can be met: the blocked randomized range finder with
// power steps of Martinsson & Voronin (SIAM J. Sci. Comput. 2016, randQB_b
// with power iterations).  The basis Q is kept explicit in the plan's Q1
// buffer (m x L, row stride ldq1_of(l_max)), B = Q^T A as T = A^T Q in Tp
// (n x L, FP64, row stride l_max); block j:
//   Y = A G_j - Q (T^T G_j);  Q_j = orth(Y)
//   q times:  Z = orth(A^T Q_j);  Y = A Z - Q (T^T Z);  Q_j = orth(Y)
//   Q_j = orth(Q_j - Q (Q^T Q_j))            (re-orthogonalisation)
//   T_j = A^T Q_j;  Q = [Q Q_j];  T = [T T_j];  L += b
// with orth = CholeskyQR2 and its explicit factor, and scal[1] += ||T_j||_F^2,
// the energy ||Q^T A||_F^2 that span(Q) holds (scal[0] = ||A||_F^2, Eq.
// sumeigen, from block 0's first pass).  Block j's sketch G_j is drawn from
// seed + j * 0x9E3779B97F4A7C15 (block 0: the plan's own sketch).  The
// caller decides between blocks (on the host) whether to grow; then the
// finish step: SVD T = V~ S~ W^T, U~ = Q W, K over all L values.
struct GrowJob {
  const void* A = nullptr;
  int64_t m = 0, n = 0, lda = 0;
  LowpA lp{nullptr, nullptr, 0};
  int b = 0, q = 0, kcap = 0;
  double t = 0.0;
  int L = 0, j = 0;
  void* U = nullptr;
  int64_t ldu = 0;
  double* S = nullptr;
  void* V = nullptr;
  int64_t ldv = 0;
  int32_t* K = nullptr;
};

constexpr uint64_t kBlockSeedStep = 0x9E3779B97F4A7C15ull;

// Y (rows x cols, ld) -= W (same layout).
template <typename T>
__global__ void k_sub(T* __restrict__ Y, const T* __restrict__ W, int64_t rows, int cols,
                      int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx / cols;
  const int j = (int)(idx - i * cols);
  Y[i * ld + j] -= W[i * ld + j];
}

// dst (rows x cols, ldd) = src (rows x cols, lds).
template <typename T>
__global__ void k_copy2d(const T* __restrict__ src, int64_t lds, T* __restrict__ dst, int64_t ldd,
                         int64_t rows, int cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx / cols;
  const int j = (int)(idx - i * cols);
  dst[i * ldd + j] = src[i * lds + j];
}

// scal[1] += ||Z||_F^2 (Z rows x cols, ld cols; one block, fixed order);
// diag[6] = L, diag[7] = scal[1] / scal[0].
__global__ void k_energy(const double* __restrict__ Z, int64_t rows, int cols, double* scal,
                         double* diag, int L) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < rows * cols; e += 256) s += Z[e] * Z[e];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e = scal[1] + sh[0];
    scal[1] = e;
    diag[6] = (double)L;
    diag[7] = scal[0] > 0.0 ? e / scal[0] : 0.0;
  }
}

// K <= kcap: a larger K is capped, with RSVD_WARN_THRESHOLD.
__global__ void k_cap_k(int32_t* K, int kcap, int32_t* status, double* diag) {
  if (threadIdx.x == 0 && *K > kcap) {
    *K = kcap;
    diag[4] = (double)kcap;
    atomicCAS(status, (int32_t)RSVD_OK, (int32_t)RSVD_WARN_THRESHOLD);   // errors stay
  }
}

inline unsigned grid_for(int64_t total) { return (unsigned)((total + 255) / 256); }

template <typename T>
struct Grow {
  rsvd_plan_s* p;
  GrowJob& g;
  hipStream_t s;
  Path<T> P;
  int64_t ldp, ldb;
  T* Qp;
  T* Yb;
  T* Wb;
  Grow(rsvd_plan_s* plan, GrowJob& job)
      : p(plan), g(job), s(plan->stream), P(plan), ldp(ldq1_of(plan->l_max)),
        ldb(ldq1_of(job.b)), Qp((T*)plan->Q1), Yb((T*)plan->Y), Wb((T*)plan->Y + job.m * ldb) {}

  bool low() const { return g.lp.es != 0; }

  // Y (m x b, ldb) = A X, X n x b FP64 (ld b)
  hipError_t pass_nn(const double* X64, double* fro2_part, int* np) {
    hipError_t e;
    const int b = g.b;
    const int64_t m = g.m, n = g.n;
    if (low()) {
      __bf16* Xhi = reinterpret_cast<__bf16*>(p->Xs);
      __bf16* Xlo = Xhi + (int64_t)b * n;
      if ((e = launch_cast_hilo_t(X64, n, b, g.lp.scale, Xhi, Xlo, n, s)) != hipSuccess) return e;
      return launch_gemm_nt_bf16(g.lp.A, g.lp.es, m, n, g.lda, Xhi, Xlo, n, b, g.lp.scale,
                                 reinterpret_cast<float*>(Yb), ldb, fro2_part, np, s);
    }
    const T* A = (const T*)g.A;
    T* Xs = (T*)p->Xs;
    if (std::is_same<T, float>::value &&
        nt_tall_applies(reinterpret_cast<const float*>(A), n, g.lda,
                        reinterpret_cast<const float*>(Xs), n, b)) {
      if ((e = launch_cast_t_from_f64<T>(X64, n, b, b, Xs, n, s)) != hipSuccess) return e;
      return launch_gemm_nt_tall(reinterpret_cast<const float*>(A), m, n, g.lda,
                                 reinterpret_cast<const float*>(Xs), n, b,
                                 reinterpret_cast<float*>(Yb), ldb, fro2_part, np, s);
    }
    if ((e = launch_cast_from_f64<T>(X64, n, b, b, Xs, b, s)) != hipSuccess) return e;
    return launch_gemm_nn<T>(A, m, n, g.lda, Xs, b, b, Yb, ldb, fro2_part, np, s);
  }

  // Z (n x b, FP64) = A^T Q, Q m x b (ld ldq)
  hipError_t pass_tn(const T* Q, int64_t ldq, double* Z) {
    if (low())
      return P.tn_bf16(g.lp, g.m, g.n, g.lda, reinterpret_cast<const float*>(Q), ldq, g.b, Z);
    return P.tn((const T*)g.A, g.m, g.n, g.lda, Q, ldq, g.b, Z);
  }

  // Yb -= Qp C, C (L x b, FP64, ld b) in p->Mk
  hipError_t sub_qc() {
    hipError_t e;
    const int L = g.L, b = g.b;
    T* CT = (T*)p->MkT;
    if (std::is_same<T, float>::value &&
        nt_tall_applies(reinterpret_cast<const float*>(Qp), L, ldp,
                        reinterpret_cast<const float*>(CT), L, b)) {
      if ((e = launch_cast_t_from_f64<T>(p->Mk, L, b, b, CT, L, s)) != hipSuccess) return e;
      e = launch_gemm_nt_tall(reinterpret_cast<const float*>(Qp), g.m, L, ldp,
                              reinterpret_cast<const float*>(CT), L, b,
                              reinterpret_cast<float*>(Wb), ldb, nullptr, nullptr, s);
    } else {
      if ((e = launch_cast_from_f64<T>(p->Mk, L, b, b, CT, b, s)) != hipSuccess) return e;
      e = launch_gemm_nn<T>(Qp, g.m, L, ldp, CT, b, b, Wb, ldb, nullptr, nullptr, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sub<T>), dim3(grid_for(g.m * b)), dim3(256), 0, s, Yb, Wb, g.m, b, ldb);
    return hipGetLastError();
  }

  // Yb -= Qp (T^T X), X n x b FP64 (ld b): the part outside span(Q)
  hipError_t project(const double* X64) {
    if (g.L == 0) return hipSuccess;
    hipError_t e = Path<double>(p).tn(p->Tp, g.n, g.L, p->l_max, X64, g.b, g.b, p->Mk);
    if (e != hipSuccess) return e;
    return sub_qc();
  }

  // Yb <- an orthonormal basis of its columns (CholeskyQR2, explicit)
  hipError_t orth() {
    hipError_t e;
    const bool tb = P.times_rinv_tall(Wb, g.b, ldb, (const T*)p->RinvT);
    if ((e = P.cqr2(Yb, g.m, g.b, ldb, Wb, ldb, nullptr, nullptr, nullptr, p->R2inv, (T*)p->RinvT,
                    tb)) != hipSuccess)
      return e;
    return P.times_rinv(Wb, g.m, g.b, ldb, (const T*)p->RinvT, tb, Yb, ldb);
  }

  hipError_t block() {
    hipError_t e;
    const int b = g.b;
    const int64_t m = g.m, n = g.n;
    if (g.j == 0) {
      if ((e = launch_fill_scal(p)) != hipSuccess) return e;
    }
    if ((e = launch_gaussian_fill(p->seed + kBlockSeedStep * (uint64_t)g.j, n, b, p->omega, s)) !=
        hipSuccess)
      return e;
    int np = 0;
    if ((e = pass_nn(p->omega, g.j == 0 ? p->fro2_part : nullptr, &np)) != hipSuccess) return e;
    if (g.j == 0 && (e = launch_reduce_scalar(p->fro2_part, np, p->scal, s)) != hipSuccess)
      return e;
    if ((e = project(p->omega)) != hipSuccess) return e;
    if ((e = orth()) != hipSuccess) return e;
    for (int it = 0; it < g.q; ++it) {
      if ((e = pass_tn(Yb, ldb, p->Zd)) != hipSuccess) return e;
      if ((e = cqr2_small(p, p->Zd, n, b, p->Zq)) != hipSuccess) return e;
      if ((e = pass_nn(p->Zq, nullptr, nullptr)) != hipSuccess) return e;
      if ((e = project(p->Zq)) != hipSuccess) return e;
      if ((e = orth()) != hipSuccess) return e;
    }
    if (g.L > 0) {   // Q_j - Q (Q^T Q_j), then orthonormalised again
      if ((e = P.tn(Qp, m, g.L, ldp, Yb, ldb, b, p->Mk)) != hipSuccess) return e;
      if ((e = sub_qc()) != hipSuccess) return e;
      if ((e = orth()) != hipSuccess) return e;
    }
    // append Q_j, T_j = A^T Q_j
    hipLaunchKernelGGL((k_copy2d<T>), dim3(grid_for(m * b)), dim3(256), 0, s, Yb, ldb,
                       Qp + g.L, ldp, m, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = pass_tn(Yb, ldb, p->Zd)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_copy2d<double>), dim3(grid_for(n * b)), dim3(256), 0, s, p->Zd,
                       (int64_t)b, p->Tp + g.L, (int64_t)p->l_max, n, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    g.L += b;
    ++g.j;
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, s, p->Zd, n, b, p->scal, p->diag, g.L);
    return hipGetLastError();
  }

  static hipError_t launch_fill_scal(rsvd_plan_s* pl) {
    // scal[1] (the captured energy) starts at zero
    return launch_fill_i32(reinterpret_cast<int32_t*>(pl->scal + 1), 2, 0, pl->stream);
  }

  hipError_t finish() {
    hipError_t e;
    const int L = g.L;
    const int64_t m = g.m, n = g.n;
    const int kc = g.kcap < L ? g.kcap : L;
    hipLaunchKernelGGL((k_copy2d<double>), dim3(grid_for(n * L)), dim3(256), 0, s, p->Tp,
                       (int64_t)p->l_max, p->Z2, (int64_t)L, n, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = small_svd_unsorted(p, p->Z2, n, L)) != hipSuccess) return e;
    // the first kc triplets; all L values (sorted) for the criterion
    if ((e = launch_sort_sign_scatter<T>(p->Su, L, p->Vt, n, L, 1, p->Uo, kc, g.S, (T*)g.V, g.ldv,
                                         nullptr, p->Wk, s)) != hipSuccess)
      return e;
    if ((e = launch_sort_sign_scatter<T>(p->Su, L, p->Vt, n, L, 1, nullptr, L, p->Zq, nullptr, 0,
                                         nullptr, nullptr, s)) != hipSuccess)
      return e;
    // U~ = Q W (first kc columns; none when U is not wanted)
    T* WT = (T*)p->MkT;
    if (!g.U) {
      e = hipSuccess;
    } else if (std::is_same<T, float>::value &&
        nt_tall_applies(reinterpret_cast<const float*>(Qp), L, ldp,
                        reinterpret_cast<const float*>(WT), L, kc)) {
      if ((e = launch_cast_t_from_f64<T>(p->Wk, L, kc, kc, WT, L, s)) != hipSuccess) return e;
      e = launch_gemm_nt_tall(reinterpret_cast<const float*>(Qp), m, L, ldp,
                              reinterpret_cast<const float*>(WT), L, kc,
                              reinterpret_cast<float*>(g.U), g.ldu, nullptr, nullptr, s);
    } else {
      if ((e = launch_cast_from_f64<T>(p->Wk, L, kc, kc, WT, kc, s)) != hipSuccess) return e;
      e = launch_gemm_nn<T>(Qp, m, L, ldp, WT, kc, kc, (T*)g.U, g.ldu, nullptr, nullptr, s);
    }
    if (e != hipSuccess) return e;
    if ((e = launch_select_k(p->Zq, L, p->scal, g.t, g.K, p->diag, p->status, s)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_cap_k, dim3(1), dim3(64), 0, s, g.K, g.kcap, p->status, p->diag);
    return hipGetLastError();
  }
};

// Whether another block fits: L + b columns within the sketch limit and n.
bool grow_fits(const rsvd_plan_s* p, const GrowJob& g) {
  return g.L + g.b <= p->l_max && g.L + g.b <= g.n;
}

// Enqueue the next block (the first one resets the status word).
int32_t grow_block(rsvd_plan_s* p, GrowJob& g) {
  if (g.j == 0) RSVD_CHECK(reset(p));
  if (p->dtype == RSVD_F64) RSVD_CHECK(Grow<double>(p, g).block());
  else RSVD_CHECK(Grow<float>(p, g).block());
  return RSVD_OK;
}

int32_t grow_finish(rsvd_plan_s* p, GrowJob& g) {
  if (p->dtype == RSVD_F64) RSVD_CHECK(Grow<double>(p, g).finish());
  else RSVD_CHECK(Grow<float>(p, g).finish());
  return RSVD_OK;
}

// ||A||_F^2 and the captured energy after the blocks so far (waits for the
// plan's stream).
int32_t grow_read(rsvd_plan_s* p, double* fro2, double* energy) {
  double h[2] = {0.0, 0.0};
  RSVD_CHECK(hipMemcpyAsync(h, p->scal, sizeof(h), hipMemcpyDeviceToHost, p->stream));
  RSVD_CHECK(hipStreamSynchronize(p->stream));
  *fro2 = h[0];
  *energy = h[1];
  return RSVD_OK;
}

template <typename T>
int32_t gram_run(rsvd_plan_s* p, const T* A, int64_t m, int64_t n, int64_t lda, double t,
                 int ucols, T* U, int64_t ldu, double* S, T* V, int64_t ldv, int32_t* K) {
  hipStream_t s = p->stream;
  Path<T> P(p);
  RSVD_CHECK(reset(p));
  // step 1: A^T A (Eq. AB), and its trace = ||A||_F^2 (Eq. sumeigen)
  if (std::is_same<T, float>::value &&
      syrk_f32_applies(reinterpret_cast<const float*>(A), n, lda)) {
    const KtPair tp = kt_reserve(p, KT_SYRK);
    RSVD_CHECK(launch_syrk_f32(reinterpret_cast<const float*>(A), m, n, lda, p->part,
                               p->max_split * p->n_max * p_cmax(p), p->Gd, s, tp.e0, tp.e1));
  } else {
    RSVD_CHECK(P.tn(A, m, n, lda, A, lda, (int)n, p->Gd));
  }
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, p->Gd, n, p->scal);
  RSVD_CHECK(hipGetLastError());
  // step 2: eigen-decomposition (Jacobi, FP64)
  hipLaunchKernelGGL(k_init_eig, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, p->Gd, n,
                     p->Xe, p->Je);
  RSVD_CHECK(hipGetLastError());
  {
    const KtPair tp = kt_reserve(p, KT_EIG);
    RSVD_CHECK(launch_jacobi_eig(p->Xe, p->Je, n, p->lam, p->diag, p->flags, p->Es, p->status, s,
                                 -1, tp.e0, tp.e1));
  }
  // step 3: s_i = sqrt(lambda_i) (Eq. LambdaSigma), sorted, sign rule
  RSVD_CHECK(launch_sqrt_clamp(p->lam, (int)n, p->Se, s));
  RSVD_CHECK(launch_sort_sign_scatter<T>(p->Se, (int)n, p->Je, n, 1, n, nullptr, (int)n, S, V,
                                         ldv, p->Vd, nullptr, s));
  // step 4: u_i = A v_i / s_i
  if (ucols > 0) {
    const double floor_rel = (double)(m > n ? m : n) * 2.220446049250313e-16;
    if (std::is_same<T, float>::value && ucols > 128) {
      // wide fp32 product: the scaled V goes in transposed (ucols x n)
      RSVD_CHECK(launch_scale_cols_inv<T>(p->Vd, n, ucols, n, S, floor_rel, (T*)p->Xs, n, 1, s));
      KtScope ts(p, KT_NT_WIDE);
      RSVD_CHECK(launch_gemm_nt_wide(reinterpret_cast<const float*>(A), m, n, lda,
                                     reinterpret_cast<const float*>(p->Xs), n, ucols,
                                     reinterpret_cast<float*>(U), ldu, s));
    } else {
      RSVD_CHECK(launch_scale_cols_inv<T>(p->Vd, n, ucols, n, S, floor_rel, (T*)p->Xs, ucols, 0, s));
      RSVD_CHECK(launch_gemm_nn<T>(A, m, n, lda, (const T*)p->Xs, ucols, ucols, U, ldu, nullptr,
                                   nullptr, s));
    }
  }
  RSVD_CHECK(launch_select_k(S, (int)n, p->scal, t, K, p->diag, p->status, s));
  return RSVD_OK;
}

bool bad_t(double t) { return !(t > 0.0 && t <= 1.0); }

int32_t check_common(rsvd_plan_s* p, const void* A, int64_t m, int64_t n, int64_t lda) {
  if (!p || !A) return RSVD_ERR_ARG;
  if (n < 1 || m < n) return RSVD_ERR_SHAPE;
  if (m > p->m_max || n > p->n_max) return RSVD_ERR_SHAPE;
  if (lda < n) return RSVD_ERR_ARG;
  return RSVD_OK;
}

int32_t check_rsvd(rsvd_plan_s* p, const void* A, int64_t m, int64_t n, int64_t lda, int32_t k,
                   int32_t pov, int32_t q, double t, const void* U, int64_t ldu, const void* S,
                   const void* V, int64_t ldv, const void* K) {
  int32_t rc = check_common(p, A, m, n, lda);
  if (rc != RSVD_OK) return rc;
  if (!U || !S || !V || !K) return RSVD_ERR_ARG;
  if (k < 1 || k > n || pov < 0 || q < 0 || bad_t(t)) return RSVD_ERR_ARG;
  if (ldu < k || ldv < k) return RSVD_ERR_ARG;
  const int64_t l = (k + (int64_t)pov < n) ? k + (int64_t)pov : n;
  if (l > p->l_max) return RSVD_ERR_SHAPE;
  return RSVD_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* rsvd_status_string(int32_t st) {
  switch (st) {
    case RSVD_OK: return "RSVD_OK";
    case RSVD_WARN_THRESHOLD: return "RSVD_WARN_THRESHOLD";
    case RSVD_WARN_ZERO_MATRIX: return "RSVD_WARN_ZERO_MATRIX";
    case RSVD_ERR_ARG: return "RSVD_ERR_ARG";
    case RSVD_ERR_SHAPE: return "RSVD_ERR_SHAPE";
    case RSVD_ERR_NOMEM: return "RSVD_ERR_NOMEM";
    case RSVD_ERR_DEVICE: return "RSVD_ERR_DEVICE";
    case RSVD_ERR_BREAKDOWN: return "RSVD_ERR_BREAKDOWN";
    case RSVD_ERR_NONFINITE: return "RSVD_ERR_NONFINITE";
    case RSVD_ERR_NOCONV: return "RSVD_ERR_NOCONV";
    default: return "RSVD_UNKNOWN_STATUS";
  }
}

int32_t rsvd_plan_create(rsvd_plan_t* plan, int64_t m_max, int64_t n_max, int32_t l_max,
                         int32_t dtype, int32_t want_gram, uint64_t seed, void* stream) {
  if (!plan) return RSVD_ERR_ARG;
  *plan = nullptr;
  if (dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16 && dtype != RSVD_FP8)
    return RSVD_ERR_ARG;
  if (lowp_es(dtype) && want_gram) return RSVD_ERR_ARG;   // the A^T A route is fp32/fp64
  if (l_max < 1) return RSVD_ERR_ARG;
  if (n_max < 1 || m_max < n_max || m_max > kMaxRows || n_max > kMaxCols) return RSVD_ERR_SHAPE;
  if (l_max > kMaxL) return RSVD_ERR_SHAPE;
  if (want_gram && n_max > jacobi_eig_max_n()) return RSVD_ERR_SHAPE;
  rsvd_plan_s* p = new (std::nothrow) rsvd_plan_s();
  if (!p) return RSVD_ERR_NOMEM;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return RSVD_ERR_DEVICE; }
  p->dtype = dtype;
  p->m_max = m_max;
  p->n_max = n_max;
  p->l_max = (int)((l_max < n_max) ? l_max : n_max);
  p->gram = want_gram != 0;
  p->seed = seed;
  p->stream = (hipStream_t)stream;
  p->max_split = tn_max_split(m_max, n_max, p->l_max);
  p->bytes = carve(p, nullptr);
  void* mem = nullptr;
  if (hipMalloc(&mem, p->bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return RSVD_ERR_NOMEM;
  }
  p->base = (char*)mem;
  carve(p, p->base);
  if (hipMemsetAsync(p->base, 0, p->bytes, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess) {
    (void)hipFree(mem);
    delete p;
    return RSVD_ERR_DEVICE;
  }
  *plan = p;
  return RSVD_OK;
}

int32_t rsvd_plan_destroy(rsvd_plan_t plan) {
  if (!plan) return RSVD_OK;
  int32_t rc = RSVD_OK;
  if (hipSetDevice(plan->device) != hipSuccess) rc = RSVD_ERR_DEVICE;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) rc = RSVD_ERR_DEVICE;
  if (plan->base && hipFree(plan->base) != hipSuccess) rc = RSVD_ERR_DEVICE;
  if (plan->kt) {
    for (int k = 0; k < KT_COUNT; ++k)
      for (int i = 0; i < kTimerPairs; ++i)
        for (int j = 0; j < 2; ++j)
          if (plan->kt[k].ev[i][j]) (void)hipEventDestroy(plan->kt[k].ev[i][j]);
    delete[] plan->kt;
  }
  delete plan;
  return rc;
}

int32_t rsvd_plan_status(rsvd_plan_t plan) {
  if (!plan) return RSVD_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return RSVD_ERR_DEVICE;
  int32_t st = 0;
  if (hipMemcpy(&st, plan->status, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return RSVD_ERR_DEVICE;
  const int32_t zero = 0;
  if (hipMemcpy(plan->status, &zero, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
    return RSVD_ERR_DEVICE;
  return st;
}

int32_t rsvd_plan_diag(rsvd_plan_t plan, double* out, int32_t count) {
  if (!plan || !out || count < 0) return RSVD_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return RSVD_ERR_DEVICE;
  const int32_t nc = count < kDiagWords ? count : kDiagWords;
  if (nc > 0 && hipMemcpy(out, plan->diag, nc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return RSVD_ERR_DEVICE;
  return nc;
}

int32_t rsvd_plan_kernel_times(rsvd_plan_t plan, int32_t enable, double* ms, int32_t* launches,
                               int32_t count) {
  if (!plan || count < 0 || (count > 0 && (!ms || !launches))) return RSVD_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  if (hipStreamSynchronize(plan->stream) != hipSuccess) return RSVD_ERR_DEVICE;
  const int32_t nc = count < KT_COUNT ? count : KT_COUNT;
  for (int k = 0; k < nc; ++k) {
    double sum = 0.0;
    int used = 0;
    if (plan->kt) {
      for (int i = 0; i < plan->kt[k].used; ++i) {
        float e = 0.f;   // a pair left unrecorded by a failed launch is skipped
        if (hipEventElapsedTime(&e, plan->kt[k].ev[i][0], plan->kt[k].ev[i][1]) != hipSuccess)
          continue;
        sum += e;
        ++used;
      }
    }
    ms[k] = used ? sum / used : 0.0;
    launches[k] = used;
  }
  if (plan->kt)
    for (int k = 0; k < KT_COUNT; ++k) plan->kt[k].used = 0;
  if (enable && !plan->kt) plan->kt = new (std::nothrow) KernelTimer[KT_COUNT];
  if (enable && !plan->kt) return RSVD_ERR_NOMEM;
  plan->timing = enable != 0;
  return nc;
}

int32_t rsvd_solve_omega(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                         const float* col_scale, int32_t k, int32_t p, int32_t q, double t,
                         const double* omega, void* U, int64_t ldu, double* S, void* V,
                         int64_t ldv, int32_t* K) {
  int32_t rc = check_rsvd(plan, A, m, n, lda, k, p, q, t, U, ldu, S, V, ldv, K);
  if (rc != RSVD_OK) return rc;
  if (plan->dtype == RSVD_BF16)
    return rsvd_solve_bf16(plan, A, col_scale, m, n, lda, k, p, q, t, omega, (float*)U, ldu, S,
                           (float*)V, ldv, K);
  if (plan->dtype == RSVD_FP8)
    return rsvd_solve_fp8(plan, A, col_scale, m, n, lda, k, p, q, t, omega, (float*)U, ldu, S,
                          (float*)V, ldv, K);
  if (col_scale) return RSVD_ERR_ARG;   // column scales belong to bf16 / FP8 storage
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  if (plan->dtype == RSVD_F64)
    return rsvd_run<double>(plan, (const double*)A, m, n, lda, k, p, q, t, omega, (double*)U, ldu,
                            S, (double*)V, ldv, K);
  return rsvd_run<float>(plan, (const float*)A, m, n, lda, k, p, q, t, omega, (float*)U, ldu, S,
                         (float*)V, ldv, K);
}

}  // extern "C"

namespace {
int32_t solve_lowp(rsvd_plan_t plan, int dtype, const void* A, const float* col_scale, int64_t m,
                   int64_t n, int64_t lda, int32_t k, int32_t p, int32_t q, double t,
                   const double* omega, float* U, int64_t ldu, double* S, float* V, int64_t ldv,
                   int32_t* K) {
  int32_t rc = check_rsvd(plan, A, m, n, lda, k, p, q, t, U, ldu, S, V, ldv, K);
  if (rc != RSVD_OK) return rc;
  if (plan->dtype != dtype) return RSVD_ERR_ARG;
  const int es = lowp_es(dtype);
  const int l = (int)((k + (int64_t)p < n) ? k + p : n);
  if (!bf16_pass_applies(A, es, n, lda, l)) return RSVD_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  const LowpA lp{A, col_scale, es};
  return rsvd_run<float>(plan, nullptr, m, n, lda, k, p, q, t, omega, U, ldu, S, V, ldv, K, &lp);
}

int32_t quantize(rsvd_plan_t plan, int es, const float* A, int64_t m, int64_t n, int64_t lda,
                 void* Aq, int64_t ldq, float* col_scale) {
  if (!plan || !A || !Aq || !col_scale) return RSVD_ERR_ARG;
  if (m < 1 || n < 1 || lda < n || ldq < n) return RSVD_ERR_ARG;
  if (m > plan->m_max || n > plan->n_max) return RSVD_ERR_SHAPE;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  unsigned* cmax = reinterpret_cast<unsigned*>(plan->part);
  if (es == 2)
    RSVD_CHECK(launch_quantize_bf16(A, m, n, lda, (__bf16*)Aq, ldq, col_scale, cmax, plan->stream));
  else
    RSVD_CHECK(launch_quantize_fp8(A, m, n, lda, Aq, ldq, col_scale, cmax, plan->stream));
  return RSVD_OK;
}
}  // namespace

extern "C" {

int32_t rsvd_solve_bf16(rsvd_plan_t plan, const void* A, const float* col_scale, int64_t m,
                        int64_t n, int64_t lda, int32_t k, int32_t p, int32_t q, double t,
                        const double* omega, float* U, int64_t ldu, double* S, float* V,
                        int64_t ldv, int32_t* K) {
  return solve_lowp(plan, RSVD_BF16, A, col_scale, m, n, lda, k, p, q, t, omega, U, ldu, S, V,
                    ldv, K);
}

int32_t rsvd_solve_fp8(rsvd_plan_t plan, const void* A, const float* col_scale, int64_t m,
                       int64_t n, int64_t lda, int32_t k, int32_t p, int32_t q, double t,
                       const double* omega, float* U, int64_t ldu, double* S, float* V,
                       int64_t ldv, int32_t* K) {
  return solve_lowp(plan, RSVD_FP8, A, col_scale, m, n, lda, k, p, q, t, omega, U, ldu, S, V,
                    ldv, K);
}

int32_t rsvd_quantize_bf16(rsvd_plan_t plan, const float* A, int64_t m, int64_t n, int64_t lda,
                           void* Aq, int64_t ldq, float* col_scale) {
  return quantize(plan, 2, A, m, n, lda, Aq, ldq, col_scale);
}

int32_t rsvd_quantize_fp8(rsvd_plan_t plan, const float* A, int64_t m, int64_t n, int64_t lda,
                          void* Aq, int64_t ldq, float* col_scale) {
  return quantize(plan, 1, A, m, n, lda, Aq, ldq, col_scale);
}

int32_t rsvd_solve_krylov(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                          int32_t k, int32_t p, int32_t i, double t, const double* omega,
                          void* U, int64_t ldu, double* S, void* V, int64_t ldv, int32_t* K) {
  int32_t rc = check_rsvd(plan, A, m, n, lda, k, p, 0, t, U, ldu, S, V, ldv, K);
  if (rc != RSVD_OK) return rc;
  if (i < 0 || lowp_es(plan->dtype)) return RSVD_ERR_ARG;
  const int64_t l = (k + (int64_t)p < n) ? k + p : n;
  const int64_t L = (i + 1) * l;
  if (L > n) return RSVD_ERR_ARG;                  // the panel must have at most n columns
  if (L > plan->l_max) return RSVD_ERR_SHAPE;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  if (plan->dtype == RSVD_F64)
    return krylov_run<double>(plan, (const double*)A, m, n, lda, k, p, i, t, omega, (double*)U,
                              ldu, S, (double*)V, ldv, K);
  return krylov_run<float>(plan, (const float*)A, m, n, lda, k, p, i, t, omega, (float*)U, ldu,
                           S, (float*)V, ldv, K);
}

int32_t rsvd_solve_adaptive(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                            const float* col_scale, int32_t k, int32_t p, int32_t q, double t,
                            int32_t k_max, void* U, int64_t ldu, double* S, void* V, int64_t ldv,
                            int32_t* K) {
  int32_t rc = check_rsvd(plan, A, m, n, lda, k, p, q, t, U, ldu, S, V, ldv, K);
  if (rc != RSVD_OK) return rc;
  if (k_max < k || k_max > n || ldu < k_max || ldv < k_max) return RSVD_ERR_ARG;
  const int64_t b = (k + (int64_t)p < n) ? k + (int64_t)p : n;
  if (2 * ldq1_of(b) > plan->l_max) return RSVD_ERR_SHAPE;
  const int es = lowp_es(plan->dtype);
  if (!es && col_scale) return RSVD_ERR_ARG;
  if (es && !bf16_pass_applies(A, es, n, lda, (int)b)) return RSVD_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  GrowJob g;
  g.A = A; g.m = m; g.n = n; g.lda = lda;
  g.lp = LowpA{es ? A : nullptr, col_scale, es};
  g.b = (int)b; g.q = q; g.kcap = k_max; g.t = t;
  g.U = U; g.ldu = ldu; g.S = S; g.V = V; g.ldv = ldv; g.K = K;
  if ((rc = grow_block(plan, g)) != RSVD_OK) return rc;
  while (grow_fits(plan, g)) {
    double f2 = 0.0, e = 0.0;
    if ((rc = grow_read(plan, &f2, &e)) != RSVD_OK) return rc;
    if (!(e < t * f2)) break;        // reached (a NaN stops the growth as well)
    if ((rc = grow_block(plan, g)) != RSVD_OK) return rc;
  }
  return grow_finish(plan, g);
}

int32_t rsvd_solve(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                   const float* col_scale, int32_t k, int32_t p, int32_t q, double t, void* U,
                   int64_t ldu, double* S, void* V, int64_t ldv, int32_t* K) {
  return rsvd_solve_omega(plan, A, m, n, lda, col_scale, k, p, q, t, nullptr, U, ldu, S, V, ldv,
                          K);
}

int32_t gram_eig_solve(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                       double t, int32_t ucols, void* U, int64_t ldu, double* S, void* V,
                       int64_t ldv, int32_t* K) {
  int32_t rc = check_common(plan, A, m, n, lda);
  if (rc != RSVD_OK) return rc;
  if (!plan->gram) return RSVD_ERR_SHAPE;
  if (!S || !V || !K || bad_t(t) || ucols < 0 || ucols > n || ldv < n) return RSVD_ERR_ARG;
  if (ucols > 0 && (!U || ldu < ucols)) return RSVD_ERR_ARG;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  if (plan->dtype == RSVD_F64)
    return gram_run<double>(plan, (const double*)A, m, n, lda, t, ucols, (double*)U, ldu, S,
                            (double*)V, ldv, K);
  return gram_run<float>(plan, (const float*)A, m, n, lda, t, ucols, (float*)U, ldu, S, (float*)V,
                         ldv, K);
}

int32_t rsvd_gaussian_fill(uint64_t seed, int64_t rows, int64_t cols, double* G, void* stream) {
  if (!G || rows < 0 || cols < 0) return RSVD_ERR_ARG;
  RSVD_CHECK(launch_gaussian_fill(seed, rows, cols, G, (hipStream_t)stream));
  return RSVD_OK;
}

int32_t rsvd_gemm_nn(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                     const void* X, int64_t ldx, int32_t c, void* Y, int64_t ldy, double* Gram,
                     double* fro2) {
  if (!plan || !A || !X || !Y) return RSVD_ERR_ARG;
  if (m < 1 || n < 1 || c < 1 || lda < n || ldx < c || ldy < c) return RSVD_ERR_ARG;
  const int64_t cmax = plan->gram ? (plan->n_max > plan->l_max ? plan->n_max : plan->l_max)
                                  : plan->l_max;
  if (m > plan->m_max || c > cmax || (Gram && c > plan->l_max)) return RSVD_ERR_SHAPE;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  hipStream_t s = plan->stream;
  int np = 0;
  if (plan->dtype == RSVD_F64) {
    RSVD_CHECK(launch_gemm_nn<double>((const double*)A, m, n, lda, (const double*)X, ldx, c,
                                      (double*)Y, ldy, fro2 ? plan->fro2_part : nullptr, &np, s));
    if (Gram) RSVD_CHECK(Path<double>(plan).gram((const double*)Y, m, c, ldy, Gram));
  } else if (lowp_es(plan->dtype)) {
    // A bfloat16 or FP8 (unit column scales), X and Y float: X through FP64
    // into the hi + lo bf16 pairs the pass takes
    const int es = lowp_es(plan->dtype);
    if (c > plan->l_max) return RSVD_ERR_SHAPE;
    if (!bf16_pass_applies(A, es, n, lda, c)) return RSVD_ERR_ARG;
    RSVD_CHECK(launch_cast_to_f64<float>((const float*)X, n, c, ldx, plan->Zd, c, s));
    __bf16* Xhi = reinterpret_cast<__bf16*>(plan->Xs);
    __bf16* Xlo = Xhi + n * c;
    RSVD_CHECK(launch_cast_hilo_t(plan->Zd, n, c, nullptr, Xhi, Xlo, n, s));
    {
      KtScope ts(plan, KT_PASS_NN);
      RSVD_CHECK(launch_gemm_nt_bf16(A, es, m, n, lda, Xhi, Xlo, n, c, nullptr,
                                     (float*)Y, ldy, fro2 ? plan->fro2_part : nullptr, &np, s));
    }
    if (Gram) RSVD_CHECK(Path<float>(plan).gram((const float*)Y, m, c, ldy, Gram));
  } else {
    if (c > 128 && !fro2 && n <= plan->n_max) {
      // wide product: X transposed into plan scratch (c x n <= cmax x n_max)
      RSVD_CHECK(launch_transpose_f32((const float*)X, n, c, ldx, (float*)plan->Xs, n, s));
      KtScope ts(plan, KT_NT_WIDE);
      RSVD_CHECK(launch_gemm_nt_wide((const float*)A, m, n, lda, (const float*)plan->Xs, n, c,
                                     (float*)Y, ldy, s));
    } else if (c <= 128 && n <= plan->n_max &&
               nt_tall_applies((const float*)A, n, lda, (const float*)plan->Xs, n, c)) {
      RSVD_CHECK(launch_transpose_f32((const float*)X, n, c, ldx, (float*)plan->Xs, n, s));
      KtScope ts(plan, KT_PASS_NN);
      RSVD_CHECK(launch_gemm_nt_tall((const float*)A, m, n, lda, (const float*)plan->Xs, n, c,
                                     (float*)Y, ldy, fro2 ? plan->fro2_part : nullptr, &np, s));
    } else {
      RSVD_CHECK(launch_gemm_nn<float>((const float*)A, m, n, lda, (const float*)X, ldx, c,
                                       (float*)Y, ldy, fro2 ? plan->fro2_part : nullptr, &np, s));
    }
    if (Gram) RSVD_CHECK(Path<float>(plan).gram((const float*)Y, m, c, ldy, Gram));
  }
  if (fro2) RSVD_CHECK(launch_reduce_scalar(plan->fro2_part, np, fro2, s));
  return RSVD_OK;
}

int32_t rsvd_gemm_tn(rsvd_plan_t plan, const void* A, int64_t m, int64_t n, int64_t lda,
                     const void* Q, int64_t ldq, int32_t c, double* Z) {
  if (!plan || !A || !Q || !Z) return RSVD_ERR_ARG;
  if (m < 1 || n < 1 || c < 1 || lda < n || ldq < c) return RSVD_ERR_ARG;
  const int64_t cmax = plan->gram ? (plan->n_max > plan->l_max ? plan->n_max : plan->l_max)
                                  : plan->l_max;
  if (m > plan->m_max || n > plan->n_max || c > cmax) return RSVD_ERR_SHAPE;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  if (plan->dtype == RSVD_F64)
    RSVD_CHECK(Path<double>(plan).tn((const double*)A, m, n, lda, (const double*)Q, ldq, c, Z));
  else if (lowp_es(plan->dtype)) {
    // A bfloat16 or FP8 (unit column scales): Q copied into the plan's padded rows
    const int es = lowp_es(plan->dtype);
    if (c > plan->l_max) return RSVD_ERR_SHAPE;
    if (!bf16_pass_applies(A, es, n, lda, c)) return RSVD_ERR_ARG;
    const int64_t lq = ldq1_of(c);
    if (hipMemcpy2DAsync(plan->Q1, lq * sizeof(float), Q, ldq * sizeof(float), c * sizeof(float),
                         m, hipMemcpyDeviceToDevice, plan->stream) != hipSuccess)
      return RSVD_ERR_DEVICE;
    RSVD_CHECK(Path<float>(plan).tn_bf16(LowpA{A, nullptr, es}, m, n, lda,
                                         (const float*)plan->Q1, lq, c, Z));
  } else
    RSVD_CHECK(Path<float>(plan).tn((const float*)A, m, n, lda, (const float*)Q, ldq, c, Z));
  return RSVD_OK;
}

int32_t rsvd_cholqr2(rsvd_plan_t plan, const void* Y, int64_t m, int32_t c, int64_t ldy, void* Q,
                     int64_t ldq, double* R) {
  if (!plan || !Y || !Q || !R) return RSVD_ERR_ARG;
  if (c < 1 || m < c || ldy < c || ldq < c) return RSVD_ERR_ARG;
  if (m > plan->m_max || c > plan->l_max) return RSVD_ERR_SHAPE;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  hipStream_t s = plan->stream;
  RSVD_CHECK(reset(plan));
  if (plan->dtype == RSVD_F64) {
    Path<double> P(plan);
    RSVD_CHECK(P.cqr2((const double*)Y, m, c, ldy, (double*)plan->Q1, c, plan->R1, plan->R1inv,
                      plan->R2, plan->R2inv, (double*)plan->RinvT, 0));
    RSVD_CHECK(P.times_rinv((const double*)plan->Q1, m, c, c, (const double*)plan->RinvT, false,
                            (double*)Q, ldq));
  } else {
    Path<float> P(plan);
    const bool tall = P.times_rinv_tall((const float*)plan->Q1, c, c, (const float*)plan->RinvT);
    RSVD_CHECK(P.cqr2((const float*)Y, m, c, ldy, (float*)plan->Q1, c, plan->R1, plan->R1inv,
                      plan->R2, plan->R2inv, (float*)plan->RinvT, tall));
    RSVD_CHECK(P.times_rinv((const float*)plan->Q1, m, c, c, (const float*)plan->RinvT, tall,
                            (float*)Q, ldq));
  }
  RSVD_CHECK(launch_small_gemm<double>(plan->R2, plan->R1, c, c, c, R, nullptr, s));
  return RSVD_OK;
}

int32_t rsvd_small_svd(rsvd_plan_t plan, const double* T, int64_t r, int32_t c, double* Vt,
                       double* S, double* W) {
  if (!plan || !T || !Vt || !S || !W) return RSVD_ERR_ARG;
  if (c < 1 || r < c) return RSVD_ERR_ARG;
  if (r > plan->n_max || c > plan->l_max) return RSVD_ERR_SHAPE;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  RSVD_CHECK(reset(plan));
  RSVD_CHECK(small_svd_unsorted(plan, T, r, c, true));
  RSVD_CHECK(launch_sort_sign_scatter<double>(plan->Su, c, plan->Vt, r, c, 1, plan->Uo, c, S,
                                              nullptr, 0, Vt, W, plan->stream));
  return RSVD_OK;
}

int32_t rsvd_sym_eig(rsvd_plan_t plan, const double* G, int64_t n, double* lam, double* V) {
  if (!plan || !G || !lam || !V) return RSVD_ERR_ARG;
  if (n < 1) return RSVD_ERR_ARG;
  if (!plan->gram || n > plan->n_max) return RSVD_ERR_SHAPE;
  if (hipSetDevice(plan->device) != hipSuccess) return RSVD_ERR_DEVICE;
  hipStream_t s = plan->stream;
  RSVD_CHECK(reset(plan));
  hipLaunchKernelGGL(k_init_eig, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, G, n,
                     plan->Xe, plan->Je);
  RSVD_CHECK(hipGetLastError());
  const KtPair tp = kt_reserve(plan, KT_EIG);
  RSVD_CHECK(launch_jacobi_eig(plan->Xe, plan->Je, n, plan->lam, plan->diag, plan->flags,
                               plan->Es, plan->status, s, -1, tp.e0, tp.e1));
  RSVD_CHECK(launch_sort_sign_scatter<double>(plan->lam, (int)n, plan->Je, n, 1, n, nullptr,
                                              (int)n, lam, nullptr, 0, V, nullptr, s));
  return RSVD_OK;
}

}  // extern "C"

// ===========================================================================
// Batches: instances of different shapes on several slots (a plan and a
// stream each), forked from and joined back into the caller's stream.
struct rsvd_batch_s {
  int device = 0;
  int dtype = RSVD_F32;
  std::vector<rsvd_plan_s*> plan;
  std::vector<hipStream_t> stream;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;   // stream the graph captures are recorded on
};

struct rsvd_batch_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kMaxSlots = 64;

__global__ void k_status_take(const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// The storage dtype of an instance's A on a slot plan: its own, or the plan's.
int instance_dtype(const rsvd_plan_s* p, const rsvd_instance& x) {
  return x.dtype ? x.dtype : p->dtype;
}

// Validate one instance for a slot plan (as rsvd_solve / rsvd_solve_bf16).
int32_t check_instance(rsvd_plan_s* p, const rsvd_instance& x) {
  // U may be NULL (S, V and K only); its leading dimension is then unused
  const void* u = x.U ? x.U : x.A;
  const int64_t ldu = x.U ? x.ldu : (int64_t)(x.k_max > x.k ? x.k_max : x.k);
  const int32_t rc = check_rsvd(p, x.A, x.m, x.n, x.lda, x.k, x.p, x.q, x.t, u, ldu, x.S,
                                x.V, x.ldv, x.K);
  if (rc != RSVD_OK) return rc;
  if (!x.status) return RSVD_ERR_ARG;
  const int dt = instance_dtype(p, x);
  if ((p->dtype == RSVD_F64) != (dt == RSVD_F64)) return RSVD_ERR_ARG;
  if (dt != RSVD_F64 && dt != RSVD_F32 && !lowp_es(dt)) return RSVD_ERR_ARG;
  if (const int es = lowp_es(dt)) {
    const int l = (int)((x.k + (int64_t)x.p < x.n) ? x.k + x.p : x.n);
    if (!bf16_pass_applies(x.A, es, x.n, x.lda, l)) return RSVD_ERR_ARG;
  }
  return RSVD_OK;
}

// Enqueue one instance's solve and its status copy on the slot plan's stream.
int32_t run_instance(rsvd_plan_s* p, const rsvd_instance& x) {
  int32_t rc;
  if (p->dtype == RSVD_F64) {
    rc = rsvd_run<double>(p, (const double*)x.A, x.m, x.n, x.lda, x.k, x.p, x.q, x.t, nullptr,
                          (double*)x.U, x.ldu, x.S, (double*)x.V, x.ldv, x.K);
  } else if (const int es = lowp_es(instance_dtype(p, x))) {
    const LowpA lp{x.A, x.col_scale, es};
    rc = rsvd_run<float>(p, nullptr, x.m, x.n, x.lda, x.k, x.p, x.q, x.t, nullptr, (float*)x.U,
                         x.ldu, x.S, (float*)x.V, x.ldv, x.K, &lp);
  } else {
    rc = rsvd_run<float>(p, (const float*)x.A, x.m, x.n, x.lda, x.k, x.p, x.q, x.t, nullptr,
                         (float*)x.U, x.ldu, x.S, (float*)x.V, x.ldv, x.K);
  }
  if (rc != RSVD_OK) return rc;
  hipLaunchKernelGGL(k_status_take, dim3(1), dim3(64), 0, p->stream, p->status, x.status);
  RSVD_CHECK(hipGetLastError());
  return RSVD_OK;
}

void batch_free(rsvd_batch_s* b) {
  (void)hipSetDevice(b->device);
  for (rsvd_plan_s* p : b->plan) rsvd_plan_destroy(p);   // synchronises its stream
  for (hipStream_t s : b->stream) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

// Validate every instance, then give each a slot: largest work (m n l)
// first, each to the slot with the least work so far (lowest index on ties).
int32_t batch_schedule(rsvd_batch_s* b, const rsvd_instance* in, int32_t count,
                       std::vector<int>& order, std::vector<int>& slot) {
  if (count < 0 || (count > 0 && !in)) return RSVD_ERR_ARG;
  std::vector<double> work(count);
  for (int i = 0; i < count; ++i) {
    const rsvd_instance& x = in[i];
    const int32_t rc = check_instance(b->plan[0], x);
    if (rc != RSVD_OK) return rc;
    const int64_t l = (x.k + (int64_t)x.p < x.n) ? x.k + (int64_t)x.p : x.n;
    work[i] = (double)x.m * (double)x.n * (double)l;
  }
  order.resize(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
  std::vector<double> load(b->plan.size(), 0.0);
  slot.assign(count, 0);
  for (int i : order) {
    int best = 0;
    for (int s = 1; s < (int)load.size(); ++s)
      if (load[s] < load[best]) best = s;
    slot[i] = best;
    load[best] += work[i];
  }
  return RSVD_OK;
}

int32_t batch_launch(rsvd_batch_s* b, const rsvd_instance* in, int32_t count, hipStream_t st) {
  std::vector<int> order, slot;
  int32_t rc = batch_schedule(b, in, count, order, slot);
  if (rc != RSVD_OK || count == 0) return rc;
  std::vector<char> used(b->plan.size(), 0);
  for (int i = 0; i < count; ++i) used[slot[i]] = 1;
  RSVD_CHECK(hipEventRecord(b->fork, st));
  for (size_t s = 0; s < used.size(); ++s)
    if (used[s]) RSVD_CHECK(hipStreamWaitEvent(b->stream[s], b->fork, 0));
  for (int i : order) {
    rc = run_instance(b->plan[slot[i]], in[i]);
    if (rc != RSVD_OK) return rc;
  }
  for (size_t s = 0; s < used.size(); ++s)
    if (used[s]) {
      RSVD_CHECK(hipEventRecord(b->done[s], b->stream[s]));
      RSVD_CHECK(hipStreamWaitEvent(st, b->done[s], 0));
    }
  return RSVD_OK;
}

int32_t batch_dispatch(rsvd_batch_s* b, const rsvd_instance* in, int32_t count, hipStream_t st) {
  return batch_launch(b, in, count, st);
}

}  // namespace

extern "C" {

int32_t rsvd_batch_create(rsvd_batch_t* batch, int32_t nslots, int64_t m_max, int64_t n_max,
                          int32_t l_max, int32_t dtype, uint64_t seed) {
  if (!batch) return RSVD_ERR_ARG;
  *batch = nullptr;
  if (nslots < 1 || nslots > kMaxSlots) return RSVD_ERR_ARG;
  if (dtype != RSVD_F64 && dtype != RSVD_F32 && !lowp_es(dtype)) return RSVD_ERR_ARG;
  rsvd_batch_s* b = new (std::nothrow) rsvd_batch_s();
  if (!b) return RSVD_ERR_NOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) { delete b; return RSVD_ERR_DEVICE; }
  b->dtype = dtype;
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    batch_free(b);
    return RSVD_ERR_DEVICE;
  }
  for (int s = 0; s < nslots; ++s) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      batch_free(b);
      return RSVD_ERR_DEVICE;
    }
    b->stream.push_back(st);
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      return RSVD_ERR_DEVICE;
    }
    b->done.push_back(ev);
    rsvd_plan_t p = nullptr;
    const int32_t rc = rsvd_plan_create(&p, m_max, n_max, l_max, dtype, 0, seed, st);
    if (rc != RSVD_OK) {
      batch_free(b);
      return rc;
    }
    b->plan.push_back(p);
  }
  *batch = b;
  return RSVD_OK;
}

int32_t rsvd_batch_destroy(rsvd_batch_t batch) {
  if (!batch) return RSVD_OK;
  batch_free(batch);
  return RSVD_OK;
}

int32_t rsvd_batch_solve(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                         void* stream) {
  if (!batch) return RSVD_ERR_ARG;
  if (hipSetDevice(batch->device) != hipSuccess) return RSVD_ERR_DEVICE;
  return batch_dispatch(batch, inst, count, (hipStream_t)stream);
}

int32_t rsvd_batch_graph_create(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                                void* stream, rsvd_batch_graph_t* graph) {
  (void)stream;   // a graph is launched on any stream; it is captured on the batch's own
  if (!batch || !graph) return RSVD_ERR_ARG;
  *graph = nullptr;
  if (hipSetDevice(batch->device) != hipSuccess) return RSVD_ERR_DEVICE;
  {  // validate before capturing anything
    std::vector<int> order, slot;
    const int32_t rc = batch_schedule(batch, inst, count, order, slot);
    if (rc != RSVD_OK) return rc;
    // sketches past kSmallSvdMaxC columns take a cooperative launch, which
    // is not put into a graph
    for (int i = 0; i < count; ++i)
      if (inst[i].k + (int64_t)inst[i].p > kSmallSvdMaxC && inst[i].n > kSmallSvdMaxC)
        return RSVD_ERR_SHAPE;
  }
  if (hipStreamBeginCapture(batch->cap, hipStreamCaptureModeRelaxed) != hipSuccess)
    return RSVD_ERR_DEVICE;
  const int32_t rc = batch_dispatch(batch, inst, count, batch->cap);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(batch->cap, &g);
  if (rc != RSVD_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc != RSVD_OK ? rc : RSVD_ERR_DEVICE;
  }
  rsvd_batch_graph_s* h = new (std::nothrow) rsvd_batch_graph_s();
  if (!h) {
    (void)hipGraphDestroy(g);
    return RSVD_ERR_NOMEM;
  }
  h->graph = g;
  if (hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete h;
    return RSVD_ERR_DEVICE;
  }
  *graph = h;
  return RSVD_OK;
}

int32_t rsvd_batch_graph_launch(rsvd_batch_graph_t graph, void* stream) {
  if (!graph) return RSVD_ERR_ARG;
  return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? RSVD_OK
                                                                      : RSVD_ERR_DEVICE;
}

int32_t rsvd_batch_graph_destroy(rsvd_batch_graph_t graph) {
  if (!graph) return RSVD_OK;
  int32_t rc = RSVD_OK;
  if (graph->exec && hipGraphExecDestroy(graph->exec) != hipSuccess) rc = RSVD_ERR_DEVICE;
  if (graph->graph && hipGraphDestroy(graph->graph) != hipSuccess) rc = RSVD_ERR_DEVICE;
  delete graph;
  return rc;
}

}  // extern "C"

// ===========================================================================
// Serving: requests queued in arrival order, admitted first come first
// served onto free slots while their footprints fit the HBM budget, retired
// by polling each busy slot's completion event.  A request with k_max > k
// grows its basis block by block on its slot (the steps of
// rsvd_solve_adaptive; after each block the captured energy decides: finish,
// grow again, or, with the fallback, move to the A^T A-route slot).
struct rsvd_server_s {
  enum Phase { kIdle = 0, kPlain, kGrow, kFinish };
  struct Req {
    rsvd_instance x;
    int64_t ticket = 0;
    int64_t bytes = 0;
    GrowJob g;
    double e_prev = 0.0;   // energy after the previous block
  };
  rsvd_batch_s* b = nullptr;
  int64_t budget = 0, in_use = 0, next_ticket = 0;
  std::deque<Req> queue;
  std::vector<int64_t> slot_ticket;   // -1: free
  std::vector<int> slot_phase;
  std::vector<Req> slot_req;
  std::deque<int64_t> finished;
  // A^T A-route slots (RSVD_SERVER_GRAM_FALLBACK)
  struct GramSlot {
    rsvd_plan_s* plan = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    float* buf = nullptr;   // fp32 copy of a bfloat16 / FP8 request's A
    bool busy = false;
    Req req;
  };
  std::vector<GramSlot> gslot;
  std::deque<Req> gqueue;
};

// A^T A-route slots of a server created with RSVD_SERVER_GRAM_FALLBACK.
constexpr int kGramSlots = 2;

namespace {

int64_t request_bytes(const rsvd_server_s* sv, const rsvd_instance& x) {
  const int dt = instance_dtype(sv->b->plan[0], x);
  const int64_t ea = dt == RSVD_F64 ? 8 : (lowp_es(dt) ? lowp_es(dt) : 4);   // A's elements
  const int64_t ep = dt == RSVD_F64 ? 8 : 4;                                  // the panels'
  const int64_t l = (x.k_max > x.k) ? sv->b->plan[0]->l_max
                                    : ((x.k + (int64_t)x.p < x.n) ? x.k + (int64_t)x.p : x.n);
  return x.m * x.lda * ea + 2 * x.m * l * ep + tn_max_split(x.m, x.n, (int)l) * x.n * l * 8;
}

bool grows(const rsvd_instance& x) { return x.k_max > x.k; }

GrowJob grow_job(const rsvd_plan_s* p, const rsvd_instance& x) {
  GrowJob g;
  const int es = lowp_es(instance_dtype(p, x));
  g.A = x.A; g.m = x.m; g.n = x.n; g.lda = x.lda;
  g.lp = LowpA{es ? x.A : nullptr, x.col_scale, es};
  g.b = (int)((x.k + (int64_t)x.p < x.n) ? x.k + (int64_t)x.p : x.n);
  g.q = x.q; g.kcap = x.k_max; g.t = x.t;
  g.U = x.U; g.ldu = x.ldu; g.S = x.S; g.V = x.V; g.ldv = x.ldv; g.K = x.K;
  return g;
}

// The A^T A route for one request on the fallback slot: all n eigenpairs
// (gram_run's steps), K over all n values capped at k_max, the first k_max
// sorted triplets written to the request's U, S, V.
template <typename T>
int32_t gram_run_capped(rsvd_plan_s* p, const T* A, int64_t m, int64_t n, int64_t lda, double t,
                        int kcap, T* U, int64_t ldu, double* S, T* V, int64_t ldv, int32_t* K) {
  hipStream_t s = p->stream;
  Path<T> P(p);
  RSVD_CHECK(reset(p));
  if (std::is_same<T, float>::value &&
      syrk_f32_applies(reinterpret_cast<const float*>(A), n, lda)) {
    RSVD_CHECK(launch_syrk_f32(reinterpret_cast<const float*>(A), m, n, lda, p->part,
                               p->max_split * p->n_max * p_cmax(p), p->Gd, s));
  } else {
    RSVD_CHECK(P.tn(A, m, n, lda, A, lda, (int)n, p->Gd));
  }
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, p->Gd, n, p->scal);
  RSVD_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_init_eig, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, p->Gd, n,
                     p->Xe, p->Je);
  RSVD_CHECK(hipGetLastError());
  RSVD_CHECK(launch_jacobi_eig(p->Xe, p->Je, n, p->lam, p->diag, p->flags, p->Es, p->status, s));
  RSVD_CHECK(launch_sqrt_clamp(p->lam, (int)n, p->Se, s));
  // all n values sorted (into Es, free after the eigensolver) and V in FP64
  RSVD_CHECK(launch_sort_sign_scatter<T>(p->Se, (int)n, p->Je, n, 1, n, nullptr, (int)n, p->Es,
                                         nullptr, 0, p->Vd, nullptr, s));
  const int kc = (int)(kcap < n ? kcap : n);
  hipLaunchKernelGGL((k_copy2d<double>), dim3(grid_for(kc)), dim3(256), 0, s, p->Es, (int64_t)kc,
                     S, (int64_t)kc, (int64_t)1, kc);
  RSVD_CHECK(hipGetLastError());
  RSVD_CHECK(launch_cast_from_f64<T>(p->Vd, n, kc, n, V, ldv, s));
  // u_i = A v_i / s_i for the first kc columns
  const double floor_rel = (double)(m > n ? m : n) * 2.220446049250313e-16;
  if (!U) {
    // S, V and K only
  } else if (std::is_same<T, float>::value && kc > 128) {
    RSVD_CHECK(launch_scale_cols_inv<T>(p->Vd, n, kc, n, p->Es, floor_rel, (T*)p->Xs, n, 1, s));
    RSVD_CHECK(launch_gemm_nt_wide(reinterpret_cast<const float*>(A), m, n, lda,
                                   reinterpret_cast<const float*>(p->Xs), n, kc,
                                   reinterpret_cast<float*>(U), ldu, s));
  } else {
    RSVD_CHECK(launch_scale_cols_inv<T>(p->Vd, n, kc, n, p->Es, floor_rel, (T*)p->Xs, kc, 0, s));
    RSVD_CHECK(launch_gemm_nn<T>(A, m, n, lda, (const T*)p->Xs, kc, kc, U, ldu, nullptr, nullptr,
                                 s));
  }
  RSVD_CHECK(launch_select_k(p->Es, (int)n, p->scal, t, K, p->diag, p->status, s));
  hipLaunchKernelGGL(k_cap_k, dim3(1), dim3(64), 0, s, K, kcap, p->status, p->diag);
  RSVD_CHECK(hipGetLastError());
  return RSVD_OK;
}

int32_t gram_admit_one(rsvd_server_s* sv, rsvd_server_s::GramSlot& gs) {
  rsvd_server_s::Req r = sv->gqueue.front();
  sv->gqueue.pop_front();
  rsvd_plan_s* p = gs.plan;
  const rsvd_instance& x = r.x;
  int32_t rc;
  if (p->dtype == RSVD_F64) {
    rc = gram_run_capped<double>(p, (const double*)x.A, x.m, x.n, x.lda, x.t, x.k_max,
                                 (double*)x.U, x.ldu, x.S, (double*)x.V, x.ldv, x.K);
  } else {
    const float* A32 = (const float*)x.A;
    int64_t lda = x.lda;
    if (const int es = lowp_es(instance_dtype(sv->b->plan[0], x))) {
      RSVD_CHECK(launch_dequantize(x.A, es, x.m, x.n, x.lda, x.col_scale, gs.buf, x.n,
                                   gs.stream));
      A32 = gs.buf;
      lda = x.n;
    }
    rc = gram_run_capped<float>(p, A32, x.m, x.n, lda, x.t, x.k_max, (float*)x.U, x.ldu, x.S,
                                (float*)x.V, x.ldv, x.K);
  }
  if (rc != RSVD_OK) return rc;
  hipLaunchKernelGGL(k_status_take, dim3(1), dim3(64), 0, gs.stream, p->status, x.status);
  RSVD_CHECK(hipGetLastError());
  RSVD_CHECK(hipEventRecord(gs.done, gs.stream));
  gs.busy = true;
  gs.req = r;
  return RSVD_OK;
}

int32_t gram_admit(rsvd_server_s* sv) {
  for (auto& gs : sv->gslot) {
    if (sv->gqueue.empty()) break;
    if (gs.busy) continue;
    const int32_t rc = gram_admit_one(sv, gs);
    if (rc != RSVD_OK) return rc;
  }
  return RSVD_OK;
}

// Admit from the head of the queue while a slot is free and the head fits
// the budget (or nothing runs).
int32_t server_admit(rsvd_server_s* sv) {
  rsvd_batch_s* b = sv->b;
  while (!sv->queue.empty()) {
    int s = -1;
    for (int i = 0; i < (int)sv->slot_ticket.size(); ++i)
      if (sv->slot_ticket[i] < 0) { s = i; break; }
    if (s < 0) break;
    rsvd_server_s::Req& r = sv->queue.front();
    if (sv->in_use > 0 && sv->in_use + r.bytes > sv->budget) break;
    int32_t rc;
    if (grows(r.x)) {
      r.g = grow_job(b->plan[s], r.x);
      r.e_prev = 0.0;
      rc = grow_block(b->plan[s], r.g);
      sv->slot_phase[s] = rsvd_server_s::kGrow;
    } else {
      rc = run_instance(b->plan[s], r.x);
      sv->slot_phase[s] = rsvd_server_s::kPlain;
    }
    if (rc != RSVD_OK) return rc;
    RSVD_CHECK(hipEventRecord(b->done[s], b->stream[s]));
    sv->slot_ticket[s] = r.ticket;
    sv->slot_req[s] = r;
    sv->in_use += r.bytes;
    sv->queue.pop_front();
  }
  return gram_admit(sv);
}

// After a block of a growing request on slot s: finish it, grow again, or
// move it to the A^T A-route slot.
int32_t grow_next(rsvd_server_s* sv, int s) {
  rsvd_batch_s* b = sv->b;
  rsvd_plan_s* p = b->plan[s];
  rsvd_server_s::Req& r = sv->slot_req[s];
  double f2 = 0.0, e = 0.0;
  int32_t rc = grow_read(p, &f2, &e);   // the slot's stream is idle: returns at once
  if (rc != RSVD_OK) return rc;
  const double need = r.x.t * f2;
  const bool fits = grow_fits(p, r.g);
  if (e < need) {
    // K predicted from the energy per column of the last block (a lower
    // estimate: later columns capture less on a decaying spectrum)
    const double per_col = (e - r.e_prev) / r.g.b;
    const double kpred = per_col > 0.0 ? r.g.L + (need - e) / per_col : 1e300;
    if (!sv->gslot.empty() && (kpred > 0.5 * r.x.n || !fits)) {
      sv->slot_ticket[s] = -1;
      sv->slot_phase[s] = rsvd_server_s::kIdle;
      sv->gqueue.push_back(r);   // its bytes stay counted until it is done
      return RSVD_OK;
    }
    if (fits) {
      r.e_prev = e;
      if ((rc = grow_block(p, r.g)) != RSVD_OK) return rc;
      RSVD_CHECK(hipEventRecord(b->done[s], b->stream[s]));
      return RSVD_OK;
    }
  }
  if ((rc = grow_finish(p, r.g)) != RSVD_OK) return rc;
  hipLaunchKernelGGL(k_status_take, dim3(1), dim3(64), 0, p->stream, p->status, r.x.status);
  RSVD_CHECK(hipGetLastError());
  RSVD_CHECK(hipEventRecord(b->done[s], b->stream[s]));
  sv->slot_phase[s] = rsvd_server_s::kFinish;
  return RSVD_OK;
}

// Retire the busy slots whose completion event has fired (a growing
// request takes its next step instead), and the A^T A-route slot.
int32_t server_retire(rsvd_server_s* sv, bool wait) {
  rsvd_batch_s* b = sv->b;
  for (int s = 0; s < (int)sv->slot_ticket.size(); ++s) {
    if (sv->slot_ticket[s] < 0) continue;
    const hipError_t e = wait ? hipEventSynchronize(b->done[s]) : hipEventQuery(b->done[s]);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return RSVD_ERR_DEVICE;
    if (sv->slot_phase[s] == rsvd_server_s::kGrow) {
      const int32_t rc = grow_next(sv, s);
      if (rc != RSVD_OK) return rc;
      continue;
    }
    const rsvd_server_s::Req& r = sv->slot_req[s];
    sv->in_use -= r.bytes;
    sv->slot_ticket[s] = -1;
    sv->slot_phase[s] = rsvd_server_s::kIdle;
    sv->finished.push_back(r.ticket);
  }
  for (auto& gs : sv->gslot) {
    if (!gs.busy) continue;
    const hipError_t e = wait ? hipEventSynchronize(gs.done) : hipEventQuery(gs.done);
    if (e == hipSuccess) {
      gs.busy = false;
      sv->in_use -= gs.req.bytes;
      sv->finished.push_back(gs.req.ticket);
    } else if (e != hipErrorNotReady) {
      return RSVD_ERR_DEVICE;
    }
  }
  return RSVD_OK;
}

int32_t server_running(const rsvd_server_s* sv) {
  int32_t r = 0;
  for (int64_t t : sv->slot_ticket) r += t >= 0;
  for (const auto& gs : sv->gslot) r += gs.busy ? 1 : 0;
  return r;
}

void server_free(rsvd_server_s* sv) {
  if (sv->b) batch_free(sv->b);
  for (auto& gs : sv->gslot) {
    if (gs.plan) rsvd_plan_destroy(gs.plan);
    if (gs.buf) (void)hipFree(gs.buf);
    if (gs.done) (void)hipEventDestroy(gs.done);
    if (gs.stream) (void)hipStreamDestroy(gs.stream);
  }
  delete sv;
}

}  // namespace

extern "C" {

int32_t rsvd_server_create(rsvd_server_t* server, int32_t nslots, int64_t m_max, int64_t n_max,
                           int32_t l_max, int32_t dtype, uint64_t seed, int64_t hbm_budget,
                           int32_t flags) {
  if (!server) return RSVD_ERR_ARG;
  *server = nullptr;
  if (hbm_budget < 1 || (flags & ~RSVD_SERVER_GRAM_FALLBACK)) return RSVD_ERR_ARG;
  const bool fallback = (flags & RSVD_SERVER_GRAM_FALLBACK) != 0;
  if (fallback && n_max > jacobi_eig_max_n()) return RSVD_ERR_SHAPE;
  rsvd_batch_t b = nullptr;
  int32_t rc = rsvd_batch_create(&b, nslots, m_max, n_max, l_max, dtype, seed);
  if (rc != RSVD_OK) return rc;
  rsvd_server_s* sv = new (std::nothrow) rsvd_server_s();
  if (!sv) {
    batch_free(b);
    return RSVD_ERR_NOMEM;
  }
  sv->b = b;
  sv->budget = hbm_budget;
  sv->slot_ticket.assign(nslots, -1);
  sv->slot_phase.assign(nslots, rsvd_server_s::kIdle);
  sv->slot_req.assign(nslots, rsvd_server_s::Req());
  if (fallback) {
    sv->gslot.resize(kGramSlots);
    const int gdt = dtype == RSVD_F64 ? RSVD_F64 : RSVD_F32;
    const int32_t gl = (int32_t)(n_max < 8 ? n_max : 8);
    for (auto& gs : sv->gslot) {
      if (hipStreamCreateWithFlags(&gs.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&gs.done, hipEventDisableTiming) != hipSuccess) {
        server_free(sv);
        return RSVD_ERR_DEVICE;
      }
      if ((rc = rsvd_plan_create(&gs.plan, m_max, n_max, gl, gdt, 1, seed, gs.stream)) !=
          RSVD_OK) {
        gs.plan = nullptr;
        server_free(sv);
        return rc;
      }
      if (gdt == RSVD_F32 &&
          hipMalloc(&gs.buf, (size_t)m_max * (size_t)n_max * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        gs.buf = nullptr;
        server_free(sv);
        return RSVD_ERR_NOMEM;
      }
    }
  }
  *server = sv;
  return RSVD_OK;
}

int32_t rsvd_server_submit(rsvd_server_t server, const rsvd_instance* req, int64_t* ticket) {
  if (!server || !req || !ticket) return RSVD_ERR_ARG;
  const rsvd_instance& x = *req;
  rsvd_plan_s* p0 = server->b->plan[0];
  int32_t rc = check_instance(p0, x);
  if (rc != RSVD_OK) return rc;
  if (grows(x)) {   // outputs for k_max columns; two row-padded blocks within l_max
    if (x.k_max > x.n || (x.U && x.ldu < x.k_max) || x.ldv < x.k_max) return RSVD_ERR_ARG;
    const int64_t bw = (x.k + (int64_t)x.p < x.n) ? x.k + (int64_t)x.p : x.n;
    if (2 * ldq1_of(bw) > p0->l_max) return RSVD_ERR_SHAPE;
  }
  if (hipSetDevice(server->b->device) != hipSuccess) return RSVD_ERR_DEVICE;
  rsvd_server_s::Req r;
  r.x = x;
  r.ticket = server->next_ticket++;
  r.bytes = request_bytes(server, x);
  server->queue.push_back(r);
  *ticket = r.ticket;
  return server_admit(server);
}

int32_t rsvd_server_progress(rsvd_server_t server, int64_t* done, int32_t cap, int32_t* ndone,
                             int32_t* queued, int32_t* running) {
  if (!server || !ndone || cap < 0 || (cap > 0 && !done)) return RSVD_ERR_ARG;
  *ndone = 0;
  if (hipSetDevice(server->b->device) != hipSuccess) return RSVD_ERR_DEVICE;
  int32_t rc = server_retire(server, false);
  if (rc == RSVD_OK) rc = server_admit(server);
  while (*ndone < cap && !server->finished.empty()) {
    done[(*ndone)++] = server->finished.front();
    server->finished.pop_front();
  }
  if (queued) *queued = (int32_t)(server->queue.size() + server->gqueue.size());
  if (running) *running = server_running(server);
  return rc;
}

int32_t rsvd_server_destroy(rsvd_server_t server) {
  if (!server) return RSVD_OK;
  int32_t rc = RSVD_OK;
  if (hipSetDevice(server->b->device) != hipSuccess) rc = RSVD_ERR_DEVICE;
  while (rc == RSVD_OK && (!server->queue.empty() || !server->gqueue.empty() ||
                           server_running(server) > 0)) {
    rc = server_retire(server, true);
    if (rc == RSVD_OK) rc = server_admit(server);
  }
  server_free(server);
  return rc;
}

}  // extern "C"

// ===========================================================================
// Grouped batches: every step of Randomized PCA (Sec. 3.1.2) is one launch
// for all instances of a batch (blockIdx.y = instance), instead of one chain
// of launches per instance.  The argument records of all launches are built
// once, from the instances' shapes and pointers, and uploaded once; a launch
// of the grouped batch replays the recorded sequence.  Instances with the
// same sketch width l and rank k share launches (their kernels' template
// choices are the same); the groups run one after the other.
struct rsvd_grouped_s {
  struct Op {
    int kind = 0;
    size_t off = 0;
    int count = 0, maxblk = 0, a0 = 0, a1 = 0;
    size_t wl_off = 0;   // work list (GWork items) of the tall passes
    int nwork = 0;
    bool fuse = false;   // the fused-Gram kernels
  };
  int device = 0;
  char* ws = nullptr;          // the instances' workspaces
  char* args = nullptr;        // all argument records, device
  std::vector<rsvd_plan_s> plans;
  std::vector<Op> ops;
};

namespace {

enum GKind {
  G_RESET, G_FILL, G_CAST_T, G_TALL, G_NARROW, G_NARROW_TRI, G_RED_S, G_GRAM_F, G_GRAM_D, G_RED,
  G_CHOL_F, G_CHOL_D, G_TN, G_SG_F, G_SG_D, G_NN_D, G_JAC, G_JAC_ACC, G_SORT, G_SEL, G_TAKE
};

__global__ void k_status_grouped(const GArgStat* __restrict__ a) {
  const GArgStat& g = a[blockIdx.y];
  if (g.src) {
    if (threadIdx.x == 0) *g.dst = *g.src;
  } else {
    if (threadIdx.x == 0) *g.dst = RSVD_OK;
    if ((int)threadIdx.x < g.nd) g.diag[threadIdx.x] = 0.0;
  }
}

struct GroupedBuilder {
  std::vector<char> host;
  std::vector<rsvd_grouped_s::Op> ops;
  template <typename A>
  void add(int kind, const std::vector<A>& rec, int a0 = 0, int a1 = 0) {
    if (rec.empty()) return;
    rsvd_grouped_s::Op op;
    op.kind = kind;
    op.off = (host.size() + 63) / 64 * 64;
    op.count = (int)rec.size();
    op.a0 = a0;
    op.a1 = a1;
    int mb = 0;
    for (const A& r : rec) mb = r.nblk > mb ? r.nblk : mb;
    op.maxblk = mb;
    host.resize(op.off + rec.size() * sizeof(A));
    memcpy(host.data() + op.off, rec.data(), rec.size() * sizeof(A));
    ops.push_back(op);
  }
  // a tall pass: records plus its work list, whose items are ordered by
  // their records' cost (largest first; the items of one record in order)
  template <typename A>
  void add_wl(int kind, const std::vector<A>& rec, const std::vector<int>& items_per_rec,
              const std::vector<double>& cost, int a0, int a1, bool fuse) {
    if (rec.empty()) return;
    rsvd_grouped_s::Op op;
    op.kind = kind;
    op.off = (host.size() + 63) / 64 * 64;
    op.count = (int)rec.size();
    op.a0 = a0;
    op.a1 = a1;
    host.resize(op.off + rec.size() * sizeof(A));
    memcpy(host.data() + op.off, rec.data(), rec.size() * sizeof(A));
    std::vector<int> order(rec.size());
    for (size_t r = 0; r < rec.size(); ++r) order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<GWork> wl;
    for (int r : order)
      for (int it = 0; it < items_per_rec[r]; ++it) wl.push_back(GWork{r, it});
    op.wl_off = (host.size() + 63) / 64 * 64;
    op.nwork = (int)wl.size();
    op.fuse = fuse;
    host.resize(op.wl_off + wl.size() * sizeof(GWork));
    memcpy(host.data() + op.wl_off, wl.data(), wl.size() * sizeof(GWork));
    ops.push_back(op);
  }
};

// Tile parameters of one instance's tall passes: 128-row tiles per work
// item of the A X and Y R^-1 products, and the shortest row split of the
// A^T Q partial sums.
struct GTune {
  int tpp = (int)(kGroupedSplitRows / 128);
  int64_t split_rows = kGroupedSplitRows;
};

constexpr int64_t kTnTileCols = 512;   // columns of A per A^T Q block

int blocks256(int64_t total) { return (int)((total + 255) / 256); }

// Whether the grouped path takes this fp32 instance: the tall kernels'
// layout conditions for A, and a sketch width that is a multiple of 4.
// A tuning entry: rows per item a whole number of 128-row tiles and
// kGroupedSplitRows <= rows <= 2^20 for both (the per-instance partials are
// sized for splits of kGroupedSplitRows rows).
bool tune_entry_valid(const rsvd_tune_entry& t) {
  const int64_t lo = kGroupedSplitRows, hi = (int64_t)1 << 20;
  return t.n > 0 && t.l > 0 && t.panel_rows >= lo && t.panel_rows <= hi &&
         t.panel_rows % 128 == 0 && t.split_rows >= lo && t.split_rows <= hi &&
         t.split_rows % 16 == 0;
}

// The entry for an instance's (n, l), else the defaults.
GTune tune_for(const rsvd_instance& x, const rsvd_tune_entry* tune, int ntune) {
  GTune g;
  const int64_t l = (x.k + (int64_t)x.p < x.n) ? x.k + (int64_t)x.p : x.n;
  for (int t = 0; t < ntune; ++t)
    if (tune[t].n == x.n && tune[t].l == l) {
      g.tpp = tune[t].panel_rows / 128;
      g.split_rows = tune[t].split_rows;
      break;
    }
  return g;
}

bool grouped_applies(const rsvd_instance& x, int64_t max_split, const GTune& tu) {
  const int64_t l = (x.k + (int64_t)x.p < x.n) ? x.k + (int64_t)x.p : x.n;
  if (l > kSmallSvdMaxC) return false;       // the grouped small kernels hold l <= 96
  if (l % 4 != 0 || x.n % 4 != 0 || x.lda % 4 != 0) return false;
  if (reinterpret_cast<uintptr_t>(x.A) % 16 != 0) return false;
  if ((int64_t)128 * x.lda * 4 >= (1LL << 31)) return false;
  int ntile = 0;
  int64_t rps = 0;
  // the A^T Q splits record_group takes (32-bit buffer offsets within one)
  tn_tall_splits(x.m, x.n, max_split, &rps, &ntile, tu.split_rows);
  return rps * x.lda * 4 < (1LL << 31) && (int64_t)31 * x.lda * 4 + (int64_t)ntile * 512 * 4 < (1LL << 31);
}

// Record Randomized PCA (the steps and kernels of rsvd_run<float>) for the
// instances `ix` (same l and k) on their workspaces `pl`.
void record_group(GroupedBuilder& B, const rsvd_instance* in, const std::vector<int>& ix,
                  std::vector<rsvd_plan_s>& pl, const std::vector<GTune>& tune, int l, int k) {
  const int ntl = (l + 15) / 16;            // column tiles of l columns
  const int ntk = (k + 15) / 16;
  const int nsl = (l + 15) / 16;            // k slabs of an l-long contraction
  auto P = [&](int i) -> rsvd_plan_s& { return pl[i]; };
  auto X = [&](int i) -> const rsvd_instance& { return in[i]; };
  // the m-row Gram matrices come from the products that write Y and Q1
  // (fused epilogue) when l fits the fused kernels
  const bool fuse = ntl <= kGramFuseMaxNt;
  auto panels = [&](int i) {
    const int64_t nt = (X(i).m + 127) / 128;
    return (int)((nt + tune[i].tpp - 1) / tune[i].tpp);
  };
  auto gram_red = [&]() {   // the fused partials' fixed-order sum into Wg
    std::vector<GArgRed> rr;
    for (int i : ix)
      rr.push_back({P(i).part, panels(i), l, l, P(i).Wg, l, blocks256((int64_t)l * l)});
    B.add(G_RED, rr);
  };
  {
    std::vector<GArgStat> r;
    for (int i : ix) r.push_back({nullptr, P(i).status, P(i).diag, kDiagWords, 1});
    B.add(G_RESET, r);
  }
  {
    std::vector<GArgFill> r;
    for (int i : ix) {
      const int64_t tot = X(i).n * (int64_t)l;
      r.push_back({P(i).seed, tot, P(i).omega, blocks256((tot + 1) / 2)});
    }
    B.add(G_FILL, r);
  }
  // A X (X FP64, n x l) into Y; with fro2 on the first pass, and the Gram
  // matrix Y^T Y when fused
  auto pass_nn = [&](bool first, bool from_zq) {
    std::vector<GArgCast> rc;
    for (int i : ix) {
      const int64_t n = X(i).n;
      rc.push_back({from_zq ? P(i).Zq : P(i).omega, n, l, l, P(i).Xs, n, blocks256(n * l)});
    }
    B.add(G_CAST_T, rc);
    std::vector<GArgTall> rt;
    std::vector<int> it;
    std::vector<double> ct;
    std::vector<std::vector<GArgNarrow>> rn(7);
    std::vector<std::vector<int>> itn(7);
    std::vector<std::vector<double>> cn(7);
    for (int i : ix) {
      const rsvd_instance& x = X(i);
      double* gm = fuse ? P(i).part : nullptr;
      if (first || x.n > 96) {
        rt.push_back({(const float*)x.A, x.m, x.n, x.lda, (const float*)P(i).Xs, x.n, l,
                      (float*)P(i).Y, l, first ? P(i).fro2_part : nullptr, gm, tune[i].tpp});
        it.push_back(panels(i));
        ct.push_back((double)x.n);
      } else {
        const int ns = (int)((x.n + 15) / 16);
        rn[ns].push_back({(const float*)x.A, x.m, x.n, x.lda, (const float*)P(i).Xs, x.n, l,
                          (float*)P(i).Y, l, gm, tune[i].tpp});
        itn[ns].push_back(panels(i));
        cn[ns].push_back((double)x.n);
      }
    }
    B.add_wl(G_TALL, rt, it, ct, ntl, 0, fuse);
    for (int ns = 1; ns <= 6; ++ns) B.add_wl(G_NARROW, rn[ns], itn[ns], cn[ns], ntl, ns, fuse);
    if (first) {
      std::vector<GArgRedS> rs;
      for (int i : ix) rs.push_back({P(i).fro2_part, panels(i), P(i).scal, 1});
      B.add(G_RED_S, rs);
    }
    if (fuse) gram_red();
  };
  // W (c x c) = Y^T Y, FP64 partials then their fixed-order sum
  auto gram = [&](bool dbl, std::function<const void*(int)> Yp, std::function<int64_t(int)> rows) {
    std::vector<GArgGram> rg;
    std::vector<GArgRed> rr;
    for (int i : ix) {
      int64_t rpb = 0;
      const int nb = (int)gram_blocks(rows(i), P(i).max_split, &rpb, kGroupedSplitRows);
      rg.push_back({Yp(i), rows(i), l, l, P(i).part, rpb, nb});
      rr.push_back({P(i).part, nb, l, l, P(i).Wg, l, blocks256((int64_t)l * l)});
    }
    B.add(dbl ? G_GRAM_D : G_GRAM_F, rg, ntl, l);
    B.add(G_RED, rr);
  };
  auto chol = [&](bool dbl, std::function<GArgChol(int)> f) {
    std::vector<GArgChol> r;
    for (int i : ix) r.push_back(f(i));
    B.add(dbl ? G_CHOL_D : G_CHOL_F, r, l);   // every factor of the group is l x l
  };
  // CholeskyQR2 of Y (m x l): Q1 = Y R1^-1, R2 = chol(Q1^T Q1), Q = Q1 R2^-1
  // (fused: Y^T Y came with the pass that wrote Y, Q1^T Q1 comes with Q1)
  auto cqr2 = [&]() {
    if (!fuse) gram(false, [&](int i) { return (const void*)P(i).Y; }, [&](int i) { return X(i).m; });
    chol(false, [&](int i) {
      return GArgChol{P(i).Wg, l, P(i).R1, P(i).R1inv, P(i).RinvT, 1, P(i).status, 1};
    });
    std::vector<GArgNarrow> rn;
    std::vector<int> it;
    std::vector<double> ct;
    for (int i : ix) {
      rn.push_back({(const float*)P(i).Y, X(i).m, l, l, (const float*)P(i).RinvT, l, l,
                    (float*)P(i).Q1, l, fuse ? P(i).part : nullptr, tune[i].tpp});
      it.push_back(panels(i));
      ct.push_back((double)l);
    }
    B.add_wl(G_NARROW_TRI, rn, it, ct, ntl, nsl, fuse);   // Y R1^-1: triangular factor
    if (fuse)
      gram_red();
    else
      gram(false, [&](int i) { return (const void*)P(i).Q1; }, [&](int i) { return X(i).m; });
    chol(false, [&](int i) {
      return GArgChol{P(i).Wg, l, P(i).R2, P(i).R2inv, nullptr, 0, P(i).status, 1};
    });
  };
  // Z = A^T Q1 (FP64 n x l) into Zd, then Z2 = Zd R2^-1
  auto pass_tn = [&]() {
    std::vector<GArgTn> rt;
    std::vector<int> blocks;
    std::vector<GArgRed> rr;
    std::vector<GArgSg> rs;
    for (int i : ix) {
      const rsvd_instance& x = X(i);
      int ntile = 0;
      int64_t rps = 0;
      const int ns = (int)tn_tall_splits(x.m, x.n, P(i).max_split, &rps, &ntile, tune[i].split_rows);
      rt.push_back({(const float*)x.A, x.m, x.n, x.lda, (const float*)P(i).Q1, l, l, rps, ntile,
                    P(i).part});
      blocks.push_back(ns * ntile);
      rr.push_back({P(i).part, ns, x.n, l, P(i).Zd, l, blocks256(x.n * (int64_t)l)});
      rs.push_back({P(i).Zd, P(i).R2inv, x.n, l, l, P(i).Z2, nullptr, 0, blocks256(x.n * (int64_t)l)});
    }
    // one launch per A^T Q kernel (column waves 1, 2, 4, 8 by n); a block
    // costs about its split's rows times n
    for (int cw : {1, 2, 4, 8}) {
      std::vector<GArgTn> rc;
      std::vector<int> it;
      std::vector<double> ct;
      for (size_t r = 0; r < rt.size(); ++r)
        if (tn_col_waves(rt[r].n) == cw) {
          rc.push_back(rt[r]);
          it.push_back(blocks[r]);
          ct.push_back((double)rt[r].rps * (double)(rt[r].n < kTnTileCols ? rt[r].n : kTnTileCols));
        }
      B.add_wl(G_TN, rc, it, ct, ntl, cw, false);
    }
    B.add(G_RED, rr);
    B.add(G_SG_F, rs);
  };
  // orthonormalise the FP64 n x l matrix Z2: Zq (explicit), R2s R1s = R
  auto cqr2_small = [&]() {
    auto nn = [&](std::function<const double*(int)> A, std::function<double*(int)> Y) {
      std::vector<GArgNn> r;
      const int nt = ntl > 8 ? 8 : ntl;
      for (int i : ix) {
        const int ct = nn_col_tiles(l, nt);
        r.push_back({A(i), X(i).n, l, l, P(i).RinvTs, l, l, Y(i), l, nullptr, ct,
                     (int)(nn_row_blocks(X(i).n) * ct)});
      }
      B.add(G_NN_D, r, nt);
    };
    gram(true, [&](int i) { return (const void*)P(i).Z2; }, [&](int i) { return X(i).n; });
    chol(true, [&](int i) {
      return GArgChol{P(i).Wg, l, P(i).R1s, P(i).R1invs, P(i).RinvTs, 0, P(i).status, 1};
    });
    nn([&](int i) { return (const double*)P(i).Z2; }, [&](int i) { return P(i).Z1; });
    gram(true, [&](int i) { return (const void*)P(i).Z1; }, [&](int i) { return X(i).n; });
    chol(true, [&](int i) {
      return GArgChol{P(i).Wg, l, P(i).R2s, P(i).R2invs, P(i).RinvTs, 0, P(i).status, 1};
    });
    nn([&](int i) { return (const double*)P(i).Z1; }, [&](int i) { return P(i).Zq; });
  };
  auto sg = [&](bool dbl, std::function<GArgSg(int)> f) {
    std::vector<GArgSg> r;
    for (int i : ix) r.push_back(f(i));
    B.add(dbl ? G_SG_D : G_SG_F, r);
  };

  // step 2: H = A G (with ||A||_F^2), CholeskyQR2
  pass_nn(true, false);
  cqr2();
  // step 3: power iterations
  for (int it = 0; it < X(ix[0]).q; ++it) {
    pass_tn();
    cqr2_small();
    pass_nn(false, true);
    cqr2();
  }
  // step 5: T = A^T Q
  pass_tn();
  // step 6: T = V~ S~ W^T (J formed from Uo S^-1; repeated with J accumulated
  // when the values span more than six decades)
  cqr2_small();
  sg(true, [&](int i) {
    return GArgSg{P(i).R2s, P(i).R1s, l, l, l, P(i).Rt, nullptr, 0, blocks256((int64_t)l * l)};
  });
  {
    std::vector<GArgJac> r;
    for (int i : ix)
      r.push_back({P(i).Rt, l, 1, P(i).Uo, P(i).Su, P(i).Mk, P(i).diag, P(i).status,
                   P(i).diag + 5, 1});
    B.add(G_JAC, r, l);
  }
  sg(true, [&](int i) {
    return GArgSg{P(i).Rt, P(i).Mk, l, l, l, P(i).Jm, nullptr, 0, blocks256((int64_t)l * l)};
  });
  {
    std::vector<GArgJac> r;
    for (int i : ix)
      r.push_back({P(i).Rt, l, 1, P(i).Uo, P(i).Su, P(i).Jm, P(i).diag, P(i).status,
                   P(i).diag + 5, 1});
    B.add(G_JAC_ACC, r, l);
  }
  sg(true, [&](int i) {
    return GArgSg{P(i).Zq, P(i).Jm, X(i).n, l, l, P(i).Vt, nullptr, 0,
                  blocks256(X(i).n * (int64_t)l)};
  });
  {
    std::vector<GArgSort> r;
    for (int i : ix) {
      const rsvd_instance& x = X(i);
      r.push_back({P(i).Su, l, P(i).Vt, x.n, l, 1, P(i).Uo, k, x.S, x.V, x.ldv, nullptr, P(i).Wk,
                   (k + 15) / 16});
    }
    B.add(G_SORT, r, l);
  }
  // step 7: U~ = Q1 (R2^-1 W), first k columns
  sg(false, [&](int i) {
    return GArgSg{P(i).R2inv, P(i).Wk, l, l, k, nullptr, P(i).MkT, 1, blocks256((int64_t)l * k)};
  });
  {
    std::vector<GArgNarrow> r;
    std::vector<int> it;
    std::vector<double> ct;
    for (int i : ix) {
      r.push_back({(const float*)P(i).Q1, X(i).m, l, l, (const float*)P(i).MkT, l, k,
                   (float*)X(i).U, X(i).ldu, nullptr, tune[i].tpp});
      it.push_back(panels(i));
      ct.push_back((double)k);
    }
    B.add_wl(G_NARROW, r, it, ct, ntk, nsl, false);
  }
  {
    std::vector<GArgSel> r;
    for (int i : ix)
      r.push_back({X(i).S, k, P(i).scal, X(i).t, X(i).K, P(i).diag, P(i).status, 1});
    B.add(G_SEL, r, k);
  }
  {
    std::vector<GArgStat> r;
    for (int i : ix) r.push_back({P(i).status, X(i).status, nullptr, 0, 1});
    B.add(G_TAKE, r);
  }
}

hipError_t grouped_launch(const rsvd_grouped_s* g, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (const rsvd_grouped_s::Op& op : g->ops) {
    const void* a = g->args + op.off;
    switch (op.kind) {
      case G_RESET:
      case G_TAKE:
        hipLaunchKernelGGL(k_status_grouped, dim3(1, (unsigned)op.count), dim3(64), 0, s,
                           (const GArgStat*)a);
        e = hipGetLastError();
        break;
      case G_FILL: e = launch_gaussian_fill_grouped((const GArgFill*)a, op.count, op.maxblk, s); break;
      case G_CAST_T:
        e = launch_cast_t_from_f64_grouped<float>((const GArgCast*)a, op.count, op.maxblk, s);
        break;
      case G_TALL:
        e = launch_gemm_nt_tall_grouped((const GArgTall*)a, (const GWork*)(g->args + op.wl_off),
                                        op.nwork, op.a0, op.fuse, s);
        break;
      case G_NARROW:
      case G_NARROW_TRI:
        e = launch_gemm_nt_narrow_grouped((const GArgNarrow*)a,
                                          (const GWork*)(g->args + op.wl_off), op.nwork, op.a0,
                                          op.a1, op.fuse, op.kind == G_NARROW_TRI, s);
        break;
      case G_RED_S: e = launch_reduce_scalar_grouped((const GArgRedS*)a, op.count, s); break;
      case G_GRAM_F:
        e = launch_gram_f64_grouped<float>((const GArgGram*)a, op.count, op.maxblk, op.a0, op.a1, s);
        break;
      case G_GRAM_D:
        e = launch_gram_f64_grouped<double>((const GArgGram*)a, op.count, op.maxblk, op.a0, op.a1,
                                            s);
        break;
      case G_RED: e = launch_reduce_partials_grouped((const GArgRed*)a, op.count, op.maxblk, s); break;
      case G_CHOL_F: e = launch_chol_inv_grouped<float>((const GArgChol*)a, op.count, op.a0, s); break;
      case G_CHOL_D: e = launch_chol_inv_grouped<double>((const GArgChol*)a, op.count, op.a0, s); break;
      case G_TN:
        e = launch_gemm_tn_tall_grouped((const GArgTn*)a, (const GWork*)(g->args + op.wl_off),
                                        op.nwork, op.a0, op.a1, s);
        break;
      case G_SG_F: e = launch_small_gemm_grouped<float>((const GArgSg*)a, op.count, op.maxblk, s); break;
      case G_SG_D: e = launch_small_gemm_grouped<double>((const GArgSg*)a, op.count, op.maxblk, s); break;
      case G_NN_D:
        e = launch_gemm_nn_f64_grouped((const GArgNn*)a, op.count, op.maxblk, op.a0, s);
        break;
      case G_JAC:
        e = launch_jacobi_svd_small_grouped((const GArgJac*)a, op.count, op.a0, 0, s);
        break;
      case G_JAC_ACC:
        e = launch_jacobi_svd_small_grouped((const GArgJac*)a, op.count, op.a0, 1, s);
        break;
      case G_SORT:
        e = launch_sort_sign_scatter_grouped<float>((const GArgSort*)a, op.count, op.maxblk, op.a0,
                                                    s);
        break;
      case G_SEL: e = launch_select_k_grouped((const GArgSel*)a, op.count, op.a0, s); break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void grouped_free(rsvd_grouped_s* g) {
  (void)hipSetDevice(g->device);
  if (g->ws) (void)hipFree(g->ws);
  if (g->args) (void)hipFree(g->args);
  delete g;
}

}  // namespace

extern "C" {

int32_t rsvd_batch_grouped_create(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                                  const rsvd_tune_entry* tune, int32_t ntune,
                                  rsvd_grouped_t* grouped) {
  if (!batch || !grouped || count < 0 || (count > 0 && !inst)) return RSVD_ERR_ARG;
  if (ntune < 0 || (ntune > 0 && !tune)) return RSVD_ERR_ARG;
  *grouped = nullptr;
  if (batch->dtype != RSVD_F32) return RSVD_ERR_ARG;
  for (int t = 0; t < ntune; ++t)
    if (!tune_entry_valid(tune[t])) return RSVD_ERR_ARG;
  std::vector<GTune> tu(count);
  for (int i = 0; i < count; ++i) {
    const int32_t rc = check_instance(batch->plan[0], inst[i]);
    if (rc != RSVD_OK) return rc;
    if (instance_dtype(batch->plan[0], inst[i]) != RSVD_F32 || !inst[i].U) return RSVD_ERR_ARG;
    tu[i] = tune_for(inst[i], tune, ntune);
    if (!grouped_applies(inst[i], batch->plan[0]->max_split, tu[i])) return RSVD_ERR_ARG;
  }
  if (hipSetDevice(batch->device) != hipSuccess) return RSVD_ERR_DEVICE;
  rsvd_grouped_s* g = new (std::nothrow) rsvd_grouped_s();
  if (!g) return RSVD_ERR_NOMEM;
  g->device = batch->device;
  // one workspace per instance, sized for it, carved from one allocation
  g->plans.resize(count);
  std::vector<size_t> off(count);
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    rsvd_plan_s& p = g->plans[i];
    const rsvd_instance& x = inst[i];
    p.device = batch->device;
    p.dtype = RSVD_F32;
    p.m_max = x.m;
    p.n_max = x.n;
    p.l_max = (int)((x.k + (int64_t)x.p < x.n) ? x.k + x.p : x.n);
    p.gram = false;
    p.seed = batch->plan[0]->seed;
    // partials for the grouped row splits only: at least kGroupedSplitRows
    // rows each, so at most ceil(m / kGroupedSplitRows) of them (within the
    // batch's split limit; the grouped launchers cap at the same count)
    const int64_t gsplit = (x.m + kGroupedSplitRows - 1) / kGroupedSplitRows;
    p.max_split = gsplit < batch->plan[0]->max_split ? gsplit : batch->plan[0]->max_split;
    // the panels of the NT products write one partial each: at most
    // max_split of them
    const int64_t ntiles = (x.m + 127) / 128;
    const int64_t tpp_min = (ntiles + p.max_split - 1) / p.max_split;
    if (tu[i].tpp < tpp_min) tu[i].tpp = (int)tpp_min;
    off[i] = total;
    total += carve(&p, nullptr);
  }
  if (total > 0 && hipMalloc(&g->ws, total) != hipSuccess) {
    (void)hipGetLastError();
    grouped_free(g);
    return RSVD_ERR_NOMEM;
  }
  for (int i = 0; i < count; ++i) carve(&g->plans[i], g->ws + off[i]);
  if (total > 0 && (hipMemset(g->ws, 0, total) != hipSuccess)) {
    grouped_free(g);
    return RSVD_ERR_DEVICE;
  }
  // groups of equal (l, k), in order of first appearance
  GroupedBuilder B;
  std::vector<char> done(count, 0);
  for (int i = 0; i < count; ++i) {
    if (done[i]) continue;
    const int l = g->plans[i].l_max, k = inst[i].k, q = inst[i].q;
    std::vector<int> ix;
    for (int j = i; j < count; ++j)
      if (!done[j] && g->plans[j].l_max == l && inst[j].k == k && inst[j].q == q) {
        ix.push_back(j);
        done[j] = 1;
      }
    record_group(B, inst, ix, g->plans, tu, l, k);
  }
  g->ops = B.ops;
  if (!B.host.empty()) {
    if (hipMalloc(&g->args, B.host.size()) != hipSuccess) {
      (void)hipGetLastError();
      grouped_free(g);
      return RSVD_ERR_NOMEM;
    }
    if (hipMemcpy(g->args, B.host.data(), B.host.size(), hipMemcpyHostToDevice) != hipSuccess) {
      grouped_free(g);
      return RSVD_ERR_DEVICE;
    }
  }
  *grouped = g;
  return RSVD_OK;
}

int32_t rsvd_batch_grouped_launch(rsvd_grouped_t grouped, void* stream) {
  if (!grouped) return RSVD_ERR_ARG;
  if (hipSetDevice(grouped->device) != hipSuccess) return RSVD_ERR_DEVICE;
  return grouped_launch(grouped, (hipStream_t)stream) == hipSuccess ? RSVD_OK : RSVD_ERR_DEVICE;
}

int32_t rsvd_batch_grouped_destroy(rsvd_grouped_t grouped) {
  if (!grouped) return RSVD_OK;
  if (hipSetDevice(grouped->device) == hipSuccess) (void)hipDeviceSynchronize();
  grouped_free(grouped);
  return RSVD_OK;
}

int32_t rsvd_batch_grouped_tune(rsvd_batch_t batch, const rsvd_instance* inst, int32_t count,
                                rsvd_tune_entry* out, int32_t cap, int32_t* nout, void* stream) {
  if (!batch || !out || !nout || cap < 0 || count < 0 || (count > 0 && !inst)) return RSVD_ERR_ARG;
  *nout = 0;
  // buckets of equal (n, l), in order of first appearance
  std::vector<rsvd_tune_entry> key;
  std::vector<std::vector<rsvd_instance>> members;
  for (int i = 0; i < count; ++i) {
    const rsvd_instance& x = inst[i];
    const int32_t l = (int32_t)((x.k + (int64_t)x.p < x.n) ? x.k + (int64_t)x.p : x.n);
    size_t b = 0;
    while (b < key.size() && !(key[b].n == x.n && key[b].l == l)) ++b;
    if (b == key.size()) {
      key.push_back(rsvd_tune_entry{(int32_t)x.n, l, (int32_t)kGroupedSplitRows,
                                    (int32_t)kGroupedSplitRows});
      members.emplace_back();
    }
    members[b].push_back(x);
  }
  if ((int32_t)key.size() > cap) return RSVD_ERR_ARG;
  if (hipSetDevice(batch->device) != hipSuccess) return RSVD_ERR_DEVICE;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return RSVD_ERR_DEVICE;
  }
  // mean time of a launch of the bucket's grouped batch under one entry
  // (one untimed launch first)
  auto timed = [&](const std::vector<rsvd_instance>& xs, const rsvd_tune_entry& t,
                   float* ms) -> int32_t {
    rsvd_grouped_t g = nullptr;
    int32_t rc = rsvd_batch_grouped_create(batch, xs.data(), (int32_t)xs.size(), &t, 1, &g);
    if (rc != RSVD_OK) return rc;
    constexpr int kReps = 3;
    rc = grouped_launch(g, s) == hipSuccess ? RSVD_OK : RSVD_ERR_DEVICE;
    if (rc == RSVD_OK && hipEventRecord(e0, s) != hipSuccess) rc = RSVD_ERR_DEVICE;
    for (int r = 0; r < kReps && rc == RSVD_OK; ++r)
      if (grouped_launch(g, s) != hipSuccess) rc = RSVD_ERR_DEVICE;
    if (rc == RSVD_OK && (hipEventRecord(e1, s) != hipSuccess ||
                          hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(ms, e0, e1) != hipSuccess))
      rc = RSVD_ERR_DEVICE;
    *ms /= kReps;
    (void)rsvd_batch_grouped_destroy(g);
    return rc;
  };
  static const int32_t kRows[] = {1024, 2048, 4096, 8192};
  int32_t rc = RSVD_OK;
  for (size_t b = 0; b < key.size() && rc == RSVD_OK; ++b) {
    rsvd_tune_entry best = key[b];
    float tbest = 0.f;
    rc = timed(members[b], best, &tbest);
    // rows per work item of the A X and Y R^-1 products, then the A^T Q
    // split length with the best of those
    for (int pass = 0; pass < 2 && rc == RSVD_OK; ++pass)
      for (int32_t r : kRows) {
        rsvd_tune_entry t = best;
        (pass == 0 ? t.panel_rows : t.split_rows) = r;
        if (t.panel_rows == best.panel_rows && t.split_rows == best.split_rows) continue;
        float ms = 0.f;
        if ((rc = timed(members[b], t, &ms)) != RSVD_OK) break;
        if (ms < tbest) {
          tbest = ms;
          best = t;
        }
      }
    out[b] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != RSVD_OK) return rc;
  *nout = (int32_t)key.size();
  return RSVD_OK;
}

int32_t rsvd_batch_grouped_graph_create(rsvd_grouped_t grouped, rsvd_batch_graph_t* graph) {
  if (!grouped || !graph) return RSVD_ERR_ARG;
  *graph = nullptr;
  if (hipSetDevice(grouped->device) != hipSuccess) return RSVD_ERR_DEVICE;
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return RSVD_ERR_DEVICE;
  hipGraph_t gr = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const hipError_t el = grouped_launch(grouped, cap);
    e = hipStreamEndCapture(cap, &gr);
    if (el != hipSuccess) e = el;
  }
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess || !gr) {
    if (gr) (void)hipGraphDestroy(gr);
    (void)hipGetLastError();
    return RSVD_ERR_DEVICE;
  }
  rsvd_batch_graph_s* h = new (std::nothrow) rsvd_batch_graph_s();
  if (!h) {
    (void)hipGraphDestroy(gr);
    return RSVD_ERR_NOMEM;
  }
  h->graph = gr;
  if (hipGraphInstantiate(&h->exec, gr, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(gr);
    delete h;
    return RSVD_ERR_DEVICE;
  }
  *graph = h;
  return RSVD_OK;
}

}  // extern "C"

// ===========================================================================
// Allocation-free Randomized PCA: the solve of rsvd_solve with its workspace
// carved, exactly as a plan's, from a file-scope device array instead of a
// plan's allocation, for callers that must not allocate device memory.
// Each GPU the library runs on holds its own copy of the array (module
// global memory) until the process ends; every call on one GPU uses that
// GPU's copy, so calls that overlap on one GPU race.

static __device__ __align__(256) char scratch[RSVD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current).  In host code the array's name is
// only a host-side stand-in, so kernels are given this address, never it.
int32_t scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return RSVD_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return RSVD_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return RSVD_OK;
}

}  // namespace

extern "C" {

int32_t rsvd_solve_noalloc(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype,
                           int32_t k, int32_t p, int32_t q, double t, uint64_t seed, void* U,
                           int64_t ldu, double* S, void* V, int64_t ldv, int32_t* K,
                           int32_t* status, void* stream) {
  if (dtype != RSVD_F64 && dtype != RSVD_F32) return RSVD_ERR_ARG;
  if (!A || !status) return RSVD_ERR_ARG;
  if (n < 1 || m < n || m > kMaxRows || n > kMaxCols) return RSVD_ERR_SHAPE;
  if (k < 1 || k > n || p < 0) return RSVD_ERR_ARG;
  const int64_t l = (k + (int64_t)p < n) ? k + (int64_t)p : n;
  if (l > kMaxL) return RSVD_ERR_SHAPE;
  // a plan sized for exactly this problem, its workspace in `scratch`: the
  // same buffers, row splits and kernels as rsvd_solve on a plan with this
  // seed (so the same results, bit for bit)
  rsvd_plan_s pl;
  pl.dtype = dtype;
  pl.m_max = m;
  pl.n_max = n;
  pl.l_max = (int)l;
  pl.gram = false;
  pl.seed = seed;
  pl.stream = (hipStream_t)stream;
  pl.max_split = tn_max_split(m, n, (int)l);
  int32_t rc = check_rsvd(&pl, A, m, n, lda, k, p, q, t, U, ldu, S, V, ldv, K);
  if (rc != RSVD_OK) return rc;
  if (carve(&pl, nullptr) > (size_t)RSVD_NOALLOC_SCRATCH_BYTES) return RSVD_ERR_SHAPE;
  if (hipGetDevice(&pl.device) != hipSuccess) return RSVD_ERR_DEVICE;
  char* base = nullptr;
  if ((rc = scratch_address(pl.device, &base)) != RSVD_OK) return rc;
  carve(&pl, base);
  // the status word and diagnostics are cleared by the solve's first kernel;
  // every other buffer is written before it is read
  if (dtype == RSVD_F64)
    rc = rsvd_run<double>(&pl, (const double*)A, m, n, lda, k, p, q, t, nullptr, (double*)U, ldu,
                          S, (double*)V, ldv, K);
  else
    rc = rsvd_run<float>(&pl, (const float*)A, m, n, lda, k, p, q, t, nullptr, (float*)U, ldu, S,
                         (float*)V, ldv, K);
  if (rc != RSVD_OK) return rc;
  hipLaunchKernelGGL(k_status_take, dim3(1), dim3(64), 0, pl.stream, pl.status, status);
  RSVD_CHECK(hipGetLastError());
  return RSVD_OK;
}

}  // extern "C"
