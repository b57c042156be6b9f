// small.hip -- the FP64 work on n x l, l x l and n x n matrices between the
// passes over A: the Gaussian sketch, Cholesky factors and their inverses
// (CholeskyQR2), small products, the one-sided Jacobi SVD of the l x l
// factor, the Jacobi eigensolver of the A^T A route, the sign rule and the
// explained-variance criterion.
#include <math.h>

#include "rsvd_internal.h"

namespace rsvd {

namespace {

constexpr double kEps = 2.220446049250313e-16;

// Errors win over warnings; among errors the most negative code wins.
__device__ __forceinline__ void set_error(int32_t* status, int32_t code) { atomicMin(status, code); }
__device__ __forceinline__ void set_warning(int32_t* status, int32_t code) { atomicCAS(status, 0, code); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011): ten rounds; each
// multiplies words 0 and 2 by the two round constants and mixes the high
// halves with words 1, 3 and the key; the key advances by the two Weyl
// constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6) + 0.5) * 1.1102230246251565e-16;
}

// The standard normal sketch matrix G of Sec. 3.1.2 step 1 (Box-Muller).
__global__ void k_gaussian_fill(uint64_t seed, int64_t total, double* __restrict__ G) {
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * pair >= total) return;
  uint32_t c[4] = {(uint32_t)(pair & 0xFFFFFFFFu), (uint32_t)((uint64_t)pair >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32));
  const double u1 = uniform53(c[0], c[1]);
  const double u2 = uniform53(c[2], c[3]);
  const double r = sqrt(-2.0 * log(u1));
  const double th = 2.0 * 3.141592653589793 * u2;
  G[2 * pair] = r * cos(th);
  if (2 * pair + 1 < total) G[2 * pair + 1] = r * sin(th);
}

template <typename S, typename D>
__global__ void k_cast(const S* __restrict__ src, int64_t rows, int64_t cols, int64_t lds,
                       D* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx / cols, j = idx - i * cols;
  dst[i * ldd + j] = (D)src[i * lds + j];
}

// ---------------------------------------------------------------------------
// Cholesky W = R^T R (R upper, positive diagonal) and Rinv = R^-1, one block,
// both c x c matrices in LDS (row stride c + 1).  Right-looking elimination
// with one barrier per step: at step j every thread updates the trailing
// entries (i, i2), j < i <= i2, with W[j][i] W[j][i2] / W[j][j], which needs
// only the (already final) row j.  The inverse solves R X = I from the last
// row up in the same way (B <- B - R[i][k] B[k][:] / R[k][k]).
constexpr int kCholThreads = 256;

template <typename T>
__global__ __launch_bounds__(kCholThreads) void k_chol_inv(const double* __restrict__ W, int c,
                                                           double* __restrict__ R,
                                                           double* __restrict__ Rinv,
                                                           T* __restrict__ RinvT,
                                                           int32_t* __restrict__ status) {
  extern __shared__ double sm[];
  const int ld = c + 1;
  double* L = sm;             // c x c, upper triangle used
  double* B = sm + c * ld;    // c x c
  double* dg = sm + 2 * c * ld;  // sqrt of the pivots
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < c * c; idx += kCholThreads) {
    const int i = idx / c, j = idx - i * c;
    L[i * ld + j] = 0.5 * (W[i * c + j] + W[j * c + i]);
    B[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    const double d = L[j * ld + j];
    if (!(d > 0.0)) {           // also catches NaN
      if (tid == 0) bad = 1;
      break;
    }
    const double inv_d = 1.0 / d;
    const int nt = c - 1 - j;   // trailing size
    for (int idx = tid; idx < nt * nt; idx += kCholThreads) {
      const int i = j + 1 + idx / nt, i2 = j + 1 + idx % nt;
      if (i2 >= i) L[i * ld + i2] -= L[j * ld + i] * L[j * ld + i2] * inv_d;
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    // R = 0 (no factor), Rinv = I keeps the later products finite
    for (int idx = tid; idx < c * c; idx += kCholThreads) {
      const int i = idx / c, j = idx - i * c;
      const double v = (i == j) ? 1.0 : 0.0;
      R[idx] = 0.0;
      Rinv[idx] = v;
      if (RinvT) RinvT[idx] = (T)v;
    }
    if (tid == 0) set_error(status, RSVD_ERR_BREAKDOWN);
    return;
  }
  // R[i][j] = L[i][j] / sqrt(L[i][i]) for j >= i (pivots read before any write)
  for (int i = tid; i < c; i += kCholThreads) dg[i] = sqrt(L[i * ld + i]);
  __syncthreads();
  for (int idx = tid; idx < c * c; idx += kCholThreads) {
    const int i = idx / c, j = idx - i * c;
    L[i * ld + j] = (j >= i) ? L[i * ld + j] / dg[i] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < c * c; idx += kCholThreads) {
    const int i = idx / c, j = idx - i * c;
    R[idx] = L[i * ld + j];
  }
  // back substitution for X = R^-1, rows from the bottom: after step k, row k
  // of B divided by R[k][k] is row k of X.
  for (int k = c - 1; k >= 1; --k) {
    const double rkk = L[k * ld + k];
    const int w = c - k;        // columns j >= k
    for (int idx = tid; idx < k * w; idx += kCholThreads) {
      const int i = idx / w, j = k + idx % w;
      B[i * ld + j] -= L[i * ld + k] * B[k * ld + j] / rkk;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < c * c; idx += kCholThreads) {
    const int i = idx / c, j = idx - i * c;
    const double v = (j >= i) ? B[i * ld + j] / L[i * ld + i] : 0.0;
    Rinv[idx] = v;
    if (RinvT) RinvT[idx] = (T)v;
  }
}

template <typename T>
__global__ void k_small_gemm(const double* __restrict__ A, const double* __restrict__ B,
                             int64_t r, int c1, int c2, double* __restrict__ C, T* __restrict__ CT) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r * c2) return;
  const int64_t i = idx / c2;
  const int j = (int)(idx - i * c2);
  double s = 0.0;
  for (int k = 0; k < c1; ++k) s += A[i * c1 + k] * B[(int64_t)k * c2 + j];
  if (C) C[idx] = s;
  if (CT) CT[idx] = (T)s;
}

// ---------------------------------------------------------------------------
// Round-robin ("circle") pairing of npad (even) indices: in step s, pair 0 is
// (npad-1, s) and pair k > 0 is ((s+k) mod (npad-1), (s-k) mod (npad-1)); the
// npad-1 steps meet every pair exactly once, and the pairs of one step are
// disjoint, so their rotations commute.
__device__ __forceinline__ void rr_pair(int s, int k, int npad, int* p, int* q) {
  int a, b;
  const int h = npad - 1;
  if (k == 0) { a = h; b = s; }
  else { a = (s + k) % h; b = (s - k + h) % h; }
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

// One-sided (Hestenes) Jacobi rotation that orthogonalises columns x, y with
// alpha = |x|^2, beta = |y|^2, gamma = x.y:  zeta = (beta - alpha)/(2 gamma),
// t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)), cs = 1/sqrt(1+t^2), sn = cs t;
// x' = cs x - sn y, y' = sn x + cs y.
__device__ __forceinline__ void jacobi_cs(double alpha, double beta, double gamma, double* cs,
                                          double* sn) {
  const double zeta = (beta - alpha) / (2.0 * gamma);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  *cs = 1.0 / sqrt(1.0 + t * t);
  *sn = *cs * t;
}

// One-sided Jacobi SVD of a c x c matrix in one block, both the matrix and
// the accumulated rotations J held column-major in LDS.  A group of G lanes
// (G | 64) owns one column pair per step.
constexpr int kJsThreads = 1024;
constexpr int kJsMaxSweeps = 60;

__global__ __launch_bounds__(kJsThreads) void k_jacobi_svd_small(
    const double* __restrict__ Min, int c, double* __restrict__ Uo, double* __restrict__ S,
    double* __restrict__ Jout, double* __restrict__ diag, int32_t* __restrict__ status, int G) {
  extern __shared__ double sm[];
  const int npad = c + (c & 1);
  double* Mc = sm;                   // column j at Mc + j*c
  double* Jc = sm + (size_t)npad * c;
  __shared__ int rotated;
  __shared__ double offmax;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < c * c; idx += kJsThreads) {
    const int i = idx / c, j = idx - i * c;   // Min row-major (i, j) -> column j
    Mc[j * c + i] = Min[idx];
    Jc[j * c + i] = (i == j) ? 1.0 : 0.0;
  }
  const int npairs = npad / 2;
  const int grp = tid / G, gl = tid % G;
  const double tol = kEps * sqrt((double)c);
  int sweep = 0;
  bool converged = false;
  double last_off = 0.0;
  __syncthreads();
  while (sweep < kJsMaxSweeps) {
    if (tid == 0) { rotated = 0; offmax = 0.0; }
    __syncthreads();
    for (int s = 0; s < npad - 1; ++s) {
      for (int pk = grp; pk < npairs; pk += kJsThreads / G) {
        int p, q;
        rr_pair(s, pk, npad, &p, &q);
        if (q >= c) continue;           // the padding index of odd c
        double* xp = Mc + (size_t)p * c;
        double* xq = Mc + (size_t)q * c;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < c; i += G) {
          const double a = xp[i], b = xq[i];
          al += a * a; be += b * b; ga += a * b;
        }
        for (int off = G / 2; off > 0; off >>= 1) {
          al += __shfl_xor(al, off);
          be += __shfl_xor(be, off);
          ga += __shfl_xor(ga, off);
        }
        const double scale = sqrt(al) * sqrt(be);
        const double rel = scale > 0.0 ? fabs(ga) / scale : 0.0;
        if (ga != 0.0 && rel > tol) {
          double cs, sn;
          jacobi_cs(al, be, ga, &cs, &sn);
          for (int i = gl; i < c; i += G) {
            const double a = xp[i], b = xq[i];
            xp[i] = cs * a - sn * b;
            xq[i] = sn * a + cs * b;
          }
          double* jp = Jc + (size_t)p * c;
          double* jq = Jc + (size_t)q * c;
          for (int i = gl; i < c; i += G) {
            const double a = jp[i], b = jq[i];
            jp[i] = cs * a - sn * b;
            jq[i] = sn * a + cs * b;
          }
          if (gl == 0) {
            rotated = 1;
            // benign race: any writer's value is a valid lower bound
            if (rel > offmax) offmax = rel;
          }
        }
      }
      __syncthreads();
    }
    ++sweep;
    last_off = offmax;
    const bool done = (rotated == 0);
    __syncthreads();
    if (done) { converged = true; break; }
  }
  // singular values = column norms, Uo = normalised columns
  for (int j = tid / 64; j < c; j += kJsThreads / 64) {
    const int lane = tid & 63;
    double s2 = 0.0;
    for (int i = lane; i < c; i += 64) s2 += Mc[(size_t)j * c + i] * Mc[(size_t)j * c + i];
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
    const double nrm = sqrt(s2);
    if (lane == 0) S[j] = nrm;
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = lane; i < c; i += 64) {
      Uo[(size_t)i * c + j] = Mc[(size_t)j * c + i] * inv;
      Jout[(size_t)i * c + j] = Jc[(size_t)j * c + i];
    }
  }
  if (tid == 0) {
    diag[2] = (double)sweep;
    diag[3] = last_off;
    if (!converged) set_error(status, RSVD_ERR_NOCONV);
  }
}

// ---------------------------------------------------------------------------
// Jacobi eigensolver of the A^T A route: one-sided Jacobi on the columns of
// the symmetric matrix X (column j at X + j*n), rotations accumulated in J.
// Every wave owns one column pair per step; the steps of a sweep are
// separated by a grid barrier (cooperative launch, all blocks resident).
// The barrier spin is bounded: on timeout the kernel records an error and
// every block leaves.
constexpr int kJeThreads = 256;
constexpr int kJeMaxSweeps = 40;
constexpr long kSpinLimit = 1L << 22;

__device__ __forceinline__ bool grid_barrier(int32_t* counter, int32_t* abort_flag, int target) {
  __threadfence();
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > kSpinLimit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  __threadfence();
  return ok != 0;
}

// flags[0] = barrier counter, flags[1] = abort flag, flags[2 + sweep] =
// rotations counted in that sweep (all zeroed by the host before launch).
__global__ __launch_bounds__(kJeThreads) void k_jacobi_eig(double* __restrict__ X,
                                                           double* __restrict__ J, int64_t n,
                                                           double* __restrict__ lam,
                                                           double* __restrict__ diag,
                                                           int32_t* __restrict__ flags,
                                                           int32_t* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int wpb = kJeThreads / 64;
  const int gwave = blockIdx.x * wpb + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * wpb;
  const int npad = (int)(n + (n & 1));
  const int npairs = npad / 2;
  const double tol = kEps * sqrt((double)n);
  int32_t* counter = flags;
  int32_t* abort_flag = flags + 1;
  int bar = 0;
  int sweep = 0;
  bool converged = false, aborted = false;
  while (sweep < kJeMaxSweeps && !aborted) {
    int local = 0;
    for (int s = 0; s < npad - 1 && !aborted; ++s) {
      for (int pk = gwave; pk < npairs; pk += nwaves) {
        int p, q;
        rr_pair(s, pk, npad, &p, &q);
        if (q >= n) continue;
        double* xp = X + (int64_t)p * n;
        double* xq = X + (int64_t)q * n;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int64_t i = lane; i < n; i += 64) {
          const double a = xp[i], b = xq[i];
          al += a * a; be += b * b; ga += a * b;
        }
        for (int off = 32; off > 0; off >>= 1) {
          al += __shfl_xor(al, off);
          be += __shfl_xor(be, off);
          ga += __shfl_xor(ga, off);
        }
        const double scale = sqrt(al) * sqrt(be);
        if (ga != 0.0 && scale > 0.0 && fabs(ga) > tol * scale) {
          double cs, sn;
          jacobi_cs(al, be, ga, &cs, &sn);
          for (int64_t i = lane; i < n; i += 64) {
            const double a = xp[i], b = xq[i];
            xp[i] = cs * a - sn * b;
            xq[i] = sn * a + cs * b;
          }
          double* jp = J + (int64_t)p * n;
          double* jq = J + (int64_t)q * n;
          for (int64_t i = lane; i < n; i += 64) {
            const double a = jp[i], b = jq[i];
            jp[i] = cs * a - sn * b;
            jq[i] = sn * a + cs * b;
          }
          ++local;
        }
      }
      if (s == npad - 2 && lane == 0 && local > 0)
        __hip_atomic_fetch_add(&flags[2 + sweep], local, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ++bar;
      if (!grid_barrier(counter, abort_flag, bar * (int)gridDim.x)) aborted = true;
    }
    if (aborted) break;
    const int rot = __hip_atomic_load(&flags[2 + sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++sweep;
    if (rot == 0) { converged = true; break; }
  }
  if (aborted) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_error(status, RSVD_ERR_DEVICE);
    return;
  }
  // lambda_j = |column j of X J| (X J = W diag(lambda) for a PSD matrix)
  for (int64_t j = gwave; j < n; j += nwaves) {
    double s2 = 0.0;
    for (int64_t i = lane; i < n; i += 64) s2 += X[j * n + i] * X[j * n + i];
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
    // sign from the Rayleigh quotient j^T X j keeps a negative eigenvalue negative
    double rq = 0.0;
    for (int64_t i = lane; i < n; i += 64) rq += J[j * n + i] * X[j * n + i];
    for (int off = 32; off > 0; off >>= 1) rq += __shfl_xor(rq, off);
    if (lane == 0) lam[j] = rq < 0.0 ? -sqrt(s2) : sqrt(s2);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    diag[2] = (double)sweep;
    if (!converged) set_error(status, RSVD_ERR_NOCONV);
  }
}

// ---------------------------------------------------------------------------
// Sort by S descending (ties: lower index first), apply the sign rule to the
// first kout vectors and scatter them.  Source vector column `col`, element
// i is at Vsrc[i * vrs + col * vcs].  One wave per output column.
template <typename T>
__global__ void k_sort_sign_scatter(const double* __restrict__ S, int c,
                                    const double* __restrict__ Vsrc, int64_t r, int64_t vrs,
                                    int64_t vcs, const double* __restrict__ Wsrc, int kout,
                                    double* __restrict__ S_out, T* __restrict__ Vout,
                                    int64_t ldv, double* __restrict__ Vd_out,
                                    double* __restrict__ Wout) {
  extern __shared__ int perm[];
  const int tid = threadIdx.x;
  for (int i = tid; i < c; i += blockDim.x) perm[i] = i;   // NaN keys may leave slots unranked
  __syncthreads();
  for (int i = tid; i < c; i += blockDim.x) {
    const double si = S[i];
    int rank = 0;
    for (int j = 0; j < c; ++j) {
      const double sj = S[j];
      rank += (sj > si) || (sj == si && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
  const int lane = tid & 63;
  for (int kk = tid / 64; kk < kout; kk += blockDim.x / 64) {
    int src = perm[kk];
    if (src < 0 || src >= c) src = kk;
    double vmax = 0.0;
    for (int64_t i = lane; i < r; i += 64) vmax = fmax(vmax, fabs(Vsrc[i * vrs + src * vcs]));
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
    int64_t first = r;
    for (int64_t i = lane; i < r; i += 64)
      if (fabs(Vsrc[i * vrs + src * vcs]) >= 0.999 * vmax) { first = i; break; }
    for (int off = 32; off > 0; off >>= 1) {
      const int64_t o = __shfl_xor(first, off);
      first = o < first ? o : first;
    }
    const double sg = (first < r && Vsrc[first * vrs + src * vcs] < 0.0) ? -1.0 : 1.0;
    if (lane == 0) S_out[kk] = S[src];
    for (int64_t i = lane; i < r; i += 64) {
      const double v = sg * Vsrc[i * vrs + src * vcs];
      if (Vout) Vout[i * ldv + kk] = (T)v;
      if (Vd_out) Vd_out[i * kout + kk] = v;
    }
    if (Wsrc && Wout)
      for (int i = lane; i < c; i += 64) Wout[(int64_t)i * kout + kk] = sg * Wsrc[(int64_t)i * c + src];
  }
}

// Cumulative explained variance criterion (Sec. 2.4): minimal K <= k with
// sum_{i<=K} s_i^2 >= t * ||A||_F^2 (Eq. sumeigen gives the denominator).
__global__ void k_select_k(const double* __restrict__ S, int k, const double* __restrict__ fro2,
                           double t, int32_t* __restrict__ K, double* __restrict__ diag,
                           int32_t* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double f2 = fro2[0];
  diag[0] = f2;
  if (!isfinite(f2)) {
    *K = 0; diag[1] = 0.0; diag[4] = 0.0;
    set_error(status, RSVD_ERR_NONFINITE);
    return;
  }
  if (f2 == 0.0) {
    // a zero matrix also breaks the Cholesky factorisations down; that is a
    // consequence, so the zero-matrix warning replaces it
    *K = 0; diag[1] = 0.0; diag[4] = 0.0;
    atomicExch(status, (int32_t)RSVD_WARN_ZERO_MATRIX);
    return;
  }
  double cum = 0.0;
  int kk = k;
  bool hit = false;
  for (int i = 0; i < k; ++i) {
    cum += S[i] * S[i];
    if (cum >= t * f2) { kk = i + 1; hit = true; break; }
  }
  *K = kk;
  diag[1] = cum / f2;
  diag[4] = (double)kk;
  if (!hit) set_warning(status, RSVD_WARN_THRESHOLD);
}

template <typename T>
__global__ void k_scale_cols_inv(const double* __restrict__ V, int64_t n, int cols, int64_t ldv,
                                 const double* __restrict__ S, double floor_rel,
                                 T* __restrict__ X, int64_t ldx) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * cols) return;
  const int64_t i = idx / cols;
  const int j = (int)(idx - i * cols);
  const double sj = S[j];
  X[i * ldx + j] = (sj > floor_rel * S[0]) ? (T)(V[i * ldv + j] / sj) : T(0);
}

__global__ void k_sqrt_clamp(const double* __restrict__ lam, int n, double* __restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) S[i] = lam[i] > 0.0 ? sqrt(lam[i]) : 0.0;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t total, int per) { return (unsigned)((total + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_gaussian_fill(uint64_t seed, int64_t rows, int64_t cols, double* G,
                                hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gaussian_fill, dim3(blocks_for((total + 1) / 2, 256)), dim3(256), 0, s,
                     seed, total, G);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cast_from_f64(const double* src, int64_t rows, int64_t cols, int64_t lds, T* dst,
                                int64_t ldd, hipStream_t s) {
  if (rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<double, T>), dim3(blocks_for(rows * cols, 256)), dim3(256), 0, s, src,
                     rows, cols, lds, dst, ldd);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cast_to_f64(const T* src, int64_t rows, int64_t cols, int64_t lds, double* dst,
                              int64_t ldd, hipStream_t s) {
  if (rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<T, double>), dim3(blocks_for(rows * cols, 256)), dim3(256), 0, s, src,
                     rows, cols, lds, dst, ldd);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_chol_inv(const double* W, int c, double* R, double* Rinv, T* RinvT,
                           int32_t* status, hipStream_t s) {
  const size_t shmem = (2 * (size_t)c * (c + 1) + c) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_inv<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_chol_inv<T>), dim3(1), dim3(kCholThreads), shmem, s, W, c, R, Rinv, RinvT,
                     status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_small_gemm(const double* A, const double* B, int64_t r, int c1, int c2, double* C,
                             T* CT, hipStream_t s) {
  if (r * c2 <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_small_gemm<T>), dim3(blocks_for(r * c2, 256)), dim3(256), 0, s, A, B, r,
                     c1, c2, C, CT);
  return hipGetLastError();
}

hipError_t launch_jacobi_svd_small(const double* M, int c, double* Uo, double* S, double* J,
                                   double* diag, int32_t* status, hipStream_t s) {
  const int npad = c + (c & 1);
  const size_t shmem = 2 * (size_t)npad * c * sizeof(double);
  // lanes per column pair: the largest power of two with npairs * G <= threads, at most 64
  int G = 64;
  while (G > 1 && (npad / 2) * G > kJsThreads) G >>= 1;
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_svd_small,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jacobi_svd_small, dim3(1), dim3(kJsThreads), shmem, s, M, c, Uo, S, J, diag,
                     status, G);
  return hipGetLastError();
}

hipError_t launch_jacobi_eig(double* X, double* J, int64_t n, double* lam, double* diag,
                             int32_t* flags, int32_t* status, hipStream_t s) {
  const int npairs = (int)((n + 1) / 2);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_jacobi_eig, kJeThreads, 0);
  if (e != hipSuccess) return e;
  const int wpb = kJeThreads / 64;
  int blocks = (npairs + wpb - 1) / wpb;
  const int resident = ncu * (per_cu > 0 ? per_cu : 1);
  if (blocks > resident) blocks = resident;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, flags, 2 + kJeMaxSweeps, 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {&X, &J, &n, &lam, &diag, &flags, &status};
  return hipLaunchCooperativeKernel((const void*)k_jacobi_eig, dim3(blocks), dim3(kJeThreads), args,
                                    0, s);
}

int jacobi_eig_flag_words() { return 2 + kJeMaxSweeps; }

template <typename T>
hipError_t launch_sort_sign_scatter(const double* S, int c, const double* Vsrc, int64_t r,
                                    int64_t vrs, int64_t vcs, const double* Wsrc, int kout,
                                    double* S_out, T* Vout, int64_t ldv, double* Vd_out,
                                    double* Wout, hipStream_t s) {
  hipLaunchKernelGGL((k_sort_sign_scatter<T>), dim3(1), dim3(1024), (size_t)c * sizeof(int), s, S,
                     c, Vsrc, r, vrs, vcs, Wsrc, kout, S_out, Vout, ldv, Vd_out, Wout);
  return hipGetLastError();
}

hipError_t launch_select_k(const double* S, int k, const double* fro2, double t, int32_t* K,
                           double* diag, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_select_k, dim3(1), dim3(64), 0, s, S, k, fro2, t, K, diag, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_cols_inv(const double* V, int64_t n, int cols, int64_t ldv, const double* S,
                                 double floor_rel, T* X, int64_t ldx, hipStream_t s) {
  if (n * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_scale_cols_inv<T>), dim3(blocks_for(n * cols, 256)), dim3(256), 0, s, V, n,
                     cols, ldv, S, floor_rel, X, ldx);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_sqrt_clamp(const double* lam, int n, double* S, hipStream_t s) {
  hipLaunchKernelGGL(k_sqrt_clamp, dim3(blocks_for(n, 256)), dim3(256), 0, s, lam, n, S);
  return hipGetLastError();
}

#define RSVD_INST(T)                                                                               \
  template hipError_t launch_cast_from_f64<T>(const double*, int64_t, int64_t, int64_t, T*,        \
                                              int64_t, hipStream_t);                               \
  template hipError_t launch_cast_to_f64<T>(const T*, int64_t, int64_t, int64_t, double*, int64_t, \
                                            hipStream_t);                                          \
  template hipError_t launch_chol_inv<T>(const double*, int, double*, double*, T*, int32_t*,      \
                                         hipStream_t);                                             \
  template hipError_t launch_small_gemm<T>(const double*, const double*, int64_t, int, int,       \
                                           double*, T*, hipStream_t);                              \
  template hipError_t launch_sort_sign_scatter<T>(const double*, int, const double*, int64_t,     \
                                                  int64_t, int64_t, const double*, int, double*,  \
                                                  T*, int64_t, double*, double*, hipStream_t);     \
  template hipError_t launch_scale_cols_inv<T>(const double*, int64_t, int, int64_t,              \
                                               const double*, double, T*, int64_t, hipStream_t);
RSVD_INST(float)
RSVD_INST(double)
#undef RSVD_INST

}  // namespace rsvd
