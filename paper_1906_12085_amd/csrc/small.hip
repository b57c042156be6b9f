// small.hip -- the FP64 work on n x l, l x l and n x n matrices between the
// passes over A: the Gaussian sketch, Cholesky factors and their inverses
// (CholeskyQR2), small products, the one-sided Jacobi SVD of the l x l
// factor, the sign rule and the explained-variance criterion.
#include "device_common.h"

namespace rsvd {

namespace {

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
__global__ void k_gaussian_fill(uint64_t seed, int64_t total, double* __restrict__ G,
                                const GArgFill* __restrict__ grp) {
  if (grp) {
    const GArgFill& a = grp[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk) return;
    seed = a.seed; total = a.total; G = a.G;
  }
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

// dst (cols x rows) = src^T, consecutive threads writing consecutive dst.
template <typename S, typename D>
__global__ void k_cast_t(const S* __restrict__ src, int64_t rows, int64_t cols, int64_t lds,
                         D* __restrict__ dst, int64_t ldd, const GArgCast* __restrict__ grp) {
  if (grp) {
    const GArgCast& a = grp[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk) return;
    src = (const S*)a.src; rows = a.rows; cols = a.cols; lds = a.lds; dst = (D*)a.dst;
    ldd = a.ldd;
  }
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  dst[j * ldd + i] = (D)src[i * lds + j];
}

// ---------------------------------------------------------------------------
// Cholesky factor R (upper, W = R^T R) and its inverse of a c x c SPD matrix
// (c <= 96), one workgroup of 256 threads, blocked in 16 x 16 blocks.  The
// matrix, padded to cp = 16 ceil(c / 16) with the identity, sits in LDS as
// its lower triangle A (turned into L = R^T in place), beside B (the identity,
// turned into L^-1 = R^-T).  For each block column k:
//   1. one wave factors the diagonal block, A_kk = L_kk L_kk^T, and inverts
//      it, X_kk = L_kk^-1, by the symmetric elimination applied to [A_kk | I]
//      with row r of both halves in the registers of lane r: at step j the
//      pivot, the pivot column (entry j of each row below) and the old row j
//      of X are read into scalar registers (readlane from fixed lanes), and
//      each row below subtracts its multiple (one FMA per entry); no
//      workgroup barrier.  Exchanging the pivot data through cross-lane
//      permutes instead (four entries per lane) took ~800 cycles a step;
//   2. L_ik = A_ik X_kk^T below it, and the block row k of B, B_kj <- X_kk B_kj
//      (j < k), B_kk = X_kk;
//   3. the trailing update A_ij -= L_ik L_jk^T (k < j <= i) and the rows below
//      in B, B_ij -= L_ik B_kj (i > k, j <= k).
// Steps 2 and 3 are 16 x 16 x 16 products on the FP64 matrix cores, spread
// over the four waves; three barriers per block column.  This is the block
// form of the elimination on [W | I] (Gauss-Jordan with the symmetric pivot).
// The element loops before and after run over rows and lanes (no index
// division), every global store coalesced.
constexpr int kCiT = 256;
constexpr int kCiMax = 96;

// 1/sqrt(x): hardware estimate plus two Newton steps.
__device__ __forceinline__ double rsq_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = fma(y, fma(-h * y, y, 0.5), y);
  return fma(y, fma(-h * y, y, 0.5), y);
}

// acc += sgn P Q for 16 x 16 blocks P, Q in LDS (row stride ld); QT: Q is
// read as the transpose of the block at Q.  FP64 16x16x4 operands: lane
// (x, y) = (l % 16, l / 16) supplies P[x][4s + y] and Q[4s + y][x].
template <bool QT>
__device__ __forceinline__ f64x4 mm16(const double* P, const double* Q, int ld, double sgn,
                                      f64x4 acc) {
  const int lane = threadIdx.x & 63, x = lane & 15, y = lane >> 4;
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const double av = sgn * P[x * ld + 4 * s4 + y];
    const double bv = QT ? Q[x * ld + 4 * s4 + y] : Q[(4 * s4 + y) * ld + x];
    acc = Mfma<double>::run(av, bv, acc);
  }
  return acc;
}
// a 16 x 16 block in the matrix-core output layout (value e of lane l at row
// l / 16 + 4 e, column l % 16)
__device__ __forceinline__ f64x4 ld16(const double* C, int ld) {
  const int lane = threadIdx.x & 63;
  f64x4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = C[Mfma<double>::row(lane, e) * ld + (lane & 15)];
  return v;
}
__device__ __forceinline__ void st16(double* C, int ld, f64x4 v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 4; ++e) C[Mfma<double>::row(lane, e) * ld + (lane & 15)] = v[e];
}

// a double broadcast from lane `src` (a constant) of the wave
__device__ __forceinline__ double readlane_d(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

template <typename T>
__global__ __launch_bounds__(kCiT) void k_chol_inv(const double* __restrict__ W, int c,
                                                   double* __restrict__ R,
                                                   double* __restrict__ Rinv,
                                                   T* __restrict__ RinvT, int trans,
                                                   int32_t* __restrict__ status,
                                                   const GArgChol* __restrict__ grp) {
  if (grp) {
    const GArgChol& a = grp[blockIdx.y];
    W = a.W; c = a.c; R = a.R; Rinv = a.Rinv; RinvT = (T*)a.RinvT; trans = a.trans;
    status = a.status;
  }
  extern __shared__ double csm[];
  const int nb = (c + 15) >> 4, cp = 16 * nb, ld = cp + 1;
  double* Ls = csm;                  // A, then L (lower blocks)
  double* Bs = csm + cp * ld;        // I, then L^-1 (lower blocks)
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int kWaves = kCiT / 64, kRows = kCiMax / kWaves, kCols = (kCiMax + 63) / 64;
  // global memory through address-space-1 pointers: generic (flat) accesses
  // may alias LDS, and the compiler then orders them against every LDS access
  const gmem<double>* Wg = to_global(W);
  // thread (u, h) covers element (i, j) = (w + 4 u, l + 64 h) of the padded
  // matrix (wave w, lane l), clamped into it: a clamped copy computes and
  // writes the same value as the element's owner, so no access is predicated
  double v[kRows][kCols];
  {
    double wt[kRows][kCols];
    // every load of a thread in flight at once (one memory latency): w_ij
    // and w_ji (indices clamped into W)
#pragma unroll
    for (int u = 0; u < kRows; ++u)
#pragma unroll
      for (int h = 0; h < kCols; ++h) {
        const int i = min(wave + kWaves * u, c - 1), j = min(lane + 64 * h, c - 1);
        v[u][h] = Wg[(size_t)i * c + j];
        wt[u][h] = Wg[(size_t)j * c + i];
      }
    // A: the lower triangle (w_ij + w_ji) / 2, the rest w_ij; the identity
    // past c in A, and in B throughout
#pragma unroll
    for (int u = 0; u < kRows; ++u)
#pragma unroll
      for (int h = 0; h < kCols; ++h) {
        const int i = min(wave + kWaves * u, cp - 1), j = min(lane + 64 * h, cp - 1);
        const double a0 = (i > j) ? 0.5 * (v[u][h] + wt[u][h]) : v[u][h];
        Ls[i * ld + j] = (i < c && j < c) ? a0 : ((i == j) ? 1.0 : 0.0);
        Bs[i * ld + j] = (i == j) ? 1.0 : 0.0;
      }
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const int k0 = 16 * k;
    if (wave == 0) {
      // 1. lane r (and its copies r + 16, r + 32, r + 48) holds row r of the
      // block in a and of X in x
      const int r = lane & 15;
      double a[16], x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        a[q] = Ls[(k0 + r) * ld + k0 + q];
        x[q] = (q == r) ? 1.0 : 0.0;
      }
      bool badl = false;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double p = readlane_d(a[j], j);                     // pivot a_jj
        badl |= !(p > 0.0);
        double sc[16], tx[16];
#pragma unroll
        for (int q = j + 1; q < 16; ++q) sc[q] = readlane_d(a[j], q);   // a_qj, q > j
#pragma unroll
        for (int q = 0; q <= j; ++q) tx[q] = readlane_d(x[q], j);       // old row j of X
        const double rs = rsq_newton(p);
        // branch-free: rows above and at the pivot take multiple 0 (an
        // exact no-op of the FMAs), rows other than the pivot's scale 1
        const double f = (r > j) ? a[j] * (rs * rs) : 0.0;           // l_rj / l_jj
        const double g = (r == j) ? rs : 1.0;
#pragma unroll
        for (int q = j + 1; q < 16; ++q) a[q] = fma(-f, sc[q], a[q]);
#pragma unroll
        for (int q = 0; q <= j; ++q) x[q] = fma(-f, tx[q], x[q]) * g;
        a[j] *= (r >= j) ? rs : 1.0;                                 // l_rj (l_jj at r = j)
      }
      if (lane < 16) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          Ls[(k0 + r) * ld + k0 + q] = (q <= r) ? a[q] : 0.0;
          Bs[(k0 + r) * ld + k0 + q] = (q <= r) ? x[q] : 0.0;
        }
      }
      if (badl && lane == 0) bad = 1;
    }
    __syncthreads();
    // 2. panel and block row k of B
    const int m1 = nb - k - 1;
    for (int t = wave; t < m1 + k; t += 4) {
      if (t < m1) {
        const int i0 = 16 * (k + 1 + t);
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mm16<true>(Ls + i0 * ld + k0, Bs + k0 * ld + k0, ld, 1.0, acc);   // A_ik X_kk^T
        st16(Ls + i0 * ld + k0, ld, acc);
      } else {
        const int j0 = 16 * (t - m1);
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mm16<false>(Bs + k0 * ld + k0, Bs + k0 * ld + j0, ld, 1.0, acc);  // X_kk B_kj
        st16(Bs + k0 * ld + j0, ld, acc);
      }
    }
    __syncthreads();
    // 3. trailing update of A and the rows of B below block row k
    const int nA = m1 * (m1 + 1) / 2, nBt = m1 * (k + 1);
    for (int t = wave; t < nA + nBt; t += 4) {
      if (t < nA) {
        int ii = 0, rem = t;
        while (rem > ii) {
          rem -= ii + 1;
          ++ii;
        }
        const int i0 = 16 * (k + 1 + ii), j0 = 16 * (k + 1 + rem);
        f64x4 acc = ld16(Ls + i0 * ld + j0, ld);
        acc = mm16<true>(Ls + i0 * ld + k0, Ls + j0 * ld + k0, ld, -1.0, acc);  // -L_ik L_jk^T
        st16(Ls + i0 * ld + j0, ld, acc);
      } else {
        const int u = t - nA, ii = u / (k + 1), jj = u - ii * (k + 1);
        const int i0 = 16 * (k + 1 + ii), j0 = 16 * jj;
        f64x4 acc = ld16(Bs + i0 * ld + j0, ld);
        acc = mm16<false>(Ls + i0 * ld + k0, Bs + k0 * ld + j0, ld, -1.0, acc); // -L_ik B_kj
        st16(Bs + i0 * ld + j0, ld, acc);
      }
    }
    __syncthreads();
  }
  gmem<double>* Rg = to_global(R);
  gmem<double>* Rig = to_global(Rinv);
  gmem<T>* RTg = to_global(RinvT);
  if (bad) {
    // R = 0 (no factor), Rinv = I keeps the later products finite
    for (int i = wave; i < c; i += kWaves)
      for (int j = lane; j < c; j += 64) {
        const double v1 = (i == j) ? 1.0 : 0.0;
        if (R) Rg[i * c + j] = 0.0;
        if (Rinv) Rig[i * c + j] = v1;
        if (RinvT) RTg[i * c + j] = (T)v1;
      }
    if (tid == 0) set_error(status, RSVD_ERR_BREAKDOWN);
    return;
  }
  // R = L^T: R_ij = L_ji; R^-1 = (L^-1)^T: (R^-1)_ij = B_ji, row i of both
  // from column i in LDS (stride ld odd: no bank conflicts); RinvT is R^-1
  // or, with trans, its transpose B.  Indices clamped into c x c as above;
  // four rows per batch: the LDS reads of a batch in flight together, then
  // its coalesced stores.  A null R or Rinv is not written.
  constexpr int kBatch = 4;
  static_assert(kRows % kBatch == 0, "whole batches of rows");
#pragma unroll
  for (int u0 = 0; u0 < kRows; u0 += kBatch) {
    double rv[kBatch][kCols], xv[kBatch][kCols], bv[kBatch][kCols];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int h = 0; h < kCols; ++h) {
        const int i = min(wave + kWaves * (u0 + u), c - 1), j = min(lane + 64 * h, c - 1);
        rv[u][h] = (j >= i) ? Ls[j * ld + i] : 0.0;
        xv[u][h] = Bs[j * ld + i];
        bv[u][h] = Bs[i * ld + j];
      }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int h = 0; h < kCols; ++h) {
        const int i = min(wave + kWaves * (u0 + u), c - 1), j = min(lane + 64 * h, c - 1);
        if (R) Rg[i * c + j] = rv[u][h];
        if (Rinv) Rig[i * c + j] = xv[u][h];
        if (RinvT) RTg[i * c + j] = (T)(trans ? bv[u][h] : xv[u][h]);
      }
  }
}

// LDS bytes of k_chol_inv for c columns
size_t chol_inv_lds(int c) {
  const size_t cp = 16 * (size_t)((c + 15) / 16);
  return 2 * cp * (cp + 1) * sizeof(double);
}

// ---------------------------------------------------------------------------
// The same factorisation for 96 < c <= 192, one workgroup of 1024 threads.
// W and B cannot both sit in registers at this width, but they never
// overlap: the symmetric elimination only ever needs W on and right of the
// diagonal (its trailing part is kept as an upper triangle), and row i of
// B = L^-1 has nonzeros only in columns k <= i.  So one c x c array P holds
// W (then R) in k >= i and B in k < i; B's diagonal, 1/sqrt(d_i), is kept
// apart in LDS.  Thread (ti, tk) = (tid / 32, tid % 32) keeps the elements
// (ti + 32u, tk + 32v), u, v < U; the 32 owners of a row are one half of a
// wave.  Step j: the owners of row j take d = p_jj, scale the row by
// r = 1/sqrt(d) (R right of the diagonal, B left of it), set p_jj = sqrt(d)
// and publish x = the row with r in the diagonal slot; every row i > j then
// subtracts r_ji x_k from its columns k >= i (the trailing triangle of W)
// and k <= j (its row of B), and leaves j < k < i at zero.  One barrier per
// step (the published rows alternate between two LDS buffers).
constexpr int kCwT = 1024;
constexpr int kCwMax = 192;                   // 32 * 6

template <int U, int JU>
__device__ __forceinline__ void chol_wide_block(double (&a)[U][U], int c, int ti, int tk, int lane,
                                                int wv, double (*xrow)[kCwMax], double* rdiag,
                                                int* bad) {
  for (int jj = 0; jj < 32; ++jj) {
    const int j = 32 * JU + jj;
    if (j >= c) return;
    const int p = j & 1;
    if (ti == jj) {
      const double d = __shfl(a[JU][JU], (lane & 32) + jj);
      if (!(d > 0.0)) *bad = 1;
      const double r = rsq_newton(d);
      const double sd = d * r;
#pragma unroll
      for (int v = 0; v < U; ++v) {
        const int k = tk + 32 * v;
        const double nv = (k == j) ? sd : a[JU][v] * r;
        if (k < c) a[JU][v] = nv;
        xrow[p][k] = (k < c) ? ((k == j) ? r : nv) : 0.0;
      }
      if (tk == 0) rdiag[j] = r;
    }
    __syncthreads();
    double xv[U];
#pragma unroll
    for (int v = 0; v < U; ++v) xv[v] = xrow[p][tk + 32 * v];
#pragma unroll
    for (int u = JU; u < U; ++u) {
      if (32 * u + 2 * wv + 1 <= j) continue;   // no row of this wave is below j
      const int i = ti + 32 * u;
      const double rji = (i > j && i < c) ? xrow[p][i] : 0.0;
#pragma unroll
      for (int v = 0; v < U; ++v) {
        const int k = tk + 32 * v;
        const double coef = (k >= i || k <= j) ? xv[v] : 0.0;
        a[u][v] = fma(-rji, coef, a[u][v]);
      }
    }
  }
}

template <int U, int JU>
__device__ __forceinline__ void chol_wide_all(double (&a)[U][U], int c, int ti, int tk, int lane,
                                              int wv, double (*xrow)[kCwMax], double* rdiag,
                                              int* bad) {
  if constexpr (JU < U) {
    chol_wide_block<U, JU>(a, c, ti, tk, lane, wv, xrow, rdiag, bad);
    chol_wide_all<U, JU + 1>(a, c, ti, tk, lane, wv, xrow, rdiag, bad);
  }
}

template <typename T, int U>
__global__ __launch_bounds__(kCwT) void k_chol_inv_wide(const double* __restrict__ W, int c,
                                                        double* __restrict__ R,
                                                        double* __restrict__ Rinv,
                                                        T* __restrict__ RinvT, int trans,
                                                        int32_t* __restrict__ status,
                                                        const GArgChol* __restrict__ grp) {
  if (grp) {
    const GArgChol& a = grp[blockIdx.y];
    W = a.W; c = a.c; R = a.R; Rinv = a.Rinv; RinvT = (T*)a.RinvT; trans = a.trans;
    status = a.status;
  }
  __shared__ double xrow[2][kCwMax];
  __shared__ double rdiag[kCwMax];
  __shared__ int bad;
  const int tid = threadIdx.x, ti = tid >> 5, tk = tid & 31, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // device memory through global pointers (generic ones would order every
  // access against the LDS traffic of the elimination)
  const gmem<double>* Wg = to_global(W);
  gmem<double>* Rg = to_global(R);
  gmem<double>* Rig = to_global(Rinv);
  gmem<T>* RTg = to_global(RinvT);
  double a[U][U];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const int i = ti + 32 * u, k = tk + 32 * v;
      a[u][v] = (i < c && k < c && k >= i) ? 0.5 * (Wg[i * c + k] + Wg[k * c + i]) : 0.0;
    }
  if (tid == 0) bad = 0;
  __syncthreads();
  chol_wide_all<U, 0>(a, c, ti, tk, lane, wv, xrow, rdiag, &bad);
  __syncthreads();
  if (bad) {
    for (int idx = tid; idx < c * c; idx += kCwT) {
      const int i = idx / c, j = idx - i * c;
      const double v = (i == j) ? 1.0 : 0.0;
      if (R) Rg[idx] = 0.0;
      if (Rinv) Rig[idx] = v;
      if (RinvT) RTg[idx] = (T)v;
    }
    if (tid == 0) set_error(status, RSVD_ERR_BREAKDOWN);
    return;
  }
  // P(i, k): R for k >= i; (L^-1)_ik = (R^-1)_ki for k < i, 1/r_ii on the diagonal
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const int i = ti + 32 * u, k = tk + 32 * v;
      if (i < c && k < c) {
        if (R) Rg[i * c + k] = k >= i ? a[u][v] : 0.0;
        const double x = k < i ? a[u][v] : (k == i ? rdiag[i] : 0.0);
        if (Rinv) Rig[k * c + i] = x;
        if (RinvT) RTg[trans ? i * c + k : k * c + i] = (T)x;
      }
    }
}

// C (r x c2) = A (r x c1) B (c1 x c2), FP64, all row-major and contiguous,
// one thread per output; optionally also CT = C cast to T (transposed with
// trans).  For the small products between the passes (c1, c2 <= 192).
template <typename T>
__global__ void k_small_gemm(const double* __restrict__ A, const double* __restrict__ B,
                             int64_t r, int c1, int c2, double* __restrict__ C, T* __restrict__ CT,
                             int trans, const GArgSg* __restrict__ grp) {
  if (grp) {
    const GArgSg& a = grp[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk) return;
    A = a.A; B = a.B; r = a.r; c1 = a.c1; c2 = a.c2; C = a.C; CT = (T*)a.CT; trans = a.trans;
  }
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r * c2) return;
  const int64_t i = idx / c2;
  const int j = (int)(idx - i * c2);
  const gmem<double>* a = to_global(A) + i * c1;
  const gmem<double>* b = to_global(B) + j;
  // the sum in k order (one FMA chain); the loads of 16 steps in flight at
  // once, not one step's at a time
  constexpr int KU = 16;
  double s = 0.0;
  int k = 0;
  for (; k + KU <= c1; k += KU) {
    double av[KU], bv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      av[u] = a[k + u];
      bv[u] = b[(int64_t)(k + u) * c2];
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) s = fma(av[u], bv[u], s);
  }
  for (; k < c1; ++k) s = fma(a[k], b[(int64_t)k * c2], s);
  if (C) to_global(C)[idx] = s;
  if (CT) to_global(CT)[trans ? (int64_t)j * r + i : idx] = (T)s;
}

// One-sided Jacobi SVD of a c x c matrix M (c <= 96) in one block: the
// columns of M held column-major in LDS, padded with zero rows to cs = 16 RU2
// (RU2 = ceil(c / 16), a template parameter).  Each group of 8 lanes owns one
// column pair per step (round-robin ordering); lane g of the group keeps rows
// 2 g + 16 u and 2 g + 1 + 16 u (u < RU2) of both columns in registers, read
// and written as 16-byte pairs, so each load or store of a group is one
// contiguous 128-byte line (bank-conflict free whatever the columns; with
// 8-byte accesses two groups of a half-wave met in the same banks whenever
// their columns were a multiple of 128 bytes apart).  The squared column
// norms sit in LDS: computed exactly at the start of each sweep and, after a
// rotation by tangent t, updated as alpha - t gamma and beta + t gamma (the
// norms of the rotated columns), so a step reduces only gamma = x_p . x_q
// across the group.  A round reads and writes the whole matrix in LDS and
// that traffic, not the arithmetic, bounds it.  Whether a group rotated, and
// the largest cosine it rotated, stay in registers until the sweep ends.
// With transpose != 0 the kernel works on M^T (the rows of Min are its
// columns).  AccJ: the rotations are accumulated in a second LDS matrix J
// and written out.  Otherwise they are not: at convergence N J = Uo S with
// N = M or M^T, so J = N^-1 Uo S and, for N = R^T, J = R Uo S^-1 -- the
// kernel writes Uo S^-1 (zero columns for zero values) in J's place and the
// caller forms the columns of J it needs with one small product.  Keeping J
// out of the rounds removes a third of their loads, stores and FP64
// operations; J's column j then carries an error of order eps S_1 / S_j, so
// this form serves callers that use the leading columns only, and it sets
// *redo when the values span more than 1 / kJsRedoRatio (or one is zero): a
// second launch with AccJ and the same redo word then repeats the
// decomposition with J accumulated (and returns at once when *redo is 0).
constexpr int kJsG = 8;
constexpr int kJsMaxRu2 = 6;                 // c <= 16 * kJsMaxRu2
constexpr int kJsMaxC = 16 * kJsMaxRu2;
constexpr int kJsMaxSweeps = 60;
constexpr double kJsRedoRatio = 1e-6;

template <bool AccJ, int RU2>
__global__ __launch_bounds__(kJsMaxC / 2 * kJsG) void k_jacobi_svd_small(
    const double* __restrict__ Min, int c, int transpose, double* __restrict__ Uo,
    double* __restrict__ S, double* __restrict__ Jout, double* __restrict__ diag,
    int32_t* __restrict__ status, double* __restrict__ redo, const GArgJac* __restrict__ garg) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  if (garg) {
    const GArgJac& a = garg[blockIdx.y];
    Min = a.M; c = a.c; transpose = a.transpose; Uo = a.Uo; S = a.S; Jout = a.J; diag = a.diag;
    status = a.status; redo = a.redo;
  }
  if (AccJ && redo && *redo == 0.0) return;  // uniform: the first pass needed no J
  constexpr int cs = 16 * RU2;               // LDS rows per column
  extern __shared__ __attribute__((aligned(16))) double sm[];
  double* Mc = sm;                           // column j at Mc + j*cs
  double* Jc = sm + (size_t)cs * c;          // AccJ only
  __shared__ int rotated;
  __shared__ double offmax;
  __shared__ double nrm2[kJsMaxC];           // squared column norms
  __shared__ double snrm[kJsMaxC];
  const int npad = c + (c & 1);
  const int tid = threadIdx.x, nthr = blockDim.x;
  // Min read in its row-major order, four loads in flight per thread
  for (int idx0 = tid; idx0 < c * c; idx0 += 4 * nthr) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = idx0 + u * nthr;
      v[u] = idx < c * c ? Min[idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = idx0 + u * nthr;
      if (idx < c * c) {
        const int i = idx / c, j = idx - i * c;   // Min row-major (i, j)
        if (transpose) Mc[i * cs + j] = v[u];    // column i of M^T is row i of Min
        else Mc[j * cs + i] = v[u];
      }
    }
  }
  for (int idx = tid; idx < cs * c; idx += nthr) {
    const int j = idx / cs, i = idx - j * cs;
    if (i >= c) Mc[idx] = 0.0;                   // the padding rows
    if (AccJ) Jc[idx] = (i == j) ? 1.0 : 0.0;
  }
  const int npairs = npad / 2, ngroups = nthr / kJsG;
  const int grp = tid / kJsG, gl = tid % kJsG;
  const double tol = kEps * (double)c, tol2 = tol * tol;
  int sweep = 0;
  bool converged = false;
  double last_off = 0.0;
  __syncthreads();
  while (sweep < kJsMaxSweeps) {
    if (tid == 0) { rotated = 0; offmax = 0.0; }
    for (int j = grp; j < c; j += ngroups) {   // exact squared norms
      const d2* x = reinterpret_cast<const d2*>(Mc + (size_t)j * cs) + gl;
      double s2 = 0.0;
#pragma unroll
      for (int u = 0; u < RU2; ++u) {
        const d2 v = x[kJsG * u];
        s2 = fma(v.x, v.x, s2);
        s2 = fma(v.y, v.y, s2);
      }
      s2 = group_sum<kJsG>(s2);
      if (gl == 0) nrm2[j] = s2;
    }
    __syncthreads();
    bool my_rot = false;
    double my_off = 0.0;                     // squared cosine, approximate (diagnostic only)
    for (int s = 0; s < npad - 1; ++s) {
      int p = 0, q = c;
      if (grp < npairs) rr_pair(s, grp, npad, &p, &q);
      if (grp < npairs && q < c) {           // uniform within the 8-lane group
        d2* xp = reinterpret_cast<d2*>(Mc + (size_t)p * cs) + gl;
        d2* xq = reinterpret_cast<d2*>(Mc + (size_t)q * cs) + gl;
        d2* jp = reinterpret_cast<d2*>(Jc + (size_t)p * cs) + gl;
        d2* jq = reinterpret_cast<d2*>(Jc + (size_t)q * cs) + gl;
        const double al = nrm2[p], be = nrm2[q];
        // all reads of the two columns (and their J columns) before any write
        d2 a[RU2], b[RU2], ja[RU2], jb[RU2];
#pragma unroll
        for (int u = 0; u < RU2; ++u) {
          a[u] = xp[kJsG * u];
          b[u] = xq[kJsG * u];
          if (AccJ) {
            ja[u] = jp[kJsG * u];
            jb[u] = jq[kJsG * u];
          }
        }
        double ga = 0.0;
#pragma unroll
        for (int u = 0; u < RU2; ++u) {
          ga = fma(a[u].x, b[u].x, ga);
          ga = fma(a[u].y, b[u].y, ga);
        }
        ga = group_sum<kJsG>(ga);
        // rotate when the cosine of the pair's angle exceeds tol
        if (rot_needed(al, be, ga, tol2, 0.0)) {
          double cs_, sn, tt;
          rot_cst(al, be, ga, true, &cs_, &sn, &tt);
#pragma unroll
          for (int u = 0; u < RU2; ++u) {
            xp[kJsG * u] = cs_ * a[u] - sn * b[u];
            xq[kJsG * u] = sn * a[u] + cs_ * b[u];
            if (AccJ) {
              jp[kJsG * u] = cs_ * ja[u] - sn * jb[u];
              jq[kJsG * u] = sn * ja[u] + cs_ * jb[u];
            }
          }
          if (gl == 0) {
            nrm2[p] = fma(-tt, ga, al);
            nrm2[q] = fma(tt, ga, be);
          }
          my_rot = true;
          my_off = fmax(my_off, ga * ga * __builtin_amdgcn_rcp(al * be));
        }
      }
      __syncthreads();
    }
    // the groups' flags (the last round's barrier orders these writes after
    // the reset; the racing maximum is a diagnostic only)
    if (my_rot && gl == 0) {
      rotated = 1;
      if (my_off > offmax) offmax = my_off;
    }
    __syncthreads();
    ++sweep;
    last_off = sqrt(offmax);
    const bool done = (rotated == 0);
    __syncthreads();
    if (done) { converged = true; break; }
  }
  // singular values = column norms, Uo = normalised columns, J or Uo S^-1
  for (int j = tid / 64; j < c; j += nthr / 64) {
    const int lane = tid & 63;
    double s2 = 0.0;
    for (int i = lane; i < c; i += 64) s2 += Mc[(size_t)j * cs + i] * Mc[(size_t)j * cs + i];
    s2 = group_sum<64>(s2);
    const double nrm = sqrt(s2);
    if (lane == 0) {
      S[j] = nrm;
      snrm[j] = nrm;
    }
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = lane; i < c; i += 64) {
      const double u = Mc[(size_t)j * cs + i] * inv;
      Uo[(size_t)i * c + j] = u;
      Jout[(size_t)i * c + j] = AccJ ? Jc[(size_t)j * cs + i] : u * inv;
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (!AccJ && redo) {
      double mx = 0.0, mn = snrm[0];
      for (int j = 0; j < c; ++j) {
        mx = fmax(mx, snrm[j]);
        mn = fmin(mn, snrm[j]);
      }
      const bool again = !(mn > kJsRedoRatio * mx);
      *redo = again ? 1.0 : 0.0;
    }
    diag[2] = (double)sweep;
    diag[3] = last_off;
    if (!converged) set_error(status, RSVD_ERR_NOCONV);
  }
}

// ---------------------------------------------------------------------------
// Sort by S descending (ties: lower index first), apply the sign rule to the
// first kout vectors and scatter them.  Source vector column `col`, element
// i is at Vsrc[i * vrs + col * vcs].  Block b handles output columns
// [16 b, 16 b + 16): every block ranks all c keys in LDS (c^2 comparisons,
// cheap next to the scatter), a wave per column finds the sign, and the
// scatter writes 16 consecutive outputs of a row together.
constexpr int kSsCols = 16;
constexpr int kSsReg = 8;     // rows per lane held in registers by the sign scan
constexpr int kSsUnroll = 8;  // scatter rows per thread with their loads in flight

template <typename T>
__global__ __launch_bounds__(256) void k_sort_sign_scatter(
    const double* __restrict__ S, int c, const double* __restrict__ Vsrc, int64_t r, int64_t vrs,
    int64_t vcs, const double* __restrict__ Wsrc, int kout, double* __restrict__ S_out,
    T* __restrict__ Vout, int64_t ldv, double* __restrict__ Vd_out, double* __restrict__ Wout,
    const GArgSort* __restrict__ grp) {
  if (grp) {
    const GArgSort& a = grp[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk) return;
    S = a.S; c = a.c; Vsrc = a.Vsrc; r = a.r; vrs = a.vrs; vcs = a.vcs; Wsrc = a.Wsrc;
    kout = a.kout; S_out = a.S_out; Vout = (T*)a.Vout; ldv = a.ldv; Vd_out = a.Vd_out;
    Wout = a.Wout;
  }
  extern __shared__ double Sl[];              // c keys, then c ints
  int* perm = reinterpret_cast<int*>(Sl + c);
  __shared__ int src_l[kSsCols];
  __shared__ double sg_l[kSsCols];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kk0 = blockIdx.x * kSsCols;
  const int ncol = min(kSsCols, kout - kk0);
  stage_to_lds(Sl, S, c);
  for (int i = tid; i < c; i += blockDim.x) perm[i] = i;   // NaN keys may leave slots unranked
  __syncthreads();
  for (int i = tid; i < c; i += blockDim.x) {
    const double si = Sl[i];
    int rank = 0;
    for (int j = 0; j < c; ++j) {
      const double sj = Sl[j];
      rank += (sj > si) || (sj == si && j < i);
    }
    if (rank < c) perm[rank] = i;
  }
  __syncthreads();
  // sign rule: the first entry within 0.999 of the largest magnitude is positive.
  // Wave w takes the block's columns w, w + 4, w + 8, w + 12; the first
  // 64 kSsReg rows of all of them are read into registers at once (every
  // load in flight together), rows past those (r > 64 kSsReg) in the loops
  // after, and the sign of the chosen entry comes from the lane that holds it.
  constexpr int kQ = kSsCols / 4;
  double av[kQ][kSsReg];
  int srcq[kQ];
#pragma unroll
  for (int jq = 0; jq < kQ; ++jq) {
    const int q = wave + 4 * jq;
    int src = q < ncol ? perm[kk0 + q] : 0;
    if (src < 0 || src >= c) src = q < ncol ? kk0 + q : 0;
    srcq[jq] = src;
    const double* col = Vsrc + (int64_t)src * vcs;
#pragma unroll
    for (int t = 0; t < kSsReg; ++t) {
      const int64_t i = lane + 64 * t;
      av[jq][t] = (q < ncol && i < r) ? col[i * vrs] : 0.0;
    }
  }
#pragma unroll
  for (int jq = 0; jq < kQ; ++jq) {
    const int q = wave + 4 * jq;
    if (q >= ncol) continue;                  // uniform per wave
    const int kk = kk0 + q, src = srcq[jq];
    const double* col = Vsrc + (int64_t)src * vcs;
    double vmax = 0.0;
#pragma unroll
    for (int t = 0; t < kSsReg; ++t) vmax = fmax(vmax, fabs(av[jq][t]));
    for (int64_t i = lane + 64 * kSsReg; i < r; i += 64) vmax = fmax(vmax, fabs(col[i * vrs]));
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
    int64_t first = r;
#pragma unroll
    for (int t = kSsReg - 1; t >= 0; --t) {
      const int64_t i = lane + 64 * t;
      if (i < r && fabs(av[jq][t]) >= 0.999 * vmax) first = i;
    }
    if (first == r)
      for (int64_t i = lane + 64 * kSsReg; i < r; i += 64)
        if (fabs(col[i * vrs]) >= 0.999 * vmax) { first = i; break; }
    for (int off = 32; off > 0; off >>= 1) {
      const int64_t o = __shfl_xor(first, off);
      first = o < first ? o : first;
    }
    // the chosen entry (first is the same in every lane)
    double fv = 0.0;
#pragma unroll
    for (int t = 0; t < kSsReg; ++t)
      if (lane + 64 * t == first) fv = av[jq][t];
    if (first < 64 * kSsReg) fv = __shfl(fv, (int)(first & 63));
    else if (first < r) fv = col[first * vrs];
    if (lane == 0) {
      src_l[q] = src;
      sg_l[q] = (first < r && fv < 0.0) ? -1.0 : 1.0;
      S_out[kk] = Sl[src];
    }
  }
  __syncthreads();
  // scatter: thread (ri, cj) moves element (i, cj) of 16 rows per pass
  const int cj = tid % kSsCols, ri = tid / kSsCols;
  if (cj < ncol) {
    const int src = src_l[cj];
    const double sg = sg_l[cj];
    const int kk = kk0 + cj;
    const double* col = Vsrc + (int64_t)src * vcs;
    constexpr int RS = 256 / kSsCols;           // rows between a thread's rows
    for (int64_t i0 = ri; i0 < r; i0 += RS * kSsUnroll) {
      double v[kSsUnroll];
#pragma unroll
      for (int u = 0; u < kSsUnroll; ++u) {
        const int64_t i = i0 + RS * u;
        v[u] = i < r ? sg * col[i * vrs] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kSsUnroll; ++u) {
        const int64_t i = i0 + RS * u;
        if (i < r) {
          if (Vout) Vout[i * ldv + kk] = (T)v[u];
          if (Vd_out) Vd_out[i * kout + kk] = v[u];
        }
      }
    }
    if (Wsrc && Wout)
      for (int i = ri; i < c; i += 256 / kSsCols) Wout[(int64_t)i * kout + kk] = sg * Wsrc[(int64_t)i * c + src];
  }
}

// Cumulative explained variance criterion (Sec. 2.4): minimal K <= k with
// sum_{i<=K} s_i^2 >= t * ||A||_F^2 (Eq. sumeigen gives the denominator).
__global__ void k_select_k(const double* __restrict__ S, int k, const double* __restrict__ fro2,
                           double t, int32_t* __restrict__ K, double* __restrict__ diag,
                           int32_t* __restrict__ status, const GArgSel* __restrict__ grp) {
  if (grp) {
    const GArgSel& a = grp[blockIdx.y];
    S = a.S; k = a.k; fro2 = a.fro2; t = a.t; K = a.K; diag = a.diag; status = a.status;
  }
  extern __shared__ double Sl[];
  stage_to_lds(Sl, S, k);
  __syncthreads();
  if (threadIdx.x != 0) return;
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
    cum += Sl[i] * Sl[i];
    if (cum >= t * f2) { kk = i + 1; hit = true; break; }
  }
  *K = kk;
  diag[1] = cum / f2;
  diag[4] = (double)kk;
  if (!hit) set_warning(status, RSVD_WARN_THRESHOLD);
}

// X = V diag(1/S) (zero columns below the floor); trans != 0 writes X^T
// (cols x n) instead, indexed so that consecutive threads write
// consecutive elements either way.
template <typename T>
__global__ void k_scale_cols_inv(const double* __restrict__ V, int64_t n, int cols, int64_t ldv,
                                 const double* __restrict__ S, double floor_rel,
                                 T* __restrict__ X, int64_t ldx, int trans) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * cols) return;
  int64_t i;
  int j;
  if (trans) { j = (int)(idx / n); i = idx - (int64_t)j * n; }
  else { i = idx / cols; j = (int)(idx - i * cols); }
  const double sj = S[j];
  const T v = (sj > floor_rel * S[0]) ? (T)(V[i * ldv + j] / sj) : T(0);
  if (trans) X[(int64_t)j * ldx + i] = v;
  else X[i * ldx + j] = v;
}

// Xt (cols x rows) = X^T through a 32 x 33 LDS tile (both sides coalesced).
__global__ void k_transpose_f32(const float* __restrict__ X, int64_t rows, int64_t cols,
                                int64_t ldx, float* __restrict__ Xt, int64_t ldxt) {
  __shared__ float tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;     // 256 threads: 8 rows at a time
  for (int rr = ty; rr < 32; rr += 8) {
    const int64_t r = r0 + rr, c = c0 + tx;
    tile[rr][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.f;
  }
  __syncthreads();
  for (int cc = ty; cc < 32; cc += 8) {
    const int64_t c = c0 + cc, r = r0 + tx;
    if (c < cols && r < rows) Xt[c * ldxt + r] = tile[tx][cc];
  }
}

__global__ void k_sqrt_clamp(const double* __restrict__ lam, int n, double* __restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) S[i] = lam[i] > 0.0 ? sqrt(lam[i]) : 0.0;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// W (c x c Gram of an m x c matrix) += shift I, shift = 11 (m c + c (c+1)) u
// ||X||_F^2 with u = 2^-53 and ||X||_F^2 = trace(W) (the shift of shifted
// CholeskyQR, Fukaya et al., SIAM J. Sci. Comput. 2020: it bounds the first
// factor's condition number so that CholeskyQR2 completes afterwards).
__global__ void k_shift_diag(double* __restrict__ W, int c, int64_t m) {
  __shared__ double tr;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < c; ++i) t += W[(int64_t)i * c + i];
    tr = t;
  }
  __syncthreads();
  const double shift = 11.0 * ((double)m * c + (double)c * (c + 1)) * 0x1p-53 * tr;
  for (int i = threadIdx.x; i < c; i += blockDim.x) W[(int64_t)i * c + i] += shift;
}

inline unsigned blocks_for(int64_t total, int per) { return (unsigned)((total + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_gaussian_fill(uint64_t seed, int64_t rows, int64_t cols, double* G,
                                hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gaussian_fill, dim3(blocks_for((total + 1) / 2, 256)), dim3(256), 0, s,
                     seed, total, G, nullptr);
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
hipError_t launch_cast_t_from_f64(const double* src, int64_t rows, int64_t cols, int64_t lds, T* dst,
                                  int64_t ldd, hipStream_t s) {
  if (rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast_t<double, T>), dim3(blocks_for(rows * cols, 256)), dim3(256), 0, s, src,
                     rows, cols, lds, dst, ldd, nullptr);
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
                           int32_t* status, hipStream_t s, int trans) {
  if (c < 1 || c > kCwMax) return hipErrorInvalidValue;
  if (c <= kCiMax) {
    const size_t shmem = chol_inv_lds(c);
    const hipError_t e = hipFuncSetAttribute((const void*)k_chol_inv<T>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_chol_inv<T>), dim3(1), dim3(kCiT), shmem, s, W, c, R, Rinv, RinvT,
                       trans, status, nullptr);
    return hipGetLastError();
  }
#define RSVD_CHOL_WIDE(U)                                                                        \
  case U:                                                                                        \
    hipLaunchKernelGGL((k_chol_inv_wide<T, U>), dim3(1), dim3(kCwT), 0, s, W, c, R, Rinv, RinvT, \
                       trans, status, nullptr);                                                  \
    break;
  switch ((c + 31) / 32) {
    RSVD_CHOL_WIDE(4) RSVD_CHOL_WIDE(5) RSVD_CHOL_WIDE(6)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_CHOL_WIDE
  return hipGetLastError();
}

int chol_inv_max_c() { return kCwMax; }

template <typename T>
hipError_t launch_small_gemm(const double* A, const double* B, int64_t r, int c1, int c2, double* C,
                             T* CT, hipStream_t s, int trans) {
  if (r * c2 <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_small_gemm<T>), dim3(blocks_for(r * c2, 256)), dim3(256), 0, s, A, B, r,
                     c1, c2, C, CT, trans, nullptr);
  return hipGetLastError();
}

// the kernel for c columns (RU2 = ceil(c / 16) row pairs per lane)
template <bool AccJ>
const void* jacobi_small_fn(int ru2) {
  switch (ru2) {
    case 1: return (const void*)k_jacobi_svd_small<AccJ, 1>;
    case 2: return (const void*)k_jacobi_svd_small<AccJ, 2>;
    case 3: return (const void*)k_jacobi_svd_small<AccJ, 3>;
    case 4: return (const void*)k_jacobi_svd_small<AccJ, 4>;
    case 5: return (const void*)k_jacobi_svd_small<AccJ, 5>;
    case 6: return (const void*)k_jacobi_svd_small<AccJ, 6>;
    default: return nullptr;
  }
}

// one launch of k_jacobi_svd_small for c columns: grid (1, count), LDS for
// M (and J) padded to 16 ceil(c / 16) rows
hipError_t launch_jacobi_small(const double* M, int c, int transpose, double* Uo, double* S,
                               double* J, int acc_j, double* diag, int32_t* status, double* redo,
                               const GArgJac* garg, int count, hipStream_t s) {
  if (c < 1 || c > kJsMaxC) return hipErrorInvalidValue;
  const int ru2 = (c + 15) / 16;
  const int npad = c + (c & 1);
  const size_t shmem = (acc_j ? 2 : 1) * (size_t)(16 * ru2) * c * sizeof(double);
  const int threads = ((npad / 2) * kJsG + 63) / 64 * 64;
  const void* fn = acc_j ? jacobi_small_fn<true>(ru2) : jacobi_small_fn<false>(ru2);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&M, (void*)&c, (void*)&transpose, (void*)&Uo, (void*)&S, (void*)&J,
                  (void*)&diag, (void*)&status, (void*)&redo, (void*)&garg};
  e = hipLaunchKernel(fn, dim3(1, (unsigned)count), dim3(threads), args, shmem, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_jacobi_svd_small(const double* M, int c, int transpose, double* Uo, double* S,
                                   double* J, int acc_j, double* diag, int32_t* status,
                                   double* redo, hipStream_t s) {
  return launch_jacobi_small(M, c, transpose, Uo, S, J, acc_j, diag, status, redo, nullptr, 1, s);
}


template <typename T>
hipError_t launch_sort_sign_scatter(const double* S, int c, const double* Vsrc, int64_t r,
                                    int64_t vrs, int64_t vcs, const double* Wsrc, int kout,
                                    double* S_out, T* Vout, int64_t ldv, double* Vd_out,
                                    double* Wout, hipStream_t s) {
  if (kout <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sort_sign_scatter<T>), dim3((kout + kSsCols - 1) / kSsCols), dim3(256),
                     (size_t)c * (sizeof(double) + sizeof(int)), s, S,
                     c, Vsrc, r, vrs, vcs, Wsrc, kout, S_out, Vout, ldv, Vd_out, Wout, nullptr);
  return hipGetLastError();
}

hipError_t launch_select_k(const double* S, int k, const double* fro2, double t, int32_t* K,
                           double* diag, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_select_k, dim3(1), dim3(256), (size_t)k * sizeof(double), s, S, k, fro2, t,
                     K, diag, status, nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_cols_inv(const double* V, int64_t n, int cols, int64_t ldv, const double* S,
                                 double floor_rel, T* X, int64_t ldx, int trans,
                                 hipStream_t s) {
  if (n * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_scale_cols_inv<T>), dim3(blocks_for(n * cols, 256)), dim3(256), 0, s, V, n,
                     cols, ldv, S, floor_rel, X, ldx, trans);
  return hipGetLastError();
}

hipError_t launch_transpose_f32(const float* X, int64_t rows, int64_t cols, int64_t ldx, float* Xt,
                                int64_t ldxt, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_f32, dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)),
                     dim3(256), 0, s, X, rows, cols, ldx, Xt, ldxt);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_shift_diag(double* W, int c, int64_t m, hipStream_t s) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shift_diag, dim3(1), dim3(128), 0, s, W, c, m);
  return hipGetLastError();
}

hipError_t launch_sqrt_clamp(const double* lam, int n, double* S, hipStream_t s) {
  hipLaunchKernelGGL(k_sqrt_clamp, dim3(blocks_for(n, 256)), dim3(256), 0, s, lam, n, S);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grouped launchers (one launch, blockIdx.y = problem).
hipError_t launch_gaussian_fill_grouped(const GArgFill* a, int count, int maxblk, hipStream_t s) {
  if (count <= 0 || maxblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gaussian_fill, dim3((unsigned)maxblk, (unsigned)count), dim3(256), 0, s,
                     0, 0, nullptr, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cast_t_from_f64_grouped(const GArgCast* a, int count, int maxblk,
                                          hipStream_t s) {
  if (count <= 0 || maxblk <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast_t<double, T>), dim3((unsigned)maxblk, (unsigned)count), dim3(256), 0,
                     s, nullptr, 0, 0, 0, nullptr, 0, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_chol_inv_grouped(const GArgChol* a, int count, int cmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (cmax < 1 || cmax > kCiMax) return hipErrorInvalidValue;
  const size_t shmem = chol_inv_lds(cmax);
  const hipError_t e = hipFuncSetAttribute((const void*)k_chol_inv<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_chol_inv<T>), dim3(1, (unsigned)count), dim3(kCiT), shmem, s, nullptr, 0,
                     nullptr, nullptr, nullptr, 0, nullptr, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_small_gemm_grouped(const GArgSg* a, int count, int maxblk, hipStream_t s) {
  if (count <= 0 || maxblk <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_small_gemm<T>), dim3((unsigned)maxblk, (unsigned)count), dim3(256), 0, s,
                     nullptr, nullptr, 0, 0, 0, nullptr, nullptr, 0, a);
  return hipGetLastError();
}

// every problem of the launch has c = cmax (the thread count and the LDS
// size follow c)
hipError_t launch_jacobi_svd_small_grouped(const GArgJac* a, int count, int cmax, int acc_j,
                                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  return launch_jacobi_small(nullptr, cmax, 0, nullptr, nullptr, nullptr, acc_j, nullptr, nullptr,
                             nullptr, a, count, s);
}

template <typename T>
hipError_t launch_sort_sign_scatter_grouped(const GArgSort* a, int count, int maxblk, int cmax,
                                            hipStream_t s) {
  if (count <= 0 || maxblk <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sort_sign_scatter<T>), dim3((unsigned)maxblk, (unsigned)count), dim3(256),
                     (size_t)cmax * (sizeof(double) + sizeof(int)), s, nullptr, 0, nullptr, 0, 0,
                     0, nullptr, 0, nullptr, nullptr, 0, nullptr, nullptr, a);
  return hipGetLastError();
}

hipError_t launch_select_k_grouped(const GArgSel* a, int count, int kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_select_k, dim3(1, (unsigned)count), dim3(256), (size_t)kmax * sizeof(double),
                     s, nullptr, 0, nullptr, 0.0, nullptr, nullptr, nullptr, a);
  return hipGetLastError();
}

template hipError_t launch_cast_t_from_f64_grouped<float>(const GArgCast*, int, int, hipStream_t);
template hipError_t launch_chol_inv_grouped<float>(const GArgChol*, int, int, hipStream_t);
template hipError_t launch_chol_inv_grouped<double>(const GArgChol*, int, int, hipStream_t);
template hipError_t launch_small_gemm_grouped<float>(const GArgSg*, int, int, hipStream_t);
template hipError_t launch_small_gemm_grouped<double>(const GArgSg*, int, int, hipStream_t);
template hipError_t launch_sort_sign_scatter_grouped<float>(const GArgSort*, int, int, int,
                                                            hipStream_t);

#define RSVD_INST(T)                                                                               \
  template hipError_t launch_cast_t_from_f64<T>(const double*, int64_t, int64_t, int64_t, T*,      \
                                                 int64_t, hipStream_t);                             \
  template hipError_t launch_cast_from_f64<T>(const double*, int64_t, int64_t, int64_t, T*,        \
                                              int64_t, hipStream_t);                               \
  template hipError_t launch_cast_to_f64<T>(const T*, int64_t, int64_t, int64_t, double*, int64_t, \
                                            hipStream_t);                                          \
  template hipError_t launch_chol_inv<T>(const double*, int, double*, double*, T*, int32_t*,      \
                                         hipStream_t, int);                                        \
  template hipError_t launch_small_gemm<T>(const double*, const double*, int64_t, int, int,       \
                                           double*, T*, hipStream_t, int);                         \
  template hipError_t launch_sort_sign_scatter<T>(const double*, int, const double*, int64_t,     \
                                                  int64_t, int64_t, const double*, int, double*,  \
                                                  T*, int64_t, double*, double*, hipStream_t);     \
  template hipError_t launch_scale_cols_inv<T>(const double*, int64_t, int, int64_t,              \
                                                const double*, double, T*, int64_t, int, hipStream_t);
RSVD_INST(float)
RSVD_INST(double)
#undef RSVD_INST

}  // namespace rsvd
