// gemm.hip -- the passes over A: Y = A X (tall-skinny, row-major) and the
// split-m partial products of A^T Q, on the gfx950 matrix cores.
//
// These are the "m n l" products of Randomized PCA (paper Sec. 3.1.2, steps
// 2, 3 and 5: H = A G, A (A^T H), T = A^T Q) and of the truncated SVD
// (Sec. 3.1.3: A^T A and u_i = A v_i / s_i).  Every product is a
// contraction, so all of them run on 16x16x4 matrix-core instructions
// (fp32 or fp64).
#include "rsvd_internal.h"

namespace rsvd {

namespace {

template <typename T> struct Vec16;          // 16-byte vector of T
template <> struct Vec16<float> { typedef f32x4 type; };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

constexpr int kNNThreads = 256;              // 4 waves
constexpr int kNNBK = 32;                    // k-chunk staged in LDS

// ---------------------------------------------------------------------------
// Y = A X.  Block = 4 waves; wave w owns rows [row0 + 16*MR*w, +16*MR), the
// block owns 16*NT columns of Y (one column tile).  A goes straight from HBM
// into registers: within a slab of 4*VW columns of A, lane (r = l%16,
// g = l/16) loads the VW consecutive elements A[row r][slab + VW*g .. +VW-1]
// with one 16-byte load, and matrix-core step t uses element t -- so step t
// contracts over k = slab + VW*g + t (a permutation of the slab, matched on
// the X side).  The X chunk (kNNBK x 16*NT) is staged transposed in LDS so a
// lane reads its VW operands with one 16-byte LDS load.  Chunk c+1 of A and
// of X is loaded into registers while chunk c is multiplied; X chunks
// alternate between two LDS buffers (one barrier per chunk).
template <typename T, int NT, int MR, bool VEC>
__global__ __launch_bounds__(kNNThreads) void k_gemm_nn(
    const T* __restrict__ A, int64_t m, int64_t n, int64_t lda, const T* __restrict__ X,
    int64_t ldx, int c, T* __restrict__ Y, int64_t ldy, double* __restrict__ fro2_part,
    int ncol_tiles, const GArgNn* __restrict__ grp) {
  if (grp) {
    const GArgNn& a = grp[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk) return;
    A = (const T*)a.A; m = a.m; n = a.n; lda = a.lda; X = (const T*)a.X; ldx = a.ldx; c = a.c;
    Y = (T*)a.Y; ldy = a.ldy; fro2_part = a.fro2; ncol_tiles = a.ncol_tiles;
  }
  typedef Mfma<T> M;
  typedef typename M::acc_t acc_t;
  typedef typename Vec16<T>::type vec_t;
  constexpr int VW = 16 / sizeof(T);
  constexpr int SLAB = 4 * VW;
  constexpr int NS = kNNBK / SLAB;
  constexpr int BC = 16 * NT;
  constexpr int XLD = kNNBK + VW;            // padded, keeps 16-byte alignment
  constexpr int XE = (kNNBK * BC + kNNThreads - 1) / kNNThreads;
  __shared__ __attribute__((aligned(16))) T Xt[2][BC * XLD];
  __shared__ double red[kNNThreads / 64];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, g = lane >> 4;
  const int64_t rb = blockIdx.x / ncol_tiles;
  const int ct = blockIdx.x % ncol_tiles;
  const int64_t row0 = rb * (64 * MR) + (int64_t)wave * 16 * MR;
  const int col0 = ct * BC;
  const bool do_ss = (fro2_part != nullptr) && ct == 0;
  const int nch = (int)((n + kNNBK - 1) / kNNBK);

  acc_t acc[MR][NT];
#pragma unroll
  for (int r = 0; r < MR; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[r][j] = acc_t{0, 0, 0, 0};
  double ss = 0.0;

  auto load_x = [&](int ch, T(&xr)[XE]) {
    const int64_t k0 = (int64_t)ch * kNNBK;
#pragma unroll
    for (int u = 0; u < XE; ++u) {
      const int idx = threadIdx.x + u * kNNThreads;
      const int kk = idx / BC, col = idx - kk * BC;
      const int64_t k = k0 + kk;
      const int cc = col0 + col;
      xr[u] = (idx < kNNBK * BC && k < n && cc < c) ? X[k * ldx + cc] : T(0);
    }
  };
  auto store_x = [&](int buf, const T(&xr)[XE]) {
#pragma unroll
    for (int u = 0; u < XE; ++u) {
      const int idx = threadIdx.x + u * kNNThreads;
      const int kk = idx / BC, col = idx - kk * BC;
      if (idx < kNNBK * BC) Xt[buf][col * XLD + kk] = xr[u];
    }
  };
  auto load_a = [&](int ch, T(&a)[NS][MR][VW]) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int64_t kb = (int64_t)ch * kNNBK + s * SLAB + g * VW;
#pragma unroll
      for (int r = 0; r < MR; ++r) {
        const int64_t row = row0 + 16 * r + lr;
        if (VEC && row < m && kb + VW <= n) {
          const vec_t v = *reinterpret_cast<const vec_t*>(A + row * lda + kb);
#pragma unroll
          for (int t = 0; t < VW; ++t) a[s][r][t] = v[t];
        } else {
#pragma unroll
          for (int t = 0; t < VW; ++t)
            a[s][r][t] = (row < m && kb + t < n) ? A[row * lda + kb + t] : T(0);
        }
      }
    }
  };
  auto compute = [&](int buf, const T(&a)[NS][MR][VW]) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (do_ss) {
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
          for (int t = 0; t < VW; ++t) ss += (double)a[s][r][t] * (double)a[s][r][t];
      }
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const vec_t b =
            *reinterpret_cast<const vec_t*>(&Xt[buf][(16 * j + lr) * XLD + s * SLAB + g * VW]);
#pragma unroll
        for (int t = 0; t < VW; ++t)
#pragma unroll
          for (int r = 0; r < MR; ++r) acc[r][j] = M::run(a[s][r][t], b[t], acc[r][j]);
      }
    }
  };

  T xr[XE];
  T a0[NS][MR][VW], a1[NS][MR][VW];
  load_x(0, xr);
  load_a(0, a0);
  store_x(0, xr);
  __syncthreads();
  for (int ch = 0; ch < nch; ch += 2) {
    const bool has1 = ch + 1 < nch;
    if (has1) { load_x(ch + 1, xr); load_a(ch + 1, a1); }
    compute(0, a0);
    if (has1) store_x(1, xr);
    __syncthreads();
    if (!has1) break;
    const bool has2 = ch + 2 < nch;
    if (has2) { load_x(ch + 2, xr); load_a(ch + 2, a0); }
    compute(1, a1);
    if (has2) store_x(0, xr);
    __syncthreads();
  }

#pragma unroll
  for (int r = 0; r < MR; ++r)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = col0 + 16 * j + lr;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = row0 + 16 * r + M::row(lane, e);
        if (row < m && col < c) Y[row * ldy + col] = acc[r][j][e];
      }
    }

  if (do_ss) {
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kNNThreads / 64; ++w) t += red[w];
      fro2_part[blockIdx.x / ncol_tiles] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Y = A Xt^T for wide outputs (more than 128 columns; the truncated SVD forms
// u_i = A v_i / s_i for every i, Sec. 3.1.3), with the right factor given
// transposed (Xt is c x n, row-major) so that both operands are read along
// k.  Two-level tiling on the full-rate 32x32x2 fp32 matrix cores: block
// tile kWM x kWN = 256 x 256 (8 waves in 4 x 2, each 64 x 128 = 2 x 4 tiles
// of 32 x 32: two waves per SIMD, one block per CU in 144 KB of LDS); chunks
// of kWK = 32 along k of both operands are staged in LDS (row-major, padded
// rows) in two buffers.  Chunk i+1 is loaded into
// registers before chunk i is multiplied and written to LDS during its last
// slab; one barrier per chunk.  Blocks are numbered so that the column tiles
// of a row panel run back to back on the same XCD (block b runs on XCD
// b mod 8), so A comes from HBM once.
//
// Fast path (n a multiple of kWK, 16-byte aligned rows): buffer loads from a
// per-block descriptor whose size ends at the last valid row, so rows past m
// (or past c) read as zero; the chunk advance is a scalar offset.  General
// path: clamped addresses and selects.
constexpr int kWM = 256, kWN = 256, kWK = 32, kWLD = kWK + 4, kWT = 512;
constexpr int kWUA = kWM * (kWK / 4) / kWT, kWUX = kWN * (kWK / 4) / kWT;   // loads per thread
constexpr int kBufDword3 = 0x00020000;        // raw 32-bit buffer (gfx9 family)

template <bool FAST>
__device__ __forceinline__ void nt_wide_body(
    const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const float* __restrict__ Xt,
    int64_t ldxt, int c, float* __restrict__ Y, int64_t ldy, int64_t arow0, int bcol0,
    float (*As)[kWM * kWLD], float (*Bs)[kWN * kWLD]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, g = lane >> 5;
  const int wr = wave >> 1, wc = wave & 1;
  const int nch = (int)((n + kWK - 1) / kWK);
  const int64_t arows = m - arow0 < kWM ? m - arow0 : kWM;
  const int bcols = c - bcol0 < kWN ? c - bcol0 : kWN;

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // thread's share of a chunk: A rows (idx >> 3) and Xt rows (idx >> 3),
  // k-quad idx & 7 (idx = tid + u kWT); eight lanes cover the 128 bytes of
  // one row
  const __amdgpu_buffer_rsrc_t ra_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(A + arow0 * lda), 0, FAST ? (int)(arows * lda * 4) : 0, kBufDword3);
  const __amdgpu_buffer_rsrc_t rx_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(Xt + (int64_t)bcol0 * ldxt), 0, FAST ? (int)(bcols * ldxt * 4) : 0,
      kBufDword3);
  int voa[kWUA], vox[kWUX];
  if (FAST) {
#pragma unroll
    for (int u = 0; u < kWUA; ++u) {
      const int idx = tid + u * kWT;
      voa[u] = (int)(((idx >> 3) * lda + 4 * (idx & 7)) * 4);
    }
#pragma unroll
    for (int u = 0; u < kWUX; ++u) {
      const int idx = tid + u * kWT;
      vox[u] = (int)(((idx >> 3) * ldxt + 4 * (idx & 7)) * 4);
    }
  }
  f32x4 ra[kWUA], rx[kWUX];
  auto load = [&](int ch) {
    const int64_t k0 = (int64_t)ch * kWK;
    if (FAST) {
      const int so = (int)(k0 * 4);
#pragma unroll
      for (int u = 0; u < kWUA; ++u)
        ra[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra_rsrc, voa[u], so, 0));
#pragma unroll
      for (int u = 0; u < kWUX; ++u)
        rx[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rx_rsrc, vox[u], so, 0));
    } else {
#pragma unroll
      for (int u = 0; u < kWUA; ++u) {
        const int idx = tid + u * kWT;
        const int64_t gr = arow0 + (idx >> 3), k = k0 + 4 * (idx & 7);
        const float* rowp = A + (gr < m ? gr : m - 1) * lda;
#pragma unroll
        for (int i = 0; i < 4; ++i) ra[u][i] = rowp[k + i < n ? k + i : n - 1];
      }
#pragma unroll
      for (int u = 0; u < kWUX; ++u) {
        const int idx = tid + u * kWT;
        const int64_t gc = bcol0 + (idx >> 3), k = k0 + 4 * (idx & 7);
        const float* rowp = Xt + (gc < c ? gc : c - 1) * ldxt;
#pragma unroll
        for (int i = 0; i < 4; ++i) rx[u][i] = rowp[k + i < n ? k + i : n - 1];
      }
    }
  };
  auto store = [&](int ch, int buf) {
    const int64_t k0 = (int64_t)ch * kWK;
#pragma unroll
    for (int u = 0; u < kWUA; ++u) {
      const int idx = tid + u * kWT, row = idx >> 3, kq = idx & 7;
      f32x4 v = ra[u];
      if (!FAST) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = (row < arows && k0 + 4 * kq + i < n) ? v[i] : 0.f;
      }
      *reinterpret_cast<f32x4*>(&As[buf][row * kWLD + 4 * kq]) = v;
    }
#pragma unroll
    for (int u = 0; u < kWUX; ++u) {
      const int idx = tid + u * kWT, col = idx >> 3, kq = idx & 7;
      f32x4 v = rx[u];
      if (!FAST) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = (col < bcols && k0 + 4 * kq + i < n) ? v[i] : 0.f;
      }
      *reinterpret_cast<f32x4*>(&Bs[buf][col * kWLD + 4 * kq]) = v;
    }
  };
  // slab of 8 k: lane (lr, g) reads k = 8 s + 4 g .. +3 of its row with one
  // 16-byte load, and step t contracts over k = 8 s + 4 g + t (the same
  // permutation on both operands)
  auto slab = [&](int buf, int s) {
    f32x4 af[2], bf[4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      af[i] = *reinterpret_cast<const f32x4*>(&As[buf][(wr * 64 + 32 * i + lr) * kWLD + 8 * s + 4 * g]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bf[j] = *reinterpret_cast<const f32x4*>(&Bs[buf][(wc * 128 + 32 * j + lr) * kWLD + 8 * s + 4 * g]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma32f::run(af[i][t], bf[j][t], acc[i][j]);
  };

  load(0);
  store(0, 0);
  __syncthreads();
  static_assert(kWK == 32, "four slabs per chunk");
  for (int ch = 0; ch < nch; ++ch) {
    const int nx = ch + 1 < nch ? ch + 1 : ch;  // the last prefetch is a harmless repeat
    const int buf = ch & 1;
    load(nx);
    __builtin_amdgcn_sched_barrier(0);        // keep the loads ahead of the multiply
    slab(buf, 0);
    slab(buf, 1);
    slab(buf, 2);
    __builtin_amdgcn_sched_barrier(0);
    slab(buf, 3);
    store(nx, buf ^ 1);                       // the other buffer: free since the last barrier
    // last slab: its 6 LDS reads, then 4 matrix-core steps per LDS write
    __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
    for (int w = 0; w < kWUA + kWUX; ++w) {
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = bcol0 + wc * 128 + 32 * j + lr;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t row = arow0 + wr * 64 + 32 * i + Mfma32f::row(lane, e);
        if (row < m && col < c) Y[row * ldy + col] = acc[i][j][e];
      }
    }
}

__global__ __launch_bounds__(kWT) void k_gemm_nt_wide(
    const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const float* __restrict__ Xt,
    int64_t ldxt, int c, float* __restrict__ Y, int64_t ldy, int64_t ntiles, int ncb,
    int64_t per_xcd, int fast) {
  __shared__ __attribute__((aligned(16))) float As[2][kWM * kWLD];
  __shared__ __attribute__((aligned(16))) float Bs[2][kWN * kWLD];
  const int64_t L = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (L >= ntiles) return;
  const int64_t rb = L / ncb;
  const int cb = (int)(L - rb * ncb);
  if (fast)
    nt_wide_body<true>(A, m, n, lda, Xt, ldxt, c, Y, ldy, rb * kWM, cb * kWN, As, Bs);
  else
    nt_wide_body<false>(A, m, n, lda, Xt, ldxt, c, Y, ldy, rb * kWM, cb * kWN, As, Bs);
}

// ---------------------------------------------------------------------------
// G = A^T A for fp32 A (the truncated SVD's Gram matrix, Sec. 3.1.3, Eq.
// AB), upper 128 x 128 tile pairs only (G is symmetric).  Block = one tile
// pair (I <= J) over one split of the rows; chunks of kSyK = 32 rows of the
// two 128-column slices are staged row-major in LDS (row stride padded to
// 288 floats, so the two half-waves of a read touch disjoint banks), two
// buffers, next chunk's buffer loads issued ahead of the multiply and its LDS
// writes interleaved into the last quarter.  32x32x2 steps contract over two
// rows: lane (lr, g) supplies A[row 2t + g][column lr of its slice] for both
// operands.  fp32 accumulation within a block, FP64 partial tiles, reduced in
// split order by k_syrk_reduce (deterministic).  Columns past n are never
// masked: they only feed output rows/columns past n, which are not written
// (and the buffer descriptor ends at the split's last row).
constexpr int kSyT = 128, kSyK = 32, kSyLD = 2 * kSyT + 32;
constexpr int kSyU = kSyK * 64 / 256;          // 16-byte loads per thread per chunk

__global__ __launch_bounds__(256, 2) void k_syrk_f32(const float* __restrict__ A, int64_t m,
                                                  int64_t n, int64_t lda, int ntile, int npair,
                                                  int64_t rps, int64_t nblk, int64_t per_xcd,
                                                  double* __restrict__ P) {
  __shared__ __attribute__((aligned(16))) float As[2][kSyK * kSyLD];
  const int64_t L = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (L >= nblk) return;
  const int64_t sp = L / npair;                  // row split (consecutive blocks share it)
  const int pr = (int)(L - sp * npair);          // tile pair, upper triangle row by row
  int I = 0, rem = pr;
  while (rem >= ntile - I) { rem -= ntile - I; ++I; }
  const int J = I + rem;
  const int64_t row0 = sp * rps;
  const int64_t rows = (m - row0 < rps) ? m - row0 : rps;
  const int nch = (int)((rows + kSyK - 1) / kSyK);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, g = lane >> 5;
  const int wr = wave >> 1, wc = wave & 1;

  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(A + row0 * lda), 0, (int)(rows * lda * 4), kBufDword3);
  // chunk = kSyK rows x 64 float4 (32 from slice I, 32 from slice J)
  int voff[kSyU];
#pragma unroll
  for (int u = 0; u < kSyU; ++u) {
    const int idx = tid + u * 256, r = idx >> 6, q = idx & 63;
    const int col = q < 32 ? I * kSyT + 4 * q : J * kSyT + 4 * (q - 32);
    voff[u] = (int)((r * lda + col) * 4);
  }
  f32x4 rg[kSyU];
  auto load = [&](int ch) {
    const int so = (int)((int64_t)ch * kSyK * lda * 4);
#pragma unroll
    for (int u = 0; u < kSyU; ++u)
      rg[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[u], so, 0));
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kSyU; ++u) {
      const int idx = tid + u * 256, r = idx >> 6, q = idx & 63;
      *reinterpret_cast<f32x4*>(&As[buf][r * kSyLD + 4 * q]) = rg[u];
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  auto steps = [&](int buf, int t0, int t1) {
#pragma unroll
    for (int t = t0; t < t1; ++t) {
      const float* rowp = &As[buf][(2 * t + g) * kSyLD];
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = rowp[wr * 64 + 32 * i + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = rowp[kSyT + wc * 64 + 32 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Mfma32f::run(a[i], b[j], acc[i][j]);
    }
  };

  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    load(ch + 1 < nch ? ch + 1 : ch);          // the last prefetch is a harmless repeat
    __builtin_amdgcn_sched_barrier(0);
    static_assert(kSyK == 32, "16 steps per chunk, the last 4 interleaved with the LDS writes");
    steps(buf, 0, 12);
    __builtin_amdgcn_sched_barrier(0);
    steps(buf, 12, 16);
    store(buf ^ 1);
    // last quarter: 4 LDS reads and 4 matrix-core steps per 2 LDS writes
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);
    }
    __syncthreads();
  }
  double* out = P + L * (int64_t)(kSyT * kSyT);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wc * 64 + 32 * j + lr;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = wr * 64 + 32 * i + Mfma32f::row(lane, e);
        out[row * kSyT + col] = (double)acc[i][j][e];
      }
    }
}

// G (n x n, FP64) from the partial tiles: element (i, j) of tile pair p is
// the sum over the splits in order; tile (I, J) also fills (J, I).
__global__ void k_syrk_reduce(const double* __restrict__ P, int64_t nsplit, int npair, int ntile,
                              int64_t n, double* __restrict__ G, int64_t ldg) {
  const int pr = blockIdx.y;
  int I = 0, rem = pr;
  while (rem >= ntile - I) { rem -= ntile - I; ++I; }
  const int J = I + rem;
  const int e0 = (blockIdx.x * blockDim.x + threadIdx.x) * 2;   // two adjacent entries
  if (e0 >= kSyT * kSyT) return;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t sp = 0; sp < nsplit; ++sp) {
    const double* t = P + (sp * npair + pr) * (int64_t)(kSyT * kSyT) + e0;
    s0 += t[0];
    s1 += t[1];
  }
  const int i = e0 / kSyT, j = e0 % kSyT;
  const int64_t gi = (int64_t)I * kSyT + i, gj = (int64_t)J * kSyT + j;
  if (gi < n && gj < n) { G[gi * ldg + gj] = s0; if (I != J) G[gj * ldg + gi] = s0; }
  if (gi < n && gj + 1 < n) { G[gi * ldg + gj + 1] = s1; if (I != J) G[(gj + 1) * ldg + gi] = s1; }
}

// ---------------------------------------------------------------------------
// Tall passes with a narrow right factor (c <= 128; the sketch and power
// iterations, Sec. 3.1.2 steps 2, 3 and 5), fp32 on 16x16x4 matrix cores
// (exact tiles for any c that is a multiple of 16).
//
// Y = A Xt^T (Xt is c x n): block = 128 rows of A x all c columns, 4 waves of
// 32 rows (2 x NT tiles); chunks of kTK = 32 along k of both operands staged
// row-major in LDS (two buffers; at l <= 80 small enough for three blocks per
// CU: rows unpadded, the 16-byte k-quad q of row r stored at quad q ^ (r % 8),
// so the eight rows a read or write touches at one quad fall in distinct
// banks).  A
// chunk is a whole 128-byte segment of each row: with 16-k chunks each row's
// cache line was consumed in two halves a chunk apart, and at n = 512 (rows
// 2 KB apart) the half left for the next chunk was often evicted and fetched
// again (1.5x the bytes of A).  The next chunk's buffer loads are issued
// before the multiply, its LDS writes interleaved into the last slab, the
// FP64 sum of squares of A (Eq. sumeigen) taken from the loaded chunk.
// Requires n % 4 == 0 and 16-byte rows (the descriptor ends at the last
// valid row; a last chunk that ends past n is zeroed there on its way to LDS).
constexpr int kTM = 128, kTK = 32, kTLD = kTK;
constexpr int kTQ = kTK / 4, kTUA = kTM * kTQ / 256;   // k-quads per row, A loads per thread
// float offset of k-quad q of row r in an LDS chunk
__device__ __forceinline__ int tq_off(int r, int q) { return r * kTLD + 4 * (q ^ (r & 7)); }

// Work-list epilogue of the NT products (see GWork): a wave's FP32 output
// tiles acc[i][J] (16 rows x 16 columns each, value e of lane l at row
// 4 (l / 16) + e, column l % 16) are, for each e, exactly the operands the
// FP64 16x16x4 matrix core takes for Y_I^T Y_J over the four rows
// 4 k + e (a = column l % 16 of tile I, b = of tile J, k = l / 16), so the
// Gram matrix of the stored (FP32) outputs is summed from the registers with
// exact products.  Columns past c and rows past m hold zeros there.
template <int NT, int RT>
__device__ __forceinline__ void gram_from_acc(const f32x4 (&acc)[RT][NT],
                                              f64x4 (&g)[NT * (NT + 1) / 2]) {
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double y[NT];
#pragma unroll
      for (int J = 0; J < NT; ++J) y[J] = (double)acc[i][J][e];
      int q = 0;
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J) {
          g[q] = Mfma<double>::run(y[I], y[J], g[q]);
          ++q;
        }
    }
}

// The waves' Gram tiles added in wave order in LDS (red: c x c doubles) and
// written as the symmetric c x c partial Pb (the upper tile pairs mirrored).
template <int NT, int WAVES>
__device__ __forceinline__ void gram_store(const f64x4 (&g)[NT * (NT + 1) / 2], int c,
                                           double* red, double* __restrict__ Pb) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int w = 0; w < WAVES; ++w) {
    if (wave == w) {
      int q = 0;
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = 16 * I + Mfma<double>::row(lane, e), j = 16 * J + (lane & 15);
            if (i < c && j < c) red[i * c + j] = (w == 0) ? g[q][e] : red[i * c + j] + g[q][e];
          }
          ++q;
        }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < c * c; idx += WAVES * 64) {
    const int i = idx / c, j = idx - i * c;
    Pb[idx] = ((i >> 4) <= (j >> 4)) ? red[i * c + j] : red[j * c + i];
  }
}

template <int NT, bool GR>
__global__ __launch_bounds__(256, 2) void k_gemm_nt_tall(
    const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const float* __restrict__ Xt,
    int64_t ldxt, int c, float* __restrict__ Y, int64_t ldy, double* __restrict__ fro2_part,
    const GArgTall* __restrict__ grp, const GWork* __restrict__ wl) {
  // tiles [t0, t1) of 128 rows; partial slot of the sum of squares / Gram
  int64_t t0 = blockIdx.x, t1 = (int64_t)blockIdx.x + 1, slot = blockIdx.x;
  double* gram = nullptr;
  if (grp) {
    const GWork w = wl[blockIdx.x];
    const GArgTall& a = grp[w.inst];
    A = a.A; m = a.m; n = a.n; lda = a.lda; Xt = a.Xt; ldxt = a.ldxt; c = a.c; Y = a.Y;
    ldy = a.ldy; fro2_part = a.fro2; gram = a.gram;
    slot = w.item;
    t0 = (int64_t)w.item * a.tpp;
    const int64_t nt_all = (m + kTM - 1) / kTM;
    t1 = t0 + a.tpp < nt_all ? t0 + a.tpp : nt_all;
  }
  constexpr int BC = 16 * NT;
  constexpr int XU = (BC * (kTK / 4) + 255) / 256;   // float4 of the Xt chunk per thread
  __shared__ __attribute__((aligned(16))) float As[2][kTM * kTLD];
  __shared__ __attribute__((aligned(16))) float Bs[2][BC * kTLD];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  const int nch = (int)((n + kTK - 1) / kTK);
  const bool do_ss = fro2_part != nullptr;
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(Xt), 0, (int)(((int64_t)(c - 1) * ldxt + n) * 4), kBufDword3);
  __amdgpu_buffer_rsrc_t ar = xr;   // the tile's rows, set per tile
  int voa[kTUA], vox[XU];
#pragma unroll
  for (int u = 0; u < kTUA; ++u) {
    const int idx = tid + u * 256;
    voa[u] = (int)(((idx / kTQ) * lda + 4 * (idx % kTQ)) * 4);
  }
#pragma unroll
  for (int u = 0; u < XU; ++u) {
    const int idx = tid + u * 256;
    vox[u] = (int)(((idx / kTQ) * ldxt + 4 * (idx % kTQ)) * 4);
  }
  f32x4 ra[kTUA], rx[XU];
  auto load = [&](int ch) {
    const int so = ch * kTK * 4;
#pragma unroll
    for (int u = 0; u < kTUA; ++u)
      ra[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ar, voa[u], so, 0));
#pragma unroll
    for (int u = 0; u < XU; ++u)
      if (tid + u * 256 < BC * (kTK / 4))
        rx[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, vox[u], so, 0));
  };
  double ss = 0.0;
  // chunk ch goes to LDS; in a last chunk that ends past n both operands are
  // zeroed beyond n (the loads there read the next row)
  auto store = [&](int buf, int ch) {
    const int kend = (int)(n - (int64_t)ch * kTK);
    const bool tail = kend < kTK;
#pragma unroll
    for (int u = 0; u < kTUA; ++u) {
      const int idx = tid + u * 256;
      f32x4 v = ra[u];
      if (tail) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = 4 * (idx % kTQ) + i < kend ? v[i] : 0.f;
      }
      *reinterpret_cast<f32x4*>(&As[buf][tq_off(idx / kTQ, idx % kTQ)]) = v;
      if (do_ss) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ss = fma((double)v[i], (double)v[i], ss);
      }
    }
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int idx = tid + u * 256;
      if (idx < BC * (kTK / 4)) {
        f32x4 v = rx[u];
        if (tail) {
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = 4 * (idx % kTQ) + i < kend ? v[i] : 0.f;
        }
        *reinterpret_cast<f32x4*>(&Bs[buf][tq_off(idx / kTQ, idx % kTQ)]) = v;
      }
    }
  };
  constexpr int RT = kTM / 64;                 // 16-row tiles per wave
  constexpr int NP = GR ? NT * (NT + 1) / 2 : 1;
  f64x4 gacc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) gacc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  f32x4 acc[RT][NT];
  // slab of 16 k: lane (lr, g) reads k = 16 s + 4 g .. +3 with one 16-byte
  // load; step t contracts over k = 16 s + 4 g + t on both operands
  auto slab = [&](int buf, int s) {
    f32x4 af[RT], bf[NT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
      af[i] = *reinterpret_cast<const f32x4*>(&As[buf][tq_off(wave * 16 * RT + 16 * i + lr, 4 * s + g)]);
#pragma unroll
    for (int j = 0; j < NT; ++j)
      bf[j] = *reinterpret_cast<const f32x4*>(&Bs[buf][tq_off(16 * j + lr, 4 * s + g)]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = Mfma<float>::run(af[i][t], bf[j][t], acc[i][j]);
  };
  static_assert(kTK == 32, "two slabs per chunk");
  for (int64_t tl = t0; tl < t1; ++tl) {
    const int64_t row0 = tl * kTM;
    const int64_t rows = m - row0 < kTM ? m - row0 : kTM;
    // the range ends at the last element of the tile's last row
    ar = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(A + row0 * lda), 0,
                                           (int)(((rows - 1) * lda + n) * 4), kBufDword3);
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    load(0);
    store(0, 0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      const int buf = ch & 1;
      const bool more = ch + 1 < nch;
      load(more ? ch + 1 : ch);                  // the last prefetch is a harmless repeat
      __builtin_amdgcn_sched_barrier(0);
      slab(buf, 0);
      __builtin_amdgcn_sched_barrier(0);
      slab(buf, 1);
      if (more) store(buf ^ 1, ch + 1);
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int col = 16 * j + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = row0 + wave * 16 * RT + 16 * i + Mfma<float>::row(lane, e);
          if (row < m && col < c) Y[row * ldy + col] = acc[i][j][e];
        }
      }
    if constexpr (GR) gram_from_acc<NT, RT>(acc, gacc);
  }
  if (do_ss) {
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) fro2_part[slot] = red[0] + red[1] + red[2] + red[3];
  }
  if constexpr (GR) {
    // As is free (the last chunk ended with a barrier): c <= 64 fits
    static_assert(16 * NT * 16 * NT * sizeof(double) <= sizeof(As), "Gram tile fits in As");
    if (gram) gram_store<NT, 4>(gacc, c, reinterpret_cast<double*>(&As[0][0]),
                                gram + slot * (int64_t)c * c);
  }
}

// Y = A Xt^T for a short k range (n <= 16 NS): the whole c x n factor is
// staged in LDS once per block and A goes straight from memory into the
// matrix-core operand registers (lane (lr, g) of a 16-row tile loads 16 bytes
// of row lr at k = 16 s + 4 g, the k order that step t of slab s contracts on
// both operands).  Persistent blocks walk tiles of kNM rows (4 waves of 32
// rows x NT column tiles); a wave's loads for its next tile are in flight
// while it multiplies the current one.  Same requirements as the tall kernel
// (n % 4 == 0, 16-byte rows).
constexpr int kNM = 128;

// With GR the Gram partial of a solo launch is per block (slot = blockIdx.x,
// at gram_part); 5 or 6 column tiles of FP64 Gram accumulators fit only at
// one wave per SIMD.  TRI: Xt is lower triangular (Xt[j][k] = 0 for k > j,
// the transposed inverse Cholesky factor R^-1 of CholeskyQR, whose zero
// blocks are exact), so k slab s only meets output tiles j >= s and the
// products of the zero blocks are skipped: NT (NT + 1) / 2 of NT^2 tile
// products at n = c.
template <int NT, int NS, bool GR, bool TRI>
__global__ __launch_bounds__(256, (GR && NT > kGramFuseMaxNt) ? 1 : 2) void k_gemm_nt_narrow(
    const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const float* __restrict__ Xt,
    int64_t ldxt, int c, float* __restrict__ Y, int64_t ldy, double* __restrict__ gram_part,
    const GArgNarrow* __restrict__ grp, const GWork* __restrict__ wl) {
  // tiles t0, t0 + step, ... below t1
  int64_t t0 = blockIdx.x, step = gridDim.x, t1 = (m + kNM - 1) / kNM, slot = blockIdx.x;
  double* gram = gram_part;
  if (grp) {
    const GWork w = wl[blockIdx.x];
    const GArgNarrow& a = grp[w.inst];
    A = a.A; m = a.m; n = a.n; lda = a.lda; Xt = a.Xt; ldxt = a.ldxt; c = a.c; Y = a.Y;
    ldy = a.ldy; gram = a.gram;
    slot = w.item;
    step = 1;
    t0 = (int64_t)w.item * a.tpp;
    const int64_t nt_all = (m + kNM - 1) / kNM;
    t1 = t0 + a.tpp < nt_all ? t0 + a.tpp : nt_all;
  }
  constexpr int BC = 16 * NT, KP = 16 * NS, LD = KP + 4;
  __shared__ __attribute__((aligned(16))) float Bs[BC * LD];
  __shared__ double gred[GR ? BC * BC : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  int vo[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) vo[i] = (int)(((int64_t)(wave * 32 + 16 * i + lr) * lda + 4 * g) * 4);
  // tile tl: buffer range ends at the last element of its last row, so rows
  // past it read zeros
  auto load = [&](int64_t tl, f32x4 (&dst)[NS][2]) {
    const int64_t r0 = tl * kNM;
    const int64_t rows = m - r0 < kNM ? m - r0 : kNM;
    const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(A + r0 * lda), 0, (int)(((rows - 1) * lda + n) * 4), kBufDword3);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        dst[sl][i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ar, vo[i], 64 * sl, 0));
  };
  constexpr int NP = GR ? NT * (NT + 1) / 2 : 1;
  f64x4 gacc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) gacc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  f32x4 nxt[NS][2];
  int64_t tl = t0;
  if (tl < t1) load(tl, nxt);
  // Xt into LDS, zero beyond c rows and n columns, while A is in flight
  for (int e = tid; e < BC * (KP / 4); e += 256) {
    const int r = e / (KP / 4), q = e - r * (KP / 4);
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (r < c && 4 * q < n) v = *reinterpret_cast<const f32x4*>(Xt + (int64_t)r * ldxt + 4 * q);
    *reinterpret_cast<f32x4*>(&Bs[r * LD + 4 * q]) = v;
  }
  __syncthreads();
  for (; tl < t1; tl += step) {
    f32x4 af[NS][2];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
#pragma unroll
      for (int i = 0; i < 2; ++i) af[sl][i] = nxt[sl][i];
    const int64_t tn = tl + step;
    load(tn < t1 ? tn : tl, nxt);             // the last prefetch is a harmless repeat
    __builtin_amdgcn_sched_barrier(0);
    f32x4 acc[2][NT];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      if (sl == NS - 1 && 16 * sl + 4 * g >= n) {
        // the last slab's k beyond n holds the next row's values
#pragma unroll
        for (int i = 0; i < 2; ++i) af[sl][i] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      f32x4 bf[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j)
        if (!TRI || j >= sl)
          bf[j] = *reinterpret_cast<const f32x4*>(&Bs[(16 * j + lr) * LD + 16 * sl + 4 * g]);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < NT; ++j)
            if (!TRI || j >= sl) acc[i][j] = Mfma<float>::run(af[sl][i][t], bf[j][t], acc[i][j]);
    }
    const int64_t row0 = tl * kNM + wave * 32;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int col = 16 * j + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = row0 + 16 * i + Mfma<float>::row(lane, e);
          if (row < m && col < c) Y[row * ldy + col] = acc[i][j][e];
        }
      }
    if constexpr (GR) gram_from_acc<NT, 2>(acc, gacc);
  }
  if constexpr (GR) {
    if (gram) gram_store<NT, 4>(gacc, c, gred, gram + slot * (int64_t)c * c);
  }
}

// Z partials (n x c per row split, FP64) of A^T Q: block = one row split of
// A and Q, all n (up to kUA per column tile) x c outputs; 8 waves of 64 A
// columns (4 x NT tiles); chunks of kUK = 16 rows staged row-major in LDS
// (row strides = 16 mod 64 floats, so the four 16-lane groups of a read hit
// disjoint banks).  16x16x4 steps contract over four rows: lane (lr, g)
// supplies A[row 4t + g][column lr of its tile] and Q[row 4t + g][column lr].
// Columns past n or c only feed outputs that are not written; rows past the
// split end read as zero (descriptor size).
constexpr int kUK = 16, kUA = 512, kUALD = kUA + 16;

template <int NT>
__global__ __launch_bounds__(512) void k_gemm_tn_tall(
    const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const float* __restrict__ Q,
    int64_t ldq, int c, int64_t rps, int ntile, double* __restrict__ P,
    const GArgTn* __restrict__ grp, const GWork* __restrict__ wl) {
  int bx = blockIdx.x;
  if (grp) {
    const GWork w = wl[blockIdx.x];
    const GArgTn& a = grp[w.inst];
    A = a.A; m = a.m; n = a.n; lda = a.lda; Q = a.Q; ldq = a.ldq; c = a.c; rps = a.rps;
    ntile = a.ntile; P = a.P;
    bx = w.item;
  }
  constexpr int BC = 16 * NT;
  constexpr int QLD = BC + ((16 - BC) % 64 + 64) % 64;
  constexpr int QU = BC / 4 * kUK;               // float4 of the Q chunk
  __shared__ __attribute__((aligned(16))) float As[2][kUK * kUALD];
  __shared__ __attribute__((aligned(16))) float Qs[2][kUK * QLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  const int ta = bx % ntile;
  const int64_t sp = bx / ntile;
  const int64_t row0 = sp * rps;
  const int64_t rows = m - row0 < rps ? m - row0 : rps;
  const int nch = (int)((rows + kUK - 1) / kUK);
  const int col0 = ta * kUA;
  const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(A + row0 * lda), 0, (int)(rows * lda * 4), kBufDword3);
  const __amdgpu_buffer_rsrc_t qr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(Q + row0 * ldq), 0, (int)(rows * ldq * 4), kBufDword3);
  // A chunk: 16 rows x 128 float4 (4 per thread); Q chunk: 16 rows x BC/4
  int voa[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = tid + u * 512;
    voa[u] = (int)(((idx >> 7) * lda + col0 + 4 * (idx & 127)) * 4);
  }
  // Q chunk: float4 piece tid + 512 u of the chunk (two per thread past 128 columns)
  constexpr int QP = (QU + 511) / 512;
  int voq[QP], qoff[QP];
  bool has_q[QP];
#pragma unroll
  for (int u = 0; u < QP; ++u) {
    const int idx = tid + 512 * u, qr_row = idx / (BC / 4), qr_q = idx % (BC / 4);
    has_q[u] = idx < QU;
    voq[u] = (int)((qr_row * ldq + 4 * qr_q) * 4);
    qoff[u] = qr_row * QLD + 4 * qr_q;
  }
  f32x4 ra[4], rq[QP];
  auto load = [&](int ch) {
    const int sa = (int)((int64_t)ch * kUK * lda * 4), sq = (int)((int64_t)ch * kUK * ldq * 4);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      ra[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ar, voa[u], sa, 0));
#pragma unroll
    for (int u = 0; u < QP; ++u)
      if (has_q[u])
        rq[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(qr, voq[u], sq, 0));
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + u * 512;
      *reinterpret_cast<f32x4*>(&As[buf][(idx >> 7) * kUALD + 4 * (idx & 127)]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < QP; ++u)
      if (has_q[u]) *reinterpret_cast<f32x4*>(&Qs[buf][qoff[u]]) = rq[u];
  };
  f32x4 acc[4][NT];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto steps = [&](int buf) {
#pragma unroll
    for (int t = 0; t < kUK / 4; ++t) {
      const float* arow = &As[buf][(4 * t + g) * kUALD + wave * 64 + lr];
      const float* qrow = &Qs[buf][(4 * t + g) * QLD + lr];
      float af[4], bf[NT];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = arow[16 * i];
#pragma unroll
      for (int j = 0; j < NT; ++j) bf[j] = qrow[16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = Mfma<float>::run(af[i], bf[j], acc[i][j]);
    }
  };
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    load(more ? ch + 1 : ch);
    __builtin_amdgcn_sched_barrier(0);
    steps(buf);
    __builtin_amdgcn_sched_barrier(0);
    if (more) store(buf ^ 1);
    __syncthreads();
  }
  double* out = P + sp * n * (int64_t)c;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = 16 * j + lr;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = col0 + wave * 64 + 16 * i + Mfma<float>::row(lane, e);
        if (row < n && col < c) out[row * c + col] = (double)acc[i][j][e];
      }
    }
}

// Z partials of A^T Q for n <= 64 CW columns (CW = 1, 2 or 4): the same
// contraction and partial layout as k_gemm_tn_tall, whose 512-column tile
// would spend most of its matrix-core steps on columns past n.  The block's
// 4 CW x NT output tiles (16 x 16) are dealt to its 8 waves -- CW = 4: two
// row tiles and all NT column tiles per wave; CW = 2: one row tile, all
// column tiles; CW = 1: one row tile and every second column tile (waves w
// and w + 4, which share a SIMD, split them) -- and every wave contracts over
// all rows of a chunk, so no cross-wave sum is needed.  Chunks of R rows
// (32; 16 for CW = 4) of the 64 CW columns of A and of Q's BC columns are
// staged row-major in LDS (row strides 16 mod 64 floats), double-buffered.
// With one column tile (n <= 256) a block is one row split.
template <int CW>
struct TnNarrow {
  static constexpr int R = CW == 4 ? 16 : 32;          // rows per chunk
  static constexpr int COLS = 64 * CW;
  static constexpr int ALD = COLS + 16;
  static constexpr int RT = 4 * CW;                     // row tiles of the block's Z
  static constexpr int IPW = RT > 8 ? RT / 8 : 1;       // row tiles per wave
  static constexpr int JS = RT < 8 ? 8 / RT : 1;        // column-tile stride
  static constexpr int UA = R * COLS / 4 / 512;         // float4 of A per thread
  static_assert(UA * 512 * 4 == R * COLS, "A chunk must be whole float4 per thread");
};

template <int NT, int CW>
__global__ __launch_bounds__(512) void k_gemm_tn_narrow(
    const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const float* __restrict__ Q,
    int64_t ldq, int c, int64_t rps, int ntile, double* __restrict__ P,
    const GArgTn* __restrict__ grp, const GWork* __restrict__ wl) {
  using G = TnNarrow<CW>;
  int bx = blockIdx.x;
  if (grp) {
    const GWork w = wl[blockIdx.x];
    const GArgTn& a = grp[w.inst];
    A = a.A; m = a.m; n = a.n; lda = a.lda; Q = a.Q; ldq = a.ldq; c = a.c; rps = a.rps;
    ntile = a.ntile; P = a.P;
    bx = w.item;
  }
  constexpr int BC = 16 * NT;
  constexpr int QLD = BC + ((16 - BC) % 64 + 64) % 64;
  constexpr int QU = G::R * BC / 4;                     // float4 of the Q chunk
  constexpr int UQ = (QU + 511) / 512;
  constexpr int JPW = (NT + G::JS - 1) / G::JS;
  __shared__ __attribute__((aligned(16))) float As[2][G::R * G::ALD];
  __shared__ __attribute__((aligned(16))) float Qs[2][G::R * QLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  const int64_t sp = bx / ntile;
  const int64_t row0 = sp * rps;
  const int64_t rows = m - row0 < rps ? m - row0 : rps;
  const int nch = (int)((rows + G::R - 1) / G::R);
  const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(A + row0 * lda), 0, (int)(rows * lda * 4), kBufDword3);
  const __amdgpu_buffer_rsrc_t qr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(Q + row0 * ldq), 0, (int)(rows * ldq * 4), kBufDword3);
  int voa[G::UA], voq[UQ];
#pragma unroll
  for (int u = 0; u < G::UA; ++u) {
    const int idx = tid + u * 512, r = idx / (G::COLS / 4), q4 = idx % (G::COLS / 4);
    voa[u] = (int)((r * lda + 4 * q4) * 4);
  }
#pragma unroll
  for (int u = 0; u < UQ; ++u) {
    const int idx = tid + u * 512, r = idx / (BC / 4), q4 = idx % (BC / 4);
    voq[u] = (int)((r * ldq + 4 * q4) * 4);
  }
  f32x4 ra[G::UA], rq[UQ];
  auto load = [&](int ch) {
    const int sa = (int)((int64_t)ch * G::R * lda * 4), sq = (int)((int64_t)ch * G::R * ldq * 4);
#pragma unroll
    for (int u = 0; u < G::UA; ++u)
      ra[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ar, voa[u], sa, 0));
#pragma unroll
    for (int u = 0; u < UQ; ++u)
      if (tid + u * 512 < QU)
        rq[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(qr, voq[u], sq, 0));
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < G::UA; ++u) {
      const int idx = tid + u * 512, r = idx / (G::COLS / 4), q4 = idx % (G::COLS / 4);
      *reinterpret_cast<f32x4*>(&As[buf][r * G::ALD + 4 * q4]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < UQ; ++u) {
      const int idx = tid + u * 512, r = idx / (BC / 4), q4 = idx % (BC / 4);
      if (idx < QU) *reinterpret_cast<f32x4*>(&Qs[buf][r * QLD + 4 * q4]) = rq[u];
    }
  };
  // this wave's tiles: row tile i0 + 8 ii, column tile j0 + JS jj (if < NT)
  const int i0 = G::RT < 8 ? wave % G::RT : wave;
  const int j0 = G::RT < 8 ? wave / G::RT : 0;
  f32x4 acc[G::IPW][JPW];
#pragma unroll
  for (int ii = 0; ii < G::IPW; ++ii)
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) acc[ii][jj] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto steps = [&](int buf) {
#pragma unroll
    for (int t = 0; t < G::R / 4; ++t) {
      const float* arow = &As[buf][(4 * t + g) * G::ALD + lr];
      const float* qrow = &Qs[buf][(4 * t + g) * QLD + lr];
      float af[G::IPW], bf[JPW];
#pragma unroll
      for (int ii = 0; ii < G::IPW; ++ii) af[ii] = arow[16 * (i0 + 8 * ii)];
#pragma unroll
      for (int jj = 0; jj < JPW; ++jj) {
        const int j = j0 + G::JS * jj;
        bf[jj] = j < NT ? qrow[16 * j] : 0.f;
      }
#pragma unroll
      for (int ii = 0; ii < G::IPW; ++ii)
#pragma unroll
        for (int jj = 0; jj < JPW; ++jj)
          if (j0 + G::JS * jj < NT) acc[ii][jj] = Mfma<float>::run(af[ii], bf[jj], acc[ii][jj]);
    }
  };
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    load(more ? ch + 1 : ch);
    __builtin_amdgcn_sched_barrier(0);
    steps(buf);
    __builtin_amdgcn_sched_barrier(0);
    if (more) store(buf ^ 1);
    __syncthreads();
  }
  double* out = P + sp * n * (int64_t)c;
#pragma unroll
  for (int ii = 0; ii < G::IPW; ++ii)
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) {
      const int j = j0 + G::JS * jj;
      if (j >= NT) continue;
      const int col = 16 * j + lr;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = 16 * (i0 + 8 * ii) + Mfma<float>::row(lane, e);
        if (row < n && col < c) out[row * c + col] = (double)acc[ii][jj][e];
      }
    }
}

template <typename T, int NT, int MR>
hipError_t nn_dispatch(const T* A, int64_t m, int64_t n, int64_t lda, const T* X, int64_t ldx,
                       int c, T* Y, int64_t ldy, double* fro2_part, int* nparts, hipStream_t s) {
  const int ncol_tiles = nn_col_tiles(c, NT);
  const int64_t nrow_blocks = nn_row_blocks(m);
  static_assert(MR == 2, "nn_row_blocks assumes two 16-row tiles per wave");
  if (nparts) *nparts = (int)nrow_blocks;
  const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && ((lda * sizeof(T)) % 16 == 0);
  dim3 grid((unsigned)(nrow_blocks * ncol_tiles));
  if (vec)
    hipLaunchKernelGGL((k_gemm_nn<T, NT, MR, true>), grid, dim3(kNNThreads), 0, s, A, m, n, lda,
                       X, ldx, c, Y, ldy, fro2_part, ncol_tiles, nullptr);
  else
    hipLaunchKernelGGL((k_gemm_nn<T, NT, MR, false>), grid, dim3(kNNThreads), 0, s, A, m, n, lda,
                       X, ldx, c, Y, ldy, fro2_part, ncol_tiles, nullptr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Split-m partials of Z = A^T Q.  Block = WAVES waves over rows [rs, re) of A;
// wave w owns 16*VW consecutive columns of A (rows of Z), the block covers
// 16*NT columns of Q.  Lane (x = l%16, g = l/16) loads A[r + g][i_w + VW*x
// .. +VW-1] (one 16-byte load when VW*sizeof(T) = 16) and Q[r + g][j0 + 16j + x];
// matrix-core step t produces the Z rows i_w + VW*x' + t, x' = 0..15.
// C is the compute type (double gives exact products of float data).
template <typename T, typename C, int VW, int NT, int WAVES, bool VEC>
__global__ __launch_bounds__(WAVES * 64) void k_gemm_tn_partial(
    const T* __restrict__ A, int64_t m, int64_t n, int64_t lda, const T* __restrict__ Q,
    int64_t ldq, int c, double* __restrict__ P, int64_t rows_per_split) {
  typedef Mfma<C> M;
  typedef typename M::acc_t acc_t;
  constexpr int U = 4;                       // 4-row groups per register set
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  const int64_t split = blockIdx.x;
  const int64_t rs = split * rows_per_split;
  const int64_t re = (rs + rows_per_split < m) ? rs + rows_per_split : m;
  const int64_t iw = (int64_t)blockIdx.y * (WAVES * 16 * VW) + (int64_t)wave * 16 * VW;
  const int64_t ia = iw + VW * x;            // this lane's first A column
  const int j0 = blockIdx.z * 16 * NT;
  const bool full_i = (ia + VW <= n);

  acc_t acc[VW][NT];
#pragma unroll
  for (int t = 0; t < VW; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[t][j] = acc_t{0, 0, 0, 0};

  // rows [r, r + 16): lane (x, g) takes rows r + 4u + g, u < U
  auto load = [&](int64_t r, T(&a)[U][VW], T(&b)[U][NT]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = r + 4 * u + g;
      const bool rok = row < re;
      bool loaded = false;
      if constexpr (VEC && VW * sizeof(T) == 16) {
        if (rok && full_i) {
          const typename Vec16<T>::type v =
              *reinterpret_cast<const typename Vec16<T>::type*>(A + row * lda + ia);
#pragma unroll
          for (int t = 0; t < VW; ++t) a[u][t] = v[t];
          loaded = true;
        }
      }
      if (!loaded) {
#pragma unroll
        for (int t = 0; t < VW; ++t) a[u][t] = (rok && ia + t < n) ? A[row * lda + ia + t] : T(0);
      }
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int col = j0 + 16 * j + x;
        b[u][j] = (rok && col < c) ? Q[row * ldq + col] : T(0);
      }
    }
  };
  auto compute = [&](const T(&a)[U][VW], const T(&b)[U][NT]) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < VW; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = M::run((C)a[u][t], (C)b[u][j], acc[t][j]);
  };

  T a0[U][VW], b0[U][NT], a1[U][VW], b1[U][NT];
  int64_t r = rs;
  load(r, a0, b0);
  while (true) {
    const bool has1 = r + 4 * U < re;
    if (has1) load(r + 4 * U, a1, b1);
    compute(a0, b0);
    if (!has1) break;
    const bool has2 = r + 8 * U < re;
    if (has2) load(r + 8 * U, a0, b0);
    compute(a1, b1);
    if (!has2) break;
    r += 8 * U;
  }

  double* Ps = P + split * n * (int64_t)c;
#pragma unroll
  for (int t = 0; t < VW; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = j0 + 16 * j + x;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = iw + VW * M::row(lane, e) + t;
        if (i < n && col < c) Ps[i * c + col] = (double)acc[t][j][e];
      }
    }
}

// Row-split count: aim at ~256 blocks in total (one per compute unit) and at
// least 64 rows per split.
int64_t tn_splits(int64_t m, int64_t tiles) {
  int64_t s = 256 / (tiles > 0 ? tiles : 1);
  if (s < 1) s = 1;
  const int64_t by_rows = (m + 63) / 64;
  if (s > by_rows) s = by_rows;
  return s < 1 ? 1 : s;
}

template <typename T, typename C, int VW, int NT, int WAVES>
hipError_t tn_dispatch(const T* A, int64_t m, int64_t n, int64_t lda, const T* Q, int64_t ldq,
                       int c, double* P, int64_t max_split, int* nsplit, hipStream_t s) {
  const int64_t itiles = (n + WAVES * 16 * VW - 1) / (WAVES * 16 * VW);
  const int64_t jtiles = (c + 16 * NT - 1) / (16 * NT);
  int64_t splits = tn_splits(m, itiles * jtiles);
  if (splits > max_split) splits = max_split;
  int64_t rps = (m + splits - 1) / splits;
  rps = (rps + 15) / 16 * 16;
  splits = (m + rps - 1) / rps;
  if (splits < 1) splits = 1;
  *nsplit = (int)splits;
  const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && ((lda * sizeof(T)) % 16 == 0);
  dim3 grid((unsigned)splits, (unsigned)itiles, (unsigned)jtiles);
  if (vec)
    hipLaunchKernelGGL((k_gemm_tn_partial<T, C, VW, NT, WAVES, true>), grid, dim3(WAVES * 64), 0, s,
                       A, m, n, lda, Q, ldq, c, P, rps);
  else
    hipLaunchKernelGGL((k_gemm_tn_partial<T, C, VW, NT, WAVES, false>), grid, dim3(WAVES * 64), 0,
                       s, A, m, n, lda, Q, ldq, c, P, rps);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 Gram matrix W = Y^T Y of a tall m x c panel (c <= 16*NT), the first
// step of each CholeskyQR pass.  Every product of two stored values is exact
// in FP64 (and for fp32 data the sum is accumulated in FP64), so the Gram
// keeps the accuracy CholeskyQR needs.  Wave w of a block takes the row
// groups w, w + WAVES, ... (4 rows each) of the block's row range; lane
// (x, g) loads Y[r + g][16 J + x] for every column tile J, and the FP64
// matrix core accumulates the upper-triangle tile pairs (I <= J) only.  The
// waves' sums are added in LDS in wave order and the block writes its
// symmetric partial P[block] (c x c).
constexpr int kGramWaves = 8;

template <typename T, int NT>
__global__ __launch_bounds__(kGramWaves * 64) void k_gram_f64(const T* __restrict__ Y, int64_t m,
                                                            int c, int64_t ldy,
                                                            double* __restrict__ P,
                                                            int64_t rows_per_block,
                                                            const GArgGram* __restrict__ grp) {
  if (grp) {
    const GArgGram& a = grp[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk) return;
    Y = (const T*)a.Y; m = a.m; c = a.c; ldy = a.ldy; P = a.P; rows_per_block = a.rpb;
  }
  typedef Mfma<double> M;
  constexpr int NP = NT * (NT + 1) / 2;
  constexpr int U = 2;                       // 4-row groups per register set
  constexpr int64_t STEP = (int64_t)4 * kGramWaves * U;
  extern __shared__ double red[];            // c x c
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  const int64_t rs = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = (rs + rows_per_block < m) ? rs + rows_per_block : m;
  f64x4 acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = f64x4{0, 0, 0, 0};
  bool colok[NT];
#pragma unroll
  for (int J = 0; J < NT; ++J) colok[J] = (16 * J + x) < c;

  // row group u of the set starting at r0: rows r0 + 4*kGramWaves*u + g
  auto load = [&](int64_t r0, T(&y)[U][NT]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = r0 + (int64_t)4 * kGramWaves * u + g;
      const bool rok = row < re;
#pragma unroll
      for (int J = 0; J < NT; ++J) y[u][J] = (rok && colok[J]) ? Y[row * ldy + 16 * J + x] : T(0);
    }
  };
  auto compute = [&](const T(&y)[U][NT]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double yd[NT];
#pragma unroll
      for (int J = 0; J < NT; ++J) yd[J] = (double)y[u][J];
      int idx = 0;
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J) {
          acc[idx] = M::run(yd[I], yd[J], acc[idx]);
          ++idx;
        }
    }
  };

  T y0[U][NT], y1[U][NT];
  int64_t r = rs + 4 * wave;
  load(r, y0);
  while (r < re) {
    const bool has1 = r + STEP < re;
    if (has1) load(r + STEP, y1);
    compute(y0);
    if (!has1) break;
    const bool has2 = r + 2 * STEP < re;
    if (has2) load(r + 2 * STEP, y0);
    compute(y1);
    if (!has2) break;
    r += 2 * STEP;
  }
  // fixed-order reduction of the waves' tiles in LDS
  for (int w = 0; w < kGramWaves; ++w) {
    if (wave == w) {
      int idx = 0;
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = 16 * I + M::row(lane, e), j = 16 * J + x;
            if (i < c && j < c) {
              const double v = acc[idx][e];
              red[i * c + j] = (w == 0) ? v : red[i * c + j] + v;
            }
          }
          ++idx;
        }
    }
    __syncthreads();
  }
  // symmetric partial: the upper tiles hold W[i][j] for tile(i) <= tile(j)
  double* Pb = P + (int64_t)blockIdx.x * c * c;
  for (int idx = threadIdx.x; idx < c * c; idx += kGramWaves * 64) {
    const int i = idx / c, j = idx - i * c;
    Pb[idx] = ((i >> 4) <= (j >> 4)) ? red[i * c + j] : red[j * c + i];
  }
}

// ---------------------------------------------------------------------------
// W partials (c x c, FP64) of Y^T Y for wide panels (96 < c <= 192): one
// workgroup per row split stages 32-row chunks of all c columns in LDS (two
// buffers, the next chunk's loads in flight while the current one is
// multiplied), and its eight waves take disjoint sets of the upper 16 x 16
// tile pairs (pair p to wave p mod 8, at most kGlMaxPairs each), so every row
// of Y is read from memory once and the waves need no sum across them; each
// wave writes its tiles (and their mirrors) to the split's partial.  The LDS
// row stride is 16 (mod 32) words, so the four 4-row groups of a read fall in
// alternate halves of the banks.
constexpr int kGlWaves = 8, kGlRows = 32;

template <typename T, int NT>
__global__ __launch_bounds__(kGlWaves * 64) void k_gram_lds(const T* __restrict__ Y, int64_t m,
                                                            int c, int64_t ldy,
                                                            double* __restrict__ P,
                                                            int64_t rows_per_block) {
  typedef Mfma<double> M;
  constexpr int NPAIR = NT * (NT + 1) / 2, MAXP = (NPAIR + kGlWaves - 1) / kGlWaves;
  constexpr int LD = (NT % 2) ? 16 * NT : 16 * NT + 16;
  constexpr int NTH = kGlWaves * 64;
  constexpr int EPT = (kGlRows * 16 * NT + NTH - 1) / NTH;   // staged elements per thread
  __shared__ T Ys[2][kGlRows * LD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int x = lane & 15, g = lane >> 4;
  const int64_t rs = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = rs + rows_per_block < m ? rs + rows_per_block : m;
  // this wave's tile pairs (upper pairs in row order, every eighth)
  int pI[MAXP], pJ[MAXP];
  const int np = (NPAIR - wave + kGlWaves - 1) / kGlWaves;
#pragma unroll
  for (int q = 0; q < MAXP; ++q) {
    int I = 0, rem = q < np ? wave + kGlWaves * q : 0;
    while (rem >= NT - I) {
      rem -= NT - I;
      ++I;
    }
    pI[q] = I;
    pJ[q] = I + rem;
  }
  f64x4 acc[MAXP];
#pragma unroll
  for (int q = 0; q < MAXP; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  // both buffers zeroed once: columns past c stay zero
  for (int e = tid; e < 2 * kGlRows * LD; e += NTH) (&Ys[0][0])[e] = T(0);
  // the chunk elements this thread stages (row er, column ec), fixed per chunk
  int er[EPT], ec[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + NTH * u;
    er[u] = e / c;
    ec[u] = e - er[u] * c;
  }
  const gmem<T>* Yg = to_global(Y);
  T v[EPT];
  auto load = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int64_t row = r0 + er[u];
      v[u] = (er[u] < kGlRows && row < re) ? Yg[row * ldy + ec[u]] : T(0);
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int u = 0; u < EPT; ++u)
      if (er[u] < kGlRows) Ys[b][er[u] * LD + ec[u]] = v[u];
  };
  __syncthreads();
  int b = 0;
  if (rs < re) {
    load(rs);
    store(0);
  }
  __syncthreads();
  for (int64_t r0 = rs; r0 < re; r0 += kGlRows, b ^= 1) {
    const bool more = r0 + kGlRows < re;
    if (more) load(r0 + kGlRows);
#pragma unroll
    for (int sk = 0; sk < kGlRows / 4; ++sk) {
      const T* row = &Ys[b][(4 * sk + g) * LD + x];
#pragma unroll
      for (int q = 0; q < MAXP; ++q)
        if (q < np) acc[q] = M::run((double)row[16 * pI[q]], (double)row[16 * pJ[q]], acc[q]);
    }
    if (more) store(b ^ 1);
    __syncthreads();
  }
  double* Pb = P + (int64_t)blockIdx.x * c * c;
#pragma unroll
  for (int q = 0; q < MAXP; ++q)
    if (q < np) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * pI[q] + M::row(lane, e), j = 16 * pJ[q] + x;
        if (i < c && j < c) {
          Pb[(int64_t)i * c + j] = acc[q][e];
          if (pI[q] != pJ[q]) Pb[(int64_t)j * c + i] = acc[q][e];
        }
      }
    }
}

template <typename T, int NT>
hipError_t gram_dispatch(const T* Y, int64_t m, int c, int64_t ldy, double* P, int64_t max_split,
                         int* nsplit, hipStream_t s) {
  int64_t rpb = 0;
  const int64_t blocks = gram_blocks(m, max_split, &rpb);
  *nsplit = (int)blocks;
  const size_t shmem = (size_t)c * c * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_gram_f64<T, NT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gram_f64<T, NT>), dim3((unsigned)blocks), dim3(kGramWaves * 64), shmem, s,
                     Y, m, c, ldy, P, rpb, nullptr);
  return hipGetLastError();
}

__global__ void k_reduce_partials(const double* __restrict__ P, int nsplit, int64_t rows,
                                  int64_t cols, double* __restrict__ Z, int64_t ldz,
                                  const GArgRed* __restrict__ grp) {
  if (grp) {
    const GArgRed& a = grp[blockIdx.y];
    if ((int)blockIdx.x >= a.nblk) return;
    P = a.P; nsplit = a.nsplit; rows = a.rows; cols = a.cols; Z = a.Z; ldz = a.ldz;
  }
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = rows * cols;
  if (idx >= total) return;
  double s = 0.0;
  int k = 0;
  for (; k + 8 <= nsplit; k += 8) {          // eight loads in flight, added in order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)(k + u) * total + idx];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; k < nsplit; ++k) s += P[(int64_t)k * total + idx];
  const int64_t i = idx / cols, j = idx - i * cols;
  Z[i * ldz + j] = s;
}

// The same sum for many partials: a workgroup of kRsWaves waves covers 64
// consecutive elements (lane = element), wave w sums the w-th contiguous run
// of the partials in order (eight loads in flight), and the runs' sums are
// added in wave order: a fixed order, with each thread's chain of dependent
// loads kRsWaves times shorter.
constexpr int kRsWaves = 8;

__global__ __launch_bounds__(kRsWaves * 64) void k_reduce_partials_split(
    const double* __restrict__ P, int nsplit, int64_t rows, int64_t cols, double* __restrict__ Z,
    int64_t ldz) {
  __shared__ double sh[kRsWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t total = rows * cols;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  const int run = (nsplit + kRsWaves - 1) / kRsWaves;
  const int k0 = wave * run, k1 = min(nsplit, k0 + run);
  double s = 0.0;
  if (idx < total) {
    const gmem<double>* p = to_global(P) + idx;
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(k + u) * total];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k < k1; ++k) s += p[(int64_t)k * total];
  }
  sh[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && idx < total) {
    double t = sh[0][lane];
#pragma unroll
    for (int w = 1; w < kRsWaves; ++w) t += sh[w][lane];
    const int64_t i = idx / cols, j = idx - i * cols;
    to_global(Z)[i * ldz + j] = t;
  }
}

__global__ void k_reduce_scalar(const double* __restrict__ parts, int n, double* out,
                                const GArgRedS* __restrict__ grp) {
  if (grp) {
    const GArgRedS& a = grp[blockIdx.y];
    parts = a.parts; n = a.n; out = a.out;
  }
  // fixed order: 256 strided lanes (each adding its entries in index order,
  // eight loads in flight), then a fixed tree
  __shared__ double sh[256];
  double s = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * 256 < n; i += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = parts[i + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; i < n; i += 256) s += parts[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// W (c x c, FP64) = Y^T Y for a short panel (m <= kGramShortRows): one
// workgroup per upper 16 x 16 tile pair (I, J), I <= J, and the waves of the
// workgroup split the rows (wave w takes the 4-row steps w, w + 8, ...;
// kGsUnroll steps' loads in flight per lane before their products); the
// waves' tiles are added in wave order in LDS and the tile and its mirror are
// written to W directly.  Against the row-split kernel plus the sum of its
// partials (two launches, and for m = 512 only two workgroups) a single
// short launch.  Same FP64 products of the stored values (exact for fp32).
constexpr int kGsWaves = 8, kGsUnroll = 8;

template <typename T>
__global__ __launch_bounds__(kGsWaves * 64) void k_gram_short(const T* __restrict__ Y, int64_t m,
                                                              int c, int64_t ldy,
                                                              double* __restrict__ W,
                                                              int64_t ldw) {
  typedef Mfma<double> M;
  // tile pair of this workgroup: the upper pairs in row order
  const int nt = (c + 15) >> 4;
  int I = 0, rem = (int)blockIdx.x;
  while (rem >= nt - I) {
    rem -= nt - I;
    ++I;
  }
  const int J = I + rem;
  __shared__ double red[kGsWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  const int ci = 16 * I + x, cj = 16 * J + x;
  const bool oki = ci < c, okj = cj < c;
  const T* yi = Y + (oki ? ci : 0);
  const T* yj = Y + (okj ? cj : 0);
  const int64_t nks = (m + 3) / 4;                      // 4-row steps
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = wave; k0 < nks; k0 += (int64_t)kGsWaves * kGsUnroll) {
    double a[kGsUnroll], b[kGsUnroll];
#pragma unroll
    for (int u = 0; u < kGsUnroll; ++u) {
      const int64_t row = 4 * (k0 + (int64_t)kGsWaves * u) + g;
      const bool rok = row < m;
      a[u] = (rok && oki) ? (double)yi[row * ldy] : 0.0;
      b[u] = (rok && okj) ? (double)yj[row * ldy] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kGsUnroll; ++u) acc = M::run(a[u], b[u], acc);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) red[wave][e * 64 + lane] = acc[e];
  __syncthreads();
  if (wave == 0) {
    f64x4 t = acc;
#pragma unroll
    for (int w = 1; w < kGsWaves; ++w)
#pragma unroll
      for (int e = 0; e < 4; ++e) t[e] += red[w][e * 64 + lane];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * I + M::row(lane, e), j = 16 * J + x;
      if (i < c && j < c) {
        W[i * ldw + j] = t[e];
        if (I != J) W[j * ldw + i] = t[e];
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Short-k products (no sum of squares) for nt_tall: one kernel per (column
// tiles, k slabs).
constexpr int kNarrowSlabs = 6;

template <int NT, bool TRI>
hipError_t narrow_nt(int ns, const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                     int64_t ldxt, int c, float* Y, int64_t ldy, hipStream_t s) {
  const dim3 grid((unsigned)narrow_blocks(m)), block(256);
#define RSVD_NT_NARROW(NS)                                                                          \
  case NS:                                                                                          \
    hipLaunchKernelGGL((k_gemm_nt_narrow<NT, NS, false, TRI>), grid, block, 0, s, A, m, n, lda, Xt, \
                       ldxt, c, Y, ldy, nullptr, nullptr, nullptr);                                 \
    break;
  switch (ns) {
    RSVD_NT_NARROW(1) RSVD_NT_NARROW(2) RSVD_NT_NARROW(3)
    RSVD_NT_NARROW(4) RSVD_NT_NARROW(5) RSVD_NT_NARROW(6)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_NT_NARROW
  return hipGetLastError();
}

template <bool TRI>
hipError_t launch_narrow(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                         int64_t ldxt, int c, float* Y, int64_t ldy, hipStream_t s) {
  const int ns = (int)((n + 15) / 16);
  switch ((c + 15) / 16) {
    case 1: return narrow_nt<1, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    case 2: return narrow_nt<2, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    case 3: return narrow_nt<3, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    case 4: return narrow_nt<4, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    case 5: return narrow_nt<5, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    case 6: return narrow_nt<6, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    case 7: return narrow_nt<7, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    case 8: return narrow_nt<8, TRI>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm_nt_narrow(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                                 int64_t ldxt, int c, float* Y, int64_t ldy, hipStream_t s) {
  return launch_narrow<false>(A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
}

// The narrow product Y = A Xt^T with a lower-triangular Xt (A R^-1 of
// CholeskyQR) and the FP64 Gram matrix of its output: one c x c partial per
// block at gram_part (persistent blocks, at most max_parts).
template <int NT, int NS>
hipError_t narrow_gram_launch(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                              int64_t ldxt, int c, float* Y, int64_t ldy, double* gram_part,
                              int nblk, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_nt_narrow<NT, NS, true, true>), dim3((unsigned)nblk), dim3(256), 0, s,
                     A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, nullptr, nullptr);
  return hipGetLastError();
}

template <int NT>
hipError_t narrow_gram_ns(int ns, const float* A, int64_t m, int64_t n, int64_t lda,
                          const float* Xt, int64_t ldxt, int c, float* Y, int64_t ldy,
                          double* gram_part, int nblk, hipStream_t s) {
  switch (ns) {
    case 1: return narrow_gram_launch<NT, 1>(A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, nblk, s);
    case 2: return narrow_gram_launch<NT, 2>(A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, nblk, s);
    case 3: return narrow_gram_launch<NT, 3>(A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, nblk, s);
    case 4: return narrow_gram_launch<NT, 4>(A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, nblk, s);
    case 5: return narrow_gram_launch<NT, 5>(A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, nblk, s);
    case 6: return narrow_gram_launch<NT, 6>(A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, nblk, s);
    default: return hipErrorInvalidValue;
  }
}

bool nt_narrow_gram_applies(const float* A, int64_t n, int64_t lda, const float* Xt, int64_t ldxt,
                            int c) {
  return nt_tall_applies(A, n, lda, Xt, ldxt, c) && n <= 16 * kNarrowSlabs && c <= 96;
}

hipError_t launch_gemm_nt_narrow_gram(const float* A, int64_t m, int64_t n, int64_t lda,
                                      const float* Xt, int64_t ldxt, int c, float* Y, int64_t ldy,
                                      double* gram_part, int64_t max_parts, int* nparts,
                                      hipStream_t s) {
  if (!nt_narrow_gram_applies(A, n, lda, Xt, ldxt, c) || max_parts < 1) return hipErrorInvalidValue;
  // past kGramFuseMaxNt column tiles the kernel holds one workgroup per CU:
  // one persistent workgroup per CU (half the partials to sum, no second
  // round of workgroups)
  int64_t nb = narrow_blocks(m);
  if ((c + 15) / 16 > kGramFuseMaxNt && nb > 256) nb = 256;
  if (nb > max_parts) nb = max_parts;
  *nparts = m > 0 ? (int)nb : 0;
  if (m <= 0) return hipSuccess;
  const int ns = (int)((n + 15) / 16);
  switch ((c + 15) / 16) {
    case 1: return narrow_gram_ns<1>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, (int)nb, s);
    case 2: return narrow_gram_ns<2>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, (int)nb, s);
    case 3: return narrow_gram_ns<3>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, (int)nb, s);
    case 4: return narrow_gram_ns<4>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, (int)nb, s);
    case 5: return narrow_gram_ns<5>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, (int)nb, s);
    case 6: return narrow_gram_ns<6>(ns, A, m, n, lda, Xt, ldxt, c, Y, ldy, gram_part, (int)nb, s);
    default: return hipErrorInvalidValue;
  }
}

bool nt_tall_applies(const float* A, int64_t n, int64_t lda, const float* Xt, int64_t ldxt, int c) {
  return c >= 1 && c <= 192 && n % 4 == 0 && (reinterpret_cast<uintptr_t>(A) % 16) == 0 &&
         (lda % 4) == 0 && (reinterpret_cast<uintptr_t>(Xt) % 16) == 0 && (ldxt % 4) == 0 &&
         (int64_t)kTM * lda * 4 < (1LL << 31) && (int64_t)c * ldxt * 4 < (1LL << 31);
}

hipError_t launch_gemm_nt_tall(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                               int64_t ldxt, int c, float* Y, int64_t ldy, double* fro2_part,
                               int* nparts, hipStream_t s) {
  if (!nt_tall_applies(A, n, lda, Xt, ldxt, c)) return hipErrorInvalidValue;
  const int64_t nblk = tall_blocks(m);
  if (nparts) *nparts = (int)nblk;
  if (m <= 0) return hipSuccess;
  if (!fro2_part && n <= 16 * kNarrowSlabs && c <= 128)
    return launch_gemm_nt_narrow(A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
  const dim3 grid((unsigned)nblk), block(256);
#define RSVD_NT_TALL(NT)                                                                      \
  case NT:                                                                                    \
    hipLaunchKernelGGL((k_gemm_nt_tall<NT, false>), grid, block, 0, s, A, m, n, lda, Xt, ldxt, \
                       c, Y, ldy, fro2_part, nullptr, nullptr);                               \
    break;
  switch ((c + 15) / 16) {
    RSVD_NT_TALL(1) RSVD_NT_TALL(2) RSVD_NT_TALL(3) RSVD_NT_TALL(4)
    RSVD_NT_TALL(5) RSVD_NT_TALL(6) RSVD_NT_TALL(7) RSVD_NT_TALL(8)
    RSVD_NT_TALL(9) RSVD_NT_TALL(10) RSVD_NT_TALL(11) RSVD_NT_TALL(12)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_NT_TALL
  return hipGetLastError();
}

hipError_t launch_gemm_nt_tri(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                              int64_t ldxt, int c, float* Y, int64_t ldy, hipStream_t s) {
  if (!nt_tall_applies(A, n, lda, Xt, ldxt, c)) return hipErrorInvalidValue;
  if (m <= 0) return hipSuccess;
  if (n <= 16 * kNarrowSlabs && c <= 128)
    return launch_narrow<true>(A, m, n, lda, Xt, ldxt, c, Y, ldy, s);
  return launch_gemm_nt_tall(A, m, n, lda, Xt, ldxt, c, Y, ldy, nullptr, nullptr, s);
}

bool tn_tall_applies(const float* A, int64_t lda, const float* Q, int64_t ldq, int c) {
  return c >= 1 && c <= 160 && (reinterpret_cast<uintptr_t>(A) % 16) == 0 && (lda % 4) == 0 &&
         (reinterpret_cast<uintptr_t>(Q) % 16) == 0 && (ldq % 4) == 0;
}

hipError_t launch_gemm_tn_tall(const float* A, int64_t m, int64_t n, int64_t lda, const float* Q,
                               int64_t ldq, int c, double* P, int64_t max_split, int* nsplit,
                               hipStream_t s) {
  if (!tn_tall_applies(A, lda, Q, ldq, c) || m <= 0) return hipErrorInvalidValue;
  int ntile = 0;
  int64_t rps = 0;
  const int64_t ns = tn_tall_splits(m, n, max_split, &rps, &ntile);
  const int64_t ld = lda > ldq ? lda : ldq;
  // 32-bit buffer offsets: the split's rows, and a chunk's offsets (at most
  // 32 rows, the narrow kernel's) within a row split
  if (rps * ld * 4 >= (1LL << 31) || (int64_t)31 * ld * 4 + (int64_t)ntile * kUA * 4 >= (1LL << 31))
    return hipErrorInvalidValue;
  *nsplit = (int)ns;
  const dim3 grid((unsigned)(ns * ntile)), block(512);
  const int cw = tn_col_waves(n);
#define RSVD_TN_TALL(NT)                                                                          \
  case NT:                                                                                        \
    if (cw == 1)                                                                                  \
      hipLaunchKernelGGL((k_gemm_tn_narrow<NT, 1>), grid, block, 0, s, A, m, n, lda, Q, ldq, c,   \
                         rps, ntile, P, nullptr, nullptr);                                             \
    else if (cw == 2)                                                                             \
      hipLaunchKernelGGL((k_gemm_tn_narrow<NT, 2>), grid, block, 0, s, A, m, n, lda, Q, ldq, c,   \
                         rps, ntile, P, nullptr, nullptr);                                             \
    else if (cw == 4)                                                                             \
      hipLaunchKernelGGL((k_gemm_tn_narrow<NT, 4>), grid, block, 0, s, A, m, n, lda, Q, ldq, c,   \
                         rps, ntile, P, nullptr, nullptr);                                             \
    else                                                                                          \
      hipLaunchKernelGGL(k_gemm_tn_tall<NT>, grid, block, 0, s, A, m, n, lda, Q, ldq, c, rps,     \
                         ntile, P, nullptr, nullptr);                                             \
    break;
  switch ((c + 15) / 16) {
    RSVD_TN_TALL(1) RSVD_TN_TALL(2) RSVD_TN_TALL(3) RSVD_TN_TALL(4)
    RSVD_TN_TALL(5) RSVD_TN_TALL(6) RSVD_TN_TALL(7) RSVD_TN_TALL(8)
    RSVD_TN_TALL(9) RSVD_TN_TALL(10)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_TN_TALL
  return hipGetLastError();
}

hipError_t launch_syrk_f32(const float* A, int64_t m, int64_t n, int64_t lda, double* P,
                           int64_t p_cap, double* G, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int ntile = (int)((n + kSyT - 1) / kSyT);
  const int npair = ntile * (ntile + 1) / 2;
  // one resident wave of blocks (two per CU on 256 CUs: every block of a row
  // split runs at the same time as the others, so they share A in L2),
  // splits of whole chunks, and the partial tiles within the scratch capacity
  int64_t nsplit = (2 * 256) / npair;
  const int64_t by_rows = (m + kSyK - 1) / kSyK;
  if (nsplit > by_rows) nsplit = by_rows;
  const int64_t cap = p_cap / ((int64_t)npair * kSyT * kSyT);
  if (nsplit > cap) nsplit = cap;
  if (nsplit < 1) return hipErrorInvalidValue;
  int64_t rps = (m + nsplit - 1) / nsplit;
  rps = (rps + kSyK - 1) / kSyK * kSyK;
  nsplit = (m + rps - 1) / rps;
  if ((reinterpret_cast<uintptr_t>(A) % 16) != 0 || (lda % 4) != 0 ||
      rps * lda * 4 >= (1LL << 31))
    return hipErrorInvalidValue;
  const int64_t nblk = nsplit * npair;
  const int64_t per_xcd = (nblk + 7) / 8;
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL(k_syrk_f32, dim3((unsigned)(8 * per_xcd)), dim3(256), 0, s, A, m, n, lda,
                     ntile, npair, rps, nblk, per_xcd, P);
  hipError_t e = hipGetLastError();
  if (ev1) (void)hipEventRecord(ev1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_syrk_reduce, dim3((kSyT * kSyT / 2 + 255) / 256, npair), dim3(256), 0, s, P,
                     nsplit, npair, ntile, n, G, n);
  return hipGetLastError();
}

bool syrk_f32_applies(const float* A, int64_t n, int64_t lda) {
  return n > 128 && (reinterpret_cast<uintptr_t>(A) % 16) == 0 && (lda % 4) == 0 &&
         (n % 4) == 0;
}

hipError_t launch_gemm_nt_wide(const float* A, int64_t m, int64_t n, int64_t lda, const float* Xt,
                               int64_t ldxt, int c, float* Y, int64_t ldy, hipStream_t s) {
  if (m <= 0 || c <= 0) return hipSuccess;
  const int64_t nrb = (m + kWM - 1) / kWM;
  const int ncb = (c + kWN - 1) / kWN;
  const int64_t ntiles = nrb * ncb;
  const int64_t per_xcd = (ntiles + 7) / 8;
  // fast path: whole chunks, 16-byte rows, and byte offsets of a block's
  // panel within 32 bits
  const bool fast = (n % kWK == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0) &&
                    (lda % 4 == 0) && (reinterpret_cast<uintptr_t>(Xt) % 16 == 0) &&
                    (ldxt % 4 == 0) && ((int64_t)kWM * lda * 4 < (1LL << 31)) &&
                    ((int64_t)kWN * ldxt * 4 < (1LL << 31));
  hipLaunchKernelGGL(k_gemm_nt_wide, dim3((unsigned)(8 * per_xcd)), dim3(kWT), 0, s, A, m, n, lda,
                     Xt, ldxt, c, Y, ldy, ntiles, ncb, per_xcd, fast ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_nn(const T* A, int64_t m, int64_t n, int64_t lda, const T* X, int64_t ldx,
                          int c, T* Y, int64_t ldy, double* fro2_part, int* nparts,
                          hipStream_t s) {
  if (m <= 0 || c <= 0) { if (nparts) *nparts = 0; return hipSuccess; }
  // the number of 16-column tiles a block covers: all of c up to 128 columns
  const int nt = (c + 15) / 16;
  switch (nt > 8 ? 8 : nt) {
    case 1: return nn_dispatch<T, 1, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
    case 2: return nn_dispatch<T, 2, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
    case 3: return nn_dispatch<T, 3, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
    case 4: return nn_dispatch<T, 4, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
    case 5: return nn_dispatch<T, 5, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
    case 6: return nn_dispatch<T, 6, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
    case 7: return nn_dispatch<T, 7, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
    default: return nn_dispatch<T, 8, 2>(A, m, n, lda, X, ldx, c, Y, ldy, fro2_part, nparts, s);
  }
}

int64_t tn_max_split(int64_t m, int64_t n, int c) {
  (void)n; (void)c;
  return tn_splits(m, 1);
}

template <typename T, typename C>
hipError_t launch_gemm_tn_partial(const T* A, int64_t m, int64_t n, int64_t lda, const T* Q,
                                  int64_t ldq, int c, double* P, int64_t max_split, int* nsplit,
                                  hipStream_t s) {
  if (m <= 0 || n <= 0 || c <= 0) { *nsplit = 0; return hipSuccess; }
  const int nt = (c + 15) / 16;
  constexpr bool exact = sizeof(C) > sizeof(T);       // fp64 Gram of fp32 data
  constexpr int VW = exact ? 1 : 16 / sizeof(T);
  constexpr int WAVES = exact ? 4 : 8;
#define RSVD_TN(NT_) return tn_dispatch<T, C, VW, NT_, WAVES>(A, m, n, lda, Q, ldq, c, P, max_split, nsplit, s)
  switch (nt > 8 ? 8 : nt) {
    case 1: RSVD_TN(1);
    case 2: RSVD_TN(2);
    case 3: RSVD_TN(3);
    case 4: RSVD_TN(4);
    case 5: RSVD_TN(5);
    case 6: RSVD_TN(6);
    case 7: RSVD_TN(7);
    default: RSVD_TN(8);
  }
#undef RSVD_TN
}

template <typename T>
hipError_t launch_gram_f64(const T* Y, int64_t m, int c, int64_t ldy, double* P, int64_t max_split,
                           int* nsplit, hipStream_t s) {
  if (m <= 0 || c <= 0) { *nsplit = 0; return hipSuccess; }
  switch ((c + 15) / 16) {
    case 1: return gram_dispatch<T, 1>(Y, m, c, ldy, P, max_split, nsplit, s);
    case 2: return gram_dispatch<T, 2>(Y, m, c, ldy, P, max_split, nsplit, s);
    case 3: return gram_dispatch<T, 3>(Y, m, c, ldy, P, max_split, nsplit, s);
    case 4: return gram_dispatch<T, 4>(Y, m, c, ldy, P, max_split, nsplit, s);
    case 5: return gram_dispatch<T, 5>(Y, m, c, ldy, P, max_split, nsplit, s);
    case 6: return gram_dispatch<T, 6>(Y, m, c, ldy, P, max_split, nsplit, s);
    default: {
      if (c > 192) return hipErrorInvalidValue;
      // one workgroup per split of at least 1024 rows, at most one per CU
      int64_t rpb = 0;
      const int64_t blocks = gram_blocks(m, max_split < 256 ? max_split : 256, &rpb, 1024);
      *nsplit = (int)blocks;
      const dim3 grid((unsigned)blocks), block(kGlWaves * 64);
      // c <= 112 takes the 8-tile kernel (its last tile column all zeros):
      // the 7-tile build needs every register and spills
      switch ((c + 15) / 16) {
        case 7:
        case 8: hipLaunchKernelGGL((k_gram_lds<T, 8>), grid, block, 0, s, Y, m, c, ldy, P, rpb); break;
        case 9: hipLaunchKernelGGL((k_gram_lds<T, 9>), grid, block, 0, s, Y, m, c, ldy, P, rpb); break;
        case 10: hipLaunchKernelGGL((k_gram_lds<T, 10>), grid, block, 0, s, Y, m, c, ldy, P, rpb); break;
        case 11: hipLaunchKernelGGL((k_gram_lds<T, 11>), grid, block, 0, s, Y, m, c, ldy, P, rpb); break;
        default: hipLaunchKernelGGL((k_gram_lds<T, 12>), grid, block, 0, s, Y, m, c, ldy, P, rpb); break;
      }
      return hipGetLastError();
    }
  }
}

template <typename T>
hipError_t launch_gram_short(const T* Y, int64_t m, int c, int64_t ldy, double* W, int64_t ldw,
                             hipStream_t s) {
  if (m <= 0 || c <= 0 || m > kGramShortRows) return hipErrorInvalidValue;
  const int nt = (c + 15) / 16;
  hipLaunchKernelGGL(k_gram_short<T>, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(kGsWaves * 64), 0,
                     s, Y, m, c, ldy, W, ldw);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* P, int nsplit, int64_t rows, int64_t cols,
                                  double* Z, int64_t ldz, hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  if (nsplit >= 4 * kRsWaves)
    hipLaunchKernelGGL(k_reduce_partials_split, dim3((unsigned)((total + 63) / 64)),
                       dim3(kRsWaves * 64), 0, s, P, nsplit, rows, cols, Z, ldz);
  else
    hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       P, nsplit, rows, cols, Z, ldz, nullptr);
  return hipGetLastError();
}

hipError_t launch_reduce_scalar(const double* parts, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_scalar, dim3(1), dim3(256), 0, s, parts, n, out, nullptr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launch geometry (shared by the ordinary and the grouped launchers).
// Row splits of the partial-sum kernels: at most one block per CU (256) and at
// least min_rows rows per split.  A solve that has the GPU to itself takes
// many short splits (parallelism); a grouped batch, whose instances fill the
// GPU together, takes long ones, so that the FP64 partials (c x c or n x c
// per split, written and read back by the reduction) stay small beside the
// panel itself (2c / min_rows of its bytes).
int64_t gram_blocks(int64_t m, int64_t max_split, int64_t* rows_per_block, int64_t min_rows) {
  int64_t blocks = (m + min_rows - 1) / min_rows;
  if (blocks > max_split) blocks = max_split;
  if (blocks < 1) blocks = 1;
  int64_t rpb = (m + blocks - 1) / blocks;
  rpb = (rpb + 3) / 4 * 4;
  *rows_per_block = rpb;
  return (m + rpb - 1) / rpb;
}

int64_t tn_tall_splits(int64_t m, int64_t n, int64_t max_split, int64_t* rows_per_split,
                       int* ntile_out, int64_t min_rows) {
  const int ntile = (int)((n + kUA - 1) / kUA);
  // about one block per CU (256), whole 16-row chunks
  int64_t ns = 256 / ntile;
  if (ns < 1) ns = 1;
  if (ns > (m + min_rows - 1) / min_rows) ns = (m + min_rows - 1) / min_rows;
  if (ns > max_split) ns = max_split;
  int64_t rps = (m + ns - 1) / ns;
  rps = (rps + kUK - 1) / kUK * kUK;
  *rows_per_split = rps;
  *ntile_out = ntile;
  return (m + rps - 1) / rps;
}

// persistent: up to two blocks per CU of the 256
// column waves of the A^T Q kernel for n columns: 1, 2 or 4 (narrow kernel,
// 64 columns per wave group) or 8 (the 512-column tile)
int tn_col_waves(int64_t n) { return n <= 64 ? 1 : (n <= 128 ? 2 : (n <= 256 ? 4 : 8)); }

int64_t narrow_blocks(int64_t m) {
  const int64_t ntile = (m + kNM - 1) / kNM;
  return ntile < 512 ? ntile : 512;
}

int64_t tall_blocks(int64_t m) { return (m + kTM - 1) / kTM; }

int nn_col_tiles(int c, int nt) { return (c + 16 * nt - 1) / (16 * nt); }

int64_t nn_row_blocks(int64_t m) { return (m + 128 - 1) / 128; }

// ---------------------------------------------------------------------------
// Grouped launchers.  The three tall passes run over a work list (one
// block per item); the other steps take one launch with blockIdx.y =
// problem.
template <int NT, bool GR>
hipError_t tall_grouped(const GArgTall* a, const GWork* wl, int nwork, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_nt_tall<NT, GR>), dim3((unsigned)nwork), dim3(256), 0, s, nullptr, 0,
                     0, 0, nullptr, 0, 0, nullptr, 0, nullptr, a, wl);
  return hipGetLastError();
}

hipError_t launch_gemm_nt_tall_grouped(const GArgTall* a, const GWork* wl, int nwork, int nt,
                                       bool gram, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (gram && nt > kGramFuseMaxNt) return hipErrorInvalidValue;
  switch (nt) {
    case 1: return gram ? tall_grouped<1, true>(a, wl, nwork, s) : tall_grouped<1, false>(a, wl, nwork, s);
    case 2: return gram ? tall_grouped<2, true>(a, wl, nwork, s) : tall_grouped<2, false>(a, wl, nwork, s);
    case 3: return gram ? tall_grouped<3, true>(a, wl, nwork, s) : tall_grouped<3, false>(a, wl, nwork, s);
    case 4: return gram ? tall_grouped<4, true>(a, wl, nwork, s) : tall_grouped<4, false>(a, wl, nwork, s);
    case 5: return tall_grouped<5, false>(a, wl, nwork, s);
    case 6: return tall_grouped<6, false>(a, wl, nwork, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NT, bool GR, bool TRI>
hipError_t narrow_grouped(const GArgNarrow* a, const GWork* wl, int nwork, int ns, hipStream_t s) {
  const dim3 grid((unsigned)nwork), block(256);
#define RSVD_G(NS)                                                                                \
  case NS:                                                                                        \
    hipLaunchKernelGGL((k_gemm_nt_narrow<NT, NS, GR, TRI>), grid, block, 0, s, nullptr, 0, 0, 0,  \
                       nullptr, 0, 0, nullptr, 0, nullptr, a, wl);                                \
    break;
  switch (ns) {
    RSVD_G(1) RSVD_G(2) RSVD_G(3) RSVD_G(4) RSVD_G(5) RSVD_G(6)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_G
  return hipGetLastError();
}

template <bool TRI>
hipError_t narrow_grouped_nt(const GArgNarrow* a, const GWork* wl, int nwork, int nt, int ns,
                             bool gram, hipStream_t s) {
  switch (nt) {
    case 1: return gram ? narrow_grouped<1, true, TRI>(a, wl, nwork, ns, s) : narrow_grouped<1, false, TRI>(a, wl, nwork, ns, s);
    case 2: return gram ? narrow_grouped<2, true, TRI>(a, wl, nwork, ns, s) : narrow_grouped<2, false, TRI>(a, wl, nwork, ns, s);
    case 3: return gram ? narrow_grouped<3, true, TRI>(a, wl, nwork, ns, s) : narrow_grouped<3, false, TRI>(a, wl, nwork, ns, s);
    case 4: return gram ? narrow_grouped<4, true, TRI>(a, wl, nwork, ns, s) : narrow_grouped<4, false, TRI>(a, wl, nwork, ns, s);
    case 5: return narrow_grouped<5, false, TRI>(a, wl, nwork, ns, s);
    case 6: return narrow_grouped<6, false, TRI>(a, wl, nwork, ns, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm_nt_narrow_grouped(const GArgNarrow* a, const GWork* wl, int nwork, int nt,
                                         int ns, bool gram, bool tri, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (gram && nt > kGramFuseMaxNt) return hipErrorInvalidValue;
  return tri ? narrow_grouped_nt<true>(a, wl, nwork, nt, ns, gram, s)
             : narrow_grouped_nt<false>(a, wl, nwork, nt, ns, gram, s);
}

hipError_t launch_gemm_tn_tall_grouped(const GArgTn* a, const GWork* wl, int nwork, int nt,
                                       int cw, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  const dim3 grid((unsigned)nwork), block(512);
#define RSVD_G(NT)                                                                              \
  case NT:                                                                                      \
    if (cw == 1)                                                                                \
      hipLaunchKernelGGL((k_gemm_tn_narrow<NT, 1>), grid, block, 0, s, nullptr, 0, 0, 0, nullptr, \
                         0, 0, 0, 1, nullptr, a, wl);                                           \
    else if (cw == 2)                                                                           \
      hipLaunchKernelGGL((k_gemm_tn_narrow<NT, 2>), grid, block, 0, s, nullptr, 0, 0, 0, nullptr, \
                         0, 0, 0, 1, nullptr, a, wl);                                           \
    else if (cw == 4)                                                                           \
      hipLaunchKernelGGL((k_gemm_tn_narrow<NT, 4>), grid, block, 0, s, nullptr, 0, 0, 0, nullptr, \
                         0, 0, 0, 1, nullptr, a, wl);                                           \
    else                                                                                        \
      hipLaunchKernelGGL(k_gemm_tn_tall<NT>, grid, block, 0, s, nullptr, 0, 0, 0, nullptr, 0, 0, \
                         0, 1, nullptr, a, wl);                                                 \
    break;
  switch (nt) {
    RSVD_G(1) RSVD_G(2) RSVD_G(3) RSVD_G(4) RSVD_G(5) RSVD_G(6)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_G
  return hipGetLastError();
}

template <typename T, int NT>
hipError_t gram_grouped(const GArgGram* a, int count, int maxblk, int cmax, hipStream_t s) {
  const size_t shmem = (size_t)cmax * cmax * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_gram_f64<T, NT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gram_f64<T, NT>), dim3((unsigned)maxblk, (unsigned)count),
                     dim3(kGramWaves * 64), shmem, s, nullptr, 0, 0, 0, nullptr, 0, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gram_f64_grouped(const GArgGram* a, int count, int maxblk, int nt, int cmax,
                                   hipStream_t s) {
  if (count <= 0 || maxblk <= 0) return hipSuccess;
  switch (nt) {
    case 1: return gram_grouped<T, 1>(a, count, maxblk, cmax, s);
    case 2: return gram_grouped<T, 2>(a, count, maxblk, cmax, s);
    case 3: return gram_grouped<T, 3>(a, count, maxblk, cmax, s);
    case 4: return gram_grouped<T, 4>(a, count, maxblk, cmax, s);
    case 5: return gram_grouped<T, 5>(a, count, maxblk, cmax, s);
    case 6: return gram_grouped<T, 6>(a, count, maxblk, cmax, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_gram_f64_grouped<float>(const GArgGram*, int, int, int, int,
                                                   hipStream_t);
template hipError_t launch_gram_f64_grouped<double>(const GArgGram*, int, int, int, int,
                                                    hipStream_t);

hipError_t launch_reduce_partials_grouped(const GArgRed* a, int count, int maxblk, hipStream_t s) {
  if (count <= 0 || maxblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)maxblk, (unsigned)count), dim3(256), 0, s,
                     nullptr, 0, 0, 0, nullptr, 0, a);
  return hipGetLastError();
}

hipError_t launch_reduce_scalar_grouped(const GArgRedS* a, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_scalar, dim3(1, (unsigned)count), dim3(256), 0, s, nullptr, 0,
                     nullptr, a);
  return hipGetLastError();
}

// FP64 Y = A X on the tiles an ordinary launch_gemm_nn<double> picks for c
// (vectorised loads: every A of a grouped launch is 16-byte aligned with an
// even leading dimension).
hipError_t launch_gemm_nn_f64_grouped(const GArgNn* a, int count, int maxblk, int nt,
                                      hipStream_t s) {
  if (count <= 0 || maxblk <= 0) return hipSuccess;
  const dim3 grid((unsigned)maxblk, (unsigned)count);
#define RSVD_G(NT)                                                                              \
  case NT:                                                                                      \
    hipLaunchKernelGGL((k_gemm_nn<double, NT, 2, true>), grid, dim3(kNNThreads), 0, s, nullptr, \
                       0, 0, 0, nullptr, 0, 0, nullptr, 0, nullptr, 1, a);                      \
    break;
  switch (nt) {
    RSVD_G(1) RSVD_G(2) RSVD_G(3) RSVD_G(4) RSVD_G(5) RSVD_G(6) RSVD_G(7) RSVD_G(8)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_G
  return hipGetLastError();
}

template hipError_t launch_gemm_nn<float>(const float*, int64_t, int64_t, int64_t, const float*,
                                          int64_t, int, float*, int64_t, double*, int*,
                                          hipStream_t);
template hipError_t launch_gemm_nn<double>(const double*, int64_t, int64_t, int64_t,
                                           const double*, int64_t, int, double*, int64_t, double*,
                                           int*, hipStream_t);
template hipError_t launch_gram_f64<float>(const float*, int64_t, int, int64_t, double*, int64_t,
                                           int*, hipStream_t);
template hipError_t launch_gram_f64<double>(const double*, int64_t, int, int64_t, double*, int64_t,
                                            int*, hipStream_t);
template hipError_t launch_gram_short<float>(const float*, int64_t, int, int64_t, double*, int64_t,
                                             hipStream_t);
template hipError_t launch_gram_short<double>(const double*, int64_t, int, int64_t, double*,
                                              int64_t, hipStream_t);
template hipError_t launch_gemm_tn_partial<float, float>(const float*, int64_t, int64_t, int64_t,
                                                         const float*, int64_t, int, double*,
                                                         int64_t, int*, hipStream_t);
template hipError_t launch_gemm_tn_partial<float, double>(const float*, int64_t, int64_t, int64_t,
                                                          const float*, int64_t, int, double*,
                                                          int64_t, int*, hipStream_t);
template hipError_t launch_gemm_tn_partial<double, double>(const double*, int64_t, int64_t,
                                                           int64_t, const double*, int64_t, int,
                                                           double*, int64_t, int*, hipStream_t);

}  // namespace rsvd
