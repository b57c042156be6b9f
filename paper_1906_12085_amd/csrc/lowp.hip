// lowp.hip -- the passes over A when A is stored in bfloat16 with one FP32
// scale per column (dequantised A = Aq diag(s)): the sketch product and the
// power-iteration products Y = A X (Sec. 3.1.2 steps 2-3) and the projection
// Z = A^T Q (step 5) on the BF16 matrix cores with FP32 accumulation.  The
// right factors X and Q are FP32/FP64 values split into hi + lo bfloat16
// pairs (x = hi + lo to 16 significant bits), so a product costs two BF16
// matrix-core operations and loses only ~2^-17 relative against an FP32
// product; A's own rounding is the stored representation (the reference
// computes on the dequantised stored A).  Also the quantiser
// (power-of-two column scales, so the scaling itself is exact).
#include <type_traits>

#include "device_common.h"

namespace rsvd {

namespace {

inline unsigned nblocks(int64_t total, int per) { return (unsigned)((total + per - 1) / per); }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16x16x32 bf16 matrix core: lane l supplies a = Aop[l%16][8(l/16) .. +7] and
// b = Bop[8(l/16) .. +7][l%16]; value e of lane l is at row 4(l/16) + e,
// column l%16 (the fp32 16x16x4 result layout).
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ u32x4 as_u32x4(bf16x8 v) { return __builtin_bit_cast(u32x4, v); }

// hi + lo split of x: hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in FP32)
__device__ __forceinline__ void split_hilo(float x, __bf16* hi, __bf16* lo) {
  const __bf16 h = (__bf16)x;
  *hi = h;
  *lo = (__bf16)(x - (float)h);
}

// Operand fragment of 8 consecutive stored elements: 16 bytes of bfloat16, or
// 8 bytes of OCP FP8 E4M3 widened to bfloat16 in registers (every E4M3 value,
// subnormals included, is exact in bfloat16; the hardware packed convert
// follows the OCP E4M3 definition, NaN for S.1111.111).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
template <int ES> struct Frag;
template <> struct Frag<2> {
  typedef u32x4 raw;
  static __device__ __forceinline__ raw load(__amdgpu_buffer_rsrc_t r, int vo, int so) {
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
  }
  static __device__ __forceinline__ u32x4 bf(raw v) { return v; }
};
template <> struct Frag<1> {
  typedef u32x2 raw;
  static __device__ __forceinline__ raw load(__amdgpu_buffer_rsrc_t r, int vo, int so) {
    return __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  // two E4M3 codes (low or high half of w) to two bfloat16 in one packed
  // convert (unit scale); every E4M3 value is exact in bfloat16, and this
  // gives the same bits as widening through FP32 for all 2^16 code pairs
  template <bool HI>
  static __device__ __forceinline__ unsigned pair(unsigned w) {
    return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f, HI));
  }
  static __device__ __forceinline__ u32x4 bf(raw v) {
    return u32x4{pair<false>(v[0]), pair<true>(v[0]), pair<false>(v[1]), pair<true>(v[1])};
  }
};

// ---------------------------------------------------------------------------
// Octet transpose: lanes o = 0..7 of an aligned group of 8 each hold 8 bf16
// (row o of an 8 x 8 block, four dwords of two columns each); afterwards lane
// o holds column o (rows 0..7 in order).  Three exchange stages: 4 x 4 blocks
// between lanes o and o^4, 2 x 2 blocks between o and o^2, single elements
// between o and o^1.
template <int PAT>
__device__ __forceinline__ unsigned swz(unsigned v) {
  return (unsigned)__builtin_amdgcn_ds_swizzle((int)v, PAT);
}
template <int CTRL>
__device__ __forceinline__ unsigned dpp(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ u32x4 octet_transpose(u32x4 d, int o) {
  // stage A: lane o (b = bit 2) keeps its half of the columns 4b..4b+3 and
  // takes the partner's: rows {o&3, (o&3)+4}, columns 4b..4b+3
  {
    const bool b = (o & 4) != 0;
    const unsigned s0 = b ? d[0] : d[2], s1 = b ? d[1] : d[3];
    const unsigned r0 = swz<0x101F>(s0), r1 = swz<0x101F>(s1);   // xor 4
    d = b ? u32x4{r0, r1, d[2], d[3]} : u32x4{d[0], d[1], r0, r1};
  }
  // stage B: rows {r, r+2, r+4, r+6} (r = o&1), columns 4b+2c1, +1 (c1 = bit 1)
  {
    const bool c1 = (o & 2) != 0;
    const unsigned s0 = c1 ? d[0] : d[1], s1 = c1 ? d[2] : d[3];
    const unsigned r0 = dpp<0x4E>(s0), r1 = dpp<0x4E>(s1);        // quad_perm(2,3,0,1): xor 2
    d = c1 ? u32x4{r0, d[1], r1, d[3]} : u32x4{d[0], r0, d[2], r1};
  }
  // stage C: column 4b + 2c1 + c0 for rows 2p, 2p+1 (c0 = bit 0)
  {
    const bool c0 = (o & 1) != 0;
    u32x4 pe;
#pragma unroll
    for (int p = 0; p < 4; ++p) pe[p] = dpp<0xB1>(d[p]);          // quad_perm(1,0,3,2): xor 1
    // c0 = 0: low(own) | low(partner) << 16;  c0 = 1: high(partner) | high(own) << 16
    const unsigned sel = c0 ? 0x03020706u : 0x05040100u;
    u32x4 out;
#pragma unroll
    for (int p = 0; p < 4; ++p) out[p] = __builtin_amdgcn_perm(pe[p], d[p], sel);
    d = out;
  }
  return d;
}

// ---------------------------------------------------------------------------
// Quantiser: s_j = 2^e with 2^(e-1) <= max_i |A_ij| < 2^e (s_j = 1 for a zero
// column), Aq = bf16(A / s_j) rounded to nearest even.
__global__ void k_colmax_abs(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                             int64_t rows_per_block, unsigned* __restrict__ cmax) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    float v = 0.f;
    for (int64_t i = r0; i < r1; ++i) v = fmaxf(v, fabsf(A[i * lda + j]));
    // non-negative floats order like their bit patterns
    atomicMax(cmax + j, __float_as_uint(v));
  }
}

__device__ __forceinline__ float pow2_scale(unsigned maxbits) {
  const float mx = __uint_as_float(maxbits);
  if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
  int e;
  (void)frexpf(mx, &e);                 // mx = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, e);
}

__global__ void k_quantize_bf16(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                const unsigned* __restrict__ cmax, __bf16* __restrict__ Aq,
                                int64_t ldq, float* __restrict__ scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  const float s = pow2_scale(cmax[j]);
  Aq[i * ldq + j] = (__bf16)(A[i * lda + j] / s);
  if (i == 0) scale[j] = s;
}

// FP8 E4M3 storage: s_j = the least power of two with max_i |A_ij| / s_j <=
// 448 (the largest E4M3 value; 1 for a zero column), Aq = E4M3(A / s_j).
__device__ __forceinline__ float pow2_scale_fp8(unsigned maxbits) {
  const float mx = __uint_as_float(maxbits);
  if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
  int e;
  const float f = frexpf(mx / 448.f, &e);   // mx / 448 = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, f == 0.5f ? e - 1 : e);
}

// x to OCP FP8 E4M3 (bias 7, 3 mantissa bits, largest 448, no infinities,
// S.1111.111 = NaN), rounded to nearest with ties to an even mantissa;
// magnitudes past 448 saturate to 448.
__device__ __forceinline__ unsigned char e4m3_rne(float x) {
  const unsigned sg = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (!(a == a)) return (unsigned char)(sg | 0x7Fu);
  if (a >= 448.f) return (unsigned char)(sg | 0x7Eu);
  if (a < 0x1p-6f) {
    // subnormal spacing 2^-9 (a rounded count of 8 is the smallest normal, code 8)
    return (unsigned char)(sg | (unsigned)rintf(a * 512.f));
  }
  int e;
  const float f = frexpf(a, &e);              // a = (2f) 2^(e-1), 2f in [1, 2)
  int ex = e - 1;
  int mq = (int)rintf((2.f * f - 1.f) * 8.f);  // exact product, rounded to even
  if (mq == 8) { mq = 0; ++ex; }
  return (unsigned char)(sg | (unsigned)((ex + 7) << 3) | (unsigned)mq);
}

__global__ void k_quantize_fp8(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                               const unsigned* __restrict__ cmax, unsigned char* __restrict__ Aq,
                               int64_t ldq, float* __restrict__ scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  const float s = pow2_scale_fp8(cmax[j]);
  Aq[i * ldq + j] = e4m3_rne(A[i * lda + j] / s);
  if (i == 0) scale[j] = s;
}

// Xhi, Xlo (c x n, row stride ldx) = split of (diag(s) X)^T, X (n x c) FP64
// row-major with ld c: row j of the result is column j of diag(s) X.
__global__ void k_cast_hilo_t(const double* __restrict__ X, int64_t n, int c,
                              const float* __restrict__ scale, __bf16* __restrict__ Xhi,
                              __bf16* __restrict__ Xlo, int64_t ldx) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * c) return;
  const int j = (int)(idx / n);
  const int64_t i = idx - (int64_t)j * n;          // consecutive threads: consecutive i
  const float x = (float)(X[i * c + j] * (scale ? (double)scale[i] : 1.0));
  split_hilo(x, Xhi + (int64_t)j * ldx + i, Xlo + (int64_t)j * ldx + i);
}

// Z (n x c, FP64, ld c) rows scaled: Z_i *= s_i.
__global__ void k_scale_rows(double* __restrict__ Z, int64_t n, int c,
                             const float* __restrict__ scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * c) return;
  Z[idx] *= (double)scale[idx / c];
}

// ---------------------------------------------------------------------------
// Y (m x c, FP32) = Aq (m x n, bf16) (Xhi + Xlo)^T, X* c x n: block = 64
// rows per wave x NT column tiles of 16, 8 waves (4 for NT > 5, whose
// registers allow one wave per SIMD); A goes straight from
// memory into the matrix-core operand registers (lane (lr, g) of a 16-row
// tile loads the 16 bytes at row lr, k = 32 st + 8 g of the chunk), two
// 32-deep steps ahead; the kBK-wide chunks of Xhi and Xlo are staged in LDS (two
// buffers) and read back as 16-byte operands.  Optionally the FP64 sum of the
// squared dequantised entries (Eq. sumeigen) per block.  Requires n % 8 == 0
// and 16-byte rows of A, Xhi, Xlo.
constexpr int kBK = 64, kBLD = kBK + 8;
template <int NT> constexpr int nt_bf16_threads() { return 512; }
// 16-row tiles per wave: 4, or 2 for panels wider than 80 columns (their
// FP32 accumulators then stay within two waves per SIMD)
template <int NT> constexpr int nt_bf16_tiles() { return NT <= 5 ? 4 : 2; }
template <int NT> constexpr int nt_bf16_rows() { return nt_bf16_threads<NT>() / 64 * 16 * nt_bf16_tiles<NT>(); }
// persistent workgroups of the NT pass: as many per CU as fit (the
// occupancy of the instantiation), on the 256 CUs
constexpr int64_t kLowpCus = 256;

template <int NT, int ES>
__global__ __launch_bounds__(nt_bf16_threads<NT>()) void k_gemm_nt_bf16(
    const unsigned char* __restrict__ A, int64_t m, int64_t n, int64_t lda,
    const __bf16* __restrict__ Xhi, const __bf16* __restrict__ Xlo, int64_t ldx, int c,
    const float* __restrict__ scale, float* __restrict__ Y, int64_t ldy,
    double* __restrict__ fro2_part) {
  constexpr int BC = 16 * NT;
  constexpr int kBT = nt_bf16_threads<NT>(), RT = nt_bf16_tiles<NT>();
  constexpr int kBM = nt_bf16_rows<NT>();                  // rows per block: RT 16-row tiles per wave
  constexpr int XP = (2 * BC * (kBK / 8) + kBT - 1) / kBT;  // 16-byte X pieces per thread
  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][2][BC * kBLD];
  __shared__ double s2l[2][kBK];
  __shared__ double red[kBT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  const int nch = (int)((n + kBK - 1) / kBK);
  const bool do_ss = fro2_part != nullptr;
  // persistent workgroups: this one takes the kBM-row tiles blockIdx.x,
  // blockIdx.x + gridDim.x, ... as one stream of 32-deep steps, so the loads
  // run ahead across tile boundaries (no drain and refill per tile)
  const int64_t ntile = (m + kBM - 1) / kBM;
  const int nlt = (int)((ntile - blockIdx.x + gridDim.x - 1) / gridDim.x);
  auto tile_row0 = [&](int lt) { return ((int64_t)blockIdx.x + (int64_t)lt * gridDim.x) * kBM; };
  // the tile's rows; the range ends at the last element of its last row
  auto tile_rsrc = [&](int lt) {
    const int64_t r0 = tile_row0(lt);
    const int64_t rows = m - r0 < kBM ? m - r0 : kBM;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(A + r0 * lda * ES), 0,
                                             (int)(((rows - 1) * lda + n) * ES), 0x00020000);
  };
  const int xrange = (int)(((int64_t)(c - 1) * ldx + n) * 2);
  const __amdgpu_buffer_rsrc_t hr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<__bf16*>(Xhi), 0, xrange, 0x00020000);
  const __amdgpu_buffer_rsrc_t lrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<__bf16*>(Xlo), 0, xrange, 0x00020000);
  int voa[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
    voa[i] = (int)(((int64_t)(wave * 16 * RT + 16 * i + lr) * lda + 8 * g) * ES);
  // X piece p of this thread: hi/lo h, row xr, 8-column group q of the chunk
  int vox[XP];
  bool xon[XP];
#pragma unroll
  for (int u = 0; u < XP; ++u) {
    const int p = tid + kBT * u;
    const int h = p / (BC * (kBK / 8)), rem = p - h * (BC * (kBK / 8));
    const int xr = rem / (kBK / 8), q = rem - xr * (kBK / 8);
    xon[u] = p < 2 * BC * (kBK / 8);
    vox[u] = (int)(((int64_t)xr * ldx + 8 * q) * 2);
  }
  // A fragments of a 32-deep step, two register sets loaded two steps ahead
  // (set t & 1 holds step t); X pieces of the next chunk loaded at its first
  // step and stored to LDS after its second
  typedef typename Frag<ES>::raw raw_t;
  raw_t ra[2][RT];
  u32x4 rx[XP];
  auto load_a = [&](__amdgpu_buffer_rsrc_t ar, int t, raw_t (&dst)[RT]) {
#pragma unroll
    for (int i = 0; i < RT; ++i) dst[i] = Frag<ES>::load(ar, voa[i], t * 32 * ES);
  };
  auto load_x = [&](int ch) {
#pragma unroll
    for (int u = 0; u < XP; ++u) {
      const int p = tid + kBT * u;
      const bool hi = p < BC * (kBK / 8);
      rx[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                            hi ? hr : lrs, vox[u], ch * kBK * 2, 0));
    }
  };
  // X chunk ch to LDS buffer buf, zero beyond n (the pieces there hold the
  // next row); squared scales of the chunk's columns
  auto store_x = [&](int buf, int ch) {
    const int kend = (int)(n - (int64_t)ch * kBK);
#pragma unroll
    for (int u = 0; u < XP; ++u) {
      if (!xon[u]) continue;
      const int p = tid + kBT * u;
      const int h = p / (BC * (kBK / 8)), rem = p - h * (BC * (kBK / 8));
      const int xr = rem / (kBK / 8), q = rem - xr * (kBK / 8);
      const u32x4 v = 8 * q < kend ? rx[u] : u32x4{0u, 0u, 0u, 0u};
      *reinterpret_cast<u32x4*>(&Xs[buf][h][xr * kBLD + 8 * q]) = v;
    }
    if (do_ss && tid < kBK) {
      const int64_t col = (int64_t)ch * kBK + tid;
      const double s = (col < n && scale) ? (double)scale[col] : 1.0;
      s2l[buf][tid] = s * s;
    }
  };
  f32x4 acc[RT][NT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  double ss = 0.0;
  // 32-deep steps per tile, rounded up to whole chunks (two steps each): a
  // step past n multiplies zeros (its A fragments are zeroed below, its X
  // columns are zero in LDS), so the register set of global step gs is gs & 1
  // and the LDS buffer of global chunk gs >> 1 is its parity
  const int nst = 2 * nch;
  const int nsteps = nlt * nst;
  load_x(0);
  load_a(tile_rsrc(0), 0, ra[0]);
  load_a(tile_rsrc(0), 1, ra[1]);
  store_x(0, 0);
  __syncthreads();
  // global step gs with register set ST = gs & 1 (a compile-time index)
  auto step = [&](int gs, auto stc) {
    constexpr int st = decltype(stc)::value;
    const int lt = gs / nst, t = gs - lt * nst;
    const int ch = t >> 1, buf = (gs >> 1) & 1;
    const bool more_x = (gs >> 1) + 1 < nsteps / 2;   // a next chunk (maybe the next tile's)
    const int nxt_ch = ch + 1 < nch ? ch + 1 : 0;
    u32x4 a[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) a[i] = Frag<ES>::bf(ra[st][i]);
    if (st == 0 && more_x) load_x(nxt_ch);
    // refill this set with global step gs + 2, which may open the next tile
    // (the last prefetches are harmless repeats)
    {
      const int g2 = gs + 2 < nsteps ? gs + 2 : gs;
      const int lt2 = g2 / nst;
      load_a(tile_rsrc(lt2), g2 - lt2 * nst, ra[st]);
    }
    __builtin_amdgcn_sched_barrier(0);
    // a step that runs past n holds the next row's values there
    if (32 * t + 8 * g >= n) {
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = u32x4{0u, 0u, 0u, 0u};
    }
    if constexpr (NT <= 5) {
      bf16x8 bh[NT], bl[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        bh[j] = *reinterpret_cast<const bf16x8*>(&Xs[buf][0][(16 * j + lr) * kBLD + 32 * st + 8 * g]);
        bl[j] = *reinterpret_cast<const bf16x8*>(&Xs[buf][1][(16 * j + lr) * kBLD + 32 * st + 8 * g]);
      }
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          acc[i][j] = mfma_bf16(as_bf16x8(a[i]), bh[j], acc[i][j]);
          acc[i][j] = mfma_bf16(as_bf16x8(a[i]), bl[j], acc[i][j]);
        }
    } else {
      // wide panels: one column tile's hi and lo fragments live at a time
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Xs[buf][0][(16 * j + lr) * kBLD + 32 * st + 8 * g]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Xs[buf][1][(16 * j + lr) * kBLD + 32 * st + 8 * g]);
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          acc[i][j] = mfma_bf16(as_bf16x8(a[i]), bh, acc[i][j]);
          acc[i][j] = mfma_bf16(as_bf16x8(a[i]), bl, acc[i][j]);
        }
      }
    }
    if (do_ss) {
      // column 32 st + 8 g + e of the chunk, four rows per value
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float v2 = 0.f;
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const float v = (float)as_bf16x8(a[i])[e];
          v2 = fmaf(v, v, v2);
        }
        ss = fma((double)v2, s2l[buf][32 * st + 8 * g + e], ss);
      }
    }
    if (st == 1) {
      // end of the chunk: the next one's X goes to the other buffer
      if (more_x) store_x(buf ^ 1, nxt_ch);
      __syncthreads();
      if (t == nst - 1) {
        // end of the tile: its outputs, and fresh accumulators
        const int64_t row0 = tile_row0(lt);
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int col = 16 * j + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int64_t row = row0 + wave * 16 * RT + 16 * i + 4 * g + e;
              if (row < m && col < c) Y[row * ldy + col] = acc[i][j][e];
            }
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
      }
    }
  };
  for (int gs = 0; gs < nsteps; gs += 2) {
    step(gs, std::integral_constant<int, 0>());
    step(gs + 1, std::integral_constant<int, 1>());
  }
  if (do_ss) {
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < kBT / 64; ++w) t += red[w];
      fro2_part[blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Z partials (FP64, one n x c slab per row split) of Aq^T Q: block = one row
// split x 512 / QS columns of A, 8 waves; wave w takes the 64 A columns of
// group w % (8 / QS) (4 x NTW tiles of 16 x 16, NTW = ceil(NT / QS)) against
// the Q column tiles [NTW (w / (8 / QS)), +NTW).  QS = 2 for NT > 8: two
// waves then share each 64-column group of A and split Q's tiles, so a
// wave's accumulators stay within two waves per SIMD.  Chunks of 32 rows
// (one 32-deep matrix-core step): lane l = 16 g + 8 h + o loads row 8 g + o
// of the chunk, columns 16 i + 8 h .. +7 of its wave's group, and the octet
// transpose turns that into the operand the matrix core takes (column
// 8 h + o = l % 16, rows 8 g .. 8 g + 7).  Q's chunk is split into hi + lo
// bfloat16 and transposed the same way (tile j by wave j mod 8) into LDS,
// where every wave reads it.  Rows past the split read zeros (buffer range);
// columns of A past n and of Q past c only reach outputs that are not
// stored.  Block order: workgroup b runs on XCD b mod 8, and the column
// tiles of one row split are given consecutive workgroups of one XCD, so
// the Q rows that every tile of the split reads come from that XCD's L2
// after the first.  Requires 16-byte rows of A and Q (lda % 8 == 0,
// ldq % 8 == 0), n % 8 == 0, and round_up(c, 8) readable columns in every
// row of Q (ldq >= that).
constexpr int kTR = 32;
template <int NT> constexpr int tn_bf16_qs() { return NT > 8 ? 2 : 1; }
// chunks in flight (register sets, and LDS buffers of Q): three where the
// accumulators leave room for a third set within two waves per SIMD
template <int NT, int QS> constexpr int tn_bf16_depth() { return (NT <= 6 || QS == 2) ? 3 : 2; }

template <int NT, int ES, int QS>
__global__ __launch_bounds__(512) void k_gemm_tn_bf16(
    const unsigned char* __restrict__ A, int64_t m, int64_t n, int64_t lda, const float* __restrict__ Q,
    int64_t ldq, int c, double* __restrict__ P, int64_t rows_per_split, int nsplit, int ntile) {
  constexpr int GW = 8 / QS;                  // 64-column groups of A per block
  constexpr int TA = 64 * GW;                 // A columns per block
  constexpr int NTW = (NT + QS - 1) / QS;     // Q tiles per wave
  constexpr int QPW = (NT + 7) / 8;           // Q tiles staged per wave
  constexpr int D = tn_bf16_depth<NT, QS>();
  __shared__ __attribute__((aligned(16))) u32x4 Bq[D][NT][2][64];   // [buf][j][hi/lo][lane]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int o = lane & 7, h = (lane >> 3) & 1, g = lane >> 4;
  const int xcd = blockIdx.x & 7, rr = blockIdx.x >> 3;
  const int tile = rr % ntile;
  const int64_t split = (int64_t)(rr / ntile) * 8 + xcd;
  if (split >= nsplit) return;                // padding of the XCD order (whole block)
  const int ag = wave % GW, j0 = (wave / GW) * NTW;
  const int64_t rs = split * rows_per_split;
  const int64_t re = rs + rows_per_split < m ? rs + rows_per_split : m;
  const int64_t col0 = (int64_t)tile * TA + ag * 64;
  const int nchunk = (int)((re - rs + kTR - 1) / kTR);
  const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(A + rs * lda * ES), 0, (int)(((re - rs - 1) * lda + n) * ES),
      0x00020000);
  const int cpad = (c + 7) & ~7;              // Q rows hold cpad readable columns
  const __amdgpu_buffer_rsrc_t qr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(Q + rs * ldq), 0, (int)(((re - rs - 1) * ldq + cpad) * 4), 0x00020000);
  // A: row 8 g + o of the chunk, columns col0 + 16 i + 8 h; clamped inside
  // the row range of the descriptor when the tile runs past n (those
  // columns' outputs are dropped)
  int voa[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int64_t cc = col0 + 16 * i + 8 * h;
    if (cc > n - 8) cc = n - 8;
    voa[i] = (int)(((int64_t)(8 * g + o) * lda + cc) * ES);
  }
  // Q tile wave + 8 t (t < QPW, below NT): row 8 g + o, columns 16 j + 8 h
  // .. +7, clamped to the readable width (the columns past c only reach
  // dropped outputs)
  int voq[QPW];
  bool qon[QPW];
#pragma unroll
  for (int t = 0; t < QPW; ++t) {
    const int jq = wave + 8 * t;
    qon[t] = jq < NT;
    const int qc = 16 * jq + 8 * h < cpad - 8 ? 16 * jq + 8 * h : cpad - 8;
    voq[t] = (int)(((int64_t)(8 * g + o) * ldq + qc) * 4);
  }
  // D register sets, chunk ch in set ch % D, loaded D chunks ahead
  typedef typename Frag<ES>::raw raw_t;
  raw_t ra[D][4];
  f32x4 rq[D][QPW][2];
  auto load = [&](int ch, raw_t (&da)[4], f32x4 (&dq)[QPW][2]) {
    const int soa = ch * kTR * (int)lda * ES;
#pragma unroll
    for (int i = 0; i < 4; ++i) da[i] = Frag<ES>::load(ar, voa[i], soa);
    const int soq = ch * kTR * (int)ldq * 4;
#pragma unroll
    for (int t = 0; t < QPW; ++t) {
      if (qon[t]) {
        dq[t][0] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(qr, voq[t], soq, 0));
        dq[t][1] =
            __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(qr, voq[t] + 16, soq, 0));
      }
    }
  };
  auto store_q = [&](int buf, const f32x4 (&q)[QPW][2]) {
#pragma unroll
    for (int t = 0; t < QPW; ++t) {
      if (!qon[t]) continue;
      bf16x8 hi, lo;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        __bf16 a, b;
        split_hilo(q[t][0][e], &a, &b);
        hi[e] = a; lo[e] = b;
        split_hilo(q[t][1][e], &a, &b);
        hi[4 + e] = a; lo[4 + e] = b;
      }
      Bq[buf][wave + 8 * t][0][lane] = octet_transpose(as_u32x4(hi), o);
      Bq[buf][wave + 8 * t][1][lane] = octet_transpose(as_u32x4(lo), o);
    }
  };
  f32x4 acc[4][NTW];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d < D; ++d) load(d < nchunk ? d : 0, ra[d], rq[d]);
  store_q(0, rq[0]);
  __syncthreads();
  // chunk ch with register set SET = ch % D (a compile-time index); its Q
  // fragments are in LDS buffer SET, the next chunk's go to the next buffer
  auto chunk = [&](int ch, auto setc) {
    constexpr int set = decltype(setc)::value;
    constexpr int nxt = (set + 1) % D;
    u32x4 a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = octet_transpose(Frag<ES>::bf(ra[set][i]), o);
    // refill this set with chunk ch + D (the last prefetches are harmless repeats)
    const int chd = ch + D < nchunk ? ch + D : ch;
    load(chd, ra[set], rq[set]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int jj = 0; jj < NTW; ++jj) {
      const int j = j0 + jj;
      if (NT % QS != 0 && j >= NT) continue;  // uniform per wave
      const bf16x8 bh = as_bf16x8(Bq[set][j][0][lane]);
      const bf16x8 bl = as_bf16x8(Bq[set][j][1][lane]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i][jj] = mfma_bf16(as_bf16x8(a[i]), bh, acc[i][jj]);
        acc[i][jj] = mfma_bf16(as_bf16x8(a[i]), bl, acc[i][jj]);
      }
    }
    if (ch + 1 < nchunk) store_q(nxt, rq[nxt]);
    __syncthreads();
  };
  for (int ch = 0; ch < nchunk; ch += D) {
    chunk(ch, std::integral_constant<int, 0>());
    if (ch + 1 < nchunk) chunk(ch + 1, std::integral_constant<int, 1>());
    if constexpr (D > 2)
      if (ch + 2 < nchunk) chunk(ch + 2, std::integral_constant<int, 2 % D>());
  }
  // acc[i][jj][e]: A column col0 + 16 i + 4 g + e, Q column 16 (j0 + jj) + (lane % 16)
  double* Pb = P + split * n * c;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < NTW; ++jj) {
      const int qcol = 16 * (j0 + jj) + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t acol = col0 + 16 * i + 4 * g + e;
        if (acol < n && qcol < c) Pb[acol * c + qcol] = (double)acc[i][jj][e];
      }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_quantize_bf16(const float* A, int64_t m, int64_t n, int64_t lda, __bf16* Aq,
                                int64_t ldq, float* scale, unsigned* cmax, hipStream_t s) {
  if (m < 1 || n < 1) return hipErrorInvalidValue;
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(cmax), n, 0, s);
  if (e != hipSuccess) return e;
  const int64_t rpb = 256;
  hipLaunchKernelGGL(k_colmax_abs, dim3((unsigned)((m + rpb - 1) / rpb)), dim3(256), 0, s, A, m, n,
                     lda, rpb, cmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_quantize_bf16, dim3(nblocks(m * n, 256)), dim3(256), 0, s, A, m, n, lda,
                     cmax, Aq, ldq, scale);
  return hipGetLastError();
}

hipError_t launch_cast_hilo_t(const double* X, int64_t n, int c, const float* scale, __bf16* Xhi,
                              __bf16* Xlo, int64_t ldx, hipStream_t s) {
  if (n * c <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_hilo_t, dim3(nblocks(n * c, 256)), dim3(256), 0, s, X, n, c, scale,
                     Xhi, Xlo, ldx);
  return hipGetLastError();
}

hipError_t launch_scale_rows(double* Z, int64_t n, int c, const float* scale, hipStream_t s) {
  if (!scale || n * c <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_rows, dim3(nblocks(n * c, 256)), dim3(256), 0, s, Z, n, c, scale);
  return hipGetLastError();
}

bool bf16_pass_applies(const void* A, int es, int64_t n, int64_t lda, int c) {
  return (es == 1 || es == 2) && c >= 1 && c <= 192 && n % 8 == 0 && lda % 8 == 0 &&
         (reinterpret_cast<uintptr_t>(A) % (8 * es)) == 0 && (int64_t)512 * lda * es < (1LL << 31);
}

// resident workgroups per CU of a kernel (at least one)
int lowp_blocks_per_cu(const void* fn, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

template <int ES>
hipError_t nt_lowp(const void* A, int64_t m, int64_t n, int64_t lda, const __bf16* Xhi,
                   const __bf16* Xlo, int64_t ldx, int c, const float* scale, float* Y,
                   int64_t ldy, double* fro2_part, int* nparts, hipStream_t s) {
  const unsigned char* Ab = static_cast<const unsigned char*>(A);
#define RSVD_NT_BF16(NT)                                                                        \
  case NT: {                                                                                    \
    constexpr int bt = nt_bf16_threads<NT>(), br = nt_bf16_rows<NT>();                          \
    static const int per_cu = lowp_blocks_per_cu((const void*)k_gemm_nt_bf16<NT, ES>, bt);     \
    const int64_t ntl = (m + br - 1) / br;                                                      \
    const int64_t nblk = ntl < kLowpCus * per_cu ? ntl : kLowpCus * per_cu;                     \
    if (nparts) *nparts = (int)nblk;                                                            \
    hipLaunchKernelGGL((k_gemm_nt_bf16<NT, ES>), dim3((unsigned)nblk), dim3(bt), 0, s, Ab, m,   \
                       n, lda, Xhi, Xlo, ldx, c, scale, Y, ldy, fro2_part);                     \
    break;                                                                                      \
  }
  switch ((c + 15) / 16) {
    RSVD_NT_BF16(1) RSVD_NT_BF16(2) RSVD_NT_BF16(3) RSVD_NT_BF16(4)
    RSVD_NT_BF16(5) RSVD_NT_BF16(6) RSVD_NT_BF16(7) RSVD_NT_BF16(8)
    RSVD_NT_BF16(9) RSVD_NT_BF16(10) RSVD_NT_BF16(11) RSVD_NT_BF16(12)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_NT_BF16
  return hipGetLastError();
}

hipError_t launch_gemm_nt_bf16(const void* A, int es, int64_t m, int64_t n, int64_t lda,
                               const __bf16* Xhi, const __bf16* Xlo, int64_t ldx, int c,
                               const float* scale, float* Y, int64_t ldy, double* fro2_part,
                               int* nparts, hipStream_t s) {
  if (!bf16_pass_applies(A, es, n, lda, c) || ldx % 8 != 0 || (int64_t)c * ldx * 2 >= (1LL << 31))
    return hipErrorInvalidValue;
  if (m <= 0) {
    if (nparts) *nparts = 0;
    return hipSuccess;
  }
  return es == 1 ? nt_lowp<1>(A, m, n, lda, Xhi, Xlo, ldx, c, scale, Y, ldy, fro2_part, nparts, s)
                 : nt_lowp<2>(A, m, n, lda, Xhi, Xlo, ldx, c, scale, Y, ldy, fro2_part, nparts, s);
}

template <int ES>
hipError_t tn_lowp(const void* A, int64_t m, int64_t n, int64_t lda, const float* Q, int64_t ldq,
                   int c, double* P, int64_t rps, int ns, int ntile, hipStream_t s) {
  const unsigned char* Ab = static_cast<const unsigned char*>(A);
  const int nsp = (ns + 7) / 8 * 8;           // splits padded to the 8 XCDs
  const dim3 grid((unsigned)(nsp * ntile)), block(512);
#define RSVD_TN_BF16(NT)                                                                        \
  case NT:                                                                                      \
    hipLaunchKernelGGL((k_gemm_tn_bf16<NT, ES, tn_bf16_qs<NT>()>), grid, block, 0, s, Ab, m, n, \
                       lda, Q, ldq, c, P, rps, ns, ntile);                                      \
    break;
  switch ((c + 15) / 16) {
    RSVD_TN_BF16(1) RSVD_TN_BF16(2) RSVD_TN_BF16(3) RSVD_TN_BF16(4)
    RSVD_TN_BF16(5) RSVD_TN_BF16(6) RSVD_TN_BF16(7) RSVD_TN_BF16(8)
    RSVD_TN_BF16(9) RSVD_TN_BF16(10) RSVD_TN_BF16(11) RSVD_TN_BF16(12)
    default: return hipErrorInvalidValue;
  }
#undef RSVD_TN_BF16
  return hipGetLastError();
}

hipError_t launch_gemm_tn_bf16(const void* A, int es, int64_t m, int64_t n, int64_t lda,
                               const float* Q, int64_t ldq, int c, double* P, int64_t max_split,
                               int* nsplit, hipStream_t s) {
  if (!bf16_pass_applies(A, es, n, lda, c) || ldq % 8 != 0 || ldq < ((c + 7) & ~7) ||
      (reinterpret_cast<uintptr_t>(Q) % 16) != 0 || m <= 0)
    return hipErrorInvalidValue;
  const int ta = (c + 15) / 16 > 8 ? 256 : 512;   // A columns per block (QS = 2 / 1)
  const int ntile = (int)((n + ta - 1) / ta);
  int64_t ns = 256 / ntile;
  if (ns < 1) ns = 1;
  if (ns > (m + kTR - 1) / kTR) ns = (m + kTR - 1) / kTR;
  if (ns > max_split) ns = max_split;
  int64_t rps = (m + ns - 1) / ns;
  rps = (rps + kTR - 1) / kTR * kTR;
  ns = (m + rps - 1) / rps;
  const int64_t ld = lda * es > ldq * 4 ? lda * es : ldq * 4;
  if ((rps + kTR) * ld >= (1LL << 31)) return hipErrorInvalidValue;
  *nsplit = (int)ns;
  return es == 1 ? tn_lowp<1>(A, m, n, lda, Q, ldq, c, P, rps, (int)ns, ntile, s)
                 : tn_lowp<2>(A, m, n, lda, Q, ldq, c, P, rps, (int)ns, ntile, s);
}

hipError_t launch_quantize_fp8(const float* A, int64_t m, int64_t n, int64_t lda, void* Aq,
                               int64_t ldq, float* scale, unsigned* cmax, hipStream_t s) {
  if (m < 1 || n < 1) return hipErrorInvalidValue;
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(cmax), n, 0, s);
  if (e != hipSuccess) return e;
  const int64_t rpb = 256;
  hipLaunchKernelGGL(k_colmax_abs, dim3((unsigned)((m + rpb - 1) / rpb)), dim3(256), 0, s, A, m, n,
                     lda, rpb, cmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_quantize_fp8, dim3(nblocks(m * n, 256)), dim3(256), 0, s, A, m, n, lda,
                     cmax, static_cast<unsigned char*>(Aq), ldq, scale);
  return hipGetLastError();
}

// A32 (m x n, ld lda32) = Aq diag(scale) (Aq bfloat16 or FP8 E4M3, one
// thread per 8 consecutive elements of a row, widened as in the passes).
template <int ES>
__global__ void k_dequantize(const unsigned char* __restrict__ Aq, int64_t m, int64_t n,
                             int64_t lda, const float* __restrict__ scale, float* __restrict__ A32,
                             int64_t lda32) {
  const int64_t g8 = (n + 7) / 8;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * g8) return;
  const int64_t i = idx / g8, j0 = 8 * (idx - i * g8);
  const unsigned char* row = Aq + i * lda * ES;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t j = j0 + e;
    if (j >= n) break;
    float v;
    if (ES == 2) {
      v = (float)reinterpret_cast<const __bf16*>(row)[j];
    } else {
      const int byte = row[j];
      v = __builtin_amdgcn_cvt_pk_f32_fp8(byte, false)[0];
    }
    A32[i * lda32 + j] = scale ? v * scale[j] : v;
  }
}

hipError_t launch_dequantize(const void* Aq, int es, int64_t m, int64_t n, int64_t lda,
                             const float* scale, float* A32, int64_t lda32, hipStream_t s) {
  if (m < 1 || n < 1) return hipSuccess;
  const int64_t total = m * ((n + 7) / 8);
  const unsigned char* Ab = static_cast<const unsigned char*>(Aq);
  if (es == 2)
    hipLaunchKernelGGL((k_dequantize<2>), dim3(nblocks(total, 256)), dim3(256), 0, s, Ab, m, n,
                       lda, scale, A32, lda32);
  else if (es == 1)
    hipLaunchKernelGGL((k_dequantize<1>), dim3(nblocks(total, 256)), dim3(256), 0, s, Ab, m, n,
                       lda, scale, A32, lda32);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace rsvd
