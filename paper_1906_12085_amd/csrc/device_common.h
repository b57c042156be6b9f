// device_common.h -- device helpers shared by the FP64 kernels of librsvd:
// status words, LDS staging, the round-robin pairing and rotation of the
// Jacobi methods, cross-lane sums, and bounded inter-workgroup waits.
#pragma once

#include <math.h>

#include "rsvd_internal.h"

namespace rsvd {
namespace {

constexpr double kEps = 2.220446049250313e-16;

// Errors win over warnings; among errors the most negative code wins.
__device__ __forceinline__ void set_error(int32_t* status, int32_t code) { atomicMin(status, code); }
__device__ __forceinline__ void set_warning(int32_t* status, int32_t code) { atomicCAS(status, 0, code); }

// Copy `count` doubles from global memory into LDS with the whole block; each
// thread issues eight independent loads before its eight LDS stores, so the
// memory latency is paid once per eight elements rather than per element.
__device__ __forceinline__ void stage_to_lds(double* dst, const double* __restrict__ src,
                                             int count) {
  const int step = blockDim.x;
  int i = threadIdx.x;
  for (; i + 7 * step < count; i += 8 * step) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[i + u * step];
#pragma unroll
    for (int u = 0; u < 8; ++u) dst[i + u * step] = v[u];
  }
  for (; i < count; i += step) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Round-robin ("circle") pairing of npad (even) indices: in step s, pair 0 is
// (npad-1, s) and pair k > 0 is ((s+k) mod (npad-1), (s-k) mod (npad-1)); the
// npad-1 steps meet every pair exactly once, and the pairs of one step are
// disjoint, so their rotations commute.
__device__ __forceinline__ void rr_pair(int s, int k, int npad, int* p, int* q) {
  // s < h and k <= h / 2, so one conditional step reduces each index mod h
  int a, b;
  const int h = npad - 1;
  if (k == 0) { a = h; b = s; }
  else {
    a = s + k;
    a = a >= h ? a - h : a;
    b = s - k;
    b = b < 0 ? b + h : b;
  }
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

// Newton steps for the hardware reciprocal and reciprocal-square-root
// estimates (each step doubles the number of correct bits).
__device__ __forceinline__ double rcp_step(double x, double r) { return fma(r, fma(-x, r, 1.0), r); }
__device__ __forceinline__ double rsq_step(double x, double y) {
  return fma(y, fma(-0.5 * x * y, y, 0.5), y);
}

// A pair of columns with alpha = |x_p|^2, beta = |x_q|^2, gamma = x_p.x_q is
// rotated when the cosine of their angle exceeds tol (gamma^2 > tol^2 alpha
// beta) and gamma^2 exceeds floor2 max(alpha, beta).  With floor2 =
// (eps |G|_F)^2 the second test leaves alone a coupling at the rounding level
// of the input G (entries carry errors of order eps |G|_F, so the inner
// product of a column of norm |x| with any other carries eps |G|_F |x|); in
// particular two columns both below that noise level are never rotated
// against each other.  floor2 = 0: every nonzero coupling past tol.
__device__ __forceinline__ bool rot_needed(double al, double be, double ga, double tol2,
                                           double floor2) {
  return ga * ga > floor2 * fmax(al, be) && ga * ga > tol2 * (al * be);
}

// The rotation (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q) that makes the
// pair orthogonal.  With zeta = (beta - alpha) / (2 gamma) the tangent is the
// root of t^2 + 2 zeta t - 1 = 0 of smaller magnitude, t = sign(zeta) / den
// with den = |zeta| + sqrt(1 + zeta^2); then c = den / sqrt(den^2 + 1) and
// s = sign(zeta) / sqrt(den^2 + 1), so c and s share one reciprocal square
// root (two Newton steps: c^2 + s^2 = 1 to rounding) while zeta and den need
// only one step each (they decide how far the pair turns, not the
// orthogonality of the rotation).  Branch-free: need = false gives the
// identity (c = 1, s = t = 0), so the two rotations a thread needs per round
// are computed side by side.
__device__ __forceinline__ void rot_cst(double al, double be, double ga, bool need, double* c,
                                        double* s, double* t) {
  const double g = need ? ga : 1.0;
  const double d = need ? be - al : 0.0;
  const double zeta = 0.5 * d * rcp_step(g, __builtin_amdgcn_rcp(g));
  const double az = fmin(fabs(zeta), 1e150);
  const double w = fma(az, az, 1.0);
  const double den = fma(w, rsq_step(w, __builtin_amdgcn_rsq(w)), az);
  const double v = fma(den, den, 1.0);
  double q = __builtin_amdgcn_rsq(v);
  q = rsq_step(v, rsq_step(v, q));
  double ti = __builtin_amdgcn_rcp(den);
  ti = rcp_step(den, rcp_step(den, ti));
  const double sg = zeta >= 0.0 ? 1.0 : -1.0;
  *c = need ? den * q : 1.0;
  *s = need ? sg * q : 0.0;
  *t = need ? sg * ti : 0.0;
}

// Sum over the G consecutive lanes of this lane's group (G = 8, 16, 32 or
// 64, groups aligned to G).  Within a 16-lane row: quad_perm swaps (lanes
// l^1, l^2) and row rotations by 4 and 8 (DPP), then every lane takes lane
// (l & 16)'s value (ds_swizzle) so all lanes of the row hold the same bits;
// larger groups add the partner row / half-wave symmetrically.  G = 8: the
// two quad sums of the half-row are exchanged by row_half_mirror (lane i
// reads lane 7 - i), and since x + y == y + x exactly, every lane of the
// group holds the same bits without a broadcast.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int PAT>
__device__ __forceinline__ double swizzle(double v) {
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), PAT);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), PAT);
  return __hiloint2double(hi, lo);
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(G == 8 || G == 16 || G == 32 || G == 64, "group of 8, 16, 32 or 64 lanes");
  v += dpp_mov<0xB1>(v);    // quad_perm(1,0,3,2)
  v += dpp_mov<0x4E>(v);    // quad_perm(2,3,0,1): quad sum
  if (G == 8) return v + dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x124>(v);   // row_ror:4
  v += dpp_mov<0x128>(v);   // row_ror:8: row sum (association differs by quad)
  v = swizzle<0x0010>(v);   // broadcast lane (l & 16): identical bits in the row
  if (G >= 32) v += swizzle<0x401F>(v);   // xor 16
  if (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

// ---------------------------------------------------------------------------
// Waits between workgroups of one cooperative launch.  Spins are bounded:
// on timeout (or when another workgroup already gave up) the abort flag is
// raised and the wait reports failure, so that every workgroup leaves.
constexpr long kSpinLimit = 1L << 22;

// Thread 0 only: spin until *word >= target (agent scope, relaxed loads).
__device__ __forceinline__ bool spin_geq(int32_t* word, int target, int32_t* abort_flag) {
  long spins = 0;
  while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
        ++spins > kSpinLimit) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Agent-scope release / acquire fences (one direction each: the release
// writes back this XCD's L2, the acquire invalidates it).
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Loads and stores of data handed between workgroups: agent-scope relaxed
// atomics, i.e. accesses made at the agent's coherence point, so the release
// fence that publishes them finds little to write back.
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// All threads of the block call this.  The block's global writes are
// published (workgroup barrier, then a release fence by thread 0) before
// *counter is incremented; thread 0 then waits for *counter >= target and
// acquires, so the block sees the writes of everyone it waited for.
__device__ __forceinline__ bool arrive_and_wait(int32_t* counter, int target, int32_t* abort_flag) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    fence_release();
    __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = spin_geq(counter, target, abort_flag) ? 1 : 0;
    fence_acquire();
  }
  __syncthreads();
  return ok != 0;
}

}  // namespace
}  // namespace rsvd
