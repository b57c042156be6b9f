// eig.hip -- the symmetric eigensolver of the A^T A route (Sec. 2.3 and
// 3.1.3): the n x n Gram matrix G is diagonalised by one-sided block Jacobi.
//
// Method.  X starts as G and J as I.  The n columns are cut into blocks of
// kB; in each step of a sweep the blocks are paired by the round-robin
// ordering (every pair of blocks meets once per sweep, the pairs of one step
// are disjoint).  For a block pair with the kW = 2 kB columns X_W:
//   M = X_W^T X_W                (kW x kW Gram of the columns),
//   R = accumulated rotations of a Jacobi sweep on M (R^T M R -> diagonal),
//   X_W <- X_W R,  J_W <- J_W R.
// Mathematically this is the column-pair Jacobi method on X, with the
// rotations of a block pair decided on their kW x kW Gram matrix instead of
// on n-long columns.  At convergence the columns of X = G J are orthogonal,
// so J holds the eigenvectors and |x_j| = |lambda_j|.
//
// GPU layout.  Each block pair is shared by P workgroups, one per slice of
// rows: a workgroup stages its slice of X_W and J_W in LDS, forms the
// slice's partial Gram on the FP64 matrix cores, and, once the P partials of
// its pair are in (an arrival counter per pair), sums them in a fixed order,
// solves the kW x kW problem itself (all P workgroups of a pair compute the
// same R from the same data), and applies R to its slice.  A step of one
// workgroup needs only the rows it owns from the two workgroups that held
// those blocks in the previous step, so steps are chained by per-workgroup
// step counters instead of a grid barrier; a grid barrier closes each sweep
// (the convergence decision).  All waits are bounded spins (abort flag).
#include "device_common.h"

namespace rsvd {

namespace {

constexpr int kB = 16;                        // columns per block
constexpr int kW = 2 * kB;                    // columns of a block pair
constexpr int kLdM = kW + 1;                  // LDS row stride of the kW x kW matrices
constexpr int kThreads = 256;                 // 16 x 16 threads: one 2 x 2 block of M each
constexpr int kMaxSweeps = 40;
constexpr int kDefaultInner = 1;              // inner sweeps per step
constexpr int kMaxN = 1024;
constexpr int kMaxPairs = kMaxN / kW;
constexpr int kMaxGroups = 256;
constexpr int kMaxSlices = 8;                 // row slices per block pair

// flag words: grid-barrier counter, abort flag, per-sweep count of block
// pairs found unconverged, per-pair arrival counters, per-workgroup step
// counters for X and for J
constexpr int kFlagBar = 0;
constexpr int kFlagAbort = 1;
constexpr int kFlagRot = 2;
constexpr int kFlagPair = kFlagRot + kMaxSweeps;
constexpr int kFlagDone = kFlagPair + kMaxPairs;      // steps whose X rows are out
constexpr int kFlagDoneJ = kFlagDone + kMaxGroups;    // steps whose J rows are out
constexpr int kFlagWords = kFlagDoneJ + kMaxGroups;

// Launch geometry for n: block pairs, rows per slice (16 * rpt), slices per pair.
struct Geom {
  int nbp, rpt, P, nwg;
};
Geom geom(int n) {
  Geom g;
  const int nb = (n + kB - 1) / kB;
  g.nbp = nb + (nb & 1) < 2 ? 2 : nb + (nb & 1);
  // at most 4 slices up to n = 512; 256-row slices past it (4 at n = 1024:
  // fewer partial Gram matrices per pair, half the CUs)
  g.rpt = n <= 128 ? 2 : (n <= 256 ? 4 : (n <= 512 ? 8 : 16));
  const int rs = 16 * g.rpt;
  g.P = (n + rs - 1) / rs;
  g.nwg = (g.nbp / 2) * g.P;
  return g;
}

// Index of the pair that holds block blk in step s of the rr_pair ordering
// of npad blocks (the inverse of rr_pair).
__device__ __forceinline__ int rr_pair_of(int blk, int s, int npad) {
  const int h = npad - 1;
  if (blk == h || blk == s) return 0;
  const int d = (blk - s + h) % h;
  return d <= (h - 1) / 2 ? d : h - d;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = group_sum<64>(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

template <int RPT>
__global__ __launch_bounds__(kThreads) void k_jacobi_eig(
    double* __restrict__ X, double* __restrict__ J, int n, int nbp, int P, int inner_max,
    double* __restrict__ Mpart, double* __restrict__ fro_part, double* __restrict__ lam,
    double* __restrict__ diag, int32_t* __restrict__ flags, int32_t* __restrict__ status,
    int svd) {
  constexpr int RS = 16 * RPT;                 // rows per slice
  constexpr int LDX = RS + 1;
  extern __shared__ double sm[];
  double* Xs = sm;                             // column c of the slice at Xs + c * LDX
  double* Js = Xs + kW * LDX;
  double* Mb = Js + kW * LDX;                  // two kW x kW buffers (row stride kLdM)
  double* Rl = Mb + 2 * kW * kLdM;             // accumulated rotation R
  __shared__ double red[4];
  __shared__ int sh_ok;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x, nwg = gridDim.x;
  const int k = g / P, r = g - k * P;
  const int row0 = r * RS;
  const int nrow = min(RS, n - row0);
  const int nsteps = nbp - 1;
  int32_t* abort_flag = flags + kFlagAbort;
  int bar = 0;
  bool aborted = false;

  // ||G||_F^2 (fixed summation order: per-workgroup partials, then every
  // workgroup adds them in index order)
  {
    const int64_t tot = (int64_t)n * n, chunk = (tot + nwg - 1) / nwg;
    const int64_t b0 = (int64_t)g * chunk, b1 = min(tot, b0 + chunk);
    double s2 = 0.0;
    for (int64_t e = b0 + tid; e < b1; e += kThreads) s2 += X[e] * X[e];
    s2 = block_sum(s2, red);
    if (tid == 0) st_agent(fro_part + g, s2);
    ++bar;
    if (!arrive_and_wait(flags + kFlagBar, bar * nwg, abort_flag)) aborted = true;
  }
  double fro2 = 0.0;
  for (int i = 0; i < nwg; ++i) fro2 += ld_agent(fro_part + i);
  const double tol = kEps * (double)n, tol2 = tol * tol;
  const double floor2 = svd ? 0.0 : kEps * kEps * fro2;   // (eps |G|_F)^2

  // Stage this slice of the pair's kW columns of a matrix (X or J) into LDS,
  // all loads issued before the first store.
  auto stage = [&](const double* Mg, double* Ms, int I, int Jb) {
    constexpr int PER = kW * RS / kThreads;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * kThreads, c = e / RS, i = e - c * RS;
      const int gc = c < kB ? I * kB + c : Jb * kB + (c - kB);
      v[u] = (gc < n && i < nrow) ? ld_agent(Mg + (int64_t)gc * n + row0 + i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * kThreads, c = e / RS, i = e - c * RS;
      Ms[c * LDX + i] = v[u];
    }
  };
  // Mg_W <- Mg_W R on this slice from its LDS copy Ms, formed as (R^T S^T)^T
  // so that 16 consecutive lanes store 16 consecutive rows of a column.
  auto apply = [&](const double* Ms, double* Mg, int I, int Jb) {
    for (int tile = wave; tile < 2 * RPT; tile += 4) {
      const int jt = tile & 1, rt = tile >> 1;
      const double* ap = Rl + (lane >> 4) * kLdM + jt * 16 + (lane & 15);
      const double* bp = Ms + (lane >> 4) * LDX + rt * 16 + (lane & 15);
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < kW; k0 += 4) acc = Mfma<double>::run(ap[k0 * kLdM], bp[k0 * LDX], acc);
      const int row = rt * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = jt * 16 + Mfma<double>::row(lane, e);
        const int gc = j < kB ? I * kB + j : Jb * kB + (j - kB);
        if (gc < n && row < nrow) st_agent(Mg + (int64_t)gc * n + row0 + row, acc[e]);
      }
    }
  };

  // thread roles in the inner rounds: pair a of rows, pair bq of columns
  const int a = tid >> 4, bq = tid & 15;
  int sweep = 0;
  bool converged = false;
  int gs = 0;                                  // steps done by this workgroup
  while (!aborted && sweep < kMaxSweeps) {
    int unconv = 0;
    for (int s = 0; s < nsteps; ++s, ++gs) {
      int I, Jb;
      rr_pair(s, k, nbp, &I, &Jb);
      if (gs > 0) {
        // the workgroups that held these rows of blocks I and Jb last step
        const int sp = (s == 0) ? nsteps - 1 : s - 1;
        const int g1 = rr_pair_of(I, sp, nbp) * P + r;
        const int g2 = rr_pair_of(Jb, sp, nbp) * P + r;
        if (tid == 0) {
          const bool ok = spin_geq(flags + kFlagDone + g1, gs, abort_flag) &&
                          spin_geq(flags + kFlagDone + g2, gs, abort_flag);
          fence_acquire();
          sh_ok = ok ? 1 : 0;
        }
        __syncthreads();
        if (!sh_ok) { aborted = true; break; }
      }
      // stage this slice of the pair's columns of X
      stage(X, Xs, I, Jb);
      __syncthreads();
      // partial Gram of the slice; wave w forms the 16 x 16 tile (w >> 1, w & 1)
      {
        double* Mp = Mpart + ((int64_t)(gs & 1) * nwg + g) * (kW * kW);
        const int ti = wave >> 1, tj = wave & 1;
        const double* xa = Xs + (ti * 16 + (lane & 15)) * LDX + (lane >> 4);
        const double* xb = Xs + (tj * 16 + (lane & 15)) * LDX + (lane >> 4);
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < RS; k0 += 4) acc = Mfma<double>::run(xa[k0], xb[k0], acc);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          st_agent(Mp + (ti * 16 + Mfma<double>::row(lane, e)) * kW + tj * 16 + (lane & 15), acc[e]);
      }
      if (!arrive_and_wait(flags + kFlagPair + k, (gs + 1) * P, abort_flag)) {
        aborted = true;
        break;
      }
      // M = the pair's P partials summed in slice order; R = I.  Each thread
      // issues its 4 x P loads before the first add.
      {
        const double* base = Mpart + ((int64_t)(gs & 1) * nwg + (int64_t)k * P) * (kW * kW);
        constexpr int EPT = kW * kW / kThreads;
        double v[EPT][kMaxSlices];
#pragma unroll
        for (int u = 0; u < EPT; ++u)
#pragma unroll
          for (int rr = 0; rr < kMaxSlices; ++rr)
            v[u][rr] = rr < P ? ld_agent(base + (int64_t)rr * (kW * kW) + tid + u * kThreads) : 0.0;
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
          double acc = v[u][0];
#pragma unroll
          for (int rr = 1; rr < kMaxSlices; ++rr) acc += v[u][rr];
          const int e = tid + u * kThreads, i = e / kW, j = e - i * kW;
          Mb[i * kLdM + j] = acc;
          Rl[i * kLdM + j] = (i == j) ? 1.0 : 0.0;
        }
      }
      __syncthreads();
      int need = 0;
      for (int e = tid; e < kW * kW; e += kThreads) {
        const int i = e / kW, j = e - i * kW;
        if (i < j) need |= rot_needed(Mb[i * kLdM + i], Mb[j * kLdM + j], Mb[i * kLdM + j], tol2, floor2) ? 1 : 0;
      }
      const int nneed = __syncthreads_count(need);
      if (nneed > 0) {
        ++unconv;
        // Jacobi rounds on M; thread (a, bq) owns the 2 x 2 block (pair a of
        // rows, pair bq of columns) of M and rows 2a, 2a+1 of R's columns of
        // pair bq; M is double-buffered so that one barrier per round
        // suffices.  In the first step of a sweep (every block takes part)
        // the rounds run over all pairs of the kW columns (round-robin, kW - 1
        // rounds); in the other steps only over the kB x kB pairs across the
        // two blocks (kB rounds, round rd pairs column i of the first block
        // with column (i + rd) mod kB of the second): pairs inside a block
        // were rotated in that block's first step and are still checked by
        // the convergence test of every step.
        const bool full = (s == 0);
        const int nrounds = full ? kW - 1 : kB;
        int cur = 0;
        for (int sw = 0; sw < inner_max; ++sw) {
          int rotated = 0;
          for (int rd = 0; rd < nrounds; ++rd) {
            const double* Mc = Mb + cur * (kW * kLdM);
            double* Mn = Mb + (cur ^ 1) * (kW * kLdM);
            int pa, qa, pb, qb;
            if (full) {
              rr_pair(rd, a, kW, &pa, &qa);
              rr_pair(rd, bq, kW, &pb, &qb);
            } else {
              pa = a; qa = kB + ((a + rd) & (kB - 1));
              pb = bq; qb = kB + ((bq + rd) & (kB - 1));
            }
            double m00 = Mc[pa * kLdM + pb], m01 = Mc[pa * kLdM + qb];
            double m10 = Mc[qa * kLdM + pb], m11 = Mc[qa * kLdM + qb];
            const double aal = Mc[pa * kLdM + pa], abe = Mc[qa * kLdM + qa], aga = Mc[pa * kLdM + qa];
            const double bal = Mc[pb * kLdM + pb], bbe = Mc[qb * kLdM + qb], bga = Mc[pb * kLdM + qb];
            double* r0 = Rl + (2 * a) * kLdM;
            double* r1 = r0 + kLdM;
            const double x0 = r0[pb], x1 = r0[qb], y0 = r1[pb], y1 = r1[qb];
            const bool ra = rot_needed(aal, abe, aga, tol2, floor2);
            const bool rb = rot_needed(bal, bbe, bga, tol2, floor2);
            double ta, ca, sa, tb, cb, sb;
            rot_cst(aal, abe, aga, ra, &ca, &sa, &ta);
            rot_cst(bal, bbe, bga, rb, &cb, &sb, &tb);
            {
              // columns: M <- M R_b; rows: M <- R_a^T M (identity where not rotated)
              const double n00 = cb * m00 - sb * m01, n01 = sb * m00 + cb * m01;
              const double n10 = cb * m10 - sb * m11, n11 = sb * m10 + cb * m11;
              const double o00 = ca * n00 - sa * n10, o10 = sa * n00 + ca * n10;
              const double o01 = ca * n01 - sa * n11, o11 = sa * n01 + ca * n11;
              const bool dg = (a == bq);
              // a diagonal block: alpha' = alpha - t gamma, beta' = beta + t gamma, gamma' = 0
              m00 = dg ? fma(-ta, aga, aal) : o00;
              m11 = dg ? fma(ta, aga, abe) : o11;
              m01 = dg ? (ra ? 0.0 : m01) : o01;
              m10 = dg ? (ra ? 0.0 : m10) : o10;
              rotated |= (dg && ra) ? 1 : 0;
            }
            Mn[pa * kLdM + pb] = m00;
            Mn[pa * kLdM + qb] = m01;
            Mn[qa * kLdM + pb] = m10;
            Mn[qa * kLdM + qb] = m11;
            r0[pb] = cb * x0 - sb * x1;
            r0[qb] = sb * x0 + cb * x1;
            r1[pb] = cb * y0 - sb * y1;
            r1[qb] = sb * y0 + cb * y1;
            __syncthreads();
            cur ^= 1;
          }
          if (__syncthreads_count(rotated) == 0) break;
        }
        // X_W <- X_W R on this slice
        apply(Xs, X, I, Jb);
      }
      // publish this step's X rows: the next owners of these blocks start
      // their step on them while this workgroup turns to J
      __syncthreads();
      if (tid == 0) {
        fence_release();
        __hip_atomic_fetch_add(flags + kFlagDone + g, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // J_W <- J_W R on this slice, once the J rows of the previous step are
      // out.  The wait comes first also where nothing is rotated: this
      // step's J rows are published below, and the next owners of these
      // blocks must find the previous step's rows in place.
      if (gs > 0) {
        const int sp = (s == 0) ? nsteps - 1 : s - 1;
        const int g1 = rr_pair_of(I, sp, nbp) * P + r;
        const int g2 = rr_pair_of(Jb, sp, nbp) * P + r;
        if (tid == 0) {
          const bool ok = spin_geq(flags + kFlagDoneJ + g1, gs, abort_flag) &&
                          spin_geq(flags + kFlagDoneJ + g2, gs, abort_flag);
          fence_acquire();
          sh_ok = ok ? 1 : 0;
        }
        __syncthreads();
        if (!sh_ok) { aborted = true; break; }
      }
      if (nneed > 0) {
        stage(J, Js, I, Jb);
        __syncthreads();
        apply(Js, J, I, Jb);
      }
      __syncthreads();
      if (tid == 0) {
        fence_release();
        __hip_atomic_fetch_add(flags + kFlagDoneJ + g, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (aborted) break;
    if (r == 0 && tid == 0 && unconv > 0)
      __hip_atomic_fetch_add(flags + kFlagRot + sweep, unconv, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    ++bar;
    if (!arrive_and_wait(flags + kFlagBar, bar * nwg, abort_flag)) { aborted = true; break; }
    const int left = __hip_atomic_load(flags + kFlagRot + sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++sweep;
    if (left == 0) { converged = true; break; }
  }
  if (aborted) {
    if (g == 0 && tid == 0) set_error(status, RSVD_ERR_DEVICE);
    return;
  }
  // lambda_j = |x_j| signed by the Rayleigh quotient j_j^T x_j (unsigned for
  // the SVD); a wave per column
  for (int j = g * 4 + wave; j < n; j += nwg * 4) {
    double s2 = 0.0, rq = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double x = X[(int64_t)j * n + i];
      s2 += x * x;
      rq += J[(int64_t)j * n + i] * x;
    }
    s2 = group_sum<64>(s2);
    rq = group_sum<64>(rq);
    if (lane == 0) lam[j] = (rq < 0.0 && !svd) ? -sqrt(s2) : sqrt(s2);
  }
  if (g == 0 && tid == 0) {
    diag[2] = (double)sweep;
    if (!converged) set_error(status, RSVD_ERR_NOCONV);
  }
}

template <int RPT>
hipError_t eig_launch(double* X, double* J, int n, const Geom& G, int inner, double* lam,
                      double* diag, int32_t* flags, double* scratch, int32_t* status,
                      hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int svd) {
  const size_t shmem = ((size_t)2 * kW * (16 * RPT + 1) + (size_t)3 * kW * kLdM) * sizeof(double);
  const void* fn = (const void*)k_jacobi_eig<RPT>;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_jacobi_eig<RPT>, kThreads, shmem);
  if (e != hipSuccess) return e;
  if (G.P > kMaxSlices || G.nwg > kMaxGroups) return hipErrorInvalidValue;
  if (G.nwg > ncu * per_cu) return hipErrorCooperativeLaunchTooLarge;
  e = launch_fill_i32(flags, kFlagWords, 0, s);
  if (e != hipSuccess) return e;
  double* Mpart = scratch;
  double* fro_part = scratch + (size_t)2 * G.nwg * kW * kW;
  int nn = n, nbp = G.nbp, P = G.P, inn = inner, sv = svd;
  void* args[] = {&X,    &J,   &nn,   &nbp,    &P,      &inn, &Mpart,
                  &fro_part, &lam, &diag, &flags, &status, &sv};
  if (ev0) (void)hipEventRecord(ev0, s);
  e = hipLaunchCooperativeKernel(fn, dim3(G.nwg), dim3(kThreads), args, shmem, s);
  if (ev1) (void)hipEventRecord(ev1, s);
  return e;
}

}  // namespace

hipError_t launch_jacobi_eig(double* X, double* J, int64_t n, double* lam, double* diag,
                             int32_t* flags, double* scratch, int32_t* status, hipStream_t s,
                             int inner_sweeps, hipEvent_t ev0, hipEvent_t ev1, int svd) {
  if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
  const Geom G = geom((int)n);
  const int inner = inner_sweeps < 0 ? kDefaultInner : (inner_sweeps < 1 ? 1 : inner_sweeps);
  switch (G.rpt) {
    case 2: return eig_launch<2>(X, J, (int)n, G, inner, lam, diag, flags, scratch, status, s,
                                     ev0, ev1, svd);
    case 4: return eig_launch<4>(X, J, (int)n, G, inner, lam, diag, flags, scratch, status, s,
                                     ev0, ev1, svd);
    case 16: return eig_launch<16>(X, J, (int)n, G, inner, lam, diag, flags, scratch, status, s,
                                   ev0, ev1, svd);
    default: return eig_launch<8>(X, J, (int)n, G, inner, lam, diag, flags, scratch, status, s,
                                     ev0, ev1, svd);
  }
}

int64_t jacobi_eig_scratch_doubles(int64_t n) {
  int64_t most = 0;
  for (int m = 1; m <= (int)(n < kMaxN ? n : kMaxN); ++m) {
    const Geom G = geom(m);
    const int64_t need = (int64_t)2 * G.nwg * kW * kW + G.nwg;
    if (need > most) most = need;
  }
  return most;
}

int64_t jacobi_eig_max_n() { return kMaxN; }

int jacobi_eig_flag_words() { return kFlagWords; }

}  // namespace rsvd
