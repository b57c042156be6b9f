"""Sketches wider than 96 columns (96 < l <= 192): the l x l Cholesky factor
and its inverse in the 1024-thread kernel, the small SVD of the l x l factor
on the cooperative block-Jacobi solver (SVD form), the Gram matrices of wide
panels on the general split-m product, the fp32 passes on the general
kernels, and the bfloat16 / FP8 passes with 9 to 12 column tiles.

Everything is compared with the oracle on identical inputs, with the bounds
and tolerances of the narrower tests: per-stage c n u bounds from the same
operands, the FP64 path's sigma within 1e-10 and the FP32 / low-precision
paths' within 1e-4 (relative), largest principal angle of the top-k U and V
subspaces within 1e-3 rad, K equal.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import EPS64, U32, align_columns, announce, dev, host, rounded, sign_rule_holds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1906_12085_amd as rs  # noqa: E402

DTYPES = {"f64": torch.float64, "f32": torch.float32}
SIG_TOL = {torch.float64: 1e-10, torch.float32: 1e-4}
HILO = 2.0 ** -16
LOWP = {"bf16": torch.bfloat16, "fp8": torch.float8_e4m3fn}


def unit(dt):
    return EPS64 if dt == torch.float64 else U32


@pytest.fixture(scope="module")
def plans():
    out = {name: rs.Plan(30000, 600, 192, dt, seed=404) for name, dt in DTYPES.items()}
    yield out
    for p in out.values():
        p.close()


@pytest.fixture(scope="module", params=list(LOWP))
def lowp_plan(request):
    p = rs.Plan(30000, 1040, 192, LOWP[request.param], seed=405)
    yield p
    p.close()


def test_wide_plan_limits():
    with pytest.raises(rs.RSVDError) as e:
        rs.Plan(1000, 400, 193, torch.float32)
    assert e.value.code == rs.RSVD_ERR_SHAPE


@pytest.mark.parametrize("name", DTYPES)
# m <= 8192 takes the one-launch short Gram; longer panels the LDS-staged
# row-split kernel (c <= 112 on its 8-tile build), at 8193 just past the switch
@pytest.mark.parametrize("m,c,kappa", [(3000, 97, 1e2), (5000, 128, 1e3), (4001, 160, 1e3),
                                       (2500, 192, 10.0), (3000, 113, 1e4), (8193, 100, 1e2),
                                       (12001, 112, 1e3), (20000, 150, 1e2), (9500, 192, 1e3)])
def test_wide_cholqr2_parity(plans, name, m, c, kappa):
    dt = DTYPES[name]
    announce(f"wide cholqr2 {name} m={m} c={c} kappa={kappa}")
    rng = np.random.default_rng(m + c)
    Y0 = synth.haar(rng, m, c) @ np.diag(np.logspace(0, -np.log10(kappa), c)) @ synth.haar(rng, c, c).T
    Y0 = rounded(Y0, dt)
    Q = torch.empty(m, c, dtype=dt, device="cuda")
    R = torch.empty(c, c, dtype=torch.float64, device="cuda")
    p = plans[name]
    rs.rsvd_cholqr2(p.handle, dev(Y0, dt), Q, R)
    assert p.status() == rs.RSVD_OK
    Qg, Rg = host(Q), host(R)
    u = unit(dt)
    assert np.abs(Qg.T @ Qg - np.eye(c)).max() <= 50 * c * u
    assert np.linalg.norm(Qg @ Rg - Y0) <= 50 * c * u * np.linalg.norm(Y0)
    Qo, Ro = oracle.qr(Y0)
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0)
    assert np.abs(Rg - Ro).max() <= 50 * c * u * kappa * np.abs(Ro).max()
    assert np.abs(Qg - Qo).max() <= 50 * c * u * kappa


# (the CholeskyQR2 of T in front of the Jacobi SVD holds condition numbers
# up to about 1e7 in FP64, as for the narrower sketches)
@pytest.mark.parametrize("r,c,decades", [(300, 97, 6), (400, 160, 6), (192, 192, 3), (500, 150, 7)])
def test_wide_small_svd_parity(plans, r, c, decades):
    announce(f"wide small_svd r={r} c={c} decades={decades}")
    rng = np.random.default_rng(r * c)
    T0 = synth.haar(rng, r, c) @ np.diag(np.logspace(0, -decades, c)) @ synth.haar(rng, c, c).T
    Vt = torch.empty(r, c, dtype=torch.float64, device="cuda")
    S = torch.empty(c, dtype=torch.float64, device="cuda")
    W = torch.empty(c, c, dtype=torch.float64, device="cuda")
    p = plans["f64"]
    rs.rsvd_small_svd(p.handle, dev(T0, torch.float64), Vt, S, W)
    assert p.status() == rs.RSVD_OK
    Uo, so, Vo = oracle.svd(T0)
    oracle.sign_convention(Uo, Vo)
    Sg, Vg, Wg = host(S), host(Vt), host(W)
    assert np.all(np.diff(Sg) <= 0)
    kappa = so[0] / so[-1]
    # relative accuracy of every value (one-sided Jacobi on the triangular
    # factor, no absolute floor)
    assert np.max(np.abs(Sg - so) / so) <= 100 * c * EPS64 * kappa
    gap = np.min(-np.diff(so) / so[:-1])
    assert np.abs(align_columns(Vg, Uo) - Uo).max() <= 100 * c * EPS64 * kappa / gap
    assert np.abs(align_columns(Wg, Vo) - Vo).max() <= 100 * c * EPS64 * kappa / gap
    assert sign_rule_holds(Vg)
    assert np.abs(Wg.T @ Wg - np.eye(c)).max() <= 50 * c * EPS64
    assert np.linalg.norm((Vg * Sg) @ Wg.T - T0) <= 100 * c * EPS64 * np.linalg.norm(T0)


def run_pair(plan, A0, dt, k, p, q, t, omega_seed):
    m, n = A0.shape
    l = min(k + p, n)
    A0 = rounded(A0, dt)
    G = synth.gaussian_omega(omega_seed, n, l)
    res = plan.solve(dev(A0, dt), k, p, q, t, omega=dev(G, torch.float64))
    ref = oracle.rsvd(A0, rounded(G, dt), k, p, q, t)
    return res, ref


def check(res, ref, dt):
    S, U, V = host(res.S), host(res.U), host(res.V)
    assert np.all(np.isfinite(S)) and np.all(np.isfinite(U)) and np.all(np.isfinite(V))
    rel = np.max(np.abs(S - ref.S) / ref.S)
    assert rel <= SIG_TOL.get(dt, 1e-4), rel
    assert oracle.principal_angle_max(ref.V, V) <= 1e-3
    assert oracle.principal_angle_max(ref.U, U) <= 1e-3
    assert res.K == ref.K and res.status == ref.status
    assert sign_rule_holds(V)


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("m,n,k,p,q", [
    (12000, 400, 128, 32, 2),    # l = 160, the mixed-precision workload's sketch
    (9001, 300, 100, 92, 1),     # l = 192 (largest), ragged m
    (6000, 250, 90, 10, 2),      # l = 100, just past the one-workgroup small SVD
    (3000, 150, 140, 20, 1),     # l clamped to n = 150
])
def test_wide_rsvd_parity(plans, name, m, n, k, p, q):
    dt = DTYPES[name]
    announce(f"wide rsvd {name} m={m} n={n} k={k} p={p} q={q}")
    sigma = 0.97 ** np.arange(n)
    A0 = synth.low_rank(m + n + k, m, n, sigma)
    res, ref = run_pair(plans[name], A0, dt, k, p, q, 0.9, 17)
    check(res, ref, dt)


@pytest.mark.parametrize("name", DTYPES)
def test_wide_rsvd_slow_decay(plans, name):
    # the mixed-precision workload's spectrum (sigma_i = 1/sqrt(i) plus
    # N(0, 1e-4) noise) at a size the oracle finishes in seconds, k = 128,
    # p = 32, q = 3
    dt = DTYPES[name]
    announce(f"wide rsvd {name} 16384x512 sigma=1/sqrt(i) k=128 p=32 q=3")
    A0 = synth.spiked_noisy(33, 16384, 512, synth.config3_sigma(512), 1e-4)
    res, ref = run_pair(plans[name], A0, dt, 128, 32, 3, 0.95, 19)
    check(res, ref, dt)


@pytest.mark.parametrize("name", DTYPES)
def test_wide_krylov_parity(plans, name):
    # the Krylov method at the 1e6 x 512 workload's rank: k = 64, p = 16,
    # i = 1 -> a panel of L = 160 columns
    dt = DTYPES[name]
    announce(f"wide krylov {name} 20000x512 k=64 p=16 i=1")
    A0 = rounded(synth.spiked_noisy(21, 20000, 512, synth.config2_sigma(512), 1e-3), dt)
    n, k, p, i, t = 512, 64, 16, 1, 0.95
    G = synth.gaussian_omega(23, n, k + p)
    res = plans[name].solve_krylov(dev(A0, dt), k, p, i, t, omega=dev(G, torch.float64))
    ref = oracle.krylov(A0, rounded(G, dt), k, p, i, t)
    check(res, ref, dt)


@pytest.mark.parametrize("name", DTYPES)
def test_wide_breakdown(plans, name):
    # exactly rank-one sketch at l = 120: the second Cholesky pivot of the
    # wide kernel is exactly zero -> RSVD_ERR_BREAKDOWN
    dt = DTYPES[name]
    n, l = 200, 120
    A = torch.zeros(300, n, dtype=dt, device="cuda")
    A[0, 0] = 1.0
    G = torch.from_numpy(np.where(np.arange(n * l).reshape(n, l) % 3 == 0, 1.0, -1.0)).cuda()
    res = plans[name].solve(A, 100, 20, 0, 0.9, omega=G)
    assert res.status == rs.RSVD_ERR_BREAKDOWN


# ---- low-precision storage, 9 to 12 column tiles ----
def stored(x, fmt):
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.float32).to(fmt)


@pytest.mark.parametrize("m,n,c", [(1037, 520, 160), (4099, 1024, 144), (300, 64, 192),
                                   (2000, 200, 176)])
def test_wide_lowp_gemm_nn_parity(lowp_plan, m, n, c):
    announce(f"{lowp_plan.storage} wide gemm_nn m={m} n={n} c={c}")
    rng = np.random.default_rng(m + 5 * n + c)
    Aq = stored(rng.standard_normal((m, n)), lowp_plan.storage)
    A64 = Aq.to(torch.float64).numpy()
    X0 = rng.standard_normal((n, c)).astype(np.float32)
    Y = torch.full((m, c), float("nan"), dtype=torch.float32, device="cuda")
    f2 = torch.empty(1, dtype=torch.float64, device="cuda")
    rs.rsvd_gemm_nn(lowp_plan.handle, Aq.cuda(), dev(X0, torch.float32), Y, fro2=f2)
    torch.cuda.synchronize()
    X64 = X0.astype(np.float64)
    Yref = oracle.gemm_nn(A64, X64)
    bound = (HILO + 2 * n * U32) * (np.abs(A64) @ np.abs(X64)) + 1e-300
    assert np.all(np.abs(host(Y) - Yref) <= bound)
    f2ref = oracle.fro2(A64)
    assert abs(host(f2)[0] - f2ref) <= 4 * U32 * f2ref


@pytest.mark.parametrize("m,n,c", [(1037, 1024, 160), (4099, 520, 144), (33, 64, 192),
                                   (2000, 256, 176), (5000, 1032, 160),
                                   (26000, 1024, 160)])   # 13 chunks per row split
def test_wide_lowp_gemm_tn_parity(lowp_plan, m, n, c):
    announce(f"{lowp_plan.storage} wide gemm_tn m={m} n={n} c={c}")
    rng = np.random.default_rng(3 * m + n + 7 * c)
    Aq = stored(rng.standard_normal((m, n)), lowp_plan.storage)
    A64 = Aq.to(torch.float64).numpy()
    Q0 = rng.standard_normal((m, c)).astype(np.float32)
    Z = torch.empty(n, c, dtype=torch.float64, device="cuda")
    rs.rsvd_gemm_tn(lowp_plan.handle, Aq.cuda(), dev(Q0, torch.float32), Z)
    torch.cuda.synchronize()
    Q64 = Q0.astype(np.float64)
    Zref = oracle.gemm_tn(A64, Q64)
    bound = (HILO + 2 * m * U32) * (np.abs(A64).T @ np.abs(Q64)) + 1e-300
    assert np.all(np.abs(host(Z) - Zref) <= bound)


def test_wide_lowp_rsvd_parity(lowp_plan):
    # sigma_i = 1/sqrt(i) plus N(0, 1e-4) noise, k = 128, p = 32 (l = 160),
    # q = 3, power-of-two column scales; oracle on the dequantised matrix
    announce(f"{lowp_plan.storage} wide rsvd 16384x512 k=128 p=32 q=3")
    A0 = synth.spiked_noisy(34, 16384, 512, synth.config3_sigma(512), 1e-4)
    Aq, s = lowp_plan.quantize(dev(A0.astype(np.float32), torch.float32))
    torch.cuda.synchronize()
    A64 = Aq.cpu().to(torch.float64).numpy() * s.cpu().numpy().astype(np.float64)[None, :]
    G = synth.gaussian_omega(29, 512, 160)
    res = lowp_plan.solve(Aq, 128, 32, 3, 0.95, omega=dev(G, torch.float64), col_scale=s)
    ref = oracle.rsvd(A64, G.astype(np.float32).astype(np.float64), 128, 32, 3, 0.95)
    check(res, ref, torch.float32)
