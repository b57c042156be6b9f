"""Per-stage parity of the HIP path against the oracle, through the C ABI.

Bounds follow from the arithmetic: a length-n dot product in precision u has
error at most about n*u*sum|a_k b_k| (standard rounding analysis), so each
product is compared element by element against that bound computed from the
absolute values of the same operands.
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


def unit(dt):
    return EPS64 if dt == torch.float64 else U32


@pytest.fixture(scope="module")
def plans():
    out = {}
    for name, dt in DTYPES.items():
        out[name] = rs.Plan(6000, 300, 96, dt, want_gram=True, seed=7)
    yield out
    for p in out.values():
        p.close()


def test_gaussian_fill_matches_published_definition():
    for seed, rows, cols in [(101, 200, 30), (5, 3, 5), (2**40 + 3, 512, 80)]:
        announce(f"gaussian_fill seed={seed} {rows}x{cols}")
        G = torch.empty(rows, cols, dtype=torch.float64, device="cuda")
        rs.rsvd_gaussian_fill(seed, G)
        torch.cuda.synchronize()
        ref = synth.gaussian_omega(seed, rows, cols)
        got = host(G)
        # same Philox words and uniforms; only libm's last bits may differ
        assert np.max(np.abs(got - ref) / (1.0 + np.abs(ref))) <= 8 * EPS64


NN_CASES = [
    (1037, 203, 30, 0),    # ragged rows, odd n (scalar loads)
    (1037, 200, 80, 0),    # 16-byte loads, tail row block
    (300, 64, 17, 4),      # padded leading dimension, c not a multiple of 16
    (5000, 256, 96, 0),
    (777, 150, 200, 0),    # c > 128: several column tiles
    (4133, 64, 80, 0),     # fp32 tall kernel (n % 32 == 0): ragged last row block
    (1000, 512, 128, 0),   # fp32 tall kernel at its widest (8 column tiles)
    (515, 32, 1, 0),       # one column
    (2049, 80, 80, 0),     # tall kernel, last k chunk half full (the CholeskyQR2 shape)
    (700, 84, 52, 4),      # tall kernel, k tail of 20, padded rows
    (1500, 4, 7, 0),       # tall kernel, a single k chunk of 4
]


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("m,n,c,pad", NN_CASES)
def test_gemm_nn_parity(plans, name, m, n, c, pad):
    dt = DTYPES[name]
    announce(f"gemm_nn {name} m={m} n={n} c={c} pad={pad}")
    rng = np.random.default_rng(m + n + c)
    A0 = rounded(rng.standard_normal((m, n)), dt)
    X0 = rounded(rng.standard_normal((n, c)), dt)
    Abig = dev(np.pad(A0, ((0, 0), (0, pad))), dt)
    A = Abig[:, :n]
    X = dev(X0, dt)
    Y = torch.empty(m, c, dtype=dt, device="cuda")
    want_gram = c <= 96
    Gm = torch.empty(c, c, dtype=torch.float64, device="cuda") if want_gram else None
    f2 = torch.empty(1, dtype=torch.float64, device="cuda")
    p = plans[name] if n <= 300 else big_plans(name)
    rs.rsvd_gemm_nn(p.handle, A, X, Y, Gram=Gm, fro2=f2)
    torch.cuda.synchronize()
    Yref = oracle.gemm_nn(A0, X0)
    bound = 2.0 * n * unit(dt) * (np.abs(A0) @ np.abs(X0)) + 1e-300
    Yg = host(Y)
    assert np.all(np.abs(Yg - Yref) <= bound)
    f2ref = oracle.fro2(A0)
    assert abs(host(f2)[0] - f2ref) <= 2 * m * n * EPS64 * f2ref
    if want_gram:
        # FP64 Gram of the stored (rounded) Y, exact products
        Gref = oracle.gemm_tn(Yg, Yg)
        gb = 2.0 * m * EPS64 * (np.abs(Yg).T @ np.abs(Yg))
        assert np.all(np.abs(host(Gm) - Gref) <= gb)


# short k (n <= 96) without the sum of squares: fp32 takes the kernel that
# loads A straight into matrix-core registers; the row padding holds NaN,
# which must not reach Y (the last k slab of a row runs past n)
NN_NARROW_CASES = [
    (2049, 80, 80, 0),     # the CholeskyQR2 shape: 5 whole k slabs, 5 column tiles
    (700, 84, 52, 4),      # last slab 4 of 16 wide, ragged column tile, NaN padding
    (1500, 4, 7, 0),       # a single k group of 4
    (257, 96, 128, 0),     # 6 slabs, 8 column tiles, one row past a block
    (33, 16, 1, 4),        # one partial block, one column
]


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("m,n,c,pad", NN_NARROW_CASES)
def test_gemm_nn_narrow_parity(plans, name, m, n, c, pad):
    dt = DTYPES[name]
    announce(f"gemm_nn narrow {name} m={m} n={n} c={c} pad={pad}")
    rng = np.random.default_rng(7 * m + n + c)
    A0 = rounded(rng.standard_normal((m, n)), dt)
    X0 = rounded(rng.standard_normal((n, c)), dt)
    A = dev(np.pad(A0, ((0, 0), (0, pad)), constant_values=np.nan), dt)[:, :n]
    X = dev(X0, dt)
    Y = torch.full((m, c), float("nan"), dtype=dt, device="cuda")
    rs.rsvd_gemm_nn(plans[name].handle, A, X, Y)
    torch.cuda.synchronize()
    Yref = oracle.gemm_nn(A0, X0)
    bound = 2.0 * n * unit(dt) * (np.abs(A0) @ np.abs(X0)) + 1e-300
    assert np.all(np.abs(host(Y) - Yref) <= bound)


# wide X without the fused sum of squares: the two-level tiled product for
# fp32 (128 x 256 block tiles, XCD-ordered), the column-tiled one for fp64
NN_WIDE_CASES = [
    (777, 150, 200, 0),    # one column tile, partial
    (1037, 203, 257, 4),   # unaligned A rows and X rows (scalar loads), ragged everything
    (300, 512, 512, 0),    # the u_i = A v_i / s_i shape at small m
    (129, 33, 300, 0),     # one full and one ragged row tile, k tail
    (5000, 256, 384, 0),
]


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("m,n,c,pad", NN_WIDE_CASES)
def test_gemm_nn_wide_parity(plans, name, m, n, c, pad):
    dt = DTYPES[name]
    announce(f"gemm_nn wide {name} m={m} n={n} c={c} pad={pad}")
    rng = np.random.default_rng(m + 3 * n + c)
    A0 = rounded(rng.standard_normal((m, n)), dt)
    X0 = rounded(rng.standard_normal((n, c)), dt)
    A = dev(np.pad(A0, ((0, 0), (0, pad))), dt)[:, :n]
    X = dev(X0, dt)
    Y = torch.full((m, c), float("nan"), dtype=dt, device="cuda")
    p = plans[name] if c <= 300 and n <= 300 else big_plans(name)
    rs.rsvd_gemm_nn(p.handle, A, X, Y)
    torch.cuda.synchronize()
    Yref = oracle.gemm_nn(A0, X0)
    bound = 2.0 * n * unit(dt) * (np.abs(A0) @ np.abs(X0)) + 1e-300
    assert np.all(np.abs(host(Y) - Yref) <= bound)


_BIG = {}


def big_plans(name):
    if name not in _BIG:
        _BIG[name] = rs.Plan(6000, 640, 96, DTYPES[name], want_gram=True, seed=7)
    return _BIG[name]


TN_CASES = [(1037, 203, 30), (5000, 256, 80), (129, 300, 200), (3, 10, 5), (4100, 97, 96),
            (4099, 512, 80), (1000, 600, 128), (70, 64, 3), (2000, 36, 48),
            # the fp32 narrow kernel, n <= 64 / 128 / 256: every column-tile
            # count's extremes, ragged m, splits shorter than a chunk
            (5003, 64, 128), (4097, 60, 20), (16, 64, 8), (3001, 128, 40), (777, 100, 96),
            (2050, 144, 24), (65, 256, 4), (5999, 192, 96),
            # 129 to 160 columns (nine and ten column tiles): the narrow
            # kernel of every width and the 512-column tile, two of them at
            # n = 640
            (1500, 64, 136), (2600, 120, 160), (3001, 256, 152), (4100, 512, 160),
            (2333, 640, 144)]


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("m,n,c", TN_CASES)
def test_gemm_tn_parity(plans, name, m, n, c):
    dt = DTYPES[name]
    announce(f"gemm_tn {name} m={m} n={n} c={c}")
    rng = np.random.default_rng(3 * m + n + c)
    A0 = rounded(rng.standard_normal((m, n)), dt)
    Q0 = rounded(rng.standard_normal((m, c)), dt)
    Z = torch.empty(n, c, dtype=torch.float64, device="cuda")
    p = plans[name] if n <= 300 else big_plans(name)
    rs.rsvd_gemm_tn(p.handle, dev(A0, dt), dev(Q0, dt), Z)
    torch.cuda.synchronize()
    Zref = oracle.gemm_tn(A0, Q0)
    # partial sums over at most m rows in the product precision, then FP64
    bound = 2.0 * m * unit(dt) * (np.abs(A0).T @ np.abs(Q0)) + 1e-300
    assert np.all(np.abs(host(Z) - Zref) <= bound)


@pytest.mark.parametrize("m,n,pad,c", [(3000, 60, 4, 40), (2500, 120, 8, 24), (1800, 200, 4, 96),
                                         (777, 300, 4, 48)])
def test_gemm_tn_padded_rows(plans, m, n, pad, c):
    # A as a view with row stride lda = n + pad (a multiple of 4): the fp32
    # kernels read whole 64-column slabs from each row start, so the padding
    # and the next row's leading entries are read and must not reach Z
    dt = torch.float32
    announce(f"gemm_tn padded rows m={m} n={n} lda={n + pad} c={c}")
    rng = np.random.default_rng(m + n + pad + c)
    A0 = rounded(rng.standard_normal((m, n)), dt)
    Q0 = rounded(rng.standard_normal((m, c)), dt)
    Abig = torch.full((m, n + pad), float("nan"), dtype=dt, device="cuda")
    Abig[:, :n] = dev(A0, dt)
    Z = torch.empty(n, c, dtype=torch.float64, device="cuda")
    rs.rsvd_gemm_tn(plans["f32"].handle, Abig[:, :n], dev(Q0, dt), Z)
    torch.cuda.synchronize()
    Zref = oracle.gemm_tn(A0, Q0)
    bound = 2.0 * m * unit(dt) * (np.abs(A0).T @ np.abs(Q0)) + 1e-300
    assert np.all(np.isfinite(host(Z)))
    assert np.all(np.abs(host(Z) - Zref) <= bound)


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("m,c,kappa", [(2000, 30, 1e2), (5000, 80, 1e3), (333, 17, 10.0),
                                           (3000, 96, 1e2), (4000, 44, 1e3), (500, 1, 1.0),
                                           (1200, 16, 10.0), (2500, 65, 1e2), (6000, 33, 1e2)])
def test_cholqr2_parity(plans, name, m, c, kappa):
    dt = DTYPES[name]
    announce(f"cholqr2 {name} m={m} c={c} kappa={kappa}")
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
    # orthonormality and reconstruction at the working precision
    assert np.abs(Qg.T @ Qg - np.eye(c)).max() <= 50 * c * u
    assert np.linalg.norm(Qg @ Rg - Y0) <= 50 * c * u * np.linalg.norm(Y0)
    # same factors as the oracle's Householder QR (unique with R_jj > 0)
    Qo, Ro = oracle.qr(Y0)
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0)
    assert np.abs(Rg - Ro).max() <= 50 * c * u * kappa * np.abs(Ro).max()
    assert np.abs(Qg - Qo).max() <= 50 * c * u * kappa


# c covers every rows-per-lane count of the kernel (ceil(c / 8) = 1 .. 12);
# the wide spectrum (sigma down to 1e-6) takes the second, J-accumulating
# launch, the clustered one (sigma in [1, 1.4], the headline's shape) does not
@pytest.mark.parametrize("r,c,spec", [
    (300, 40, "wide"), (200, 31, "wide"), (96, 96, "wide"), (250, 1, "wide"), (100, 2, "wide"),
    (150, 17, "wide"), (300, 80, "wide"), (300, 89, "wide"), (64, 63, "clustered"),
    (290, 80, "clustered"), (300, 96, "clustered"), (120, 8, "clustered"), (200, 9, "clustered"),
    (220, 24, "clustered"), (260, 33, "clustered"), (300, 47, "clustered"), (280, 56, "clustered"),
    (296, 72, "clustered")])
def test_small_svd_parity(plans, r, c, spec):
    announce(f"small_svd r={r} c={c} {spec}")
    rng = np.random.default_rng(r * c)
    sig = np.logspace(0, -6, c) if spec == "wide" else np.linspace(1.4, 1.0, c)
    T0 = synth.haar(rng, r, c) @ np.diag(sig) @ synth.haar(rng, c, c).T
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
    assert np.max(np.abs(Sg - so) / so) <= 100 * c * EPS64 * kappa
    # separated values: columns match up to sign; the sign rule is applied
    assert np.abs(align_columns(Vg, Uo) - Uo).max() <= 1e-9
    assert np.abs(align_columns(Wg, Vo) - Vo).max() <= 1e-9
    assert sign_rule_holds(Vg)
    assert np.linalg.norm((Vg * Sg) @ Wg.T - T0) <= 100 * c * EPS64 * np.linalg.norm(T0)


# n = 512 and 1024: four and eight row slices per block pair (1024 fills the
# chip with one workgroup per CU)
@pytest.mark.parametrize("n", [2, 7, 64, 200, 257, 512, 1024])
def test_sym_eig_parity(plans, n):
    announce(f"sym_eig n={n}")
    rng = np.random.default_rng(n)
    Qh = synth.haar(rng, n, n)
    lam_true = np.linspace(3.0, 0.5, n) ** 2
    G0 = (Qh * lam_true) @ Qh.T
    G0 = 0.5 * (G0 + G0.T)
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    V = torch.empty(n, n, dtype=torch.float64, device="cuda")
    p = plans["f64"] if n <= 300 else rs.Plan(n, n, 8, torch.float64, want_gram=True, seed=1)
    rs.rsvd_sym_eig(p.handle, dev(G0, torch.float64), lam, V)
    assert p.status() == rs.RSVD_OK
    if n > 300:
        p.close()
        # the construction itself: eigenvalues lam_true (descending) with the
        # columns of Qh, exact up to the rounding of G0 (the oracle's cyclic
        # Jacobi takes minutes at this size)
        lo, Vo = lam_true.copy(), np.ascontiguousarray(Qh)
    else:
        lo, Vo, _ = oracle.eig_sym(G0)
    oracle.sign_convention(None, Vo)
    lg, Vg = host(lam), host(V)
    assert np.abs(lg - lo).max() <= 50 * n * EPS64 * lo[0]
    gap = np.min(np.abs(np.diff(lo))) / lo[0]
    assert np.abs(align_columns(Vg, Vo) - Vo).max() <= 100 * n * EPS64 / gap
    assert sign_rule_holds(Vg)
    assert np.abs(Vg.T @ Vg - np.eye(n)).max() <= 50 * n * EPS64


def test_sym_eig_repeated_and_clustered():
    # n = 512 (four row slices per block pair) with exactly repeated
    # eigenvalues (multiplicities 6, 10, 15 and a zero of multiplicity 3), a
    # cluster of 20 eigenvalues 1e-12 apart (relative), a separated leading
    # one, and 457 distinct values.  Eigenvectors inside a cluster are
    # determined only as a subspace, so the checks are: eigenvalues within
    # c n eps lambda_1, the residual ||G V - V Lambda||_F within c n eps ||G||_F,
    # orthonormal V, and for every cluster (split where the relative gap
    # exceeds 1e-9) the largest principal angle against the construction's
    # subspace within c n eps lambda_1 / delta (Davis-Kahan, delta = the
    # cluster's distance to the rest of the spectrum).
    n = 512
    announce(f"sym_eig repeated/clustered n={n}")
    lam = np.concatenate([[9.0], [7.0] * 6, 5.0 * (1.0 + 1e-12 * np.arange(20)), [3.0] * 10,
                          [2.5] * 15, np.linspace(2.0, 0.1, n - 55), [0.0] * 3])
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    rng = np.random.default_rng(512)
    Qh = synth.haar(rng, n, n)
    G0 = (Qh * lam) @ Qh.T
    G0 = 0.5 * (G0 + G0.T)
    lg_t = torch.empty(n, dtype=torch.float64, device="cuda")
    V_t = torch.empty(n, n, dtype=torch.float64, device="cuda")
    p = rs.Plan(n, n, 8, torch.float64, want_gram=True, seed=1)
    try:
        rs.rsvd_sym_eig(p.handle, dev(G0, torch.float64), lg_t, V_t)
        assert p.status() == rs.RSVD_OK
    finally:
        p.close()
    lg, Vg = host(lg_t), host(V_t)
    tol = 50 * n * EPS64
    assert np.all(np.diff(lg) <= 0)
    assert np.abs(lg - lam).max() <= tol * lam[0]
    assert np.linalg.norm(G0 @ Vg - Vg * lg) <= tol * np.linalg.norm(G0)
    assert np.abs(Vg.T @ Vg - np.eye(n)).max() <= tol
    assert sign_rule_holds(Vg)
    cut = np.where(-np.diff(lam) > 1e-9 * lam[0])[0] + 1
    groups = np.split(np.arange(n), cut)
    assert max(len(g) for g in groups) == 20 and len(groups) == n - 19 - 5 - 9 - 14 - 2
    for idx in groups:
        rest = np.setdiff1d(np.arange(n), idx)
        delta = np.min(np.abs(lam[idx][:, None] - lam[rest][None, :]))
        ang = oracle.principal_angle_max(Qh[:, idx], Vg[:, idx])
        assert ang <= 2 * tol * lam[0] / delta + 1e-14, (idx[0], len(idx), ang, delta)
