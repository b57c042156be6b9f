"""Pins for the oracle's Randomized PCA (Sec. 3.1.2), its K selection
(Sec. 2.4) and the truncated SVD through A^T A (Sec. 2.3 / 3.1.3).

Randomized PCA is an approximation, so the pins are what the mathematics
fixes for it: exact recovery when rank(A) <= l, interlacing of the computed
values below the true ones, the probabilistic error bound of Halko,
Martinsson & Tropp (SIAM Review 2011, Sec. 10), and convergence in q.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------- select K
def test_select_k_golden_config1_closed_form():
    g = load_golden("select_k_config1.txt")
    sigma = synth.config1_sigma(200)
    lam = sigma ** 2
    K, st = oracle.select_k(sigma, float(np.sum(lam)), float(g["T"]))
    assert (K, st) == (int(g["K"]), oracle.OK)
    f = np.cumsum(lam) / np.sum(lam)
    assert abs(f[8] - g["F9"]) < 1e-7 and abs(f[9] - g["F10"]) < 1e-7


def test_select_k_edges():
    s = np.array([2.0, 1.0, 1.0])          # lambda = 4, 1, 1 ; total 6
    assert oracle.select_k(s, 6.0, 4.0 / 6.0) == (1, oracle.OK)   # equality counts (>= t)
    assert oracle.select_k(s, 6.0, 0.7) == (2, oracle.OK)
    assert oracle.select_k(s, 6.0, 1.0) == (3, oracle.OK)
    # only k of n values known: denominator ||A||_F^2 larger than their sum
    assert oracle.select_k(s, 10.0, 0.9) == (3, oracle.WARN_THRESHOLD)
    assert oracle.select_k(np.zeros(3), 0.0, 0.5) == (0, oracle.WARN_ZERO)
    for bad_t in [0.0, -0.1, 1.5, float("nan")]:
        with pytest.raises(ValueError):
            oracle.select_k(s, 6.0, bad_t)


def test_sign_convention_rule():
    V = np.array([[0.1, -0.6], [-0.9, 0.6], [0.2, 0.1]])
    U = np.array([[1.0, 2.0], [3.0, 4.0]])
    U2, V2 = oracle.sign_convention(U.copy(), V.copy())
    assert np.array_equal(V2[:, 0], -V[:, 0]) and np.array_equal(U2[:, 0], -U[:, 0])
    assert np.array_equal(V2[:, 1], -V[:, 1])   # tie |-0.6| = |0.6|: index 0 wins, it is negative -> flip
    assert np.array_equal(U2[:, 1], -U[:, 1])
    V = np.array([[-0.6], [0.6]])
    _, V3 = oracle.sign_convention(None, V.copy())
    assert V3[0, 0] == 0.6


# ----------------------------------------------------------- sketch matrix
def test_philox_known_answers():
    with open(__import__("conftest").GOLDEN + "/philox_kat.txt") as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for r in rows:
        ctr = np.array([[int(x, 16) for x in r[:4]]], dtype=np.uint64)
        key = [int(x, 16) for x in r[4:6]]
        want = [int(x, 16) for x in r[7:11]]
        assert [int(x) for x in synth.philox4x32_10(ctr, key)[0]] == want


def test_gaussian_omega_moments_and_determinism():
    G = synth.gaussian_omega(101, 400, 250)
    assert G.shape == (400, 250)
    assert np.array_equal(G, synth.gaussian_omega(101, 400, 250))
    assert not np.array_equal(G, synth.gaussian_omega(102, 400, 250))
    N = G.size
    assert abs(G.mean()) < 5 / np.sqrt(N)
    assert abs(G.var() - 1) < 5 * np.sqrt(2 / N)
    assert abs(np.mean(G ** 4) - 3) < 0.1                       # Gaussian kurtosis
    # prefix property: element e depends only on (seed, e)
    assert np.array_equal(synth.gaussian_omega(7, 3, 5).ravel(), synth.gaussian_omega(7, 5, 3).ravel())


# --------------------------------------------------------- Randomized PCA
def test_rsvd_exact_recovery_at_rank_l():
    # rank(A) = r <= l: range(A G) = range(A) almost surely, so the sketch
    # captures A exactly and the top r values are A's to rounding
    m, n, k, p = 600, 80, 12, 8
    r = k + p
    sigma = np.logspace(0, -3, r)
    A = synth.low_rank(21, m, n, sigma)
    G = synth.gaussian_omega(5, n, r)
    for q in [0, 1, 2]:
        res = oracle.rsvd(A, G, k, p, q, 0.99)
        assert np.max(np.abs(res.S - sigma[:k]) / sigma[:k]) <= 1e-10
        U, s, V = oracle.svd(A)
        oracle.sign_convention(U, V)
        assert np.allclose(res.V, V[:, :k], atol=1e-9)
        assert np.allclose(res.U, U[:, :k], atol=1e-9)


def test_rsvd_config1_interlacing_K_and_accuracy():
    c = synth.CONFIG1
    A = synth.config1(c["seed"])
    n = A.shape[1]
    l = c["k"] + c["p"]
    G = synth.gaussian_omega(c["omega_seed"], n, l)
    res = oracle.rsvd(A, G, c["k"], c["p"], c["q"], c["t"])
    U, s, V = oracle.svd(A)
    # the computed values never exceed the true ones (Q^T A is a compression)
    assert np.all(res.S <= s[:c["k"]] * (1 + 1e-12))
    # K criterion: K_rsvd >= K_exact (interlacing); config 1 gives 10 for both
    K_exact, _ = oracle.select_k(s, oracle.fro2(A), c["t"])
    assert res.K >= K_exact and res.K == 10 and res.status == oracle.OK
    assert abs(res.fro2 - np.sum(s ** 2)) <= 1e-12 * res.fro2
    # gap sigma_10/sigma_31 = 0.85^-21 ~ 30 with q = 2 -> the top 10 are exact
    assert np.max(np.abs(res.S[:10] - s[:10]) / s[:10]) <= 1e-10
    assert oracle.principal_angle_max(V[:, :10], res.V[:, :10]) <= 1e-8
    assert np.abs(res.U.T @ res.U - np.eye(c["k"])).max() <= 1e-13
    assert np.abs(res.V.T @ res.V - np.eye(c["k"])).max() <= 1e-13
    # A^T U = V S holds exactly for U = Q W, S, V from the SVD of T = A^T Q
    assert np.linalg.norm(A.T @ res.U - res.V * res.S) <= 1e-12 * np.linalg.norm(A)


def test_rsvd_halko_error_bound_and_q_convergence():
    # Halko-Martinsson-Tropp (SIAM Rev. 2011, Sec. 1.5 / Thm 10.6 and Cor. 10.10):
    # with k + p columns, ||A - Q Q^T A|| <= [1 + 11 sqrt(k+p) sqrt(min(m,n))]^(1/(2q+1))
    # * sigma_{k+1} except with probability <= 6 p^-p.  With k_out = l (p_out = 0)
    # the oracle returns the whole rank-l approximation Q Q^T A = U S V^T.
    m, n, k, p = 800, 120, 10, 6
    l = k + p
    rng = np.random.default_rng(9)
    sigma = 1.0 / np.arange(1, n + 1) ** 0.7
    A = synth.haar(rng, m, n) @ np.diag(sigma) @ synth.haar(rng, n, n).T
    errs = []
    for q in [0, 1, 2, 3]:
        worst = 0.0
        for seed in range(5):
            res = oracle.rsvd(A, synth.gaussian_omega(1000 + seed, n, l), l, 0, q, 0.5)
            err = np.linalg.norm(A - (res.U * res.S) @ res.V.T, 2)
            bound = (1 + 11 * np.sqrt(l) * np.sqrt(n)) ** (1.0 / (2 * q + 1)) * sigma[k]
            assert err <= bound
            assert err >= sigma[l] * (1 - 1e-12)           # Eckart-Young: rank l cannot beat sigma_{l+1}
            worst = max(worst, err)
        errs.append(worst)
    assert errs[0] > errs[1] > errs[2] > errs[3]          # power iterations help


def test_rsvd_clamps_l_to_n_and_rejects_bad_args():
    A = synth.low_rank(3, 50, 8, np.linspace(2, 1, 8))
    res = oracle.rsvd(A, synth.gaussian_omega(1, 8, 8), 6, 10, 1, 0.9)  # l = min(16, 8)
    s = oracle.svd(A)[1]
    assert np.allclose(res.S, s[:6], rtol=1e-12)
    with pytest.raises(RuntimeError):
        oracle.rsvd(A, synth.gaussian_omega(1, 8, 8), 9, 0, 1, 0.9)    # k > n


# ------------------------------------------------- truncated SVD via A^T A
def test_gram_route_matches_exact_on_top_K():
    # Sec. 2.3: V from eig(A^T A), s_i = sqrt(lambda_i), u_i = A v_i / s_i.
    # The A^T A route resolves s_i to about eps*s_1^2/s_i (absolute), so it is
    # compared with the exact SVD on the values the criterion keeps (K = 10).
    A = synth.config1(1)
    m, n = A.shape
    g = oracle.gram_eig(A, 0.95)
    U, s, V = oracle.svd(A)
    oracle.sign_convention(U, V)
    assert g.K == 10 and g.status == oracle.OK
    assert np.max(np.abs(g.S[:10] - s[:10]) / s[:10]) <= 1e-12
    assert np.allclose(g.V[:, :10], V[:, :10], atol=1e-10)
    assert np.allclose(g.U[:, :10], U[:, :10], atol=1e-10)
    assert np.abs(g.V.T @ g.V - np.eye(n)).max() <= 20 * n * EPS
    # absolute accuracy of every lambda_i = s_i^2 relative to lambda_1
    assert np.max(np.abs(g.S ** 2 - s ** 2)) <= 50 * n * EPS * s[0] ** 2
    # Eq. AV for the columns that were formed
    good = g.S > m * EPS * g.S[0]
    assert np.linalg.norm(A @ g.V[:, good] - g.U[:, good] * g.S[good]) <= 1e-10 * np.linalg.norm(A)


def test_gram_route_zero_matrix_and_partial_u():
    A = np.zeros((30, 4))
    g = oracle.gram_eig(A, 0.9)
    assert g.K == 0 and g.status == oracle.WARN_ZERO
    assert np.all(g.S == 0) and np.all(g.U == 0)
    A = synth.low_rank(4, 40, 6, [3.0, 2.0, 1.0, 0.5, 0.25, 0.1])
    g = oracle.gram_eig(A, 0.9, ucols=2)
    assert g.U.shape == (40, 2)
