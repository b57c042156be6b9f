"""Pins for the oracle's SVD and symmetric eigensolver (paper Sec. 2.1-2.3).

Closed forms (tests/golden), brute-force special cases (diagonal, rank one,
known spectrum), the identities the paper states (U^T U = V^T V = I,
A v_i = s_i u_i, s_i^2 = eig(A^T A), sum lambda_i = ||A||_F^2), and LAPACK
as a third opinion.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("name", ["svd_2x2.txt", "svd_3x2.txt"])
@pytest.mark.parametrize("route", ["jacobi", "exact"])
def test_svd_golden(name, route):
    g = load_golden(name)
    fn = oracle.svd if route == "exact" else (lambda X: oracle.svd_jacobi(X)[:3])
    U, s, V = fn(g["A"])
    oracle.sign_convention(U, V)
    assert np.allclose(s, g["S"], rtol=4 * EPS, atol=0)
    assert np.allclose(V, g["V"], atol=8 * EPS)
    assert np.allclose(U, g["U"], atol=8 * EPS)


def test_eig_golden_3x3():
    g = load_golden("eig_3x3.txt")
    lam, V, _ = oracle.eig_sym(g["G"])
    oracle.sign_convention(None, V)
    assert np.allclose(lam, g["LAM"], rtol=0, atol=8 * EPS)
    assert np.allclose(V, g["V"], atol=8 * EPS)


def test_svd_diagonal_and_rank_one():
    # diagonal (padded to m > n): singular values are the sorted |d_i|
    d = np.array([0.5, -3.0, 2.0, 1e-9, 7.0])
    A = np.zeros((9, 5)); A[:5, :5] = np.diag(d)
    U, s, V = oracle.svd(A)
    assert np.allclose(s, np.sort(np.abs(d))[::-1], rtol=4 * EPS, atol=0)
    # rank one A = x y^T: s_1 = ||x|| ||y||, the rest zero
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(40), rng.standard_normal(6)
    U, s, V = oracle.svd(np.outer(x, y))
    assert abs(s[0] - np.linalg.norm(x) * np.linalg.norm(y)) <= 8 * EPS * s[0]
    assert np.all(s[1:] <= 40 * EPS * s[0])
    assert abs(abs(V[:, 0] @ y) - np.linalg.norm(y)) <= 1e-13 * np.linalg.norm(y)
    assert abs(abs(U[:, 0] @ x) - np.linalg.norm(x)) <= 1e-13 * np.linalg.norm(x)


def test_svd_known_spectrum_config1():
    # A = U diag(sigma) V^T with exactly orthonormal U (centred, so centring is
    # a no-op) and V: the realised singular values are the generator's sigma.
    A = synth.config1(1)
    m, n = A.shape
    sigma = synth.config1_sigma(n)
    U, s, V = oracle.svd(A)
    # forming A in FP64 perturbs it by ~n*eps*||A|| (absolute), so by Weyl's
    # inequality every s_i is within that of sigma_i; the large ones are
    # therefore relatively exact
    assert np.max(np.abs(s - sigma)) <= 10 * n * EPS * sigma[0]
    top = sigma > 1e-2
    assert np.max(np.abs(s[top] - sigma[top]) / sigma[top]) <= 1e-11
    # Sec. 2.1 identities
    assert np.abs(U.T @ U - np.eye(n)).max() <= 10 * n * EPS
    assert np.abs(V.T @ V - np.eye(n)).max() <= 10 * n * EPS
    assert np.abs(V @ V.T - np.eye(n)).max() <= 10 * n * EPS
    assert np.linalg.norm(A @ V - U * s) <= 10 * n * EPS * np.linalg.norm(A)       # Eq. AV
    # delta = ||A - U S V^T||_F / ||A||_F (the paper's error measure, Sec. 4)
    assert np.linalg.norm(A - (U * s) @ V.T) / np.linalg.norm(A) <= 10 * n * EPS
    # Eq. sumeigen
    assert abs(np.sum(s ** 2) - oracle.fro2(A)) <= 10 * n * EPS * oracle.fro2(A)
    assert np.all(np.diff(s) <= 0)


@pytest.mark.parametrize("m,n", [(300, 40), (120, 120), (1000, 7)])
def test_svd_lapack_third_opinion(m, n):
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) @ np.diag(np.logspace(0, -8, n)) @ synth.haar(rng, n, n).T
    U, s, V = oracle.svd(A)
    sl = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s, sl, rtol=1e-10, atol=1e-14 * sl[0])
    assert np.linalg.norm(A - (U * s) @ V.T) <= 20 * n * EPS * np.linalg.norm(A)


def test_eig_identities_and_lapack():
    # eig(A^T A): lambda_i = s_i^2 (Eq. LambdaSigma), A^T A V = V diag(lambda)
    rng = np.random.default_rng(11)
    A = rng.standard_normal((400, 60)) * np.linspace(3.0, 0.1, 60)
    G = A.T @ A
    lam, V, _ = oracle.eig_sym(G)
    n = G.shape[0]
    assert np.abs(V.T @ V - np.eye(n)).max() <= 20 * n * EPS
    assert np.linalg.norm(G @ V - V * lam) <= 20 * n * EPS * np.linalg.norm(G)
    assert abs(lam.sum() - np.trace(G)) <= 20 * n * EPS * np.trace(G)
    assert np.all(np.diff(lam) <= 0)
    ll = np.linalg.eigvalsh(G)[::-1]
    assert np.allclose(lam, ll, rtol=0, atol=50 * n * EPS * ll[0])
    s = oracle.svd(A)[1]
    assert np.allclose(np.sqrt(lam), s, rtol=1e-10)


def test_eig_singular_and_repeated():
    # rank-deficient PSD with a repeated eigenvalue: the eigenvalues are exact
    # closed forms; only the eigenspace of the repeated value is compared
    Q = synth.haar(np.random.default_rng(2), 6, 6)
    lam_true = np.array([4.0, 2.0, 2.0, 1.0, 0.0, 0.0])
    G = (Q * lam_true) @ Q.T
    lam, V, _ = oracle.eig_sym(G)
    assert np.allclose(lam, lam_true, atol=50 * EPS)
    assert oracle.principal_angle_max(Q[:, 1:3], V[:, 1:3]) <= 1e-12
