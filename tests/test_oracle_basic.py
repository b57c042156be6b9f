"""Pins for the oracle's building blocks: products, ||A||_F^2, Householder QR.

Each check compares against something other than the oracle itself: brute
force by hand, closed forms worked out in tests/golden, exact integer
arithmetic, or numpy/LAPACK as an independent third opinion.
"""
import numpy as np
import pytest

import oracle
from conftest import load_golden

EPS = np.finfo(np.float64).eps


def test_gemm_nn_brute_force_tiny():
    A = np.array([[1.0, 2.0, 3.0, 4.0], [0.5, -1.0, 2.0, 0.0], [3.0, 0.0, -2.0, 1.0]])
    B = np.array([[1.0, 0.0], [2.0, 1.0], [0.0, -1.0], [1.0, 3.0]])
    C = oracle.gemm_nn(A, B)
    for i in range(3):
        for j in range(2):
            assert C[i, j] == sum(A[i, p] * B[p, j] for p in range(4))


def test_gemm_tn_integer_exact_and_third_opinion():
    rng = np.random.default_rng(0)
    A = rng.integers(-9, 10, size=(257, 13)).astype(np.float64)
    B = rng.integers(-9, 10, size=(257, 7)).astype(np.float64)
    C = oracle.gemm_tn(A, B)
    # integer data: every partial sum is exact in FP64, so equality is exact
    assert np.array_equal(C, (A.T.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))
    A = rng.standard_normal((1000, 30))
    B = rng.standard_normal((1000, 9))
    assert np.allclose(oracle.gemm_tn(A, B), A.T @ B, rtol=0, atol=1e-12)
    X = rng.standard_normal((30, 11))
    assert np.allclose(oracle.gemm_nn(A, X), A @ X, rtol=0, atol=1e-12)


def test_fro2_integer_exact_and_trace_identity():
    # Eq. sumeigen: sum a_ij^2 = tr(A^T A) = sum lambda_i
    A = np.arange(-60, 60, dtype=np.float64).reshape(24, 5)
    assert oracle.fro2(A) == float(np.sum(np.arange(-60, 60) ** 2))
    rng = np.random.default_rng(1)
    A = rng.standard_normal((500, 40))
    s = np.linalg.svd(A, compute_uv=False)
    f2 = oracle.fro2(A)
    assert abs(f2 - np.trace(A.T @ A)) <= 1e-12 * f2
    assert abs(f2 - np.sum(s ** 2)) <= 1e-12 * f2


def test_qr_golden_3x2():
    g = load_golden("qr_3x2.txt")
    Q, R = oracle.qr(g["X"])
    assert np.allclose(Q, g["Q"], rtol=0, atol=4 * EPS)
    assert np.allclose(R, g["R"], rtol=0, atol=8 * EPS)


@pytest.mark.parametrize("m,n", [(50, 1), (200, 17), (3000, 64), (64, 64)])
def test_qr_invariants(m, n):
    rng = np.random.default_rng(m * 7 + n)
    X = rng.standard_normal((m, n)) * np.logspace(0, -6, n)  # graded columns
    Q, R = oracle.qr(X)
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 20 * m * EPS
    assert np.linalg.norm(Q @ R - X) <= 20 * m * EPS * np.linalg.norm(X)
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.diag(R) >= 0)
    # LAPACK third opinion: same factors once its signs follow R_jj >= 0
    Ql, Rl = np.linalg.qr(X)
    d = np.sign(np.diag(Rl))
    assert np.allclose(Q, Ql * d, atol=1e-9)
    assert np.allclose(R, Rl * d[:, None], atol=1e-9 * np.abs(R).max())


def test_principal_angle_metric():
    # span(e1) vs span(cos th e1 + sin th e2) -> angle th, also below 1e-8
    for th in [0.3, 1e-5, 1e-11]:
        X = np.zeros((5, 1)); X[0, 0] = 1.0
        Y = np.zeros((5, 1)); Y[0, 0] = np.cos(th); Y[1, 0] = np.sin(th)
        assert abs(oracle.principal_angle_max(X, Y) - th) <= 1e-15 + 1e-12 * th
    # same subspace, rotated basis -> 0
    rng = np.random.default_rng(3)
    X, _ = np.linalg.qr(rng.standard_normal((40, 6)))
    Rot, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    assert oracle.principal_angle_max(X, X @ Rot) < 1e-14
