"""Pins of the oracle's Krylov method (Sec. 3.1.1) against facts the method
and linear algebra fix, not against itself:

* exact recovery: for rank(A) = (i+1) l the Krylov space of dimension
  (i+1) l holds the whole range, so the values are the exact ones, while
  Randomized PCA with the same l and q = i is not exact (a dropped or
  misplaced block would give Randomized PCA's accuracy);
* the Krylov space contains Randomized PCA's final range (AA^T)^i A G, so its
  Ritz values lie between Randomized PCA's and the exact ones;
* Rayleigh-Ritz: U~^T A V~ = diag(s~) with orthonormal U~ and V~;
* i = 0 is Randomized PCA with q = 0 on the same G.
"""
import numpy as np

import oracle
import synth


def lowrank(rng, m, n, r, decay=0.7):
    s = decay ** np.arange(r)
    return synth.haar(rng, m, r) @ np.diag(s) @ synth.haar(rng, n, r).T, s


def test_exact_recovery_at_full_krylov_rank():
    rng = np.random.default_rng(3)
    m, n, k, p, i = 300, 60, 6, 2, 1
    l = k + p
    A, s = lowrank(rng, m, n, (i + 1) * l)
    G = synth.gaussian_omega(11, n, l)
    kr = oracle.krylov(A, G, k, p, i, 0.99)
    assert np.max(np.abs(kr.S - s[:k]) / s[:k]) <= 1e-10
    rp = oracle.rsvd(A, G, k, p, i, 0.99)
    assert np.max(np.abs(rp.S - s[:k]) / s[:k]) > 1e-8       # not exact without the blocks


def test_ritz_values_between_rsvd_and_exact():
    rng = np.random.default_rng(5)
    m, n = 400, 80
    A = synth.haar(rng, m, n) @ np.diag(1.0 / np.arange(1, n + 1)) @ synth.haar(rng, n, n).T
    exact = oracle.svd(A)[1]
    for k, p, i in [(5, 3, 1), (8, 4, 2), (4, 0, 3)]:
        G = synth.gaussian_omega(k + 7 * i, n, k + p)
        kr = oracle.krylov(A, G, k, p, i, 0.99)
        rp = oracle.rsvd(A, G, k, p, i, 0.99)
        tol = 1e-12 * exact[0]
        assert np.all(kr.S >= rp.S - tol)
        assert np.all(kr.S <= exact[:k] + tol)


def test_rayleigh_ritz_identity():
    rng = np.random.default_rng(7)
    m, n, k, p, i = 250, 50, 5, 3, 2
    A = rng.standard_normal((m, n))
    G = synth.gaussian_omega(1, n, k + p)
    kr = oracle.krylov(A, G, k, p, i, 0.99)
    assert np.abs(kr.U.T @ kr.U - np.eye(k)).max() <= 1e-12
    assert np.abs(kr.V.T @ kr.V - np.eye(k)).max() <= 1e-12
    assert np.abs(kr.U.T @ A @ kr.V - np.diag(kr.S)).max() <= 1e-12 * kr.S[0]
    assert np.all(np.diff(kr.S) <= 0)


def test_no_power_blocks_is_randomized_pca_q0():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((200, 40))
    G = synth.gaussian_omega(2, 40, 10)
    kr = oracle.krylov(A, G, 6, 4, 0, 0.9)
    rp = oracle.rsvd(A, G, 6, 4, 0, 0.9)
    assert np.max(np.abs(kr.S - rp.S) / rp.S) <= 1e-12
    assert kr.K == rp.K


def test_krylov_space_wider_than_n_is_rejected():
    A = np.ones((50, 10))
    G = synth.gaussian_omega(2, 10, 6)
    try:
        oracle.krylov(A, G, 4, 2, 1, 0.9)                 # 2 * 6 = 12 > 10 columns
    except RuntimeError:
        return
    raise AssertionError("expected the oracle to reject (i+1) l > n")
