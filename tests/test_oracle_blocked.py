"""Pins of the oracle's Randomized PCA with the rank grown in blocks
(orc_rsvd_blocked: Martinsson & Voronin 2016, blocked range finder with power
steps, stopping on the criterion of Sec. 2.4) against what the mathematics
fixes, independent of the routine's own arithmetic:

- one block is the Randomized PCA of Sec. 3.1.2 with the same sketch
  (orc_rsvd, itself pinned in test_oracle_rsvd.py);
- when rank(A) is a multiple of the block, the blocks span range(A) and the
  values are the exact singular values (numpy's LAPACK SVD as the reference);
- the captured energy ||Q^T A||_F^2 equals the sum of the squared values of
  T = A^T Q (an SVD identity), grows block by block and never passes
  ||A||_F^2 (Eq. sumeigen); the block that stops the growth is the first
  whose energy reaches t ||A||_F^2;
- the returned factors are orthonormal (so is the basis Q, U = Q W), the
  values interlace the exact ones, and on a separated spectrum K is the
  exact K of Sec. 2.4.
"""
import numpy as np
import pytest

import oracle
import synth


def blocks(seed, n, b, nb):
    return np.concatenate([synth.gaussian_omega(seed + 1000 * j, n, b) for j in range(nb)], axis=1)


def test_one_block_is_randomized_pca():
    A = synth.spiked_noisy(3, 400, 60, 0.9 ** np.arange(60), 1e-3)
    b, q = 16, 2
    G = blocks(5, 60, b, 3)
    r = oracle.rsvd_blocked(A, G, b, q, 0.05, 48, 12)        # t reached by the first block
    assert r.L == b and len(r.energy) == 1
    ref = oracle.rsvd(A, G[:, :b], 12, b - 12, q, 0.05)
    assert np.max(np.abs(r.S - ref.S) / ref.S) <= 1e-12
    assert oracle.principal_angle_max(ref.V, r.V) <= 1e-10
    assert oracle.principal_angle_max(ref.U, r.U) <= 1e-10
    assert r.K == ref.K


def test_exact_recovery_at_three_blocks():
    m, n, b = 300, 50, 8
    sig = np.concatenate([np.logspace(0, -3, 3 * b), np.zeros(n - 3 * b)])
    A = synth.low_rank(7, m, n, sig, centre=False)
    G = blocks(11, n, b, 5)
    r = oracle.rsvd_blocked(A, G, b, 0, 1.0 - 1e-12, 40, 3 * b)
    assert r.L == 3 * b
    s_exact = np.linalg.svd(A, compute_uv=False)[:3 * b]
    assert np.max(np.abs(r.S - s_exact) / s_exact) <= 1e-10
    assert abs(r.energy[-1] - oracle.fro2(A)) <= 1e-12 * oracle.fro2(A)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_energy_identity_monotone_and_stopping(q):
    m, n, b, t = 500, 80, 6, 0.93
    A = synth.spiked_noisy(9, m, n, np.arange(1, n + 1) ** -0.7, 1e-4)
    G = blocks(13, n, b, 12)
    r = oracle.rsvd_blocked(A, G, b, q, t, 72, 72)
    f2 = oracle.fro2(A)
    e = r.energy
    assert np.all(np.diff(e) > 0) and e[-1] <= f2 * (1 + 1e-12)
    # the growth stopped at the first block reaching t (or at the cap)
    assert np.all(e[:-1] < t * f2)
    assert e[-1] >= t * f2 or r.L + b > 72
    # ||T||_F^2 = sum of the squared values of T (all L are returned here)
    assert len(r.S) == r.L
    assert abs(np.sum(r.S ** 2) - e[-1]) <= 1e-12 * e[-1]
    # orthonormal factors, interlacing with the exact values
    assert np.abs(r.U.T @ r.U - np.eye(r.L)).max() <= 1e-12
    assert np.abs(r.V.T @ r.V - np.eye(r.L)).max() <= 1e-12
    s_exact = np.linalg.svd(A, compute_uv=False)
    assert np.all(r.S <= s_exact[:r.L] * (1 + 1e-12))


def test_k_matches_exact_criterion():
    # geometric spectrum: power steps make the captured values exact to
    # rounding where K falls, so K is the exact K of Sec. 2.4
    m, n, b, t = 600, 90, 10, 0.9
    sig = 0.85 ** np.arange(n)
    A = synth.low_rank(17, m, n, sig)
    G = blocks(19, n, b, 8)
    r = oracle.rsvd_blocked(A, G, b, 2, t, 80, 80)
    K_exact, _ = oracle.select_k(np.linalg.svd(A, compute_uv=False), oracle.fro2(A), t)
    assert r.K == K_exact and r.status == oracle.OK
    assert r.L >= K_exact


def test_cap_and_arguments():
    A = synth.low_rank(23, 200, 40, np.ones(40))               # flat: t = 0.99 needs all 40
    G = blocks(29, 40, 8, 5)
    r = oracle.rsvd_blocked(A, G, 8, 1, 0.99, 24, 10)          # stops at the 24-column cap
    assert r.L == 24 and r.K == 10 and r.status == oracle.WARN_THRESHOLD
    assert len(r.S) == 10
    with pytest.raises(RuntimeError):
        oracle.rsvd_blocked(A, G, 0, 1, 0.9, 24, 10)
    with pytest.raises(RuntimeError):
        oracle.rsvd_blocked(A, G, 8, 1, 1.5, 24, 10)
