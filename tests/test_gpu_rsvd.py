"""End-to-end parity of rsvd_solve / rsvd_solve_omega (Randomized PCA, paper
Sec. 3.1.2) against the oracle on identical inputs: the same stored A and the
same sketch G rounded to the compute dtype.

Tolerances: relative singular-value error <= 1e-10 for the FP64 path and
<= 1e-4 for the FP32 path, largest principal angle between the computed and
the oracle's top-k subspaces <= 1e-3 rad (U and V), K equal.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import EPS64, align_columns, announce, dev, host, rounded, sign_rule_holds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1906_12085_amd as rs  # noqa: E402

SIG_TOL = {torch.float64: 1e-10, torch.float32: 1e-4}
ANGLE_TOL = 1e-3


@pytest.fixture(scope="module")
def plans():
    out = {dt: rs.Plan(40000, 300, 96, dt, want_gram=False, seed=202) for dt in (torch.float64, torch.float32)}
    yield out
    for p in out.values():
        p.close()


def run_pair(plan, A0, dt, k, p, q, t, omega_seed, lda_pad=0):
    """GPU solve with a given G and the oracle on the same rounded inputs."""
    m, n = A0.shape
    l = min(k + p, n)
    A0 = rounded(A0, dt)
    G = synth.gaussian_omega(omega_seed, n, l)
    Abig = dev(np.pad(A0, ((0, 0), (0, lda_pad))), dt)
    res = plan.solve(Abig[:, :n], k, p, q, t, omega=dev(G, torch.float64))
    ref = oracle.rsvd(A0, rounded(G, dt), k, p, q, t)
    return res, ref, A0


def check_parity(res, ref, dt, k, check_vectors_exact=False):
    S, U, V = host(res.S), host(res.U), host(res.V)
    assert np.all(np.isfinite(S)) and np.all(np.isfinite(U)) and np.all(np.isfinite(V))
    rel = np.max(np.abs(S - ref.S) / ref.S)
    assert rel <= SIG_TOL[dt], rel
    assert oracle.principal_angle_max(ref.V, V) <= ANGLE_TOL
    assert oracle.principal_angle_max(ref.U, U) <= ANGLE_TOL
    assert res.K == ref.K
    assert sign_rule_holds(V)
    if check_vectors_exact:
        assert np.abs(align_columns(V, ref.V) - ref.V).max() <= 1e-8
        assert np.abs(align_columns(U, ref.U) - ref.U).max() <= 1e-8


def test_config1_fp64_parity(plans):
    c = synth.CONFIG1
    announce("rsvd config1 fp64 2000x200 k=20 p=10 q=2")
    A0 = synth.config1(c["seed"])
    res, ref, _ = run_pair(plans[torch.float64], A0, torch.float64, c["k"], c["p"], c["q"], c["t"],
                           c["omega_seed"])
    assert res.status == rs.RSVD_OK and res.K == 10
    check_parity(res, ref, torch.float64, c["k"], check_vectors_exact=True)


def test_config1_seeded_sketch_equals_supplied(plans):
    # rsvd_solve draws G from the plan seed with the same published generator
    c = synth.CONFIG1
    announce("rsvd config1 seeded vs supplied sketch")
    A0 = synth.config1(c["seed"])
    plan = plans[torch.float64]  # seed 202
    A = dev(A0, torch.float64)
    r1 = plan.solve(A, c["k"], c["p"], c["q"], c["t"])
    G = synth.gaussian_omega(202, A0.shape[1], c["k"] + c["p"])
    r2 = plan.solve(A, c["k"], c["p"], c["q"], c["t"], omega=dev(G, torch.float64))
    assert np.max(np.abs(host(r1.S) - host(r2.S)) / host(r2.S)) <= 1e-12
    assert np.abs(host(r1.V) - host(r2.V)).max() <= 1e-10


def test_fp32_parity_noisy_spectrum(plans):
    # the 1e6 x 512 FP32 recipe (sigma_i = 1/i plus N(0, 1e-3) noise) at a size
    # the oracle finishes in seconds
    announce("rsvd fp32 20000x128 k=16 p=8 q=2 sigma=1/i noise 1e-3")
    A0 = synth.spiked_noisy(12, 20000, 128, synth.config2_sigma(128), 1e-3)
    res, ref, _ = run_pair(plans[torch.float32], A0, torch.float32, 16, 8, 2, 0.95, 77)
    check_parity(res, ref, torch.float32, 16)
    assert res.status == ref.status


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("m,n,k,p,q,pad", [
    (1037, 203, 10, 5, 1, 0),     # ragged m, odd n, odd l
    (1000, 200, 20, 0, 0, 4),     # p = 0, q = 0, padded lda
    (500, 24, 24, 8, 1, 0),       # k = n, l clamped to n
    (4097, 96, 30, 66, 2, 0),     # l = n = 96 (largest l)
    (33, 33, 1, 2, 3, 0),         # square, k = 1
])
def test_edge_shapes(plans, dt, m, n, k, p, q, pad):
    announce(f"rsvd edge {dt} m={m} n={n} k={k} p={p} q={q} pad={pad}")
    sigma = np.logspace(0, -2, n)
    A0 = synth.low_rank(m + n, m, n, sigma)
    res, ref, _ = run_pair(plans[dt], A0, dt, k, p, q, 0.9, 5, lda_pad=pad)
    check_parity(res, ref, dt, k)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_status_words(plans, dt):
    plan = plans[dt]
    announce(f"rsvd status words {dt}")
    n = 20
    # zero matrix: K = 0, RSVD_WARN_ZERO_MATRIX, S = 0
    res = plan.solve(torch.zeros(100, n, dtype=dt, device="cuda"), 4, 2, 1, 0.9)
    assert res.status == rs.RSVD_WARN_ZERO_MATRIX and res.K == 0
    assert np.all(host(res.S) == 0)
    # a NaN in A: RSVD_ERR_NONFINITE
    A = torch.randn(100, n, dtype=dt, device="cuda")
    A[3, 4] = float("nan")
    res = plan.solve(A, 4, 2, 1, 0.9)
    assert res.status == rs.RSVD_ERR_NONFINITE
    # exactly rank-one sketch: a single nonzero entry of A and a +-1 sketch
    # make the second Cholesky pivot exactly zero -> RSVD_ERR_BREAKDOWN
    A = torch.zeros(100, n, dtype=dt, device="cuda")
    A[0, 0] = 1.0
    G = torch.from_numpy(np.where(np.arange(n * 6).reshape(n, 6) % 3 == 0, 1.0, -1.0)).cuda()
    res = plan.solve(A, 4, 2, 0, 0.9, omega=G)
    assert res.status == rs.RSVD_ERR_BREAKDOWN
    # threshold not reached within k values: K = k, RSVD_WARN_THRESHOLD
    A0 = synth.low_rank(9, 300, n, np.ones(n))
    res = plan.solve(dev(A0, dt), 4, 2, 1, 0.99)
    assert res.status == rs.RSVD_WARN_THRESHOLD and res.K == 4
    # the status word is cleared by reading it
    assert plan.status() == rs.RSVD_OK


def test_argument_errors(plans):
    plan = plans[torch.float64]
    A = torch.zeros(100, 20, dtype=torch.float64, device="cuda")
    with pytest.raises(rs.RSVDError) as e:
        plan.solve(A, 21, 0, 0, 0.9)            # k > n
    assert e.value.code == rs.RSVD_ERR_ARG
    with pytest.raises(rs.RSVDError) as e:
        plan.solve(A, 4, 2, 0, 1.5)             # t outside (0, 1]
    assert e.value.code == rs.RSVD_ERR_ARG
    with pytest.raises(rs.RSVDError) as e:
        plan.solve(torch.zeros(100, 200, dtype=torch.float64, device="cuda"), 90, 10, 0, 0.9)  # l = 100 > 96
    assert e.value.code == rs.RSVD_ERR_SHAPE
    with pytest.raises(rs.RSVDError) as e:
        plan.solve(torch.zeros(10, 20, dtype=torch.float64, device="cuda"), 4, 0, 0, 0.9)  # m < n
    assert e.value.code == rs.RSVD_ERR_SHAPE


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_deterministic(plans, dt):
    announce(f"rsvd determinism {dt}")
    A0 = synth.spiked_noisy(3, 9000, 100, synth.config2_sigma(100), 1e-3)
    A = dev(rounded(A0, dt), dt)
    r1 = plans[dt].solve(A, 12, 8, 2, 0.95)
    r2 = plans[dt].solve(A, 12, 8, 2, 0.95)
    assert torch.equal(r1.U, r2.U) and torch.equal(r1.V, r2.V) and torch.equal(r1.S, r2.S)


def test_small_svd_wide_value_range(plans):
    # The solves form the small SVD's right factor from Uo S^-1 unless the
    # values of T span more than six decades; then the decomposition is
    # repeated with the rotations accumulated (diag[5] = 1).  Both sides of
    # that switch are held to the FP64 parity gates.  (A spread of T past
    # 1e6 means the same of the sketch Y, which only the FP64 path's
    # CholeskyQR2 orthonormalises.)
    dt = torch.float64
    plan = plans[dt]
    m, n, k, p, q = 3000, 64, 12, 12, 0
    rng = np.random.default_rng(71)
    for decades, redo in ((3.0, 0.0), (7.0, 1.0)):
        announce(f"rsvd small-SVD values over {decades:g} decades {dt}")
        sig = np.concatenate([np.logspace(0, -decades, k + p),
                              10.0 ** -decades * np.logspace(-0.1, -1, n - k - p)])
        A0 = synth.haar(rng, m, n) @ np.diag(sig) @ synth.haar(rng, n, n).T
        res, ref, _ = run_pair(plan, A0, dt, k, p, q, 0.999, 13)
        assert plan.diag()[5] == redo
        check_parity(res, ref, dt, k)
