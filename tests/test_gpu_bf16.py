"""Parity of the low-precision storage paths (plan dtypes RSVD_BF16 and
RSVD_FP8) against the oracle.

The matrix is Aq diag(s), Aq bfloat16 or OCP FP8 E4M3 and s power-of-two
column scales; the oracle runs in FP64 on that dequantised stored matrix
(exact: a bf16 or E4M3 value times a power of two is an FP64 number), so what
is checked is the computation, not the storage rounding.  E4M3 values are
widened to bfloat16 exactly, so both formats share the bounds below.

Bounds: a bf16 x bf16 product is exact in FP32; the right factor x is held
as hi + lo with |x - (hi + lo)| <= 2^-17 |x|; sums are FP32 inside a row
block (n or the split's rows terms) -- so a product entry is within
(2^-16 + 2 n 2^-24) sum|a_k x_k|.  The end-to-end solve has the FP32 path's
tolerances (sigma <= 1e-4 relative, largest principal angle <= 1e-3 rad,
K equal).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import EPS64, U32, announce, dev, host, sign_rule_holds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1906_12085_amd as rs  # noqa: E402

HILO = 2.0 ** -16


FORMATS = {"bf16": torch.bfloat16, "fp8": torch.float8_e4m3fn}


def stored(x, fmt=torch.bfloat16):
    """Round an FP64/FP32 array to the storage format (nearest even) as a CPU
    tensor (torch's own conversions: an implementation independent of the
    library's)."""
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.float32).to(fmt)



def deq(Aq_cpu, s=None):
    A = Aq_cpu.to(torch.float64).numpy()
    return A if s is None else A * np.asarray(s, dtype=np.float64)[None, :]


@pytest.fixture(scope="module", params=list(FORMATS))
def plan(request):
    p = rs.Plan(40000, 600, 96, FORMATS[request.param], seed=5)
    yield p
    p.close()


NN_CASES = [
    (1037, 200, 80, 0),    # last 64-wide chunk holds one 32-deep step (8 of 32 columns)
    (2049, 512, 80, 0),    # the 1e6 x 512 pass shape at small m
    (300, 64, 17, 8),      # padded rows, ragged column tile
    (515, 8, 1, 0),        # one k group of 8, one column
    (700, 96, 96, 0),      # l_max columns (6 tiles)
    (4133, 520, 64, 8),    # k tail of 8 past 8 whole chunks, padded rows, ragged rows
    (129, 24, 33, 0),      # one row past a block, 3 column tiles (last ragged)
]


@pytest.mark.parametrize("m,n,c,pad", NN_CASES)
def test_bf16_gemm_nn_parity(plan, m, n, c, pad):
    announce(f"bf16 gemm_nn m={m} n={n} c={c} pad={pad}")
    rng = np.random.default_rng(m + 5 * n + c)
    Aq = stored(rng.standard_normal((m, n)), plan.storage)
    A64 = deq(Aq)
    X0 = rng.standard_normal((n, c)).astype(np.float32)
    Abig = torch.zeros((m, n + pad), dtype=plan.storage)
    Abig[:, :n] = Aq
    if pad:
        Abig[:, n:] = float("nan")          # must not reach Y
    A = Abig.cuda()[:, :n]
    Y = torch.full((m, c), float("nan"), dtype=torch.float32, device="cuda")
    f2 = torch.empty(1, dtype=torch.float64, device="cuda")
    Gm = torch.empty(c, c, dtype=torch.float64, device="cuda")
    rs.rsvd_gemm_nn(plan.handle, A, dev(X0, torch.float32), Y, Gram=Gm, fro2=f2)
    torch.cuda.synchronize()
    X64 = X0.astype(np.float64)
    Yref = oracle.gemm_nn(A64, X64)
    bound = (HILO + 2 * n * U32) * (np.abs(A64) @ np.abs(X64)) + 1e-300
    Yg = host(Y)
    assert np.all(np.abs(Yg - Yref) <= bound)
    f2ref = oracle.fro2(A64)
    assert abs(host(f2)[0] - f2ref) <= 4 * U32 * f2ref
    Gref = oracle.gemm_tn(Yg, Yg)
    assert np.all(np.abs(host(Gm) - Gref) <= 2.0 * m * EPS64 * (np.abs(Yg).T @ np.abs(Yg)))


TN_CASES = [
    (1037, 200, 80),
    (4099, 512, 80),
    (129, 64, 3),          # Q rows of 3 columns (read as 8, the rest dropped)
    (2000, 520, 48),       # two column tiles of A, the second 8 wide
    (70, 16, 1),
    (1000, 96, 96),
    (33, 8, 9),            # one partial row chunk
    (40000, 512, 80),      # 5 chunks per row split (prefetch sets past a whole round)
    (30000, 136, 20),      # 4 chunks per split, a 136-column A in a 512-column tile
]


@pytest.mark.parametrize("m,n,c", TN_CASES)
def test_bf16_gemm_tn_parity(plan, m, n, c):
    announce(f"bf16 gemm_tn m={m} n={n} c={c}")
    rng = np.random.default_rng(3 * m + n + 7 * c)
    Aq = stored(rng.standard_normal((m, n)), plan.storage)
    A64 = deq(Aq)
    Q0 = rng.standard_normal((m, c)).astype(np.float32)
    Z = torch.empty(n, c, dtype=torch.float64, device="cuda")
    rs.rsvd_gemm_tn(plan.handle, Aq.cuda(), dev(Q0, torch.float32), Z)
    torch.cuda.synchronize()
    Q64 = Q0.astype(np.float64)
    Zref = oracle.gemm_tn(A64, Q64)
    bound = (HILO + 2 * m * U32) * (np.abs(A64).T @ np.abs(Q64)) + 1e-300
    assert np.all(np.abs(host(Z) - Zref) <= bound)


def test_bf16_quantize(plan):
    fmt = plan.storage
    announce(f"{fmt} quantize 3000x64, column scales 1e-3..1e3, a zero column, wide-range columns")
    rng = np.random.default_rng(9)
    A0 = (rng.standard_normal((3000, 64)) * 10.0 ** rng.uniform(-3, 3, 64)).astype(np.float32)
    A0[:, 5] = 0.0
    # entries spread over 12 decades: FP8 subnormals and underflow to zero
    A0[:, 7] = (rng.choice([-1.0, 1.0], 3000) * 10.0 ** rng.uniform(-12, 0, 3000)).astype(np.float32)
    A = dev(A0, torch.float32)
    Aq, s = plan.quantize(A)
    torch.cuda.synchronize()
    sg = s.cpu().numpy().astype(np.float64)
    cmax = np.abs(A0).max(axis=0).astype(np.float64)
    e = np.log2(sg)
    assert np.all(e == np.round(e))                      # powers of two
    nz = cmax > 0
    r = cmax[nz] / sg[nz]                                # largest scaled magnitude per column
    if fmt == torch.bfloat16:
        assert np.all(r >= 0.5) and np.all(r < 1.0)      # 2^(e-1) <= max < 2^e
    else:
        assert np.all(r > 224.0) and np.all(r <= 448.0)  # least 2^e with max / 2^e <= 448
    assert sg[5] == 1.0
    ref = stored(A0.astype(np.float64) / sg[None, :], fmt)   # exact division by 2^e
    bits = torch.int16 if fmt == torch.bfloat16 else torch.uint8
    assert torch.equal(Aq.cpu().view(bits), ref.view(bits))


def solve_pair(plan, A0, k, p, q, t, omega_seed, scaled=True):
    m, n = A0.shape
    l = min(k + p, n)
    if scaled:
        Aq, s = plan.quantize(dev(A0.astype(np.float32), torch.float32))
        torch.cuda.synchronize()
        A64 = deq(Aq.cpu(), s.cpu().numpy())
    else:
        # unit scales: the matrix enters the storage format as it is
        A0 = A0 / np.abs(A0).max() * (1.0 if plan.storage == torch.bfloat16 else 400.0)
        Aq, s = stored(A0, plan.storage).cuda(), None
        A64 = deq(Aq.cpu())
    G = synth.gaussian_omega(omega_seed, n, l)
    res = plan.solve(Aq, k, p, q, t, omega=dev(G, torch.float64), col_scale=s)
    ref = oracle.rsvd(A64, G.astype(np.float32).astype(np.float64), k, p, q, t)
    return res, ref


def check(res, ref):
    S, U, V = host(res.S), host(res.U), host(res.V)
    assert np.all(np.isfinite(S)) and np.all(np.isfinite(U)) and np.all(np.isfinite(V))
    assert np.max(np.abs(S - ref.S) / ref.S) <= 1e-4
    assert oracle.principal_angle_max(ref.V, V) <= 1e-3
    assert oracle.principal_angle_max(ref.U, U) <= 1e-3
    assert res.K == ref.K and res.status == ref.status
    assert sign_rule_holds(V)


@pytest.mark.parametrize("scaled", [True, False], ids=["scaled", "unit"])
def test_bf16_rsvd_noisy_spectrum(plan, scaled):
    # the 1e6 x 512 recipe (sigma_i = 1/i plus N(0, 1e-3) noise) at a size the
    # oracle finishes in seconds
    announce(f"bf16 rsvd 20000x128 k=16 p=8 q=2 scaled={scaled}")
    A0 = synth.spiked_noisy(12, 20000, 128, synth.config2_sigma(128), 1e-3)
    res, ref = solve_pair(plan, A0, 16, 8, 2, 0.95, 77, scaled)
    check(res, ref)


@pytest.mark.parametrize("m,n,k,p,q", [
    (1037, 208, 10, 5, 1),     # ragged m, l = 15
    (500, 24, 24, 8, 1),       # k = n, l clamped to n
    (4097, 96, 30, 66, 2),     # l = n = 96
    (33, 32, 1, 2, 3),         # square, k = 1
])
def test_bf16_rsvd_edge_shapes(plan, m, n, k, p, q):
    announce(f"bf16 rsvd edge m={m} n={n} k={k} p={p} q={q}")
    rng = np.random.default_rng(m + n + k)
    A0 = synth.haar(rng, m, n) @ np.diag(np.logspace(0, -2, n)) @ synth.haar(rng, n, n).T
    res, ref = solve_pair(plan, A0, k, p, q, 0.9, 31)
    check(res, ref)


def test_bf16_argument_errors(plan):
    A = torch.zeros((100, 20), dtype=plan.storage, device="cuda")       # n % 8 != 0
    with pytest.raises(rs.RSVDError) as ei:
        plan.solve(A, 4, 2, 1, 0.9)
    assert ei.value.code == rs.RSVD_ERR_ARG
    with pytest.raises(rs.RSVDError):
        rs.Plan(1000, 64, 16, plan.storage, want_gram=True)


def test_bf16_deterministic(plan):
    announce("bf16 rsvd deterministic 5000x64")
    A0 = synth.spiked_noisy(4, 5000, 64, synth.config2_sigma(64), 1e-3)
    Aq, s = plan.quantize(dev(A0.astype(np.float32), torch.float32))
    r1 = plan.solve(Aq, 8, 8, 2, 0.9, col_scale=s)
    r2 = plan.solve(Aq, 8, 8, 2, 0.9, col_scale=s)
    assert torch.equal(r1.S, r2.S) and torch.equal(r1.U, r2.U) and torch.equal(r1.V, r2.V)
