"""Continuous batching (rsvd_server_*): requests submitted while others run
are admitted as slots and budget free up; every result must equal, bit for
bit, the same problem solved alone on a plan of the same sizes and seed, and
pass the oracle's parity gates (relative sigma error <= 1e-4 for FP32,
principal angles <= 1e-3 rad, K and status equal)."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev, host, rounded

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1906_12085_amd as rs  # noqa: E402

SEED = 505
M_MAX, N_MAX, L_MAX = 20000, 128, 40


def requests(dt, count, seed):
    """m log-uniform in [1000, 20000] (multiples of 64), n in {32, 64, 128},
    sigma_i = i^-alpha with alpha in [0.5, 2], t in {0.9, 0.95, 0.99}: the
    serving workload's recipe at test sizes."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice([32, 64, 128]))
        m = max(n, int(np.exp(rng.uniform(np.log(1000), np.log(M_MAX))) // 64 * 64))
        alpha = rng.uniform(0.5, 2.0)
        sig = np.arange(1, n + 1, dtype=np.float64) ** -alpha
        A0 = rounded(synth.haar(rng, m, n) @ np.diag(sig) @ synth.haar(rng, n, n).T, dt)
        t = float(rng.choice([0.9, 0.95, 0.99]))
        out.append((dev(A0, dt), min(16, n // 4), 8, 2, t, A0))
    return out


def poll(sv, pending, seen_running):
    """One progress call: drop the finished tickets from `pending` (the
    server reports each finished ticket once)."""
    done, queued, running = sv.progress()
    seen_running.append(running)
    for tk in done:
        pending.discard(tk)
    return queued, running


def drain(sv, pending, seen_running, limit_s=60.0):
    t0 = time.monotonic()
    while pending:
        queued, running = poll(sv, pending, seen_running)
        assert time.monotonic() - t0 < limit_s, (sorted(pending), queued, running)


def test_serve_same_alone_and_in_mix():
    dt = torch.float32
    announce("serve: 14 requests arriving in waves on 3 slots")
    reqs = requests(dt, 14, 3)
    sv = rs.Server(3, M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    tickets, pending, seen = [], set(), []
    for i, (A, k, p, q, t, _) in enumerate(reqs):
        tk = sv.submit(A, k, p, q, t)
        tickets.append(tk)
        pending.add(tk)
        poll(sv, pending, seen)
        if i % 4 == 3:                     # let the first waves finish partly
            time.sleep(0.002)
    drain(sv, pending, seen)
    assert tickets == list(range(len(reqs)))
    assert max(seen) > 1                   # requests ran side by side
    alone = rs.Plan(M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    for tk, (A, k, p, q, t, A0) in zip(tickets, reqs):
        o = sv.results[tk]
        ref = alone.solve(A, k, p, q, t)
        assert torch.equal(o["S"], ref.S) and torch.equal(o["U"], ref.U)
        assert torch.equal(o["V"], ref.V)
        assert int(o["K"].item()) == ref.K and int(o["status"].item()) == ref.status
        m, n = A.shape
        G = rounded(synth.gaussian_omega(SEED, n, min(k + p, n)), dt)
        orc = oracle.rsvd(A0, G, k, p, q, t)
        assert np.max(np.abs(host(o["S"]) - orc.S) / orc.S) <= 1e-4
        assert oracle.principal_angle_max(orc.V, host(o["V"])) <= 1e-3
        assert oracle.principal_angle_max(orc.U, host(o["U"])) <= 1e-3
        assert int(o["K"].item()) == orc.K and int(o["status"].item()) == orc.status
    alone.close()
    sv.close()


@pytest.mark.parametrize("budget_requests,limit", [(0.5, 1), (2.2, 2)])
def test_serve_budget_admission(budget_requests, limit):
    # identical 6000 x 64 requests: the budget holds half of one (each runs
    # alone) or a bit over two (at most two run at once) of their footprints
    dt = torch.float32
    announce(f"serve: budget of {budget_requests} requests, at most {limit} running")
    m, n, k, p, q = 6000, 64, 8, 8, 2
    l = k + p
    rng = np.random.default_rng(9)
    A0 = rounded(synth.haar(rng, m, n) @ np.diag(np.arange(1, n + 1.0) ** -1.0)
                 @ synth.haar(rng, n, n).T, dt)
    A = dev(A0, dt)
    # footprint as the server counts it: A, two m x l panels, the A^T Q
    # partials (min(256, ceil(m / 64)) splits of n x l FP64)
    splits = min(256, (m + 63) // 64)
    foot = m * n * 4 + 2 * m * l * 4 + splits * n * l * 8
    sv = rs.Server(4, M_MAX, N_MAX, L_MAX, dt, seed=SEED, hbm_budget=int(budget_requests * foot))
    pending, seen = set(), []
    for _ in range(6):
        pending.add(sv.submit(A, k, p, q, 0.9))
        poll(sv, pending, seen)
    drain(sv, pending, seen)
    assert max(seen) <= limit
    first = sv.results[0]
    for tk in range(1, 6):
        o = sv.results[tk]
        assert torch.equal(o["S"], first["S"]) and torch.equal(o["V"], first["V"])
        assert torch.equal(o["U"], first["U"])
    sv.close()


def test_serve_arguments():
    dt = torch.float32
    sv = rs.Server(2, 4000, 64, 24, dt, seed=1)
    A = torch.zeros((1000, 64), dtype=dt, device="cuda")
    with pytest.raises(rs.RSVDError) as ei:
        sv.submit(A, 20, 8, 1, 0.9)                    # l = 28 > l_max = 24
    assert ei.value.code == rs.RSVD_ERR_SHAPE
    with pytest.raises(rs.RSVDError) as ei:
        sv.submit(A, 4, 2, 1, 1.5)                     # t outside (0, 1]
    assert ei.value.code == rs.RSVD_ERR_ARG
    done, queued, running = sv.progress()
    assert done == [] and queued == 0 and running == 0
    assert sv.submit(A, 4, 2, 1, 0.9) == 0             # rejected requests take no ticket
    sv.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_serve_low_precision_same_alone_and_oracle(fmt):
    # A stored in bfloat16 / FP8 E4M3 with power-of-two column scales: every
    # result equals rsvd_solve_bf16 / _fp8 alone on a plan of the same sizes
    # and seed, and passes the FP32 gates against the oracle on the
    # dequantised stored matrix
    storage = torch.bfloat16 if fmt == "bf16" else torch.float8_e4m3fn
    announce(f"serve: 8 {fmt} requests on 3 slots")
    reqs = requests(torch.float32, 8, 17)
    quant = rs.Plan(M_MAX, N_MAX, L_MAX, storage, seed=SEED)
    stored = []
    for A, k, p, q, t, _ in reqs:
        Aq, s = quant.quantize(A)
        stored.append((Aq, s, k, p, q, t))
    torch.cuda.synchronize()
    sv = rs.Server(3, M_MAX, N_MAX, L_MAX, storage, seed=SEED)
    pending, seen = set(), []
    tickets = []
    for Aq, s, k, p, q, t in stored:
        tickets.append(sv.submit(Aq, k, p, q, t, col_scale=s))
        pending.add(tickets[-1])
        poll(sv, pending, seen)
    drain(sv, pending, seen)
    for tk, (Aq, s, k, p, q, t) in zip(tickets, stored):
        o = sv.results[tk]
        ref = quant.solve(Aq, k, p, q, t, col_scale=s)
        assert torch.equal(o["S"], ref.S) and torch.equal(o["U"], ref.U)
        assert torch.equal(o["V"], ref.V)
        assert int(o["K"].item()) == ref.K and int(o["status"].item()) == ref.status
        n = Aq.shape[1]
        A64 = (Aq.double() * s.double()[None, :]).cpu().numpy()
        G = rounded(synth.gaussian_omega(SEED, n, min(k + p, n)), torch.float32)
        orc = oracle.rsvd(A64, G, k, p, q, t)
        assert np.max(np.abs(host(o["S"]) - orc.S) / orc.S) <= 1e-4
        assert oracle.principal_angle_max(orc.V, host(o["V"])) <= 1e-3
        assert oracle.principal_angle_max(orc.U, host(o["U"])) <= 1e-3
        assert int(o["K"].item()) == orc.K and int(o["status"].item()) == orc.status
    sv.close()
    quant.close()


def test_serve_adaptive_rank():
    # with k_max the rank grows in blocks of k + p columns while t is not
    # reached: each result equals rsvd_solve_adaptive alone on a plan of the
    # same sizes and seed (bit for bit) and the oracle's blocked routine on
    # the same block sketches
    dt = torch.float32
    announce("serve: adaptive rank, 6 requests, blocks of 12 growing up to k_max = 32")
    reqs = requests(dt, 6, 23)
    sv = rs.Server(3, M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    pending, seen, tickets = set(), [], []
    for A, _, p, q, t, _ in reqs:
        tickets.append(sv.submit(A, 4, p, q, t, k_max=32))
        pending.add(tickets[-1])
        poll(sv, pending, seen)
    drain(sv, pending, seen)
    alone = rs.Plan(M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    grew = 0
    step = 0x9E3779B97F4A7C15
    for tk, (A, _, p, q, t, A0) in zip(tickets, reqs):
        n = A.shape[1]
        ref = alone.solve_adaptive(A, 4, p, q, t, 32)
        L = int(alone.diag()[6])
        grew += L > 4 + p
        o = sv.results[tk]
        kc = min(32, L)
        assert int(o["K"].item()) == ref.K and int(o["status"].item()) == ref.status
        assert torch.equal(o["S"][:kc], ref.S[:kc]) and torch.equal(o["V"][:, :kc], ref.V[:, :kc])
        assert torch.equal(o["U"][:, :kc], ref.U[:, :kc])
        b = min(4 + p, n)
        G = np.concatenate([synth.gaussian_omega((SEED + j * step) % (1 << 64), n, b)
                            for j in range(L_MAX // b)], axis=1)
        orc = oracle.rsvd_blocked(A0, rounded(G, dt), b, q, t, L_MAX, 32)
        assert orc.L == L
        assert np.max(np.abs(host(o["S"])[:kc] - orc.S) / orc.S) <= 1e-4
        assert oracle.principal_angle_max(orc.V, host(o["V"])[:, :kc]) <= 1e-3
        assert int(o["K"].item()) == orc.K and int(o["status"].item()) == orc.status
    assert grew >= 2                            # the case is exercised
    alone.close()
    sv.close()


def test_serve_mixed_storage():
    # one fp32 server, requests alternating fp32 and bfloat16 / FP8 storage:
    # every result equals the solve alone on a plan of that storage with the
    # same sizes and seed, bit for bit
    announce("serve: 9 requests, fp32 / bf16 / fp8 storage on one server")
    reqs = requests(torch.float32, 9, 41)
    plans = {fmt: rs.Plan(M_MAX, N_MAX, L_MAX, fmt, seed=SEED)
             for fmt in (torch.float32, torch.bfloat16, torch.float8_e4m3fn)}
    sv = rs.Server(3, M_MAX, N_MAX, L_MAX, torch.float32, seed=SEED)
    pending, seen, sub = set(), [], []
    fmts = [torch.float32, torch.bfloat16, torch.float8_e4m3fn]
    for i, (A, k, p, q, t, _) in enumerate(reqs):
        fmt = fmts[i % 3]
        if fmt == torch.float32:
            Aq, s = A, None
        else:
            Aq, s = plans[fmt].quantize(A)
            torch.cuda.synchronize()
        tk = sv.submit(Aq, k, p, q, t, col_scale=s)
        sub.append((tk, fmt, Aq, s, k, p, q, t))
        pending.add(tk)
        poll(sv, pending, seen)
    drain(sv, pending, seen)
    assert max(seen) > 1
    for tk, fmt, Aq, s, k, p, q, t in sub:
        o = sv.results[tk]
        ref = plans[fmt].solve(Aq, k, p, q, t, col_scale=s)
        assert torch.equal(o["S"], ref.S) and torch.equal(o["U"], ref.U)
        assert torch.equal(o["V"], ref.V)
        assert int(o["K"].item()) == ref.K and int(o["status"].item()) == ref.status
    for pl in plans.values():
        pl.close()
    sv.close()


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
def test_serve_gram_fallback(fmt):
    # slow decay (sigma_i = i^-0.5) at t = 0.99 needs K ~ 0.9 n: the growth
    # predicts K past n / 2 (or fills the 40-column sketch) and the request
    # moves to the A^T A-route slot, whose result equals gram_eig_solve alone
    # (the first k_max = n triplets; a bfloat16 A dequantised); fast decay
    # (i^-2, t = 0.9) finishes on its slot.  No request ends short of t.
    announce(f"serve: A^T A fallback, {fmt} storage")
    rng = np.random.default_rng(61)
    sv = rs.Server(2, M_MAX, N_MAX, L_MAX, torch.float32, seed=SEED, gram_fallback=True)
    quant = rs.Plan(M_MAX, N_MAX, L_MAX, torch.bfloat16, seed=SEED)
    gram = rs.Plan(M_MAX, N_MAX, 8, torch.float32, want_gram=True, seed=SEED)
    alone = rs.Plan(M_MAX, N_MAX, L_MAX, torch.float32, seed=SEED)
    pending, seen, sub = set(), [], []
    for i, (alpha, t) in enumerate([(0.5, 0.99), (2.0, 0.9), (0.5, 0.99), (1.5, 0.95)]):
        m, n = 4096 + 1024 * i, 128
        sig = np.arange(1, n + 1, dtype=np.float64) ** -alpha
        A0 = synth.haar(rng, m, n) @ np.diag(sig) @ synth.haar(rng, n, n).T
        A = dev(A0.astype(np.float32), torch.float32)
        if fmt == "bf16":
            Aq, s = quant.quantize(A)
            torch.cuda.synchronize()
            A32 = (Aq.float() * s[None, :]).contiguous()
        else:
            Aq, s, A32 = A, None, A
        tk = sv.submit(Aq, 4, 8, 2, t, col_scale=s, k_max=n)
        sub.append((tk, alpha, t, Aq, s, A32))
        pending.add(tk)
        poll(sv, pending, seen)
    drain(sv, pending, seen)
    for tk, alpha, t, Aq, s, A32 in sub:
        o = sv.results[tk]
        n = Aq.shape[1]
        assert int(o["status"].item()) == rs.RSVD_OK
        if alpha == 0.5:
            ref = gram.gram_eig(A32, t, ucols=n)
            assert int(o["K"].item()) == ref.K > n // 2
            assert torch.equal(o["S"], ref.S[:n]) and torch.equal(o["V"], ref.V[:, :n])
            assert torch.equal(o["U"], ref.U)
        else:
            ref = alone.solve_adaptive(Aq, 4, 8, 2, t, n) if s is None else None
            if ref is not None:
                L = int(alone.diag()[6])
                assert int(o["K"].item()) == ref.K <= L
                assert torch.equal(o["S"][:L], ref.S[:L]) and torch.equal(o["V"][:, :L], ref.V[:, :L])
    for pl in (quant, gram, alone):
        pl.close()
    sv.close()


def test_serve_without_u():
    # requests that ask for S, V and K only: the same values as with U, bit
    # for bit, through all three routes (fixed rank, growth, A^T A fallback)
    announce("serve: requests without U")
    reqs = requests(torch.float32, 6, 71)
    sv = rs.Server(3, M_MAX, N_MAX, L_MAX, torch.float32, seed=SEED, gram_fallback=True)
    pending, seen, pairs = set(), [], []
    for i, (A, k, p, q, t, _) in enumerate(reqs):
        k_max = 0 if i % 2 == 0 else A.shape[1]
        kk = 4 if k_max else k
        a = sv.submit(A, kk, p, q, t, k_max=k_max)
        b = sv.submit(A, kk, p, q, t, k_max=k_max, want_u=False)
        pairs.append((a, b))
        pending.update((a, b))
        poll(sv, pending, seen)
    drain(sv, pending, seen)
    for a, b in pairs:
        oa, ob = sv.results[a], sv.results[b]
        assert ob["U"] is None
        # a growing request writes its first min(k_max, L) columns (S starts
        # at zero in the binding; V's unwritten columns are undefined)
        assert torch.equal(oa["S"], ob["S"])
        c = int(torch.nonzero(oa["S"]).max()) + 1
        assert torch.equal(oa["V"][:, :c], ob["V"][:, :c])
        assert torch.equal(oa["K"], ob["K"]) and torch.equal(oa["status"], ob["status"])
    sv.close()
