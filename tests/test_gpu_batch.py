"""Batches of Randomized PCA problems of different shapes (rsvd_batch_*).

Each instance of a batch must equal, bit for bit, rsvd_solve of the same
problem on a plan of the same sizes and seed running alone (the slots are
such plans; deterministic kernels and fixed-order reductions make the
results independent of what else runs), and must pass the oracle's parity
gates (same A, the plan's seeded G): relative sigma error <= 1e-10 (FP64) /
1e-4 (FP32), principal angles <= 1e-3 rad, K and the status word equal.  A
captured batch is replayed several times, with eager work in between, and
every replay is compared with the eager batch.  A grouped batch (every step
one launch for all instances) takes longer row splits for its partial sums
than a solve alone, so it is held to the oracle's gates and to FP32 rounding
of the solo solve, and its replays to each other bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev, host, rounded, sign_rule_holds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1906_12085_amd as rs  # noqa: E402

SEED = 404
M_MAX, N_MAX, L_MAX = 12000, 128, 40
SIG_TOL = {torch.float64: 1e-10, torch.float32: 1e-4}


def problems(dt, count, seed):
    """Uneven instances: m in [700, 12000], n in {32, 48, 64, 96, 128},
    k = min(8, n / 4), p = 8, q = 2, sigma_i = exp(-r i) with r in
    [0.01, 0.2] (the batched workload's recipe at test sizes)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice([32, 48, 64, 96, 128]))
        m = int(rng.integers(max(n, 700), M_MAX + 1))
        r = rng.uniform(0.01, 0.2)
        sig = np.exp(-r * np.arange(1, n + 1))
        A0 = synth.haar(rng, m, n) @ np.diag(sig) @ synth.haar(rng, n, n).T
        A0 = rounded(A0, dt)
        out.append((dev(A0, dt), min(8, n // 4), 8, 2, 0.95, A0))
    return out


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batch_equals_alone_and_oracle(dt):
    announce(f"batch of 11 uneven instances on 3 slots {dt}")
    probs = problems(dt, 11, 5 if dt == torch.float64 else 6)
    b = rs.Batch(3, M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    outs = b.solve([pr[:5] for pr in probs])
    torch.cuda.synchronize()
    alone = rs.Plan(M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    for (A, k, p, q, t, A0), o in zip(probs, outs):
        m, n = A.shape
        ref = alone.solve(A, k, p, q, t)
        assert torch.equal(o["S"], ref.S) and torch.equal(o["U"], ref.U)
        assert torch.equal(o["V"], ref.V)
        assert int(o["K"].item()) == ref.K and int(o["status"].item()) == ref.status
        l = min(k + p, n)
        G = rounded(synth.gaussian_omega(SEED, n, l), dt)
        orc = oracle.rsvd(A0, G, k, p, q, t)
        S, U, V = host(o["S"]), host(o["U"]), host(o["V"])
        assert np.max(np.abs(S - orc.S) / orc.S) <= SIG_TOL[dt]
        assert oracle.principal_angle_max(orc.V, V) <= 1e-3
        assert oracle.principal_angle_max(orc.U, U) <= 1e-3
        assert int(o["K"].item()) == orc.K and int(o["status"].item()) == orc.status
        assert sign_rule_holds(V)
    alone.close()
    b.close()


def test_batch_graph_replays():
    dt = torch.float32
    announce("batch graph: capture 9 instances on 4 slots, 3 replays with eager work between")
    probs = problems(dt, 9, 8)
    b = rs.Batch(4, M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    eager = b.solve([pr[:5] for pr in probs])
    torch.cuda.synchronize()
    keep = [{key: o[key].clone() for key in ("U", "S", "V", "K", "status")} for o in eager]
    g = b.graph([pr[:5] for pr in probs])
    other = rs.Plan(M_MAX, N_MAX, L_MAX, dt, seed=SEED + 1)
    for rep in range(3):
        for o in g.outs:                      # the replay must write every output again
            for key in ("U", "S", "V"):
                o[key].fill_(float("nan"))
            o["K"].fill_(-9)
            o["status"].fill_(-99)
        g.launch()
        torch.cuda.synchronize()
        for o, e in zip(g.outs, keep):
            for key in ("U", "S", "V", "K", "status"):
                assert torch.equal(o[key], e[key]), (rep, key)
        A, k, p, q, t, _ = probs[rep]
        other.solve(A, k, p, q, t)            # eager work between replays
        torch.cuda.synchronize()
    g.close()
    other.close()
    b.close()


def test_batch_arguments():
    dt = torch.float64
    b = rs.Batch(2, 4000, 64, 24, dt, seed=1)
    A = torch.zeros((1000, 64), dtype=dt, device="cuda")
    B = torch.zeros((50, 64), dtype=dt, device="cuda")         # m < n
    with pytest.raises(rs.RSVDError) as ei:
        b.solve([(A, 8, 8, 1, 0.9), (B, 8, 8, 1, 0.9)])
    assert ei.value.code == rs.RSVD_ERR_SHAPE
    with pytest.raises(rs.RSVDError) as ei:
        b.solve([(A, 20, 8, 1, 0.9)])                          # l = 28 > l_max = 24
    assert ei.value.code == rs.RSVD_ERR_SHAPE
    with pytest.raises(rs.RSVDError) as ei:
        b.graph([(A, 0, 8, 1, 0.9)])                           # k < 1
    assert ei.value.code == rs.RSVD_ERR_ARG
    assert b.solve([]) == []
    b.close()
    with pytest.raises(rs.RSVDError):
        rs.Batch(0, 4000, 64, 24, dt)
    with pytest.raises(KeyError):
        rs.Batch(2, 4000, 64, 24, torch.int32)


def test_batch_grouped_replays_and_oracle():
    # every step one launch for all instances, with longer row splits for
    # the partial sums than a solve alone takes: every replay equals the
    # first bit for bit; each result passes the oracle's FP32 gates and
    # agrees with the solo solve in K and status and, to FP32 rounding, in
    # sigma; two rank groups (k = 8 and 16)
    dt = torch.float32
    announce("grouped batch: 12 uneven instances, two (l, k) groups, two launches")
    probs = problems(dt, 12, 31)
    probs = [(A, 8 if i % 2 else 16, p, q, t, A0) if A.shape[1] >= 64 else (A, k, p, q, t, A0)
             for i, (A, k, p, q, t, A0) in enumerate(probs)]
    b = rs.Batch(2, M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    g = b.grouped([pr[:5] for pr in probs])
    first = None
    for rep in range(2):
        for o in g.outs:
            for key in ("U", "S", "V"):
                o[key].fill_(float("nan"))
            o["K"].fill_(-9)
            o["status"].fill_(-99)
        g.launch()
        torch.cuda.synchronize()
        now = [{key: o[key].clone() for key in ("U", "S", "V", "K", "status")} for o in g.outs]
        if first is None:
            first = now
        for a, c in zip(now, first):
            for key in a:
                assert torch.equal(a[key], c[key]), (rep, key)
    alone = rs.Plan(M_MAX, N_MAX, L_MAX, dt, seed=SEED)
    for (A, k, p, q, t, A0), o in zip(probs, g.outs):
        ref = alone.solve(A, k, p, q, t)
        assert int(o["K"].item()) == ref.K and int(o["status"].item()) == ref.status
        assert np.max(np.abs(host(o["S"]) - host(ref.S)) / host(ref.S)) <= 1e-5
        n = A.shape[1]
        G = rounded(synth.gaussian_omega(SEED, n, min(k + p, n)), dt)
        orc = oracle.rsvd(A0, G, k, p, q, t)
        S, U, V = host(o["S"]), host(o["U"]), host(o["V"])
        assert np.max(np.abs(S - orc.S) / orc.S) <= 1e-4, A.shape
        assert oracle.principal_angle_max(orc.V, V) <= 1e-3
        assert oracle.principal_angle_max(orc.U, U) <= 1e-3
        assert int(o["K"].item()) == orc.K and int(o["status"].item()) == orc.status
        assert sign_rule_holds(V)
    g.close()
    alone.close()
    b.close()


def test_batch_grouped_wide_columns():
    # the wider A^T Q kernels in grouped launches (n = 192 and 256: 256-column
    # slabs; n = 512: the 512-column tile), m below and above the grouped
    # split length (1024 rows), two rank groups; replays bit for bit, results
    # against the oracle and the solo solve
    dt = torch.float32
    announce("grouped batch: n in {192, 256, 512}, m 900..5000, two launches")
    shapes = [(900, 512, 16), (5000, 512, 32), (1500, 192, 32), (3000, 256, 16), (1100, 256, 32),
              (4000, 192, 16)]
    rng = np.random.default_rng(77)
    probs = []
    for m, n, k in shapes:
        sig = np.exp(-rng.uniform(0.01, 0.05) * np.arange(1, n + 1))
        A0 = rounded(synth.haar(rng, m, n) @ np.diag(sig) @ synth.haar(rng, n, n).T, dt)
        probs.append((dev(A0, dt), k, 8, 2, 0.9, A0))
    b = rs.Batch(2, 5000, 512, 40, dt, seed=SEED)
    g = b.grouped([pr[:5] for pr in probs])
    g.launch()
    torch.cuda.synchronize()
    first = [{key: o[key].clone() for key in ("U", "S", "V", "K", "status")} for o in g.outs]
    g.launch()
    torch.cuda.synchronize()
    for o, f in zip(g.outs, first):
        for key in f:
            assert torch.equal(o[key], f[key]), key
    alone = rs.Plan(5000, 512, 40, dt, seed=SEED)
    for (A, k, p, q, t, A0), o in zip(probs, g.outs):
        ref = alone.solve(A, k, p, q, t)
        assert int(o["K"].item()) == ref.K and int(o["status"].item()) == ref.status
        assert np.max(np.abs(host(o["S"]) - host(ref.S)) / host(ref.S)) <= 1e-5
        n = A.shape[1]
        G = rounded(synth.gaussian_omega(SEED, n, k + p), dt)
        orc = oracle.rsvd(A0, G, k, p, q, t)
        S, U, V = host(o["S"]), host(o["U"]), host(o["V"])
        assert np.max(np.abs(S - orc.S) / orc.S) <= 1e-4, A.shape
        assert oracle.principal_angle_max(orc.V, V) <= 1e-3
        assert oracle.principal_angle_max(orc.U, U) <= 1e-3
        assert int(o["K"].item()) == orc.K and int(o["status"].item()) == orc.status
    g.close()
    alone.close()
    b.close()


def test_batch_grouped_arguments():
    b = rs.Batch(2, 4000, 64, 24, torch.float32, seed=1)
    A = torch.zeros((1000, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(rs.RSVDError) as ei:
        b.grouped([(A, 6, 4, 1, 0.9)])                  # l = 10: not a multiple of 4
    assert ei.value.code == rs.RSVD_ERR_ARG
    with pytest.raises(rs.RSVDError) as ei:
        b.grouped([(A[:, :62], 8, 8, 1, 0.9)])          # n = 62, lda = 64
    assert ei.value.code == rs.RSVD_ERR_ARG
    b.close()
    b64 = rs.Batch(2, 4000, 64, 24, torch.float64, seed=1)
    with pytest.raises(rs.RSVDError) as ei:
        b64.grouped([(A.double(), 8, 8, 1, 0.9)])       # fp32 batches only
    assert ei.value.code == rs.RSVD_ERR_ARG
    b64.close()


def test_batch_grouped_tuned_graph_unfused():
    # the work-list passes under non-default tile parameters (rows per item
    # and A^T Q split length from a tuning table) give the same K and status
    # as the defaults and sigma to FP32 rounding; sketches wider than 64
    # columns take the separate m-row Gram kernels (no fused epilogue); a
    # captured grouped batch replays bit for bit the eager launch, with
    # eager work between replays; the autotuner returns one valid entry per
    # (n, l); an entry outside the limits is an argument error
    dt = torch.float32
    announce("grouped batch: tuning table, l = 72 (unfused Gram) and 56, graph replays, autotuner")
    rng = np.random.default_rng(91)
    # l = 72 (unfused), 56 (the fused kernels' widest, four column tiles), 24 and 16
    shapes = [(9000, 128, 64), (3000, 128, 64), (6000, 256, 16), (2500, 64, 16), (12000, 256, 64),
              (700, 64, 8), (7000, 128, 48), (1500, 96, 48)]
    probs = []
    for m, n, k in shapes:
        sig = np.exp(-rng.uniform(0.01, 0.2) * np.arange(1, n + 1))
        A0 = rounded(synth.haar(rng, m, n) @ np.diag(sig) @ synth.haar(rng, n, n).T, dt)
        probs.append((dev(A0, dt), k, 8, 2, 0.95, A0))
    b = rs.Batch(2, 12000, 256, 72, dt, seed=SEED)
    g1 = b.grouped([pr[:5] for pr in probs])
    g1.launch()
    torch.cuda.synchronize()
    buckets = sorted({(A.shape[1], min(k + p, A.shape[1])) for A, k, p, *_ in probs})
    tune = [(n, l, 2048, 4096) for n, l in buckets]
    g2 = b.grouped([pr[:5] for pr in probs], tune=tune)
    g2.launch()
    torch.cuda.synchronize()
    eager = [{key: o[key].clone() for key in ("U", "S", "V", "K", "status")} for o in g2.outs]
    for (A, k, p, q, t, A0), o1, o2 in zip(probs, g1.outs, g2.outs):
        assert torch.equal(o1["K"], o2["K"]) and torch.equal(o1["status"], o2["status"])
        # other row splits and panels round the FP32 sums in another order:
        # the values differ by about u sigma_1 (not relative to each sigma_i)
        s1 = host(o1["S"])
        assert np.max(np.abs(s1 - host(o2["S"]))) <= 1e-6 * s1[0]
        n = A.shape[1]
        G = rounded(synth.gaussian_omega(SEED, n, min(k + p, n)), dt)
        orc = oracle.rsvd(A0, G, k, p, q, t)
        S, U, V = host(o2["S"]), host(o2["U"]), host(o2["V"])
        assert np.max(np.abs(S - orc.S) / orc.S) <= 1e-4, A.shape
        assert oracle.principal_angle_max(orc.V, V) <= 1e-3
        assert oracle.principal_angle_max(orc.U, U) <= 1e-3
        assert int(o2["K"].item()) == orc.K and int(o2["status"].item()) == orc.status
    gr = g2.graph()
    for rep in range(3):
        for o in g2.outs:
            for key in ("U", "S", "V"):
                o[key].fill_(float("nan"))
            o["K"].fill_(-9)
            o["status"].fill_(-99)
        torch.cuda.synchronize()
        gr.launch()
        torch.cuda.synchronize()
        for o, e in zip(g2.outs, eager):
            for key in e:
                assert torch.equal(o[key], e[key]), (rep, key)
    gr.close()
    entries = b.tune_grouped([pr[:5] for pr in probs])
    assert sorted((n, l) for n, l, _, _ in entries) == buckets
    for _, _, pr_, sr in entries:
        assert pr_ in (1024, 2048, 4096, 8192) and sr in (1024, 2048, 4096, 8192)
    with pytest.raises(rs.RSVDError) as ei:
        b.grouped([pr[:5] for pr in probs], tune=[(128, 72, 1000, 1024)])
    assert ei.value.code == rs.RSVD_ERR_ARG
    g1.close()
    g2.close()
    b.close()
