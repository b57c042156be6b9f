"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds input generation only: none of the method's arithmetic.
It serves both the FP64 oracle and the GPU path (it is the one thing they
share).

* ``philox4x32_10`` / ``gaussian_omega``: the Gaussian sketch matrix G
  (paper Sec. 3.1.2 step 1, "standard normal distribution matrix G of size
  n x l").  The counter-based Philox4x32-10 generator follows its published
  definition (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC 2011); normals come from the Box-Muller transform (Box &
  Muller 1958).  The GPU library implements the same two published
  definitions in its own code, so a seed means the same G on both sides.
* ``haar``: Haar-distributed orthonormal columns (QR of a Gaussian matrix
  with the signs of diag(R) fixed; Mezzadri, Notices AMS 2007).
* workload recipes: the matrices the paper's setting calls for (real m x n,
  m >> n, columns centred: Sec. 1 "Assumptions"), with prescribed spectra.

Element e = i*l + j of a row-major n x l sketch matrix uses Philox counter
(e // 2, 0, 0, 0) (64-bit index split into the first two words) and key
(seed mod 2^32, seed >> 32).  The four output words give two uniforms
u1 = ((x0 >> 5) * 2^26 + (x1 >> 6) + 0.5) * 2^-53 and the same for (x2, x3),
and Box-Muller gives z0 = sqrt(-2 ln u1) cos(2 pi u2) for even e and
z1 = sqrt(-2 ln u1) sin(2 pi u2) for odd e.
"""
from __future__ import annotations

import math

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.  ctr: (N, 4) uint32 counters; key: two
    uint32 words.  Returns (N, 4) uint32.  Each round multiplies words 0 and 2
    by the two Philox constants, and the new state is
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is advanced by the two Weyl constants between rounds."""
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4) & _MASK
    c0, c1, c2, c3 = (c[:, i].copy() for i in range(4))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def _uniform53(hi: np.ndarray, lo: np.ndarray) -> np.ndarray:
    a = (hi.astype(np.uint64) >> np.uint64(5)).astype(np.float64) * 67108864.0  # 2^26
    b = (lo.astype(np.uint64) >> np.uint64(6)).astype(np.float64)
    return (a + b + 0.5) * (2.0 ** -53)


def gaussian_omega(seed: int, n: int, l: int) -> np.ndarray:
    """Row-major n x l standard normal matrix G for `seed` (see module doc)."""
    N = n * l
    npairs = (N + 1) // 2
    idx = np.arange(npairs, dtype=np.uint64)
    ctr = np.zeros((npairs, 4), dtype=np.uint64)
    ctr[:, 0] = idx & _MASK
    ctr[:, 1] = idx >> np.uint64(32)
    x = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    u1 = _uniform53(x[:, 0], x[:, 1])
    u2 = _uniform53(x[:, 2], x[:, 3])
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * math.pi * u2
    z = np.empty(2 * npairs)
    z[0::2] = r * np.cos(th)
    z[1::2] = r * np.sin(th)
    return z[:N].reshape(n, l)


def haar(rng: np.random.Generator, n: int, k: int, centre: bool = False) -> np.ndarray:
    """n x k matrix with Haar-distributed orthonormal columns.  With centre=True
    the Gaussian's columns are centred first, so every column of the result is
    orthogonal to the all-ones vector (the centring of A is then a no-op)."""
    Z = rng.standard_normal((n, k))
    if centre:
        Z -= Z.mean(axis=0, keepdims=True)
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def centre_columns(A: np.ndarray) -> np.ndarray:
    """Zero mean over each feature (column): the paper's standing assumption."""
    return A - A.mean(axis=0, keepdims=True)


def low_rank(seed: int, m: int, n: int, sigma, centre: bool = True) -> np.ndarray:
    """A = U diag(sigma) V^T with Haar U (m x r, centred), V (n x r), r = len(sigma)."""
    rng = np.random.default_rng(seed)
    sigma = np.asarray(sigma, dtype=np.float64)
    r = len(sigma)
    U = haar(rng, m, r, centre=centre)
    V = haar(rng, n, r)
    A = (U * sigma) @ V.T
    return centre_columns(A) if centre else A


# --------------------------------------------------------------------------
# Workload recipes.  Each returns plain arrays; nothing here computes an SVD.

CONFIG1 = dict(m=2000, n=200, k=20, p=10, q=2, t=0.95, seed=1, omega_seed=101)


def config1_sigma(n: int = 200) -> np.ndarray:
    """sigma_i = 10 * 0.85^(i-1), i = 1..n."""
    return 10.0 * 0.85 ** np.arange(n, dtype=np.float64)


def config1(seed: int = 1) -> np.ndarray:
    """2000 x 200 FP64: A = U diag(sigma) V^T, U Haar in the complement of the
    ones vector, V Haar 200 x 200, sigma_i = 10*0.85^(i-1), columns centred."""
    c = CONFIG1
    return low_rank(seed, c["m"], c["n"], config1_sigma(c["n"]), centre=True)


CONFIG2 = dict(m=1_000_000, n=512, k=64, p=16, q=2, t=0.95, seed=2, omega_seed=202,
               noise_std=1e-3)


def config2_sigma(n: int = 512) -> np.ndarray:
    """sigma_i = 1/i, i = 1..n."""
    return 1.0 / np.arange(1, n + 1, dtype=np.float64)


CONFIG3 = dict(m=262_144, n=1024, k=128, p=32, q=3, t=0.95, seed=3, omega_seed=303,
               noise_std=1e-4)


def config3_sigma(n: int = 1024) -> np.ndarray:
    """sigma_i = 1/sqrt(i), i = 1..n (slow decay)."""
    return 1.0 / np.sqrt(np.arange(1, n + 1, dtype=np.float64))


CONFIG4 = dict(count=512, m_lo=4096, m_hi=65536, n_choices=(64, 128, 256, 512), r_lo=0.01,
               r_hi=0.2, k_max=32, p=8, q=2, t=0.95, seed=4)


def batch_shapes(c=None):
    """The batched workload's instances: (m, n, r, k) with m uniform integer in
    [m_lo, m_hi], n uniform in n_choices, r uniform in [r_lo, r_hi] (the
    spectrum is sigma_i = exp(-r i)) and k = min(k_max, n / 4)."""
    c = c or CONFIG4
    rng = np.random.default_rng(c["seed"])
    out = []
    for _ in range(c["count"]):
        m = int(rng.integers(c["m_lo"], c["m_hi"] + 1))
        n = int(rng.choice(c["n_choices"]))
        r = float(rng.uniform(c["r_lo"], c["r_hi"]))
        out.append((m, n, r, min(c["k_max"], n // 4)))
    return out


def batch_problems(torch, dev, c=None):
    """The batched workload's matrices on the device (no noise), as
    (A, k, p, q, t) per instance, by the device recipe of spiked_noisy_torch."""
    c = c or CONFIG4
    out = []
    for i, (m, n, r, k) in enumerate(batch_shapes(c)):
        A = spiked_noisy_torch(c["seed"] * 100003 + i, m, n, exp_sigma(n, r), 0.0, dev,
                               torch.float32)
        out.append((A, k, c["p"], c["q"], c["t"]))
    return out


CONFIG5 = dict(rate=200.0, seconds=60.0, m_lo=1000, m_hi=1_000_000, m_multiple=64,
               n_choices=(128, 256, 512, 1024), alpha_lo=0.5, alpha_hi=2.0,
               t_choices=(0.9, 0.95, 0.99), storage_choices=("fp32", "bf16"), k=16, p=8, q=2,
               l_max=192, pool=24, seed=5)


def serve_pool(c=None):
    """Matrices the serving workload draws its requests from: (m, n, alpha)
    with m log-uniform in [m_lo, m_hi] rounded down to a multiple of
    m_multiple, n uniform in n_choices, alpha uniform in [alpha_lo, alpha_hi]
    (sigma_i = i^-alpha)."""
    c = c or CONFIG5
    rng = np.random.default_rng(c["seed"])
    out = []
    for _ in range(c["pool"]):
        n = int(rng.choice(c["n_choices"]))
        m = int(np.exp(rng.uniform(np.log(c["m_lo"]), np.log(c["m_hi"]))))
        m = max(n, m // c["m_multiple"] * c["m_multiple"])
        out.append((m, n, float(rng.uniform(c["alpha_lo"], c["alpha_hi"]))))
    return out


def serve_arrivals(c=None):
    """Poisson arrivals at `rate` per second over `seconds`: (time, pool
    index, t, storage) per request, storage drawn uniformly from
    storage_choices."""
    c = c or CONFIG5
    rng = np.random.default_rng(c["seed"] + 1)
    out, now = [], 0.0
    while True:
        now += rng.exponential(1.0 / c["rate"])
        if now >= c["seconds"]:
            return out
        j = int(rng.integers(0, c["pool"]))
        t = float(rng.choice(c["t_choices"]))
        out.append((now, j, t, str(rng.choice(c["storage_choices"]))))


def power_sigma(n: int, alpha: float) -> np.ndarray:
    """sigma_i = i^-alpha, i = 1..n."""
    return np.arange(1, n + 1, dtype=np.float64) ** -alpha


def exp_sigma(n: int, r: float) -> np.ndarray:
    """sigma_i = exp(-r i), i = 1..n."""
    return np.exp(-r * np.arange(1, n + 1, dtype=np.float64))


def spiked_noisy(seed: int, m: int, n: int, sigma, noise_std: float) -> np.ndarray:
    """CPU (numpy) version of the config-2 recipe at any size:
    A = U diag(sigma) V^T + noise_std * N(0,1), U an orthonormalised centred
    Gaussian (m x n), V Haar (n x n), columns centred, FP64."""
    rng = np.random.default_rng(seed)
    U = haar(rng, m, n, centre=True)
    V = haar(rng, n, n)
    A = (U * np.asarray(sigma)) @ V.T + noise_std * rng.standard_normal((m, n))
    return centre_columns(A)


def spiked_noisy_torch(seed: int, m: int, n: int, sigma, noise_std: float, device,
                       out_dtype=None, chunk_rows: int = 1 << 17):
    """Device version of the same recipe for the full-size workload (1e6 x 512):
    built in FP64 with torch on `device` (seeded torch generator), U
    orthonormalised by two Cholesky-QR passes computed in FP64 (Cholesky on
    the host), V Haar from numpy, then cast to `out_dtype`.  Input preparation
    only; the library under test is not involved."""
    import torch

    out_dtype = out_dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    U = torch.randn(m, n, dtype=torch.float64, device=device, generator=g)
    U -= U.mean(dim=0, keepdim=True)
    for _ in range(2):
        Gm = (U.T @ U).cpu().numpy()
        L = np.linalg.cholesky(0.5 * (Gm + Gm.T))
        Linv_t = torch.from_numpy(np.linalg.inv(L).T.copy()).to(device)
        U = U @ Linv_t
    rng = np.random.default_rng(int(seed) + 7919)
    V = torch.from_numpy(haar(rng, n, n)).to(device)
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    M = (V * sig).T.contiguous()          # diag(sigma) V^T
    A = torch.empty(m, n, dtype=torch.float64, device=device)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        A[r0:r1] = U[r0:r1] @ M
        A[r0:r1] += noise_std * torch.randn(r1 - r0, n, dtype=torch.float64, device=device,
                                            generator=g)
    del U
    A -= A.mean(dim=0, keepdim=True)
    out = A.to(out_dtype)
    del A
    return out
