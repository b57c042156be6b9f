"""FP64 CPU oracle for the randomized range finder / truncated SVD.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The GPU package
``paper_1906_12085_amd`` never imports this module, and this module never
imports the GPU package; they share no code.

The arithmetic lives in ``oracle.c`` (plain double-precision loops, OpenMP);
this file compiles it with gcc (``build()``) and marshals numpy arrays.  Each
wrapper names the passage of the paper (arXiv 1906.12085) it follows.

Parity status of every routine is listed in ``PINS`` (which test pins it).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, WARN_THRESHOLD, WARN_ZERO = 0, 1, 2
ERR_ARG, ERR_NOMEM, ERR_NOCONV = -1, -3, -7

# routine -> tests that pin it against something other than itself
PINS = {
    "gemm_nn / gemm_tn": "tests/test_oracle_basic.py (brute force, numpy third opinion)",
    "fro2": "tests/test_oracle_basic.py (Eq. sumeigen: equals trace(A^T A) and sum s_i^2)",
    "qr_householder": "tests/test_oracle_basic.py (Q^T Q = I, QR = X, R upper with R_jj>=0, "
                      "uniqueness vs Gram-Schmidt by hand on 3x2)",
    "svd_jacobi / svd_exact": "tests/test_oracle_svd.py (golden closed forms, known spectrum, "
                              "invariants of Sec. 2.1, LAPACK third opinion)",
    "eig_sym_jacobi": "tests/test_oracle_svd.py (golden 2x2/3x3, A V = V diag(lam), LAPACK)",
    "select_k": "tests/test_oracle_rsvd.py (golden config-1 closed form K=10, edge cases)",
    "rsvd": "tests/test_oracle_rsvd.py (exact recovery at rank l, interlacing, "
            "Halko et al. error bound, convergence in q)",
    "gram_eig": "tests/test_oracle_rsvd.py (equals exact SVD on well-separated spectra)",
    "rsvd_blocked": "tests/test_oracle_blocked.py (one block equals Randomized PCA, exact "
                    "recovery when rank(A) is a multiple of the block, energy = sum of the "
                    "captured s^2 and monotone up to ||A||_F^2, the stopping block is the first "
                    "to reach t, orthonormal factors, interlacing, K equals the exact K)",
    "krylov": "tests/test_oracle_krylov.py (exact recovery at rank (i+1) l where Randomized "
              "PCA with q = i is not exact, Ritz values between those of Randomized PCA and "
              "the exact ones, U^T A V = diag(s), i = 0 equals q = 0)",
}


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, dbl, p = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lib.orc_gemm_nn.argtypes = [i64, i64, i64, p, i64, p, i64, p, i64]
        lib.orc_gemm_tn.argtypes = [i64, i64, i64, p, i64, p, i64, p, i64]
        lib.orc_gemm_tn.restype = ctypes.c_int
        lib.orc_fro2.argtypes = [i64, i64, p, i64]
        lib.orc_fro2.restype = dbl
        lib.orc_qr_householder.argtypes = [i64, i64, p, i64, p, i64, p, i64]
        lib.orc_qr_householder.restype = ctypes.c_int
        lib.orc_svd_jacobi.argtypes = [i64, i64, p, i64, p, i64, p, p, i64]
        lib.orc_svd_jacobi.restype = ctypes.c_int
        lib.orc_svd_exact.argtypes = [i64, i64, p, i64, p, i64, p, p, i64]
        lib.orc_svd_exact.restype = ctypes.c_int
        lib.orc_eig_sym_jacobi.argtypes = [i64, p, i64, p, p, i64]
        lib.orc_eig_sym_jacobi.restype = ctypes.c_int
        lib.orc_select_k.argtypes = [i64, p, dbl, dbl, ctypes.POINTER(i64)]
        lib.orc_select_k.restype = ctypes.c_int
        lib.orc_sign_convention.argtypes = [i64, i64, i64, p, i64, p, i64]
        lib.orc_rsvd.argtypes = [i64, i64, p, i64, p, i64, i64, i64, dbl,
                                 p, i64, p, p, i64, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
        lib.orc_rsvd.restype = ctypes.c_int
        lib.orc_krylov.argtypes = [i64, i64, p, i64, p, i64, i64, i64, dbl,
                                   p, i64, p, p, i64, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
        lib.orc_krylov.restype = ctypes.c_int
        lib.orc_gram_eig.argtypes = [i64, i64, p, i64, dbl, i64, p, i64, p, p, i64,
                                     ctypes.POINTER(i64), ctypes.POINTER(dbl)]
        lib.orc_gram_eig.restype = ctypes.c_int
        lib.orc_rsvd_blocked.argtypes = [i64, i64, p, i64, p, i64, i64, i64, dbl, i64, i64,
                                         p, i64, p, p, i64, ctypes.POINTER(i64),
                                         ctypes.POINTER(i64), p, ctypes.POINTER(dbl)]
        lib.orc_rsvd_blocked.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def gemm_nn(A, B) -> np.ndarray:
    """C = A B (plain loops; Sec. 3.1 counts m*n*l multiply-adds)."""
    A, B = _f64(A), _f64(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.empty((m, n))
    _load().orc_gemm_nn(m, k, n, _ptr(A), k, _ptr(B), n, _ptr(C), n)
    return C


def gemm_tn(A, B) -> np.ndarray:
    """C = A^T B, reduction over rows in a fixed chunk order."""
    A, B = _f64(A), _f64(B)
    m, k = A.shape
    m2, n = B.shape
    assert m == m2
    C = np.empty((k, n))
    rc = _load().orc_gemm_tn(m, k, n, _ptr(A), k, _ptr(B), n, _ptr(C), n)
    assert rc == OK, rc
    return C


def fro2(A) -> float:
    """||A||_F^2 = sum a_ij^2 (Eq. sumeigen)."""
    A = _f64(A)
    m, n = A.shape
    return float(_load().orc_fro2(m, n, _ptr(A), n))


def qr(X):
    """Thin Householder QR, X = Q R with R_jj >= 0 (stands in for the paper's
    'QR decomposition on H', Sec. 3.1.2 step 4)."""
    X = _f64(X)
    m, n = X.shape
    Q = np.empty((m, n))
    R = np.empty((n, n))
    rc = _load().orc_qr_householder(m, n, _ptr(X), n, _ptr(Q), n, _ptr(R), n)
    assert rc == OK, rc
    return Q, R


def svd_jacobi(X):
    """One-sided Jacobi SVD, X = U diag(s) V^T (Sec. 2.1).  Returns U, s, V, sweeps."""
    X = _f64(X)
    m, n = X.shape
    U = np.empty((m, n)); s = np.empty(n); V = np.empty((n, n))
    rc = _load().orc_svd_jacobi(m, n, _ptr(X), n, _ptr(U), n, _ptr(s), _ptr(V), n)
    if rc < 0:
        raise RuntimeError(f"orc_svd_jacobi failed: {rc}")
    return U, s, V, rc


def svd(X):
    """Exact thin SVD (Householder QR, then one-sided Jacobi on R).  Returns U, s, V."""
    X = _f64(X)
    m, n = X.shape
    U = np.empty((m, n)); s = np.empty(n); V = np.empty((n, n))
    rc = _load().orc_svd_exact(m, n, _ptr(X), n, _ptr(U), n, _ptr(s), _ptr(V), n)
    if rc < 0:
        raise RuntimeError(f"orc_svd_exact failed: {rc}")
    return U, s, V


def eig_sym(G):
    """Cyclic Jacobi eigen-decomposition of a symmetric matrix, lam descending
    (eig of A^T A, Sec. 2.3).  Returns lam, V, sweeps."""
    G = _f64(G)
    n = G.shape[0]
    lam = np.empty(n); V = np.empty((n, n))
    rc = _load().orc_eig_sym_jacobi(n, _ptr(G), n, _ptr(lam), _ptr(V), n)
    if rc < 0:
        raise RuntimeError(f"orc_eig_sym_jacobi failed: {rc}")
    return lam, V, rc


def select_k(s, fro2_value: float, t: float):
    """Cumulative explained variance criterion (Sec. 2.4).  Returns (K, status)."""
    s = _f64(s)
    K = ctypes.c_int64(0)
    rc = _load().orc_select_k(len(s), _ptr(s), float(fro2_value), float(t), ctypes.byref(K))
    if rc < 0:
        raise ValueError(f"orc_select_k rejected its arguments: {rc}")
    return int(K.value), int(rc)


def sign_convention(U, V):
    """Apply the output sign rule in place: the lowest-index entry of v_i whose
    magnitude is within 0.1% of the largest is made positive (u_i flips with it).
    Arrays must be C-contiguous float64 so the change is visible to the caller."""
    assert V.dtype == np.float64 and V.flags.c_contiguous and V.flags.writeable
    n, k = V.shape
    if U is not None:
        assert U.dtype == np.float64 and U.flags.c_contiguous and U.flags.writeable
        m = U.shape[0]
        _load().orc_sign_convention(m, n, k, _ptr(U), U.shape[1], _ptr(V), k)
    else:
        _load().orc_sign_convention(0, n, k, None, 0, _ptr(V), k)
    return U, V


class RSVDResult(NamedTuple):
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    K: int
    fro2: float
    status: int


def rsvd(A, G, k: int, p: int, q: int, t: float) -> RSVDResult:
    """Randomized PCA (Sec. 3.1.2) with the sketch matrix G (n x l, l=min(k+p,n))
    given, and an orthonormalisation after every product with A or A^T."""
    A, G = _f64(A), _f64(G)
    m, n = A.shape
    l = min(k + p, n)
    assert G.shape == (n, l), (G.shape, (n, l))
    U = np.empty((m, k)); S = np.empty(k); V = np.empty((n, k))
    K = ctypes.c_int64(0); f2 = ctypes.c_double(0.0)
    rc = _load().orc_rsvd(m, n, _ptr(A), n, _ptr(G), k, p, q, float(t),
                          _ptr(U), k, _ptr(S), _ptr(V), k, ctypes.byref(K), ctypes.byref(f2))
    if rc < 0:
        raise RuntimeError(f"orc_rsvd failed: {rc}")
    return RSVDResult(U, S, V, int(K.value), float(f2.value), int(rc))


def krylov(A, G, k: int, p: int, i: int, t: float) -> RSVDResult:
    """Krylov method (Sec. 3.1.1) with the sketch G (n x l, l = min(k+p, n))
    given: blocks H(0) = A G, H(j) = A (A^T H(j-1)) for j <= i, QR of their
    concatenation (m x (i+1) l, at most n columns), T = A^T Q, SVD of T."""
    A, G = _f64(A), _f64(G)
    m, n = A.shape
    l = min(k + p, n)
    assert G.shape == (n, l), (G.shape, (n, l))
    U = np.empty((m, k)); S = np.empty(k); V = np.empty((n, k))
    K = ctypes.c_int64(0); f2 = ctypes.c_double(0.0)
    rc = _load().orc_krylov(m, n, _ptr(A), n, _ptr(G), k, p, i, float(t),
                            _ptr(U), k, _ptr(S), _ptr(V), k, ctypes.byref(K), ctypes.byref(f2))
    if rc < 0:
        raise RuntimeError(f"orc_krylov failed: {rc}")
    return RSVDResult(U, S, V, int(K.value), float(f2.value), int(rc))


def gram_eig(A, t: float, ucols: int | None = None) -> RSVDResult:
    """Truncated SVD through A^T A (Sec. 2.3 / 3.1.3): S (n), V (n x n), U (m x ucols)."""
    A = _f64(A)
    m, n = A.shape
    uc = n if ucols is None else int(ucols)
    U = np.empty((m, max(uc, 1))); S = np.empty(n); V = np.empty((n, n))
    K = ctypes.c_int64(0); f2 = ctypes.c_double(0.0)
    rc = _load().orc_gram_eig(m, n, _ptr(A), n, float(t), uc, _ptr(U), max(uc, 1),
                              _ptr(S), _ptr(V), n, ctypes.byref(K), ctypes.byref(f2))
    if rc < 0:
        raise RuntimeError(f"orc_gram_eig failed: {rc}")
    return RSVDResult(U[:, :uc], S, V, int(K.value), float(f2.value), int(rc))


class BlockedResult(NamedTuple):
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    K: int
    fro2: float
    status: int
    L: int
    energy: np.ndarray


def rsvd_blocked(A, G, b: int, q: int, t: float, lmax: int, kcap: int) -> BlockedResult:
    """Randomized PCA with the rank grown in blocks of b columns until the
    criterion of Sec. 2.4 can be met (Martinsson & Voronin 2016, blocked
    range finder with power steps); G (n x nb*b) holds the blocks' sketches
    side by side.  Returns the first min(kcap, L) triplets, K (capped at
    kcap), the columns used L and the captured energy after each block."""
    A, G = _f64(A), _f64(G)
    m, n = A.shape
    assert G.shape[0] == n and (b < 1 or G.shape[1] % b == 0)
    kcap_ = max(int(kcap), 1)
    U = np.zeros((m, kcap_)); S = np.zeros(kcap_); V = np.zeros((n, kcap_))
    energy = np.zeros(max(1, G.shape[1] // max(b, 1)))
    K = ctypes.c_int64(0); L = ctypes.c_int64(0); f2 = ctypes.c_double(0.0)
    rc = _load().orc_rsvd_blocked(m, n, _ptr(A), n, _ptr(G), G.shape[1], b, q, float(t), lmax,
                                  kcap, _ptr(U), kcap_, _ptr(S), _ptr(V), kcap_, ctypes.byref(K),
                                  ctypes.byref(L), _ptr(energy), ctypes.byref(f2))
    if rc < 0:
        raise RuntimeError(f"orc_rsvd_blocked failed: {rc}")
    Lv = int(L.value)
    kc = min(kcap, Lv)
    return BlockedResult(U[:, :kc], S[:kc], V[:, :kc], int(K.value), float(f2.value), int(rc),
                         Lv, energy[:Lv // b])


def principal_angle_max(X, Y) -> float:
    """Largest principal angle between span(X) and span(Y) (both with
    orthonormal columns, same column count), computed in the sine form
    arcsin ||(I - X X^T) Y||_2, which keeps resolution for small angles
    (Bjorck & Golub 1973).  A test metric, not part of the method."""
    X, Y = _f64(X), _f64(Y)
    R = Y - X @ (X.T @ Y)
    s = np.linalg.norm(R, 2) if R.size else 0.0
    return float(np.arcsin(min(1.0, s)))
