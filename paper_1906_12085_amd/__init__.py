"""Python binding of librsvd.so (include/rsvd.h): randomized range finder and
truncated SVD (PCA by SVD) of a tall-skinny centred matrix on an MI355X.

Argument marshalling only: every step of a solve runs in the HIP kernels of
librsvd.so.  Tensors are torch tensors on the GPU (torch supplies device
memory and streams); the functions below pass their data pointers, sizes and
row strides to the C entry points of the same names.  If librsvd.so has not
been built this module raises on first use -- there is no fallback path.

Quick use::

    plan = Plan(m_max, n_max, l_max, torch.float32, want_gram=True)
    U, S, V, K = plan.solve(A, k=64, p=16, q=2, t=0.95)
    U, S, V, K = plan.gram_eig(A, t=0.95)
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsvd.so")

RSVD_F64, RSVD_F32, RSVD_BF16, RSVD_FP8 = 0, 1, 2, 3
STATUS = {
    0: "RSVD_OK", 1: "RSVD_WARN_THRESHOLD", 2: "RSVD_WARN_ZERO_MATRIX",
    -1: "RSVD_ERR_ARG", -2: "RSVD_ERR_SHAPE", -3: "RSVD_ERR_NOMEM", -4: "RSVD_ERR_DEVICE",
    -5: "RSVD_ERR_BREAKDOWN", -6: "RSVD_ERR_NONFINITE", -7: "RSVD_ERR_NOCONV",
}
RSVD_OK, RSVD_WARN_THRESHOLD, RSVD_WARN_ZERO_MATRIX = 0, 1, 2
RSVD_ERR_ARG, RSVD_ERR_SHAPE, RSVD_ERR_NOMEM, RSVD_ERR_DEVICE = -1, -2, -3, -4
RSVD_ERR_BREAKDOWN, RSVD_ERR_NONFINITE, RSVD_ERR_NOCONV = -5, -6, -7
RSVD_SERVER_GRAM_FALLBACK = 1

EXPORTS = ["rsvd_status_string", "rsvd_plan_create", "rsvd_plan_destroy", "rsvd_plan_status",
           "rsvd_plan_diag", "rsvd_solve", "rsvd_solve_omega", "gram_eig_solve",
           "rsvd_gaussian_fill", "rsvd_gemm_nn", "rsvd_gemm_tn", "rsvd_cholqr2",
           "rsvd_small_svd", "rsvd_sym_eig", "rsvd_plan_kernel_times", "rsvd_solve_bf16",
           "rsvd_quantize_bf16", "rsvd_solve_fp8", "rsvd_quantize_fp8", "rsvd_solve_krylov",
           "rsvd_batch_create", "rsvd_batch_destroy", "rsvd_batch_solve",
           "rsvd_batch_graph_create", "rsvd_batch_graph_launch", "rsvd_batch_graph_destroy",
           "rsvd_server_create", "rsvd_server_submit", "rsvd_server_progress",
           "rsvd_server_destroy", "rsvd_batch_grouped_create", "rsvd_batch_grouped_launch",
           "rsvd_batch_grouped_destroy", "rsvd_solve_noalloc", "rsvd_solve_adaptive",
           "rsvd_batch_grouped_tune", "rsvd_batch_grouped_graph_create"]

# The committed tile parameters of grouped batches on gfx950 (written by
# tune_grouped.py from the autotuner's measurements).
TUNE_CACHE = os.path.join(HERE, "tune_grouped_gfx950.json")


class RsvdInstance(ctypes.Structure):
    """One problem of a batch (the C struct rsvd_instance)."""
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("k", ctypes.c_int32), ("p", ctypes.c_int32),
                ("q", ctypes.c_int32), ("t", ctypes.c_double), ("U", ctypes.c_void_p),
                ("ldu", ctypes.c_int64), ("S", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("ldv", ctypes.c_int64), ("K", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("col_scale", ctypes.c_void_p), ("k_max", ctypes.c_int32),
                ("dtype", ctypes.c_int32)]


class RsvdTuneEntry(ctypes.Structure):
    """Tile parameters of a grouped batch for one (n, l) (rsvd_tune_entry)."""
    _fields_ = [("n", ctypes.c_int32), ("l", ctypes.c_int32), ("panel_rows", ctypes.c_int32),
                ("split_rows", ctypes.c_int32)]


def load_tune_cache(path: str = TUNE_CACHE):
    """The entries of a tuning cache file (JSON list of {n, l, panel_rows,
    split_rows}); [] if there is none."""
    import json
    if not os.path.exists(path):
        return []
    with open(path) as f:
        data = json.load(f)
    return [(int(e["n"]), int(e["l"]), int(e["panel_rows"]), int(e["split_rows"]))
            for e in data["entries"]]


def _tune_array(entries):
    if not entries:
        return None, 0
    arr = (RsvdTuneEntry * len(entries))()
    for i, e in enumerate(entries):
        arr[i] = RsvdTuneEntry(*[int(v) for v in e])
    return arr, len(entries)


def _dtype_codes(torch):
    """torch dtype of A -> (rsvd_dtype, dtype of U and V)."""
    return {torch.float64: (RSVD_F64, torch.float64), torch.float32: (RSVD_F32, torch.float32),
            torch.bfloat16: (RSVD_BF16, torch.float32),
            torch.float8_e4m3fn: (RSVD_FP8, torch.float32)}


class RSVDError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librsvd.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run __graft_entry__.build() "
                          "(there is no CPU fallback for the GPU path)")
    lib = ctypes.CDLL(path)
    i32, i64, u64, dbl, vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                              ctypes.c_void_p)
    sig = {
        "rsvd_status_string": (ctypes.c_char_p, [i32]),
        "rsvd_plan_create": (i32, [ctypes.POINTER(vp), i64, i64, i32, i32, i32, u64, vp]),
        "rsvd_plan_destroy": (i32, [vp]),
        "rsvd_plan_status": (i32, [vp]),
        "rsvd_plan_diag": (i32, [vp, vp, i32]),
        "rsvd_solve": (i32, [vp, vp, i64, i64, i64, vp, i32, i32, i32, dbl, vp, i64, vp, vp, i64,
                             vp]),
        "rsvd_solve_omega": (i32, [vp, vp, i64, i64, i64, vp, i32, i32, i32, dbl, vp,
                                   vp, i64, vp, vp, i64, vp]),
        "rsvd_solve_krylov": (i32, [vp, vp, i64, i64, i64, i32, i32, i32, dbl, vp,
                                    vp, i64, vp, vp, i64, vp]),
        "rsvd_solve_adaptive": (i32, [vp, vp, i64, i64, i64, vp, i32, i32, i32, dbl, i32,
                                      vp, i64, vp, vp, i64, vp]),
        "rsvd_batch_create": (i32, [ctypes.POINTER(vp), i32, i64, i64, i32, i32, u64]),
        "rsvd_batch_destroy": (i32, [vp]),
        "rsvd_batch_solve": (i32, [vp, ctypes.POINTER(RsvdInstance), i32, vp]),
        "rsvd_batch_graph_create": (i32, [vp, ctypes.POINTER(RsvdInstance), i32, vp,
                                          ctypes.POINTER(vp)]),
        "rsvd_batch_graph_launch": (i32, [vp, vp]),
        "rsvd_batch_graph_destroy": (i32, [vp]),
        "rsvd_server_create": (i32, [ctypes.POINTER(vp), i32, i64, i64, i32, i32, u64, i64,
                                     i32]),
        "rsvd_server_submit": (i32, [vp, ctypes.POINTER(RsvdInstance), ctypes.POINTER(i64)]),
        "rsvd_server_progress": (i32, [vp, ctypes.POINTER(i64), i32, ctypes.POINTER(i32),
                                       ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "rsvd_server_destroy": (i32, [vp]),
        "rsvd_batch_grouped_create": (i32, [vp, ctypes.POINTER(RsvdInstance), i32,
                                            ctypes.POINTER(RsvdTuneEntry), i32,
                                            ctypes.POINTER(vp)]),
        "rsvd_batch_grouped_tune": (i32, [vp, ctypes.POINTER(RsvdInstance), i32,
                                          ctypes.POINTER(RsvdTuneEntry), i32,
                                          ctypes.POINTER(i32), vp]),
        "rsvd_batch_grouped_graph_create": (i32, [vp, ctypes.POINTER(vp)]),
        "rsvd_batch_grouped_launch": (i32, [vp, vp]),
        "rsvd_batch_grouped_destroy": (i32, [vp]),
        "gram_eig_solve": (i32, [vp, vp, i64, i64, i64, dbl, i32, vp, i64, vp, vp, i64, vp]),
        "rsvd_gaussian_fill": (i32, [u64, i64, i64, vp, vp]),
        "rsvd_gemm_nn": (i32, [vp, vp, i64, i64, i64, vp, i64, i32, vp, i64, vp, vp]),
        "rsvd_gemm_tn": (i32, [vp, vp, i64, i64, i64, vp, i64, i32, vp]),
        "rsvd_cholqr2": (i32, [vp, vp, i64, i32, i64, vp, i64, vp]),
        "rsvd_small_svd": (i32, [vp, vp, i64, i32, vp, vp, vp]),
        "rsvd_sym_eig": (i32, [vp, vp, i64, vp, vp]),
        "rsvd_plan_kernel_times": (i32, [vp, i32, vp, vp, i32]),
        "rsvd_solve_bf16": (i32, [vp, vp, vp, i64, i64, i64, i32, i32, i32, dbl, vp,
                                  vp, i64, vp, vp, i64, vp]),
        "rsvd_quantize_bf16": (i32, [vp, vp, i64, i64, i64, vp, i64, vp]),
        "rsvd_solve_fp8": (i32, [vp, vp, vp, i64, i64, i64, i32, i32, i32, dbl, vp,
                                 vp, i64, vp, vp, i64, vp]),
        "rsvd_quantize_fp8": (i32, [vp, vp, i64, i64, i64, vp, i64, vp]),
        "rsvd_solve_noalloc": (i32, [vp, i64, i64, i64, i32, i32, i32, i32, dbl, u64, vp, i64,
                                     vp, vp, i64, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _ld(t) -> int:
    """Row stride of a row-major 2-D tensor (elements between rows)."""
    assert t.dim() == 2 and t.stride(1) == 1, "matrices must be row-major with unit column stride"
    return t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise RSVDError(rc, where)
    return rc


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


# ---------------------------------------------------------------- C names --
def rsvd_status_string(code: int) -> str:
    return load_library().rsvd_status_string(code).decode()


def rsvd_plan_create(m_max: int, n_max: int, l_max: int, dtype: int, want_gram: bool = False,
                     seed: int = 0, stream=None) -> int:
    h = ctypes.c_void_p()
    rc = load_library().rsvd_plan_create(ctypes.byref(h), m_max, n_max, l_max, dtype,
                                         int(bool(want_gram)), seed, _stream_ptr(stream))
    _check(rc, "rsvd_plan_create")
    return h.value


def rsvd_plan_destroy(plan: int) -> int:
    return _check(load_library().rsvd_plan_destroy(plan), "rsvd_plan_destroy")


def rsvd_plan_status(plan: int) -> int:
    return load_library().rsvd_plan_status(plan)


def rsvd_plan_diag(plan: int, count: int = 8):
    buf = (ctypes.c_double * count)()
    nc = _check(load_library().rsvd_plan_diag(plan, buf, count), "rsvd_plan_diag")
    return list(buf[:nc])


KERNEL_KINDS = ["eigensolver", "pass_nn", "pass_tn", "syrk", "nn_wide"]


def rsvd_plan_kernel_times(plan: int, enable: bool):
    """Mean launch durations (ms) and launch counts per timed kernel kind since
    the previous call; then timing is switched on or off for later calls."""
    n = len(KERNEL_KINDS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int32 * n)()
    nc = _check(load_library().rsvd_plan_kernel_times(plan, 1 if enable else 0, ms, cnt, n),
                "rsvd_plan_kernel_times")
    return {KERNEL_KINDS[i]: (ms[i], cnt[i]) for i in range(nc)}


def rsvd_solve(plan: int, A, k: int, p: int, q: int, t: float, U, S, V, K,
               col_scale=None) -> int:
    m, n = A.shape
    return _check(load_library().rsvd_solve(plan, _ptr(A), m, n, _ld(A), _ptr(col_scale), k, p,
                                            q, float(t), _ptr(U), _ld(U), _ptr(S), _ptr(V),
                                            _ld(V), _ptr(K)), "rsvd_solve")


def rsvd_solve_omega(plan: int, A, k: int, p: int, q: int, t: float, omega, U, S, V, K,
                     col_scale=None) -> int:
    m, n = A.shape
    if omega is not None:
        assert omega.is_contiguous() and omega.dtype.is_floating_point and omega.element_size() == 8
    return _check(load_library().rsvd_solve_omega(plan, _ptr(A), m, n, _ld(A), _ptr(col_scale), k,
                                                  p, q, float(t), _ptr(omega), _ptr(U), _ld(U),
                                                  _ptr(S), _ptr(V), _ld(V), _ptr(K)),
                  "rsvd_solve_omega")


def rsvd_solve_noalloc(A, k: int, p: int, q: int, t: float, seed: int, U, S, V, K, status,
                       stream=None) -> int:
    """rsvd_solve without a plan: the workspace is the library's static device
    array (nothing is allocated); status (1 int32, device) receives the
    status word."""
    import torch
    m, n = A.shape
    code = {torch.float64: RSVD_F64, torch.float32: RSVD_F32}[A.dtype]
    return _check(load_library().rsvd_solve_noalloc(_ptr(A), m, n, _ld(A), code, k, p, q,
                                                    float(t), seed, _ptr(U), _ld(U), _ptr(S),
                                                    _ptr(V), _ld(V), _ptr(K), _ptr(status),
                                                    _stream_ptr(stream)),
                  "rsvd_solve_noalloc")


def rsvd_solve_krylov(plan: int, A, k: int, p: int, i: int, t: float, omega, U, S, V,
                      K) -> int:
    m, n = A.shape
    if omega is not None:
        assert omega.is_contiguous() and omega.dtype.is_floating_point and omega.element_size() == 8
    return _check(load_library().rsvd_solve_krylov(plan, _ptr(A), m, n, _ld(A), k, p, i,
                                                   float(t), _ptr(omega), _ptr(U), _ld(U),
                                                   _ptr(S), _ptr(V), _ld(V), _ptr(K)),
                  "rsvd_solve_krylov")


def rsvd_solve_adaptive(plan: int, A, k: int, p: int, q: int, t: float, k_max: int, U, S, V, K,
                        col_scale=None) -> int:
    m, n = A.shape
    return _check(load_library().rsvd_solve_adaptive(plan, _ptr(A), m, n, _ld(A),
                                                     _ptr(col_scale), k, p, q, float(t),
                                                     int(k_max), _ptr(U), _ld(U), _ptr(S),
                                                     _ptr(V), _ld(V), _ptr(K)),
                  "rsvd_solve_adaptive")


def rsvd_solve_bf16(plan: int, A, col_scale, k: int, p: int, q: int, t: float, omega, U, S, V,
                    K) -> int:
    m, n = A.shape
    if omega is not None:
        assert omega.is_contiguous() and omega.element_size() == 8
    return _check(load_library().rsvd_solve_bf16(plan, _ptr(A), _ptr(col_scale), m, n, _ld(A), k,
                                                 p, q, float(t), _ptr(omega), _ptr(U), _ld(U),
                                                 _ptr(S), _ptr(V), _ld(V), _ptr(K)),
                  "rsvd_solve_bf16")


def rsvd_solve_fp8(plan: int, A, col_scale, k: int, p: int, q: int, t: float, omega, U, S, V,
                   K) -> int:
    m, n = A.shape
    if omega is not None:
        assert omega.is_contiguous() and omega.element_size() == 8
    return _check(load_library().rsvd_solve_fp8(plan, _ptr(A), _ptr(col_scale), m, n, _ld(A), k,
                                                p, q, float(t), _ptr(omega), _ptr(U), _ld(U),
                                                _ptr(S), _ptr(V), _ld(V), _ptr(K)),
                  "rsvd_solve_fp8")


def rsvd_quantize_fp8(plan: int, A, Aq, col_scale) -> int:
    m, n = A.shape
    return _check(load_library().rsvd_quantize_fp8(plan, _ptr(A), m, n, _ld(A), _ptr(Aq),
                                                   _ld(Aq), _ptr(col_scale)),
                  "rsvd_quantize_fp8")


def rsvd_quantize_bf16(plan: int, A, Aq, col_scale) -> int:
    m, n = A.shape
    return _check(load_library().rsvd_quantize_bf16(plan, _ptr(A), m, n, _ld(A), _ptr(Aq),
                                                    _ld(Aq), _ptr(col_scale)),
                  "rsvd_quantize_bf16")


def gram_eig_solve(plan: int, A, t: float, ucols: int, U, S, V, K) -> int:
    m, n = A.shape
    ldu = _ld(U) if U is not None else 0
    return _check(load_library().gram_eig_solve(plan, _ptr(A), m, n, _ld(A), float(t), ucols,
                                                _ptr(U), ldu, _ptr(S), _ptr(V), _ld(V), _ptr(K)),
                  "gram_eig_solve")


def rsvd_gaussian_fill(seed: int, G, stream=None) -> int:
    rows, cols = G.shape
    assert G.is_contiguous() and G.element_size() == 8
    return _check(load_library().rsvd_gaussian_fill(seed, rows, cols, _ptr(G), _stream_ptr(stream)),
                  "rsvd_gaussian_fill")


def rsvd_gemm_nn(plan: int, A, X, Y, Gram=None, fro2=None) -> int:
    m, n = A.shape
    c = X.shape[1]
    return _check(load_library().rsvd_gemm_nn(plan, _ptr(A), m, n, _ld(A), _ptr(X), _ld(X), c,
                                              _ptr(Y), _ld(Y), _ptr(Gram), _ptr(fro2)),
                  "rsvd_gemm_nn")


def rsvd_gemm_tn(plan: int, A, Q, Z) -> int:
    m, n = A.shape
    c = Q.shape[1]
    assert Z.is_contiguous() and tuple(Z.shape) == (n, c)
    return _check(load_library().rsvd_gemm_tn(plan, _ptr(A), m, n, _ld(A), _ptr(Q), _ld(Q), c,
                                              _ptr(Z)), "rsvd_gemm_tn")


def rsvd_cholqr2(plan: int, Y, Q, R) -> int:
    m, c = Y.shape
    assert R.is_contiguous()
    return _check(load_library().rsvd_cholqr2(plan, _ptr(Y), m, c, _ld(Y), _ptr(Q), _ld(Q),
                                              _ptr(R)), "rsvd_cholqr2")


def rsvd_small_svd(plan: int, T, Vt, S, W) -> int:
    r, c = T.shape
    assert T.is_contiguous() and Vt.is_contiguous() and W.is_contiguous()
    return _check(load_library().rsvd_small_svd(plan, _ptr(T), r, c, _ptr(Vt), _ptr(S), _ptr(W)),
                  "rsvd_small_svd")


def rsvd_sym_eig(plan: int, G, lam, V) -> int:
    n = G.shape[0]
    assert G.is_contiguous() and V.is_contiguous()
    return _check(load_library().rsvd_sym_eig(plan, _ptr(G), n, _ptr(lam), _ptr(V)),
                  "rsvd_sym_eig")


# ------------------------------------------------------- convenience class --
class Result(NamedTuple):
    U: object
    S: object
    V: object
    K: int
    status: int


class Plan:
    """Owns an rsvd plan; allocates outputs as torch tensors on the device."""

    def __init__(self, m_max: int, n_max: int, l_max: int, dtype, want_gram: bool = False,
                 seed: int = 0, stream=None):
        import torch
        self.torch = torch
        code = {torch.float64: RSVD_F64, torch.float32: RSVD_F32, torch.bfloat16: RSVD_BF16,
                torch.float8_e4m3fn: RSVD_FP8}[dtype]
        self.storage = dtype
        # outputs of a bfloat16 or fp8 plan are float
        self.dtype = torch.float32 if code in (RSVD_BF16, RSVD_FP8) else dtype
        self.handle = rsvd_plan_create(m_max, n_max, l_max, code, want_gram, seed, stream)
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if self.handle:
            rsvd_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out(self, shape, dtype=None):
        return self.torch.empty(shape, dtype=dtype or self.dtype, device=self.device)

    def status(self) -> int:
        return rsvd_plan_status(self.handle)

    def diag(self):
        return rsvd_plan_diag(self.handle)

    def solve(self, A, k: int, p: int, q: int, t: float, omega=None, sync: bool = True,
              col_scale=None):
        m, n = A.shape
        torch = self.torch
        U = self._out((m, k)); V = self._out((n, k))
        S = self._out((k,), torch.float64); K = self._out((1,), torch.int32)
        if omega is None:
            rsvd_solve(self.handle, A, k, p, q, t, U, S, V, K, col_scale=col_scale)
        else:
            rsvd_solve_omega(self.handle, A, k, p, q, t, omega, U, S, V, K, col_scale=col_scale)
        if not sync:
            return Result(U, S, V, K, 0)
        st = self.status()
        return Result(U, S, V, int(K.item()), st)

    def solve_adaptive(self, A, k: int, p: int, q: int, t: float, k_max: int, col_scale=None):
        """Randomized PCA with the rank grown in blocks of min(k + p, n)
        columns until the threshold t can be met (rsvd_solve_adaptive); U, S,
        V hold k_max columns (the first min(k_max, L) written), L = the
        basis size, from the plan's diagnostics."""
        m, n = A.shape
        torch = self.torch
        U = self._out((m, k_max)); V = self._out((n, k_max))
        S = self._out((k_max,), torch.float64); K = self._out((1,), torch.int32)
        rsvd_solve_adaptive(self.handle, A, k, p, q, t, k_max, U, S, V, K, col_scale=col_scale)
        st = self.status()
        return Result(U, S, V, int(K.item()), st)

    def solve_krylov(self, A, k: int, p: int, i: int, t: float, omega=None, sync: bool = True):
        """Krylov method with i + 1 blocks of l = min(k + p, n) columns
        (rsvd_solve_krylov)."""
        m, n = A.shape
        torch = self.torch
        U = self._out((m, k)); V = self._out((n, k))
        S = self._out((k,), torch.float64); K = self._out((1,), torch.int32)
        rsvd_solve_krylov(self.handle, A, k, p, i, t, omega, U, S, V, K)
        if not sync:
            return Result(U, S, V, K, 0)
        st = self.status()
        return Result(U, S, V, int(K.item()), st)

    def quantize(self, A):
        """Storage of an fp32 matrix in the plan's format (bfloat16 or FP8 E4M3):
        (Aq, col_scale) with power-of-two column scales (rsvd_quantize_bf16 /
        rsvd_quantize_fp8)."""
        m, n = A.shape
        Aq = self.torch.empty((m, n), dtype=self.storage, device=self.device)
        s = self.torch.empty((n,), dtype=self.torch.float32, device=self.device)
        if self.storage == self.torch.float8_e4m3fn:
            rsvd_quantize_fp8(self.handle, A, Aq, s)
        else:
            rsvd_quantize_bf16(self.handle, A, Aq, s)
        return Aq, s

    def gram_eig(self, A, t: float, ucols: Optional[int] = None, sync: bool = True):
        m, n = A.shape
        torch = self.torch
        uc = n if ucols is None else ucols
        U = self._out((m, uc)) if uc > 0 else None
        S = self._out((n,), torch.float64); V = self._out((n, n)); K = self._out((1,), torch.int32)
        gram_eig_solve(self.handle, A, t, uc, U, S, V, K)
        if not sync:
            return Result(U, S, V, K, 0)
        st = self.status()
        return Result(U, S, V, int(K.item()), st)


class Batch:
    """Many Randomized PCA problems of different shapes on `nslots` slots
    (rsvd_batch_*).  `problems` is a list of (A, k, p, q, t) or, for a
    bfloat16 / FP8 batch, (A, k, p, q, t, col_scale); outputs are allocated
    per problem.  solve() runs them now; graph() captures the same solves
    (same A and output tensors) into a replayable HIP graph."""

    def __init__(self, nslots: int, m_max: int, n_max: int, l_max: int, dtype, seed: int = 0):
        import torch
        self.torch = torch
        code, self.dtype = _dtype_codes(torch)[dtype]
        h = ctypes.c_void_p()
        _check(load_library().rsvd_batch_create(ctypes.byref(h), nslots, m_max, n_max, l_max,
                                                code, seed), "rsvd_batch_create")
        self.handle = h.value
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if self.handle:
            _check(load_library().rsvd_batch_destroy(self.handle), "rsvd_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, problems):
        """Output tensors and the C instance array for `problems`."""
        torch = self.torch
        outs, arr = [], (RsvdInstance * len(problems))()
        for i, pr in enumerate(problems):
            A, k, p, q, t = pr[:5]
            cs = pr[5] if len(pr) > 5 else None
            m, n = A.shape
            o = dict(U=torch.empty((m, k), dtype=self.dtype, device=self.device),
                     V=torch.empty((n, k), dtype=self.dtype, device=self.device),
                     S=torch.empty((k,), dtype=torch.float64, device=self.device),
                     K=torch.empty((1,), dtype=torch.int32, device=self.device),
                     status=torch.empty((1,), dtype=torch.int32, device=self.device), A=A)
            arr[i] = RsvdInstance(A.data_ptr(), m, n, _ld(A), k, p, q, float(t),
                                  o["U"].data_ptr(), _ld(o["U"]), o["S"].data_ptr(),
                                  o["V"].data_ptr(), _ld(o["V"]), o["K"].data_ptr(),
                                  o["status"].data_ptr(), _ptr(cs), 0,
                                  _dtype_codes(torch)[A.dtype][0])
            o["col_scale"] = cs
            outs.append(o)
        return outs, arr

    def solve(self, problems, stream=None, prepared=None):
        outs, arr = prepared if prepared is not None else self.prepare(problems)
        _check(load_library().rsvd_batch_solve(self.handle, arr, len(arr), _stream_ptr(stream)),
               "rsvd_batch_solve")
        return outs

    def grouped(self, problems, prepared=None, tune=None):
        """The same solves as a grouped batch (fp32 batches only); `tune` is
        a list of (n, l, panel_rows, split_rows) tile parameters."""
        outs, arr = prepared if prepared is not None else self.prepare(problems)
        g = ctypes.c_void_p()
        tarr, nt = _tune_array(tune)
        _check(load_library().rsvd_batch_grouped_create(self.handle, arr, len(arr), tarr, nt,
                                                        ctypes.byref(g)),
               "rsvd_batch_grouped_create")
        return BatchGrouped(g.value, outs)

    def tune_grouped(self, problems, prepared=None, stream=None, cap: int = 64):
        """Autotune the grouped tile parameters on these problems (runs
        them): [(n, l, panel_rows, split_rows)] per (n, l) bucket."""
        outs, arr = prepared if prepared is not None else self.prepare(problems)
        out = (RsvdTuneEntry * cap)()
        nout = ctypes.c_int32()
        _check(load_library().rsvd_batch_grouped_tune(self.handle, arr, len(arr), out, cap,
                                                      ctypes.byref(nout), _stream_ptr(stream)),
               "rsvd_batch_grouped_tune")
        return [(e.n, e.l, e.panel_rows, e.split_rows) for e in out[:nout.value]]

    def graph(self, problems, prepared=None):
        outs, arr = prepared if prepared is not None else self.prepare(problems)
        g = ctypes.c_void_p()
        _check(load_library().rsvd_batch_graph_create(self.handle, arr, len(arr), None,
                                                      ctypes.byref(g)), "rsvd_batch_graph_create")
        return BatchGraph(g.value, outs)


class BatchGrouped:
    """A grouped batch (rsvd_batch_grouped_*): every step one launch for all
    problems; launch() runs it on a stream."""

    def __init__(self, handle, outs):
        self.handle, self.outs = handle, outs

    def launch(self, stream=None):
        _check(load_library().rsvd_batch_grouped_launch(self.handle, _stream_ptr(stream)),
               "rsvd_batch_grouped_launch")
        return self.outs

    def graph(self):
        """One launch of this grouped batch captured into a HIP graph (which
        keeps this object alive)."""
        g = ctypes.c_void_p()
        _check(load_library().rsvd_batch_grouped_graph_create(self.handle, ctypes.byref(g)),
               "rsvd_batch_grouped_graph_create")
        return BatchGraph(g.value, self.outs, owner=self)

    def close(self):
        if self.handle:
            _check(load_library().rsvd_batch_grouped_destroy(self.handle),
                   "rsvd_batch_grouped_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """A captured batch; launch() replays it on a stream."""

    def __init__(self, handle, outs, owner=None):
        self.handle, self.outs, self.owner = handle, outs, owner

    def launch(self, stream=None):
        _check(load_library().rsvd_batch_graph_launch(self.handle, _stream_ptr(stream)),
               "rsvd_batch_graph_launch")
        return self.outs

    def close(self):
        if self.handle:
            _check(load_library().rsvd_batch_graph_destroy(self.handle), "rsvd_batch_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching of Randomized PCA requests (rsvd_server_*): submit()
    queues a request and returns its ticket; progress() never blocks and
    returns the tickets that finished since the last call (their outputs,
    kept in `results[ticket]`, are then complete).  Requests may store A in
    fp32, bfloat16 or FP8 on one server (other than FP64); gram_fallback adds
    the A^T A-route slot for requests whose K is predicted past n / 2."""

    def __init__(self, nslots: int, m_max: int, n_max: int, l_max: int, dtype, seed: int = 0,
                 hbm_budget: int = 1 << 40, gram_fallback: bool = False):
        import torch
        self.torch = torch
        code, self.dtype = _dtype_codes(torch)[dtype]
        h = ctypes.c_void_p()
        flags = RSVD_SERVER_GRAM_FALLBACK if gram_fallback else 0
        _check(load_library().rsvd_server_create(ctypes.byref(h), nslots, m_max, n_max, l_max,
                                                 code, seed, int(hbm_budget), flags),
               "rsvd_server_create")
        self.handle = h.value
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.results = {}
        self._buf = (ctypes.c_int64 * 1024)()

    def submit(self, A, k: int, p: int, q: int, t: float, col_scale=None, k_max: int = 0,
               want_u: bool = True) -> int:
        """Queue a request (A in fp32, bfloat16 or FP8 E4M3 with col_scale, or
        fp64 on an fp64 server); with k_max > k its rank grows in blocks of
        k + p columns until t can be met (or the A^T A route takes it), K is
        capped at k_max, and U, S, V hold k_max columns (no U with
        want_u=False), of which the first min(k_max, columns found) are
        written; S starts at zero, so its unwritten tail reads 0."""
        torch = self.torch
        m, n = A.shape
        kc = max(k, k_max)
        code = _dtype_codes(torch)[A.dtype][0]
        o = dict(U=torch.empty((m, kc), dtype=self.dtype, device=self.device) if want_u else None,
                 V=torch.empty((n, kc), dtype=self.dtype, device=self.device),
                 S=torch.zeros((kc,), dtype=torch.float64, device=self.device),
                 K=torch.empty((1,), dtype=torch.int32, device=self.device),
                 status=torch.empty((1,), dtype=torch.int32, device=self.device), A=A)
        req = RsvdInstance(A.data_ptr(), m, n, _ld(A), k, p, q, float(t), _ptr(o["U"]),
                           _ld(o["U"]) if want_u else 0, o["S"].data_ptr(), o["V"].data_ptr(),
                           _ld(o["V"]),
                           o["K"].data_ptr(), o["status"].data_ptr(), _ptr(col_scale),
                           int(k_max), code)
        o["col_scale"] = col_scale
        tk = ctypes.c_int64()
        _check(load_library().rsvd_server_submit(self.handle, ctypes.byref(req), ctypes.byref(tk)),
               "rsvd_server_submit")
        self.results[tk.value] = o
        return tk.value

    def progress(self):
        """(finished tickets, queued, running)."""
        nd, qd, rn = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().rsvd_server_progress(self.handle, self._buf, len(self._buf),
                                                   ctypes.byref(nd), ctypes.byref(qd),
                                                   ctypes.byref(rn)), "rsvd_server_progress")
        return list(self._buf[:nd.value]), qd.value, rn.value

    def close(self):
        if self.handle:
            _check(load_library().rsvd_server_destroy(self.handle), "rsvd_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
