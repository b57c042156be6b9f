"""Helpers for the GPU parity tests (test-side only)."""
import sys

import numpy as np

EPS64 = np.finfo(np.float64).eps
U32 = 2.0 ** -24


def announce(msg: str) -> None:
    """Name the case before a GPU step runs (so a hang or fault names it)."""
    print(f"[case] {msg}", file=sys.stderr, flush=True)


def dev(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t) -> np.ndarray:
    return t.detach().double().cpu().numpy()


def align_columns(X: np.ndarray, Xref: np.ndarray) -> np.ndarray:
    """Flip columns of X to the sign of Xref (both k columns)."""
    s = np.sign(np.sum(X * Xref, axis=0))
    s[s == 0] = 1.0
    return X * s


def sign_rule_holds(V: np.ndarray) -> bool:
    """The lowest-index entry within 0.1% of the largest magnitude is positive."""
    for j in range(V.shape[1]):
        v = V[:, j]
        vmax = np.abs(v).max()
        if vmax == 0:
            continue
        i = int(np.argmax(np.abs(v) >= 0.999 * vmax))
        if v[i] < 0:
            return False
    return True


def rounded(x: np.ndarray, torch_dtype) -> np.ndarray:
    """x rounded to the storage dtype the GPU path sees, back in FP64."""
    import torch
    if torch_dtype == torch.float32:
        return x.astype(np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)
