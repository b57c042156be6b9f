import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workload, tens of seconds")


def load_golden(name):
    """Parse a golden fixture: '#' comments, 'KEY: row ; row ; ...' entries."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            rows = [[float(x) for x in r.split()] for r in val.split(";")]
            arr = np.array(rows)
            if arr.size == 1:
                out[key.strip()] = float(arr.ravel()[0])
            else:
                out[key.strip()] = arr[0] if arr.shape[0] == 1 else arr
    return out


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build()
    yield


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
