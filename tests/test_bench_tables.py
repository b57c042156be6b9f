"""Host checks of bench.py's kernel tables (no GPU): every timed kernel names
its kernel and the peak it is compared with, and every measured HBM traffic
figure is tied to the current source text of the kernel it was measured on
(bench.py reports a figure only while that holds, so a kernel changed after
its counters were taken shows here, before a GPU run)."""
import importlib.util
import os
import sys

from conftest import ROOT


def _bench():
    spec = importlib.util.spec_from_file_location("bench_tables", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        spec.loader.exec_module(mod)
    finally:
        sys.argv = argv
    return mod


def test_kernel_info_entries():
    b = _bench()
    for kind, entry in b.KERNEL_INFO.items():
        assert len(entry) == 2, kind
        name, unit = entry
        assert name.startswith("k_") and unit in b.PEAK_TFLOPS or unit == "alu", kind


def test_traffic_figures_match_kernel_sources():
    b = _bench()
    for kind, entry in b.TRAFFIC.items():
        assert len(entry) == 4, kind
        nbytes, path, names, digest = entry
        assert nbytes > 0
        assert b.kernel_source_digest(path, names) == digest, (
            f"{kind}: {names} in {path} changed since its HBM counters were taken")
