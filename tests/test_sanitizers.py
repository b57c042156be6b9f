"""Host sanitizer runs (CPU only, no GPU): the FP64 oracle (oracle/oracle.c)
and the library's host-side validation (argument and shape checks of the C
ABI, including sizes large enough to overflow careless 64-bit arithmetic)
built with AddressSanitizer and UndefinedBehaviorSanitizer and driven by the
programs in tests/sanitize/.  Any sanitizer report aborts the driver
(-fno-sanitize-recover), so the test only has to see exit status 0.  The
library is compiled for gfx950 as usual, with the sanitizers on its host
pass only (-Xarch_host); nothing is launched on a device."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-std=c99", "-O1", "-g", "-fopenmp", *SAN, "-o", exe,
         os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    r = run([exe], env=ENV)
    assert "oracle driver ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
@pytest.mark.timeout(900)
def test_abi_validation_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_1906_12085_amd", "csrc")
    host_san = [f for s in SAN for f in ("-Xarch_host", s)]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        run([HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj])
        return obj

    srcs = [os.path.join(csrc, f) for f in ("gemm.hip", "small.hip", "eig.hip", "lowp.hip",
                                            "rsvd.hip")]
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"))
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "abi_driver")
    run([HIPCC, "--offload-arch=gfx950", *host_san, "-o", exe, *objs])
    r = run([exe], env=ENV)
    assert "abi driver ok" in r.stdout
