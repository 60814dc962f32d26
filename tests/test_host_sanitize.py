"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The four HIP sources are compiled with the sanitizers on the host side only
(`-Xarch_host`), linked with a C++ driver (`host_sanitize/abi_host_paths.cpp`)
that calls every entry point of the C ABI with arguments the host checks
reject, and, where no GPU is present, with arguments that pass those checks
so that the clean-up after a failed device call runs.  Any sanitizer report
or unmet expectation fails the test.  CPU only: the driver never launches a
kernel.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1409_2065_amd import build as B  # noqa: E402

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    try:
        return B.hipcc()
    except RuntimeError:
        return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_abi_host_paths_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    flags = [f"--offload-arch={B.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")] + SAN
    procs, objs = [], []
    for src in B.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for src, p in zip(B.SOURCES, procs):
        out, _ = p.communicate()
        assert p.returncode == 0, f"{src}:\n{out[-3000:]}"
    exe = str(tmp_path / "abi_host_paths")
    drv = os.path.join(ROOT, "tests", "host_sanitize", "abi_host_paths.cpp")
    r = subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-O1", "-g", "-std=c++17",
                        "-I", os.path.join(ROOT, "include"), *SAN[:4], "-x", "hip", drv, "-x", "none",
                        *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error:" not in text, text[-4000:]
    assert r.returncode == 0, text[-4000:]
    assert "0 failed" in r.stdout
