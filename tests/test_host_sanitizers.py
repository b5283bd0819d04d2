"""The library's host code under sanitizers (CPU): the multilevel partitioner with its worker
pool, the on-the-fly update, the sequence / gap / Chebyshev helpers and the argument checks of
the device entry points, built with AddressSanitizer + UndefinedBehaviorSanitizer and, apart,
with ThreadSanitizer (host pass only; the device code is compiled as usual and never runs)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.slow


def _build_and_run(tmp_path, sanitizers):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_1603_00937_amd.build import SOURCES, PROBE_SOURCES, hipcc_flags
    srcs = [os.path.join(ROOT, "paper_1603_00937_amd", "csrc", s)
            for s in SOURCES + PROBE_SOURCES]
    flags = [f for f in hipcc_flags() if f not in ("-shared", "-fPIC", "-O3")] + ["-O1", "-g"]
    san = []
    for s in sanitizers:
        san += ["-Xarch_host", f"-fsanitize={s}"]
    exe = str(tmp_path / "host_driver")
    cmd = [HIPCC, *flags, *san, "-Xarch_host", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
           *srcs, os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ok" in r.stdout, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out, out[-4000:]


def test_host_code_under_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, ["address", "undefined"])


def test_host_code_under_tsan(tmp_path):
    _build_and_run(tmp_path, ["thread"])
