"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers in tests/sanitize/ are built with the sanitizers and run: one
calls every routine of the CPU oracle on small systems and edge cases, the
other the host-only code of the runtime (configuration checks, workspace and
admission plans, the MSD schedule, the initial-state generators, md_init's
error path without a device).  Device code is not instrumented: GPU
sanitizers are not part of this toolchain's use here, and the runtime
driver's host objects are linked against the normally built kernel objects.
A test passes when its driver exits 0 with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

from paper_2001_07089_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, cwd=OUT, timeout=600)
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error:" not in text and "LeakSanitizer" not in text, text
    assert r.returncode == 0, text
    return text


def test_oracle_under_asan_and_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off", "-Wall",
           "-Wno-unknown-pragmas", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    assert "0 failed checks" in _run(exe)


def test_runtime_host_code_under_asan_and_ubsan():
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    kernels = [os.path.join(B.OBJDIR, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        B.build()
    os.makedirs(OUT, exist_ok=True)
    obj = os.path.join(OUT, "runtime_host_driver.o")
    exe = os.path.join(OUT, "runtime_host_driver")
    # sanitizers on the host side only (-Xarch_host before each option)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    cc = [hipcc, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-pthread", "-I", B.INCLUDE, "-I", B.CSRC,
          "-Xarch_host", "-fno-sanitize-recover=all"] + san + \
         ["-c", os.path.join(HERE, "sanitize", "runtime_host_driver.cpp"), "-o", obj]
    subprocess.run(cc, check=True, capture_output=True, text=True)
    ld = [hipcc, "--offload-arch=gfx950", "-pthread"] + san + [obj] + kernels + ["-o", exe]
    subprocess.run(ld, check=True, capture_output=True, text=True)
    assert "0 failed checks" in _run(exe)
