"""The library's host-side planning code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host_sanitize/plans_driver.cpp drives host-only plans (random networks in every
precision and split policy, sparse states of random bitstrings, the creation error paths);
this test builds it with the library's sources, the sanitizers on the host side only (device
code is compiled as usual and never runs: host-only plans touch no GPU), runs it and checks
that it ends cleanly with no sanitizer report (leak detection on).  CPU only.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_03978_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN = ["-fsanitize=address", "-fsanitize=undefined"]


def _host_only(flags):
    # every sanitizer flag applies to the host compilation only
    out = []
    for f in flags:
        out += ["-Xarch_host", f]
    return out


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain missing")
def test_host_planning_is_clean_under_asan_and_ubsan():
    tmp = tempfile.mkdtemp(prefix="tn_asan_")
    try:
        objs = []
        common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Wno-unused-value",
                  "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        for src in ("tn_plan.cpp", "tn_kernels.hip", "tn_costmodel.hip"):
            obj = os.path.join(tmp, src + ".o")
            cmd = [HIPCC] + common + _host_only(SAN + ["-fno-omit-frame-pointer"]) + \
                  ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stdout + r.stderr
            objs.append(obj)
        drv = os.path.join(tmp, "driver.o")
        r = subprocess.run([CLANG, "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                            "-c", os.path.join(ROOT, "tests", "host_sanitize", "plans_driver.cpp"), "-o", drv],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        exe = os.path.join(tmp, "driver")
        r = subprocess.run([CLANG, "-fsanitize=address,undefined"] + objs + [drv, "-L/opt/rocm/lib", "-lamdhip64",
                            "-Wl,-rpath,/opt/rocm/lib", "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
        assert r.stdout.startswith("ok "), out[-2000:]
        assert int(r.stdout.split()[1]) >= 300, r.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
