"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the CPU oracle's whole pipeline, and liblogfx's host-only entry points
(mask construction, argument checks, calls refused before any device work),
each built with gcc/g++ -fsanitize=address,undefined into a small driver
program (tests/sanitize/) and run; any sanitizer report fails the test."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, cwd=None, timeout=600):
    return subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=ENV)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    r = _run(["gcc", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-ffp-contract=off", "-pthread", *SAN,
              os.path.join(ROOT, "tests", "sanitize", "oracle_pipeline.c"), os.path.join(ROOT, "oracle", "logfx_oracle.c"),
              "-lm", "-o", exe])
    assert r.returncode == 0, r.stderr
    r = _run([exe])
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"),
                    reason="needs g++ and the ROCm headers")
def test_host_entry_points_under_sanitizers(tmp_path):
    """The host runtime compiled by g++ with the sanitizers, linked with the
    library's own kernel objects (built by the package build, not
    instrumented: device code is out of reach of these tools)."""
    build = os.path.join(ROOT, "paper_1304_3992_amd", "_build")
    objs = sorted(o for o in glob.glob(os.path.join(build, "*.o")) if not o.endswith("logfx_host.o"))
    if not objs:
        pytest.skip("the library has not been built (python -m paper_1304_3992_amd.build)")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1304_3992_amd", "csrc"),
           "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    host_o = str(tmp_path / "host.o")
    r = _run(["g++", "-std=c++17", *SAN, *inc, "-c", os.path.join(ROOT, "paper_1304_3992_amd", "csrc", "logfx_host.cpp"),
              "-o", host_o])
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "host_san")
    r = _run(["g++", "-std=c++17", *SAN, *inc, os.path.join(ROOT, "tests", "sanitize", "host_entry_points.cpp"),
              host_o, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    assert r.returncode == 0, r.stderr
    r = _run([exe])
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
