"""The host code of the library (argument checks, parameter validation,
level shapes, workspace carving, error strings) built with AddressSanitizer
and UndefinedBehaviorSanitizer on the host side and exercised by a C driver
that never reaches a device (`tests/host/validation_driver.c`).  Device code
is compiled as usual; only the host pass carries the sanitizers."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_08463_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm toolchain")
def test_host_validation_under_asan_ubsan(tmp_path):
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    lib = tmp_path / "libfracture_san.so"
    cmd = ([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-pthread", "--offload-arch=gfx950",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN
           + ["-I", os.path.join(ROOT, "include"), "-shared", "-o", str(lib)] + srcs)
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-4000:]
    exe = tmp_path / "driver"
    res = subprocess.run([CLANG, "-g", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
                          os.path.join(ROOT, "tests", "host", "validation_driver.c"), "-L", str(tmp_path),
                          "-lfracture_san", f"-Wl,-rpath,{tmp_path}", "-o", str(exe)],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(res.stdout, res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "host validation ok" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
