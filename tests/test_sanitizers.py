"""AddressSanitizer + UndefinedBehaviorSanitizer builds (CPU only) of the FP64
oracle and of the host runtime of the library: the oracle runs a few steps of
every equation, boundary kind and limiter option; the host runtime (device
entry points replaced by stand-ins) runs the Fourier CFL analysis over every
option and crkfr_create's refusals of bad configurations.  A memory error or
undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ROCM = "/opt/rocm"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
          os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "crkfr_oracle.c"), "-lm"])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="1"))
    assert "0 failed statuses" in r.stdout


@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "bin", "hipcc")), reason="no ROCm toolchain")
def test_host_runtime_under_asan_ubsan(tmp_path):
    hip = [os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    host_o, stub_o, drv_o = (str(tmp_path / n) for n in ("host.o", "stubs.o", "driver.o"))
    _run(hip + ["-c", os.path.join(ROOT, "paper_2502_07517_amd", "csrc", "crkfr_host.hip"), "-o", host_o])
    _run(hip + ["-c", os.path.join(SAN, "host_stubs.hip"), "-o", stub_o])
    cxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not os.path.exists(cxx):
        cxx = shutil.which("clang++") or "g++"
    _run([cxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-c",
          os.path.join(SAN, "host_driver.cpp"), "-o", drv_o])
    exe = str(tmp_path / "host_san")
    _run([cxx, "-fsanitize=address,undefined", drv_o, host_o, stub_o, "-L" + os.path.join(ROCM, "lib"),
          "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert "0 failures" in r.stdout
