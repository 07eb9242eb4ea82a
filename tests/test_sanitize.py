"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (no
GPU needed): the CPU oracle (plain and OpenMP builds) driven through every
entry point on small 2D and 3D grids, and the C ABI's host argument checks
(every entry point called with arguments it must reject before any device
work).  Either run fails on any sanitizer report, including leaks.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
SANFLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=120)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report
    assert "runtime error" not in report and "Sanitizer" not in report, report


@pytest.mark.parametrize("omp", [False, True])
def test_oracle_under_sanitizers(tmp_path, omp):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    exe = str(tmp_path / "oracle_san")
    cmd = (["gcc"] + SANFLAGS + (["-fopenmp"] if omp else []) +
           ["-std=c99", os.path.join(ROOT, "oracle", "mg_oracle.c"),
            os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    subprocess.run(cmd, check=True, capture_output=True)
    _run(exe)


def test_abi_argument_checks_under_sanitizers(tmp_path):
    # the host part of mg_api.cpp is built with the sanitizers (device code
    # as usual) and linked with the library's kernel objects
    build = os.path.join(ROOT, "paper_2206_05543_amd", "_build")
    kobjs = [os.path.join(build, f) for f in ("mg_kernels.hip.o", "mg_adjoint.hip.o")]
    if not os.path.exists(HIPCC) or not all(os.path.exists(o) for o in kobjs):
        pytest.skip("hipcc or the library's object files are missing")
    inc = "-I" + os.path.join(ROOT, "include")
    api = str(tmp_path / "api_san.o")
    drv = str(tmp_path / "abi_driver.o")
    exe = str(tmp_path / "abi_san")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", inc,
                    "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host",
                    "-fno-omit-frame-pointer", "-x", "hip", "-c",
                    os.path.join(ROOT, "paper_2206_05543_amd", "csrc", "mg_api.cpp"), "-o", api],
                   check=True, capture_output=True)
    subprocess.run(["g++"] + SANFLAGS + ["-std=c++17", inc, "-c",
                                         os.path.join(SAN, "abi_driver.cpp"), "-o", drv],
                   check=True, capture_output=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address,undefined",
                    drv, api] + kobjs + ["-o", exe], check=True, capture_output=True)
    _run(exe)
