"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the FP64 oracle
and of the host side of the C ABI (the host geometry builder and handle
queries), each driven on 2D and 3D scenes and every rejection path by a small
driver program.  Host code only: nothing here touches a GPU.  A planted
buffer overrun (a per-walk buffer one entry short handed to the oracle's
solver) must be reported, which shows the sanitizer is live."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DRIVER = os.path.join(ROOT, "oracle", "asan_check.c")
HOST_DRIVER = os.path.join(ROOT, "paper_2410_18944_amd", "csrc", "asan_host_check.cpp")
HOST_BUILDER = os.path.join(ROOT, "paper_2410_18944_amd", "csrc", "geom_build.cpp")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, timeout=300):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=ENV)


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("sanitizers")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(workdir):
    exe = str(workdir / "asan_oracle")
    b = _run(["gcc", "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-Wno-misleading-indentation", *SAN,
              ORACLE_DRIVER, "-o", exe, "-lm"])
    assert b.returncode == 0, b.stderr
    r = _run([exe])
    assert r.returncode == 0 and "asan oracle ok" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_planted_overrun_is_reported(workdir):
    exe = str(workdir / "asan_oracle_planted")
    b = _run(["gcc", "-std=c11", "-Wno-unknown-pragmas", "-Wno-misleading-indentation", *SAN,
              "-DWOST_PLANT_OVERRUN", ORACLE_DRIVER, "-o", exe, "-lm"])
    assert b.returncode == 0, b.stderr
    r = _run([exe])
    assert r.returncode != 0
    assert "AddressSanitizer: heap-buffer-overflow" in r.stderr, r.stderr[-2000:]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not available")
def test_host_abi_under_address_and_ub_sanitizers(workdir):
    exe = str(workdir / "asan_host")
    b = _run([CLANG, "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", HOST_BUILDER, HOST_DRIVER,
              "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    assert b.returncode == 0, b.stderr[-3000:]
    r = _run([exe])
    assert r.returncode == 0 and "asan host ok" in r.stdout, r.stdout + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
