"""AddressSanitizer + UndefinedBehaviorSanitizer builds on the CPU.

1. The oracle (oracle/boba_oracle.c), compiled with gcc and the sanitizers
   into tests/sanitize/oracle_driver.c, which calls every oracle function on
   seeded graphs, edge cases and invalid IDs.
2. The host-side code of libboba.so (argument checks, plans, workspace
   carving): every source compiled with the host pass instrumented (device
   code is unchanged and never runs here), then the boundary tests run through
   the C ABI in a subprocess with the sanitizer runtime preloaded.
Any sanitizer report aborts the program, which fails the test."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is required")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-Wall", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", ROOT, "-o", exe,
                    os.path.join(SAN, "oracle_driver.c"), "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle driver ok" in r.stdout


def _asan_runtime(hipcc):
    out = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    return out if out and os.path.isabs(out) and os.path.exists(out) else None


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2306_10410_amd import build as B
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc is required")
    runtime = _asan_runtime(hipcc)
    if runtime is None:
        pytest.skip("clang's AddressSanitizer runtime was not found")
    # -Xarch_host before each sanitizer option: the host pass only
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in B.HIPCC_FLAGS if f != "-O3"] + ["-O1", "-g"] + host_san

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        r = subprocess.run([hipcc, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj], capture_output=True,
                           text=True)
        assert r.returncode == 0, r.stderr
        return obj

    with ThreadPoolExecutor(min(8, len(B.SOURCES))) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    lib = str(tmp_path / "libboba_asan.so")
    r = subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *host_san[:4], "-o", lib, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # the build really is instrumented
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_handle" in syms
    env = {**os.environ, "LD_PRELOAD": runtime, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
    r = subprocess.run([sys.executable, os.path.join(SAN, "run_boundary.py"), lib], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "boundary ok" in r.stdout
