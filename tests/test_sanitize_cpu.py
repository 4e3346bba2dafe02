"""Host sanitizers (no GPU): the oracle's C sources and the host code of the
library's C ABI are built with AddressSanitizer and UndefinedBehavior-
Sanitizer (the device code of the library is built as usual), and a driver
(tests/sanitize/driver.c) runs the oracle on random pairs in both modes, a
small search and the Smith-Waterman checker, then every host-only path of
the ABI: defaults, checks, encoding, and the argument errors each entry point
returns before touching the device.  Any sanitizer report fails the run."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1508_06561_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang"
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.slow
def test_sanitized_oracle_and_host_abi(tmp_path):
    if not (os.path.exists(CLANG) and os.path.exists(HIPCC)):
        pytest.skip("ROCm clang / hipcc not available")
    lib = tmp_path / "libhs_san.so"
    # host code only: each -fsanitize= follows -Xarch_host
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=undefined",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(CSRC, "hs_lib.hip"), os.path.join(CSRC, "hs_server.cpp"),
                    "-lpthread", "-o", str(lib)], check=True, capture_output=True)
    exe = tmp_path / "driver"
    subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize", "driver.c"),
                    os.path.join(ROOT, "oracle", "hs_oracle.c"),
                    os.path.join(ROOT, "oracle", "sw_check.c"),
                    str(lib), f"-Wl,-rpath,{tmp_path}", "-o", str(exe)],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "all checks held" in r.stdout
