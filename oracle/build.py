"""Builds the oracle's C sources into a shared library with gcc.

Test infrastructure only: the oracle is loaded by the tests, the smoke check
and the benchmark's CPU-baseline leg, never by the product library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")
SOURCES = ["hs_oracle.c", "sw_check.c"]


def build(extra_flags=(), out=LIB):
    """Compile the oracle (always recompiles) and return the library path."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", out + ".tmp", *srcs, *extra_flags]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
