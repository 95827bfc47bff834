"""Compile the oracle's C part (oracle/igf_quad.c) with gcc, in-tree.

TEST INFRASTRUCTURE ONLY: the library built here is loaded by the oracle,
which only the test suite, the smoke check and the benchmark's CPU-baseline
leg use.

    python -m oracle.build
"""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "igf_quad.c")
LIB = os.path.join(HERE, "liboracle_igf.so")


def build():
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("gcc not found; the oracle's Green's function library cannot be built")
    tmp = LIB + ".tmp"
    cmd = [cc, "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall", SRC, "-o", tmp, "-lquadmath", "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"gcc failed for {SRC}:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def ensure_built():
    """Build the library when it is missing or older than its source."""
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build())
