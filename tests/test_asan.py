"""Host code under AddressSanitizer (and UndefinedBehaviorSanitizer for the
oracle): the oracle's C part, and the library's host runtime (plan
creation, validation, workspace layout, the engine-invariant checks, the
status strings) built with host-side ASan and driven by the plain C client.
CPU only; the device code is built as usual (sanitizers apply to host code
only here)."""

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1509_07685_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")


def run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_c_part_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_igf_client"
    r = run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             os.path.join(ROOT, "tests", "c", "oracle_igf_client.c"), os.path.join(ROOT, "oracle", "igf_quad.c"),
             "-o", str(exe), "-lquadmath", "-lm"])
    assert r.returncode == 0, r.stderr
    r = run([str(exe)], env=ENV, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not available")
def test_host_runtime_under_asan(tmp_path):
    from paper_1509_07685_amd import build as B
    srcs = list(B.SOURCES)
    flags = [f for f in B.COMMON] + ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                                     "-fno-omit-frame-pointer"]

    def compile_one(src):
        obj = tmp_path / (os.path.splitext(src)[0] + ".o")
        return run([B.hipcc(), *flags, *B.EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", str(obj)]), obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(compile_one, srcs))
    for (r, _), src in zip(results, srcs):
        assert r.returncode == 0, (src, r.stderr[-2000:])
    lib = tmp_path / "libdks_poisson.so"
    r = run([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
             *[str(o) for _, o in results], "-o", str(lib)])
    assert r.returncode == 0, r.stderr[-2000:]
    # the client is linked by the same compiler as the library, so that both
    # use its sanitizer runtime
    clang = os.path.join(os.path.dirname(os.path.realpath(B.hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    exe = tmp_path / "abi_client"
    r = run([clang, "-std=c99", "-g", "-fsanitize=address", "-I", os.path.join(ROOT, "include"),
             os.path.join(ROOT, "tests", "c", "abi_client.c"), "-o", str(exe), "-L", str(tmp_path), "-ldks_poisson",
             f"-Wl,-rpath,{tmp_path}"])
    assert r.returncode == 0, r.stderr
    r = run([str(exe)], env=ENV, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert r.stdout.startswith("ok ")
