"""Invariants of the Stockham pass kernels, checked on the host for every plan.

The checker (csrc/fft_plan_check.h) runs when a Poisson or raw FFT plan is
created and turns a plan that breaks an invariant into DKS_EUNSUPPORTED.
Here: every length the library accepts passes with the committed engine
constants (through the C ABI and through a host-only harness of the same
header), one planted mistake per invariant is caught, and the harness shows
which plans the engine constants of an earlier, never-committed variant
(32 KiB LDS budget, 256 / 128 threads) would have broken.
"""

import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1509_07685_amd", "libdks_poisson.so")


def lengths_23(limit):
    out = []
    for n in range(1, limit + 1):
        m = n
        while m % 2 == 0:
            m //= 2
        while m % 3 == 0:
            m //= 3
        if m == 1:
            out.append(n)
    return out


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan_check") / "plan_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_1509_07685_amd", "csrc"),
                    os.path.join(ROOT, "tests", "c", "plan_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows, planted = {}, {}
    for line in out.splitlines():
        parts = line.split()
        if parts[0] == "planted":
            planted[parts[1]] = int(parts[2])
        elif parts[0] == "ok":
            planted["ok"] = int(parts[1])
        else:
            key = (parts[0], parts[1])
            rows[key] = {}
            for p in parts[5:]:
                role, counts = p.split(":")
                rows[key][role] = [int(v) for v in counts.split("/")]
    return rows, planted


def test_committed_constants_satisfy_every_invariant(harness):
    rows, _ = harness
    for dt in ("f32", "f64"):
        for role, counts in rows[("committed", dt)].items():
            assert sum(counts[1:]) == 0, (dt, role, counts)
            assert counts[0] > 40


def test_each_planted_mistake_is_caught(harness):
    _, planted = harness
    assert planted == {"structure": 1, "tile_shape": 2, "coverage": 3, "tile_load": 4, "lds": 5, "ok": 0}


def test_variant_constants_break_coverage_only_above_2048_fp64(harness):
    """A 32 KiB budget with 128 FP64 threads leaves 16 complex values per
    thread, but a single pencil of more than 2048 FP64 values no longer fits
    the budget: its passes would need more butterfly slots than the threads
    have (wrong outputs, not a stall).  Lengths up to 2048, which include
    every mesh up to 1024^3, satisfy every invariant."""
    rows, _ = harness
    v = rows[("variant_lds32k_t256", "f64")]
    assert v["cols"][3] == 7 and sum(v["cols"][1:]) == 7
    assert v["x_fwd"][0] == 47 and sum(v["x_fwd"][1:]) == 0
    f = rows[("variant_lds32k_t256", "f32")]
    assert all(sum(c[1:]) == 0 for c in f.values())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdks_poisson.so not built")
def test_every_accepted_mesh_plans_in_both_dtypes():
    from paper_1509_07685_amd import dks
    lib = dks._lib
    plan = ctypes.c_void_p()
    meshes = [n for n in lengths_23(2048) if n >= 2 and 2 * n in lengths_23(4096)]
    for dt in (dks.DKS_F32, dks.DKS_F64):
        for n in meshes:
            for shape in ((n, 2, 3), (3, n, 2), (2, 4, n)):
                assert lib.dks_poisson_plan(*shape, 1.0, 1.0, 1.0, dt, ctypes.byref(plan)) == dks.DKS_OK, (shape, dt)
                assert lib.dks_poisson_destroy(plan) == dks.DKS_OK


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdks_poisson.so not built")
def test_every_accepted_raw_fft_length_plans_in_both_dtypes():
    from paper_1509_07685_amd import dks
    lib = dks._lib
    plan = ctypes.c_void_p()
    for dt in (dks.DKS_F32, dks.DKS_F64):
        for kind in (dks.DKS_FFT_C2C, dks.DKS_FFT_R2C):
            for n in lengths_23(4096):
                if kind == dks.DKS_FFT_R2C and n % 2:
                    continue
                assert lib.dks_fft_plan(n, 2, 3, 1, kind, dt, ctypes.byref(plan)) == dks.DKS_OK, (n, dt, kind)
                assert lib.dks_fft_destroy(plan) == dks.DKS_OK
                assert lib.dks_fft_plan(2, n, 3, 1, kind, dt, ctypes.byref(plan)) == dks.DKS_OK, (n, dt, kind)
                assert lib.dks_fft_destroy(plan) == dks.DKS_OK
