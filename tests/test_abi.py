"""C ABI contract checks that need no GPU: the library loads, exports every
entry point the header declares, and rejects bad arguments on the host
before any device work."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_1509_07685_amd", "libdks_poisson.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdks_poisson.so not built")


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dks_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dks_poisson_plan", "dks_poisson_solve_rho", "dks_poisson_solve_particles",
                     "dks_poisson_solve_particles_batched", "dks_poisson_prepare", "dks_poisson_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_1509_07685_amd import dks
    assert sorted(dks.EXPORTS) == declared_functions()
    for name in declared_functions():
        assert callable(getattr(dks, name))


@pytest.fixture()
def dks():
    from paper_1509_07685_amd import dks as mod
    return mod


def _status(fn, *args):
    return fn(*args)


def test_plan_validation(dks):
    lib = dks._lib
    plan = ctypes.c_void_p()
    # good plans
    assert lib.dks_poisson_plan(32, 32, 32, 1e-4, 1e-4, 1e-4, dks.DKS_F64, ctypes.byref(plan)) == dks.DKS_OK
    assert lib.dks_poisson_destroy(plan) == dks.DKS_OK
    assert lib.dks_poisson_plan(96, 96, 192, 0.0, 0.0, 0.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_OK
    assert lib.dks_poisson_destroy(plan) == dks.DKS_OK
    # 2n = 2^a 3^b only
    assert lib.dks_poisson_plan(5, 8, 8, 1.0, 1.0, 1.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EUNSUPPORTED
    assert lib.dks_poisson_plan(8, 8, 2049, 1.0, 1.0, 1.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EUNSUPPORTED
    # sizes, spacings, dtype, output pointer
    assert lib.dks_poisson_plan(1, 8, 8, 1.0, 1.0, 1.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_poisson_plan(3, 8, 8, 0.0, 0.0, 0.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_poisson_plan(8, 8, 8, 1.0, 0.0, 1.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_poisson_plan(8, 8, 8, -1.0, 1.0, 1.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_poisson_plan(8, 8, 8, float("nan"), 1.0, 1.0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_poisson_plan(8, 8, 8, 1.0, 1.0, 1.0, 7, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_poisson_plan(8, 8, 8, 1.0, 1.0, 1.0, dks.DKS_F32, None) == dks.DKS_EINVAL


def test_workspace_and_state_checks(dks):
    lib = dks._lib
    plan = dks.dks_poisson_plan(16, 12, 9, 1e-4, 1e-4, 2e-4, dks.DKS_F32)
    try:
        nbytes = dks.dks_poisson_workspace_bytes(plan)
        assert nbytes > 0
        per = dks.dks_poisson_batch_scratch_bytes(plan, 1, 0)
        assert dks.dks_poisson_batch_scratch_bytes(plan, 4, 0) == 4 * per
        assert per < nbytes
        assert dks.dks_poisson_batch_scratch_bytes(plan, 2, 1000) == 2 * (per + 12032 + 4096)
        assert dks.dks_poisson_particle_scratch_bytes(plan, 1000) == 12032 + 4096
        assert dks.dks_poisson_particle_scratch_bytes(plan, 0) == 0
        sz = ctypes.byref(ctypes.c_size_t())
        fake_s = ctypes.c_void_p(0x300000)
        assert lib.dks_poisson_batch_scratch_bytes(plan, 0, 10, sz) == dks.DKS_EINVAL
        assert lib.dks_poisson_batch_scratch_bytes(plan, 17, 10, sz) == dks.DKS_EINVAL
        assert lib.dks_poisson_batch_scratch_bytes(plan, 2, -1, sz) == dks.DKS_EINVAL
        assert lib.dks_poisson_particle_scratch_bytes(plan, 2 ** 32, sz) == dks.DKS_EINVAL
        assert lib.dks_poisson_particle_scratch_bytes(plan, 2 ** 32 - 2 ** 20 + 1, sz) == dks.DKS_EINVAL
        assert lib.dks_poisson_particle_scratch_bytes(plan, 2 ** 32 - 2 ** 20, sz) == dks.DKS_OK
        assert lib.dks_poisson_batch_scratch_bytes(plan, 1, 2 ** 32 - 2 ** 20 + 1, sz) == dks.DKS_EINVAL
        # batched: table and batch checked before anything else
        assert dks.PARTICLE_SET_BYTES == 80
        tab = ctypes.c_void_p(0x200000)
        assert lib.dks_poisson_solve_particles_batched(plan, 2, None, 10, fake_s, 1 << 20, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_particles_batched(plan, 0, tab, 10, fake_s, 1 << 20, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_particles_batched(plan, 17, tab, 10, fake_s, 1 << 20, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_particles_batched(plan, 2, tab, -1, fake_s, 1 << 20, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_particles_batched(plan, 2, tab, 10, fake_s, 1 << 20,
                                                       None) == dks.DKS_EWORKSPACE
        # no workspace yet
        fake = ctypes.c_void_p(0x100000)
        assert lib.dks_poisson_solve_rho(plan, fake, fake, None, None) == dks.DKS_EWORKSPACE
        assert lib.dks_poisson_prepare(plan, None) == dks.DKS_EWORKSPACE
        # too small, misaligned, null
        assert lib.dks_poisson_set_workspace(plan, fake, nbytes - 1) == dks.DKS_EWORKSPACE
        assert lib.dks_poisson_set_workspace(plan, ctypes.c_void_p(0x100010), nbytes) == dks.DKS_EWORKSPACE
        assert lib.dks_poisson_set_workspace(plan, None, nbytes) == dks.DKS_EWORKSPACE
        # particle scratch: misaligned refused; too small for the particle count refused
        assert lib.dks_poisson_set_particle_scratch(plan, ctypes.c_void_p(0x100008), 4096) == dks.DKS_EWORKSPACE
        assert lib.dks_poisson_set_particle_scratch(plan, fake, 512) == dks.DKS_OK
        assert lib.dks_poisson_set_workspace(plan, fake, nbytes) == dks.DKS_OK
        assert lib.dks_poisson_solve_particles(plan, fake, fake, fake, 40, 1e-15, fake, fake, fake,
                                               None, None, None) == dks.DKS_EWORKSPACE
        # scheme selection: unknown values refused; a new kernel needs a new prepare
        assert lib.dks_poisson_set_scheme(plan, 2, 0) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_scheme(plan, 0, 3) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_scheme(None, 0, 0) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_scheme(plan, dks.DKS_GREEN_POINT, dks.DKS_ASSIGN_TSC) == dks.DKS_OK
        assert lib.dks_poisson_set_scheme(plan, dks.DKS_GREEN_INTEGRATED, dks.DKS_ASSIGN_CIC) == dks.DKS_OK
        assert lib.dks_poisson_set_deterministic(None, 1) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_deterministic(plan, 2) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_deterministic(plan, 1) == dks.DKS_OK
        assert lib.dks_poisson_set_deterministic(plan, 0) == dks.DKS_OK
        # attached but not prepared: solves are refused before touching the device
        assert lib.dks_poisson_solve_rho(plan, fake, fake, None, None) == dks.DKS_ESTATE
        assert lib.dks_poisson_solve_particles(plan, fake, fake, fake, 10, 1e-15, fake, fake, fake,
                                               None, None, None) == dks.DKS_ESTATE
        assert lib.dks_poisson_geometry(plan, None, (ctypes.c_double * 3)(),
                                        (ctypes.c_double * 3)()) == dks.DKS_ESTATE
        # argument errors come first
        assert lib.dks_poisson_solve_rho(plan, None, fake, None, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_rho(plan, fake, None, None, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_particles(plan, fake, fake, fake, -1, 1e-15, fake, fake, fake,
                                               None, None, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_particles(plan, None, fake, fake, 10, 1e-15, fake, fake, fake,
                                               None, None, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_particles(plan, fake, fake, fake, 1, float("inf"), fake, fake, fake,
                                               None, None, None) == dks.DKS_EINVAL
        # host-resident solves: staging size, attachment and call order, all on the host
        assert dks.dks_poisson_host_staging_bytes(plan) == 10 * 6912   # 16*12*9 floats = 27 * 256 B
        assert lib.dks_poisson_set_host_staging(plan, None, 1 << 20) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_host_staging(plan, ctypes.c_void_p(0x100040), 1 << 20) == dks.DKS_EWORKSPACE
        assert lib.dks_poisson_set_host_staging(plan, fake, 10 * 6912 - 1) == dks.DKS_EWORKSPACE
        tk = ctypes.c_uint64()
        hbuf = (ctypes.c_float * (16 * 12 * 9))()
        assert lib.dks_poisson_solve_rho_host(plan, hbuf, hbuf, None, None, None) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_rho_host(plan, hbuf, None, None, None, ctypes.byref(tk)) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_rho_host(plan, None, hbuf, None, None, ctypes.byref(tk)) == dks.DKS_EINVAL
        assert lib.dks_poisson_solve_rho_host(plan, hbuf, hbuf, None, None, ctypes.byref(tk)) == dks.DKS_ESTATE
        assert lib.dks_poisson_host_query(plan, 0, ctypes.byref(ctypes.c_int())) == dks.DKS_EINVAL
        assert lib.dks_poisson_host_wait(plan, 0) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_host_staging(plan, fake, 10 * 6912) == dks.DKS_OK
        assert lib.dks_poisson_set_origin(plan, 0.0, 1.0, float("nan")) == dks.DKS_EINVAL
        assert lib.dks_poisson_set_origin(plan, 0.0, 1.0, 2.0) == dks.DKS_OK
    finally:
        dks.dks_poisson_destroy(plan)


def test_fitted_plan_rejects_mesh_density_and_origin(dks):
    lib = dks._lib
    plan = dks.dks_poisson_plan(16, 16, 16, 0.0, 0.0, 0.0, dks.DKS_F64)
    try:
        assert lib.dks_poisson_set_origin(plan, 0.0, 0.0, 0.0) == dks.DKS_ESTATE
        fake = ctypes.c_void_p(0x100000)
        assert lib.dks_poisson_solve_rho(plan, fake, fake, None, None) == dks.DKS_ESTATE
    finally:
        dks.dks_poisson_destroy(plan)


def test_status_strings(dks):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert dks.dks_status_string(code)
    assert dks.dks_status_string(12345) == "unknown status"
    with pytest.raises(dks.DKSError):
        dks.dks_poisson_plan(5, 5, 5, 1.0, 1.0, 1.0, dks.DKS_F32)


def test_workspace_grows_with_mesh_and_dtype(dks):
    sizes = {}
    for n in (16, 32, 64):
        for code in (dks.DKS_F32, dks.DKS_F64):
            p = dks.dks_poisson_plan(n, n, n, 1.0, 1.0, 1.0, code)
            sizes[(n, code)] = dks.dks_poisson_workspace_bytes(p)
            dks.dks_poisson_destroy(p)
    assert sizes[(32, dks.DKS_F32)] > sizes[(16, dks.DKS_F32)]
    assert sizes[(64, dks.DKS_F64)] > sizes[(64, dks.DKS_F32)]
    # about 27 sizeof(real) x 8 per node for the doubled-grid intermediates, well under 64x
    assert sizes[(64, dks.DKS_F32)] < 64 * 4 * 64 ** 3 * 8


def test_fft_plan_validation(dks):
    lib = dks._lib
    plan = ctypes.c_void_p()
    for args in ((64, 64, 64, 1), (1, 1, 1, 1), (4096, 1, 1, 3), (6, 9, 27, 2), (2, 3, 4096, 1)):
        for kind in (dks.DKS_FFT_C2C, dks.DKS_FFT_R2C):
            assert lib.dks_fft_plan(*args, kind, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_OK
            assert lib.dks_fft_destroy(plan) == dks.DKS_OK
    assert lib.dks_fft_plan(5, 8, 8, 1, 0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EUNSUPPORTED
    assert lib.dks_fft_plan(8192, 1, 1, 1, 0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EUNSUPPORTED
    assert lib.dks_fft_plan(0, 8, 8, 1, 0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_fft_plan(8, 8, 8, 0, 0, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_fft_plan(8, 8, 8, 1, 2, dks.DKS_F32, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_fft_plan(8, 8, 8, 1, 0, 5, ctypes.byref(plan)) == dks.DKS_EINVAL
    assert lib.dks_fft_plan(8, 8, 8, 1, 0, dks.DKS_F32, None) == dks.DKS_EINVAL
    p = dks.dks_fft_plan(12, 8, 6, 2, dks.DKS_FFT_R2C, dks.DKS_F64)
    try:
        nbytes = dks.dks_fft_workspace_bytes(p)
        # the complex-to-real scratch alone: (12/2 + 1) * 8 * 6 * 2 complex doubles
        assert nbytes >= 7 * 8 * 6 * 2 * 16
        fake = ctypes.c_void_p(0x100000)
        assert lib.dks_fft_forward(p, fake, ctypes.c_void_p(0x200000), None) == dks.DKS_EWORKSPACE
        assert lib.dks_fft_set_workspace(p, ctypes.c_void_p(0x100010), nbytes) == dks.DKS_EWORKSPACE
        assert lib.dks_fft_set_workspace(p, fake, nbytes - 1) == dks.DKS_EWORKSPACE
        assert lib.dks_fft_set_workspace(p, fake, nbytes) == dks.DKS_OK
        assert lib.dks_fft_forward(p, fake, ctypes.c_void_p(0x200000), None) == dks.DKS_ESTATE
        assert lib.dks_fft_forward(p, fake, fake, None) == dks.DKS_EINVAL      # R2C is out of place only
        assert lib.dks_fft_forward(p, None, fake, None) == dks.DKS_EINVAL
        assert lib.dks_fft_inverse(p, fake, None, None) == dks.DKS_EINVAL
    finally:
        dks.dks_fft_destroy(p)


def test_musr_plan_validation(dks):
    lib = dks._lib
    plan = ctypes.c_void_p()
    assert lib.dks_musr_plan(16, 206250, 4.8e-5, 133, ctypes.byref(plan)) == dks.DKS_OK
    assert lib.dks_musr_destroy(plan) == dks.DKS_OK
    for args in ((0, 100, 0.1, 1), (33, 100, 0.1, 1), (4, 0, 0.1, 1), (4, 100, 0.0, 1), (4, 100, float("nan"), 1),
                 (4, 100, 0.1, 0), (4, 100, 0.1, 1025), (4, 2 ** 31, 0.1, 1)):
        assert lib.dks_musr_plan(*args, ctypes.byref(plan)) == dks.DKS_EINVAL, args
    p = dks.dks_musr_plan(4, 5000, 0.01, 8)
    try:
        nbytes = dks.dks_musr_workspace_bytes(p)
        assert nbytes >= 8 * 3 * 4 * 8       # partials of 3 workgroups x 4 detectors per set
        fake = ctypes.c_void_p(0x100000)
        prm = (ctypes.c_double * 18)()
        assert lib.dks_musr_eval(p, 0, prm, fake, None) == dks.DKS_EWORKSPACE
        assert lib.dks_musr_set_workspace(p, ctypes.c_void_p(0x100008), nbytes) == dks.DKS_EWORKSPACE
        assert lib.dks_musr_set_workspace(p, fake, nbytes - 1) == dks.DKS_EWORKSPACE
        assert lib.dks_musr_set_workspace(p, fake, nbytes) == dks.DKS_OK
        assert lib.dks_musr_eval(p, 0, prm, fake, None) == dks.DKS_ESTATE     # not prepared, no data
        assert lib.dks_musr_eval(p, 2, prm, fake, None) == dks.DKS_EINVAL
        assert lib.dks_musr_eval(p, 0, None, fake, None) == dks.DKS_EINVAL
        assert lib.dks_musr_eval(p, 0, prm, None, None) == dks.DKS_EINVAL
        assert lib.dks_musr_eval_batch(p, 0, fake, 0, fake, None) == dks.DKS_EINVAL
        assert lib.dks_musr_eval_batch(p, 0, fake, 9, fake, None) == dks.DKS_EINVAL
        assert lib.dks_musr_set_data(p, None) == dks.DKS_EINVAL
    finally:
        dks.dks_musr_destroy(p)


def test_plain_c_client(tmp_path):
    """The headers compile as C99 with gcc and a C program linked against the
    library runs its host-side calls."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "abi_client"
    libdir = os.path.dirname(LIB)
    src = os.path.join(ROOT, "tests", "c", "abi_client.c")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), src,
                        "-o", str(exe), "-L", libdir, "-ldks_poisson", f"-Wl,-rpath,{libdir}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok ")
