"""ctypes binding of libdks_poisson.so (include/dks_poisson.h).

Argument marshalling only: every step of the solve runs in the HIP library.
The module-level functions carry the C names and signatures; `PoissonPlan`
wraps a plan with torch-owned device memory (PyTorch supplies allocations
and streams, nothing else).  Importing this module fails loudly if the
library has not been built.
"""

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdks_poisson.so")

DKS_OK = 0
DKS_EINVAL = -1
DKS_EUNSUPPORTED = -2
DKS_ENOMEM = -3
DKS_EHIP = -4
DKS_EWORKSPACE = -5
DKS_ESTATE = -6
DKS_F32 = 0
DKS_F64 = 1
DKS_GREEN_INTEGRATED = 0
DKS_GREEN_POINT = 1
DKS_ASSIGN_CIC = 0
DKS_ASSIGN_NGP = 1
DKS_ASSIGN_TSC = 2
DKS_MUSR_CHISQ = 0
DKS_MUSR_MLE = 1
MUSR_STATS = {"chisq": DKS_MUSR_CHISQ, "mle": DKS_MUSR_MLE}
DKS_FFT_C2C = 0
DKS_FFT_R2C = 1
GREENS = {"integrated": DKS_GREEN_INTEGRATED, "point": DKS_GREEN_POINT}
SCHEMES = {"cic": DKS_ASSIGN_CIC, "ngp": DKS_ASSIGN_NGP, "tsc": DKS_ASSIGN_TSC}

EXPORTS = (
    "dks_poisson_plan", "dks_poisson_set_origin", "dks_poisson_set_scheme", "dks_poisson_set_deterministic",
    "dks_poisson_workspace_bytes",
    "dks_poisson_batch_scratch_bytes", "dks_poisson_particle_scratch_bytes",
    "dks_poisson_set_particle_scratch", "dks_poisson_set_workspace", "dks_poisson_prepare",
    "dks_poisson_solve_rho", "dks_poisson_solve_particles", "dks_poisson_solve_particles_batched",
    "dks_poisson_deposit", "dks_poisson_gather", "dks_poisson_geometry", "dks_poisson_destroy",
    "dks_status_string", "dks_timing_enable", "dks_timing_read", "dks_poisson_host_staging_bytes",
    "dks_poisson_set_host_staging", "dks_poisson_solve_rho_host", "dks_poisson_host_query",
    "dks_poisson_host_wait", "dks_fft_plan", "dks_fft_workspace_bytes", "dks_fft_set_workspace",
    "dks_fft_prepare", "dks_fft_forward", "dks_fft_inverse", "dks_fft_destroy", "dks_musr_plan",
    "dks_musr_workspace_bytes", "dks_musr_set_workspace", "dks_musr_prepare", "dks_musr_set_data",
    "dks_musr_eval", "dks_musr_eval_batch", "dks_musr_destroy", "dks_poisson_solve_particles_noalloc",
    "dks_poisson_solve_particles_sorted",
)


class DKSError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {dks_status_string(status)} ({status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1509_07685_amd.build`")
    return ctypes.CDLL(LIB_PATH)


_lib = _load()

_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i64 = ctypes.c_int64
_d = ctypes.c_double
_i = ctypes.c_int
_PLAN = ctypes.c_void_p

_SIGS = {
    "dks_poisson_plan": (_i, [_i, _i, _i, _d, _d, _d, _i, ctypes.POINTER(_PLAN)]),
    "dks_poisson_set_origin": (_i, [_PLAN, _d, _d, _d]),
    "dks_poisson_set_scheme": (_i, [_PLAN, _i, _i]),
    "dks_poisson_set_deterministic": (_i, [_PLAN, _i]),
    "dks_poisson_workspace_bytes": (_i, [_PLAN, ctypes.POINTER(_sz)]),
    "dks_poisson_batch_scratch_bytes": (_i, [_PLAN, _i, _i64, ctypes.POINTER(_sz)]),
    "dks_poisson_particle_scratch_bytes": (_i, [_PLAN, _i64, ctypes.POINTER(_sz)]),
    "dks_poisson_set_particle_scratch": (_i, [_PLAN, _vp, _sz]),
    "dks_poisson_set_workspace": (_i, [_PLAN, _vp, _sz]),
    "dks_poisson_prepare": (_i, [_PLAN, _vp]),
    "dks_poisson_solve_rho": (_i, [_PLAN, _vp, _vp, _vp, _vp]),
    "dks_poisson_solve_particles": (_i, [_PLAN, _vp, _vp, _vp, _i64, _d, _vp, _vp, _vp, _vp, _vp, _vp]),
    "dks_poisson_solve_particles_batched": (_i, [_PLAN, _i, _vp, _i64, _vp, _sz, _vp]),
    "dks_poisson_solve_particles_noalloc": (_i, [_PLAN, _vp, _vp, _vp, _i64, _d, _vp, _vp, _vp, _vp, _vp, _vp]),
    "dks_poisson_solve_particles_sorted": (_i, [_PLAN, _vp, _vp, _vp, _i64, _d, _vp, _vp, _vp, _vp, _vp, _vp,
                                                _vp, _vp, _vp, _vp]),
    "dks_poisson_deposit": (_i, [_PLAN, _vp, _vp, _vp, _i64, _d, _vp, _vp, _vp]),
    "dks_poisson_gather": (_i, [_PLAN, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "dks_poisson_geometry": (_i, [_PLAN, _vp, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "dks_poisson_destroy": (_i, [_PLAN]),
    "dks_status_string": (ctypes.c_char_p, [_i]),
    "dks_timing_enable": (_i, [_i]),
    "dks_timing_read": (_i, [_vp, _i, ctypes.POINTER(_i)]),
    "dks_poisson_host_staging_bytes": (_i, [_PLAN, ctypes.POINTER(_sz)]),
    "dks_poisson_set_host_staging": (_i, [_PLAN, _vp, _sz]),
    "dks_poisson_solve_rho_host": (_i, [_PLAN, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "dks_poisson_host_query": (_i, [_PLAN, ctypes.c_uint64, ctypes.POINTER(_i)]),
    "dks_poisson_host_wait": (_i, [_PLAN, ctypes.c_uint64]),
    "dks_fft_plan": (_i, [_i, _i, _i, _i, _i, _i, ctypes.POINTER(_PLAN)]),
    "dks_fft_workspace_bytes": (_i, [_PLAN, ctypes.POINTER(_sz)]),
    "dks_fft_set_workspace": (_i, [_PLAN, _vp, _sz]),
    "dks_fft_prepare": (_i, [_PLAN, _vp]),
    "dks_fft_forward": (_i, [_PLAN, _vp, _vp, _vp]),
    "dks_fft_inverse": (_i, [_PLAN, _vp, _vp, _vp]),
    "dks_fft_destroy": (_i, [_PLAN]),
    "dks_musr_plan": (_i, [_i, _i64, _d, _i, ctypes.POINTER(_PLAN)]),
    "dks_musr_workspace_bytes": (_i, [_PLAN, ctypes.POINTER(_sz)]),
    "dks_musr_set_workspace": (_i, [_PLAN, _vp, _sz]),
    "dks_musr_prepare": (_i, [_PLAN, _vp]),
    "dks_musr_set_data": (_i, [_PLAN, _vp]),
    "dks_musr_eval": (_i, [_PLAN, _i, _vp, _vp, _vp]),
    "dks_musr_eval_batch": (_i, [_PLAN, _i, _vp, _i, _vp, _vp]),
    "dks_musr_destroy": (_i, [_PLAN]),
}


class dks_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def dks_status_string(status):
    return _lib.dks_status_string(int(status)).decode()


def _check(status, what):
    if status != DKS_OK:
        raise DKSError(status, what)


def dks_poisson_plan(nx, ny, nz, hx, hy, hz, dtype):
    plan = _PLAN()
    _check(_lib.dks_poisson_plan(nx, ny, nz, hx, hy, hz, dtype, ctypes.byref(plan)), "dks_poisson_plan")
    return plan


def dks_poisson_set_origin(plan, x0, y0, z0):
    _check(_lib.dks_poisson_set_origin(plan, x0, y0, z0), "dks_poisson_set_origin")


def dks_poisson_set_scheme(plan, green, assign):
    _check(_lib.dks_poisson_set_scheme(plan, green, assign), "dks_poisson_set_scheme")


def dks_poisson_set_deterministic(plan, on):
    _check(_lib.dks_poisson_set_deterministic(plan, 1 if on else 0), "dks_poisson_set_deterministic")


def dks_poisson_workspace_bytes(plan):
    out = _sz()
    _check(_lib.dks_poisson_workspace_bytes(plan, ctypes.byref(out)), "dks_poisson_workspace_bytes")
    return out.value


def dks_poisson_batch_scratch_bytes(plan, batch, max_np):
    out = _sz()
    _check(_lib.dks_poisson_batch_scratch_bytes(plan, batch, max_np, ctypes.byref(out)),
           "dks_poisson_batch_scratch_bytes")
    return out.value


def dks_poisson_particle_scratch_bytes(plan, np_):
    out = _sz()
    _check(_lib.dks_poisson_particle_scratch_bytes(plan, np_, ctypes.byref(out)),
           "dks_poisson_particle_scratch_bytes")
    return out.value


def dks_poisson_set_particle_scratch(plan, ptr, nbytes):
    _check(_lib.dks_poisson_set_particle_scratch(plan, ptr, nbytes), "dks_poisson_set_particle_scratch")


def dks_poisson_set_workspace(plan, ptr, nbytes):
    _check(_lib.dks_poisson_set_workspace(plan, ptr, nbytes), "dks_poisson_set_workspace")


def dks_poisson_prepare(plan, stream):
    _check(_lib.dks_poisson_prepare(plan, stream), "dks_poisson_prepare")


def dks_poisson_solve_rho(plan, rho, phi, E_mesh, stream):
    _check(_lib.dks_poisson_solve_rho(plan, rho, phi, E_mesh, stream), "dks_poisson_solve_rho")


def dks_poisson_host_staging_bytes(plan):
    n = _sz()
    _check(_lib.dks_poisson_host_staging_bytes(plan, ctypes.byref(n)), "dks_poisson_host_staging_bytes")
    return n.value


def dks_poisson_set_host_staging(plan, ptr, nbytes):
    _check(_lib.dks_poisson_set_host_staging(plan, ptr, nbytes), "dks_poisson_set_host_staging")


def dks_poisson_solve_rho_host(plan, rho_host, phi_host, E_host, stream):
    t = ctypes.c_uint64()
    _check(_lib.dks_poisson_solve_rho_host(plan, rho_host, phi_host, E_host, stream, ctypes.byref(t)),
           "dks_poisson_solve_rho_host")
    return t.value


def dks_poisson_host_query(plan, ticket):
    done = _i()
    _check(_lib.dks_poisson_host_query(plan, ticket, ctypes.byref(done)), "dks_poisson_host_query")
    return bool(done.value)


def dks_poisson_host_wait(plan, ticket):
    _check(_lib.dks_poisson_host_wait(plan, ticket), "dks_poisson_host_wait")


def dks_fft_plan(nx, ny, nz, batch, kind, dtype):
    plan = _PLAN()
    _check(_lib.dks_fft_plan(nx, ny, nz, batch, kind, dtype, ctypes.byref(plan)), "dks_fft_plan")
    return plan


def dks_fft_workspace_bytes(plan):
    n = _sz()
    _check(_lib.dks_fft_workspace_bytes(plan, ctypes.byref(n)), "dks_fft_workspace_bytes")
    return n.value


def dks_fft_set_workspace(plan, ptr, nbytes):
    _check(_lib.dks_fft_set_workspace(plan, ptr, nbytes), "dks_fft_set_workspace")


def dks_fft_prepare(plan, stream):
    _check(_lib.dks_fft_prepare(plan, stream), "dks_fft_prepare")


def dks_fft_forward(plan, inp, out, stream):
    _check(_lib.dks_fft_forward(plan, inp, out, stream), "dks_fft_forward")


def dks_fft_inverse(plan, inp, out, stream):
    _check(_lib.dks_fft_inverse(plan, inp, out, stream), "dks_fft_inverse")


def dks_fft_destroy(plan):
    _check(_lib.dks_fft_destroy(plan), "dks_fft_destroy")


def dks_musr_plan(n_det, n_bins, dt, max_sets):
    plan = _PLAN()
    _check(_lib.dks_musr_plan(n_det, n_bins, dt, max_sets, ctypes.byref(plan)), "dks_musr_plan")
    return plan


def dks_musr_workspace_bytes(plan):
    n = _sz()
    _check(_lib.dks_musr_workspace_bytes(plan, ctypes.byref(n)), "dks_musr_workspace_bytes")
    return n.value


def dks_musr_set_workspace(plan, ptr, nbytes):
    _check(_lib.dks_musr_set_workspace(plan, ptr, nbytes), "dks_musr_set_workspace")


def dks_musr_prepare(plan, stream):
    _check(_lib.dks_musr_prepare(plan, stream), "dks_musr_prepare")


def dks_musr_set_data(plan, data):
    _check(_lib.dks_musr_set_data(plan, data), "dks_musr_set_data")


def dks_musr_eval(plan, stat, params, result, stream):
    _check(_lib.dks_musr_eval(plan, stat, params, result, stream), "dks_musr_eval")


def dks_musr_eval_batch(plan, stat, params, nsets, results, stream):
    _check(_lib.dks_musr_eval_batch(plan, stat, params, nsets, results, stream), "dks_musr_eval_batch")


def dks_musr_destroy(plan):
    _check(_lib.dks_musr_destroy(plan), "dks_musr_destroy")


def dks_poisson_solve_particles(plan, x, y, z, np_, q, Ex, Ey, Ez, phi, n_outside, stream):
    _check(_lib.dks_poisson_solve_particles(plan, x, y, z, np_, q, Ex, Ey, Ez, phi, n_outside, stream),
           "dks_poisson_solve_particles")


def dks_poisson_solve_particles_noalloc(plan, x, y, z, np_, q, Ex, Ey, Ez, phi, n_outside, stream):
    _check(_lib.dks_poisson_solve_particles_noalloc(plan, x, y, z, np_, q, Ex, Ey, Ez, phi, n_outside, stream),
           "dks_poisson_solve_particles_noalloc")


NOALLOC_SCRATCH_BYTES = 64 << 20     # DKS_NOALLOC_SCRATCH_BYTES


def dks_poisson_solve_particles_sorted(plan, x, y, z, np_, q, x_out, y_out, z_out, Ex, Ey, Ez, phi, new_index,
                                       n_outside, stream):
    _check(_lib.dks_poisson_solve_particles_sorted(plan, x, y, z, np_, q, x_out, y_out, z_out, Ex, Ey, Ez, phi,
                                                   new_index, n_outside, stream),
           "dks_poisson_solve_particles_sorted")


class dks_particle_set(ctypes.Structure):
    """One element of a batched solve (device addresses, count, charge)."""
    _fields_ = [("x", _vp), ("y", _vp), ("z", _vp), ("Ex", _vp), ("Ey", _vp), ("Ez", _vp), ("phi", _vp),
                ("n_outside", _vp), ("np", _i64), ("q", _d)]


PARTICLE_SET_BYTES = ctypes.sizeof(dks_particle_set)


def _set_dtype():
    import numpy as np
    return np.dtype([("x", "<u8"), ("y", "<u8"), ("z", "<u8"), ("Ex", "<u8"), ("Ey", "<u8"), ("Ez", "<u8"),
                     ("phi", "<u8"), ("n_outside", "<u8"), ("np", "<i8"), ("q", "<f8")])


PARTICLE_SET_DTYPE = _set_dtype()   # numpy layout of dks_particle_set
assert PARTICLE_SET_DTYPE.itemsize == PARTICLE_SET_BYTES


def particle_set_table(entries):
    """Bytes of a dks_particle_set array.  entries: sequence of dicts with keys
    x, y, z, Ex, Ey, Ez (device addresses), optional phi, n_outside, and np, q."""
    arr = (dks_particle_set * len(entries))()
    for a, e in zip(arr, entries):
        for k in ("x", "y", "z", "Ex", "Ey", "Ez", "phi", "n_outside"):
            setattr(a, k, e.get(k) or None)
        a.np = int(e["np"])
        a.q = float(e["q"])
    return bytes(arr)


def dks_poisson_solve_particles_batched(plan, batch, sets, max_np, scratch, scratch_bytes, stream):
    """sets: device address of `batch` dks_particle_set records."""
    st = _lib.dks_poisson_solve_particles_batched(plan, batch, sets, max_np, scratch, scratch_bytes, stream)
    _check(st, "dks_poisson_solve_particles_batched")


def dks_poisson_deposit(plan, x, y, z, np_, q, rho, n_outside, stream):
    _check(_lib.dks_poisson_deposit(plan, x, y, z, np_, q, rho, n_outside, stream), "dks_poisson_deposit")


def dks_poisson_gather(plan, E_mesh, x, y, z, np_, Ex, Ey, Ez, stream):
    _check(_lib.dks_poisson_gather(plan, E_mesh, x, y, z, np_, Ex, Ey, Ez, stream), "dks_poisson_gather")


def dks_poisson_geometry(plan, stream):
    h = (_d * 3)()
    o = (_d * 3)()
    _check(_lib.dks_poisson_geometry(plan, stream, h, o), "dks_poisson_geometry")
    return tuple(h), tuple(o)


def dks_timing_enable(enable):
    _check(_lib.dks_timing_enable(1 if enable else 0), "dks_timing_enable")


def dks_timing_read(capacity=64):
    """{kernel name: (launches, total_ms, min_ms, max_ms)} since timing was enabled."""
    arr = (dks_kernel_time * capacity)()
    count = _i()
    _check(_lib.dks_timing_read(ctypes.cast(arr, _vp), capacity, ctypes.byref(count)), "dks_timing_read")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms, arr[i].min_ms, arr[i].max_ms)
            for i in range(count.value)}


def dks_poisson_destroy(plan):
    _check(_lib.dks_poisson_destroy(plan), "dks_poisson_destroy")


# --------------------------------------------------------------------------
# torch-facing convenience wrapper
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_code(dtype):
    torch = _torch()
    if dtype in ("f32", torch.float32):
        return DKS_F32, torch.float32
    if dtype in ("f64", torch.float64):
        return DKS_F64, torch.float64
    raise ValueError(f"unsupported dtype {dtype}")


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class PoissonPlan:
    """A plan plus its torch-allocated device workspace.

    n = (nx, ny, nz) nodes; h = (hx, hy, hz) metres or None for the
    particle-fitted cubic mesh; dtype "f32"/"f64" (or torch dtype); scheme
    "cic"/"ngp"/"tsc"; green "integrated"/"point".
    """

    def __init__(self, n, h=None, dtype="f32", device="cuda", stream=None, prepare=True, scheme="cic",
                 green="integrated", deterministic=False):
        torch = _torch()
        self.n = tuple(int(v) for v in n)
        self.fitted = h is None
        self.h = (0.0, 0.0, 0.0) if h is None else tuple(float(v) for v in h)
        self.code, self.dtype = _dtype_code(dtype)
        self.device = torch.device(device)
        self.handle = dks_poisson_plan(*self.n, *self.h, self.code)
        dks_poisson_set_scheme(self.handle, GREENS[green], SCHEMES[scheme])
        if deterministic:
            dks_poisson_set_deterministic(self.handle, True)
        self.workspace_bytes = dks_poisson_workspace_bytes(self.handle)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        dks_poisson_set_workspace(self.handle, _ptr(self.workspace), self.workspace_bytes)
        self.particle_scratch = None
        if prepare:
            self.prepare(stream)

    def prepare(self, stream=None):
        dks_poisson_prepare(self.handle, _stream_handle(stream))

    def set_deterministic(self, on):
        dks_poisson_set_deterministic(self.handle, on)

    def set_origin(self, origin):
        dks_poisson_set_origin(self.handle, *[float(v) for v in origin])

    def mesh_shape(self):
        nx, ny, nz = self.n
        return (nz, ny, nx)

    def _check_tensor(self, t, shape, name):
        if t.dtype != self.dtype or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name} must be a contiguous {self.dtype} CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def solve_rho(self, rho, want_phi=True, want_E=True, stream=None):
        torch = _torch()
        self._check_tensor(rho, self.mesh_shape(), "rho")
        phi = torch.empty(self.mesh_shape(), dtype=self.dtype, device=rho.device) if want_phi else None
        E = torch.empty((3,) + self.mesh_shape(), dtype=self.dtype, device=rho.device) if want_E else None
        dks_poisson_solve_rho(self.handle, _ptr(rho), _ptr(phi), _ptr(E), _stream_handle(stream))
        return phi, E

    def host_staging(self):
        """Attach the device staging area of host-resident solves (once)."""
        torch = _torch()
        if getattr(self, "staging", None) is None:
            nbytes = dks_poisson_host_staging_bytes(self.handle)
            self.staging = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            dks_poisson_set_host_staging(self.handle, _ptr(self.staging), nbytes)
        return self.staging

    def _check_host(self, t, shape, name):
        if t.dtype != self.dtype or not t.is_contiguous() or t.device.type != "cpu":
            raise ValueError(f"{name} must be a contiguous {self.dtype} host tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def solve_rho_host(self, rho_host, phi_host=None, E_host=None, stream=None):
        """Enqueue a host-resident solve (host tensors, page-locked for
        overlap); returns its ticket.  The tensors must stay alive and
        untouched until host_wait(ticket) or host_done(ticket)."""
        self._check_host(rho_host, self.mesh_shape(), "rho_host")
        if phi_host is not None:
            self._check_host(phi_host, self.mesh_shape(), "phi_host")
        if E_host is not None:
            self._check_host(E_host, (3,) + self.mesh_shape(), "E_host")
        self.host_staging()
        return dks_poisson_solve_rho_host(self.handle, rho_host.data_ptr(),
                                          None if phi_host is None else phi_host.data_ptr(),
                                          None if E_host is None else E_host.data_ptr(), _stream_handle(stream))

    def host_done(self, ticket):
        return dks_poisson_host_query(self.handle, ticket)

    def host_wait(self, ticket):
        dks_poisson_host_wait(self.handle, ticket)

    def reserve_particles(self, npart):
        """Attach (growing if needed) the binned-particle scratch for npart particles."""
        torch = _torch()
        need = dks_poisson_particle_scratch_bytes(self.handle, npart)
        if self.particle_scratch is None or self.particle_scratch.numel() < need:
            self.particle_scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            dks_poisson_set_particle_scratch(self.handle, _ptr(self.particle_scratch),
                                             self.particle_scratch.numel())

    def solve_particles(self, x, y, z, q, want_phi=False, out=None, stream=None):
        torch = _torch()
        npart = x.numel()
        self.reserve_particles(npart)
        for name, t in (("x", x), ("y", y), ("z", z)):
            self._check_tensor(t, (npart,), name)
        if out is None:
            Ex, Ey, Ez = (torch.empty(npart, dtype=self.dtype, device=x.device) for _ in range(3))
            cnt = torch.zeros(1, dtype=torch.int64, device=x.device)
        else:
            Ex, Ey, Ez, cnt = out
        phi = torch.empty(self.mesh_shape(), dtype=self.dtype, device=x.device) if want_phi else None
        dks_poisson_solve_particles(self.handle, _ptr(x), _ptr(y), _ptr(z), npart, float(q), _ptr(Ex),
                                    _ptr(Ey), _ptr(Ez), _ptr(phi), _ptr(cnt), _stream_handle(stream))
        return (Ex, Ey, Ez), phi, cnt

    def solve_particles_sorted(self, x, y, z, q, want_phi=False, want_index=False, pos_out=None, out=None,
                               stream=None):
        """The step with particles returned in binned order: the positions in
        that order go to pos_out (three new arrays unless given; they must
        not overlap the inputs) and the field comes back in it; with
        want_index, also each input index's new position (int32).
        Returns ((x, y, z) in binned order, (Ex, Ey, Ez), phi, count, index)."""
        torch = _torch()
        npart = x.numel()
        self.reserve_particles(npart)
        for name, t in (("x", x), ("y", y), ("z", z)):
            self._check_tensor(t, (npart,), name)
        if pos_out is None:
            pos_out = tuple(torch.empty(npart, dtype=self.dtype, device=x.device) for _ in range(3))
        if out is None:
            Ex, Ey, Ez = (torch.empty(npart, dtype=self.dtype, device=x.device) for _ in range(3))
            cnt = torch.zeros(1, dtype=torch.int64, device=x.device)
        else:
            Ex, Ey, Ez, cnt = out
        phi = torch.empty(self.mesh_shape(), dtype=self.dtype, device=x.device) if want_phi else None
        idx = torch.empty(npart, dtype=torch.int32, device=x.device) if want_index else None
        xo, yo, zo = pos_out
        dks_poisson_solve_particles_sorted(self.handle, _ptr(x), _ptr(y), _ptr(z), npart, float(q), _ptr(xo),
                                           _ptr(yo), _ptr(zo), _ptr(Ex), _ptr(Ey), _ptr(Ez), _ptr(phi), _ptr(idx),
                                           _ptr(cnt), _stream_handle(stream))
        return (xo, yo, zo), (Ex, Ey, Ez), phi, cnt, idx

    def deposit(self, x, y, z, q, stream=None):
        torch = _torch()
        npart = x.numel()
        self.reserve_particles(npart)
        rho = torch.empty(self.mesh_shape(), dtype=self.dtype, device=x.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=x.device)
        dks_poisson_deposit(self.handle, _ptr(x), _ptr(y), _ptr(z), npart, float(q), _ptr(rho), _ptr(cnt),
                            _stream_handle(stream))
        return rho, cnt

    def gather(self, E_mesh, x, y, z, stream=None):
        torch = _torch()
        npart = x.numel()
        self._check_tensor(E_mesh, (3,) + self.mesh_shape(), "E_mesh")
        Ex, Ey, Ez = (torch.empty(npart, dtype=self.dtype, device=x.device) for _ in range(3))
        dks_poisson_gather(self.handle, _ptr(E_mesh), _ptr(x), _ptr(y), _ptr(z), npart, _ptr(Ex), _ptr(Ey),
                           _ptr(Ez), _stream_handle(stream))
        return Ex, Ey, Ez

    def geometry(self, stream=None):
        return dks_poisson_geometry(self.handle, _stream_handle(stream))

    def batch_scratch(self, batch, max_np):
        torch = _torch()
        nbytes = dks_poisson_batch_scratch_bytes(self.handle, batch, max_np)
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device), nbytes

    def solve_particles_batched(self, table, batch, max_np, scratch, stream=None):
        """One batched launch.  table: device uint8 tensor holding `batch`
        dks_particle_set records (see particle_set_table); the library reads it
        on the device when the kernels run, so a captured launch picks up
        whatever the table holds at replay."""
        buf, nbytes = scratch
        if table.numel() < batch * PARTICLE_SET_BYTES:
            raise ValueError("particle set table too small for the batch")
        dks_poisson_solve_particles_batched(self.handle, batch, _ptr(table), int(max_np), _ptr(buf), nbytes,
                                            _stream_handle(stream))

    def close(self):
        if self.handle is not None:
            dks_poisson_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FFTPlan:
    """A raw 3-D FFT plan plus its torch-allocated workspace.

    n = (nx, ny, nz) (x fastest; extents of 1 give 2-D / 1-D transforms),
    batch consecutive arrays, kind "c2c" or "r2c", dtype "f32"/"f64".
    Complex tensors are torch complex64 / complex128 of shape
    (batch, nz, ny, nx) (or (batch, nz, ny, nx//2+1) for the r2c spectrum).
    """

    def __init__(self, n, batch=1, kind="c2c", dtype="f32", device="cuda", stream=None):
        torch = _torch()
        self.n = tuple(int(v) for v in n)
        self.batch = int(batch)
        self.kind = kind
        self.code, self.dtype = _dtype_code(dtype)
        self.cdtype = torch.complex64 if self.dtype == torch.float32 else torch.complex128
        kcode = {"c2c": DKS_FFT_C2C, "r2c": DKS_FFT_R2C}[kind]
        self.handle = dks_fft_plan(*self.n, self.batch, kcode, self.code)
        nbytes = dks_fft_workspace_bytes(self.handle)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        dks_fft_set_workspace(self.handle, _ptr(self.workspace), self.workspace.numel())
        dks_fft_prepare(self.handle, _stream_handle(stream))

    def shape(self, spectrum=False):
        nx, ny, nz = self.n
        if spectrum and self.kind == "r2c":
            nx = nx // 2 + 1
        return (self.batch, nz, ny, nx)

    def _check(self, t, dtype, shape, name):
        if t.dtype != dtype or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def forward(self, x, out=None, stream=None):
        torch = _torch()
        in_dt = self.dtype if self.kind == "r2c" else self.cdtype
        self._check(x, in_dt, self.shape(), "x")
        if out is None:
            out = torch.empty(self.shape(spectrum=True), dtype=self.cdtype, device=x.device)
        self._check(out, self.cdtype, self.shape(spectrum=True), "out")
        dks_fft_forward(self.handle, _ptr(x), _ptr(out), _stream_handle(stream))
        return out

    def inverse(self, X, out=None, stream=None):
        torch = _torch()
        out_dt = self.dtype if self.kind == "r2c" else self.cdtype
        self._check(X, self.cdtype, self.shape(spectrum=True), "X")
        if out is None:
            out = torch.empty(self.shape(), dtype=out_dt, device=X.device)
        self._check(out, out_dt, self.shape(), "out")
        dks_fft_inverse(self.handle, _ptr(X), _ptr(out), _stream_handle(stream))
        return out

    def close(self):
        if self.handle is not None:
            dks_fft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MusrFit:
    """Resident muSR histograms [n_det][n_bins] (FP64 CUDA tensor) and the
    device evaluation of the fit statistic for parameter vectors
    [sigma, B, (N0, Nbkg, A0, phi) per detector]."""

    def __init__(self, data, dt, max_sets=1, stream=None):
        torch = _torch()
        if data.dtype != torch.float64 or not data.is_contiguous() or data.device.type != "cuda" or data.dim() != 2:
            raise ValueError("data must be a contiguous 2-D float64 CUDA tensor [n_det][n_bins]")
        self.data = data
        self.n_det, self.n_bins = data.shape
        self.nparam = 2 + 4 * self.n_det
        self.handle = dks_musr_plan(self.n_det, self.n_bins, float(dt), int(max_sets))
        nbytes = dks_musr_workspace_bytes(self.handle)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=data.device)
        dks_musr_set_workspace(self.handle, _ptr(self.workspace), nbytes)
        dks_musr_prepare(self.handle, _stream_handle(stream))
        dks_musr_set_data(self.handle, _ptr(data))
        self.result = torch.empty(1, dtype=torch.float64, device=data.device)

    def eval_async(self, stat, params, out=None, stream=None):
        """Enqueue one evaluation; returns the device result tensor (1 element)."""
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        if p.shape != (self.nparam,):
            raise ValueError(f"expected {self.nparam} parameters")
        out = self.result if out is None else out
        dks_musr_eval(self.handle, MUSR_STATS[stat], p.ctypes.data, _ptr(out), _stream_handle(stream))
        return out

    def __call__(self, stat, params):
        return float(self.eval_async(stat, params).item())

    def eval_batch(self, stat, params, out=None, stream=None):
        """params: float64 CUDA tensor [nsets][nparam]; returns results [nsets]."""
        torch = _torch()
        if params.dtype != torch.float64 or not params.is_contiguous() or params.dim() != 2 \
                or params.shape[1] != self.nparam:
            raise ValueError(f"params must be a contiguous float64 CUDA tensor [nsets][{self.nparam}]")
        nsets = params.shape[0]
        if out is None:
            out = torch.empty(nsets, dtype=torch.float64, device=params.device)
        dks_musr_eval_batch(self.handle, MUSR_STATS[stat], _ptr(params), nsets, _ptr(out), _stream_handle(stream))
        return out

    def close(self):
        if self.handle is not None:
            dks_musr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
