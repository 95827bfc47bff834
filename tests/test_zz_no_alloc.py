"""The allocation-free particle step (dks_poisson_solve_particles_noalloc)
against dks_poisson_solve_particles, through the C ABI: two calls in a row on
one plan, the second with fewer particles (the static scratch keeps the first
call's contents), in both dtypes; and the size limit is refused before any
device work.  Tolerances as for every parity test: relative L2 2e-5 FP32,
1e-12 FP64 (the two entry points run the same kernels; they differ only in
the order in which float atomics merge work items)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import poisson_oracle as orc  # noqa: E402
from paper_1509_07685_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-5, "f64": 1e-12}
NP_DT = {"f32": np.float32, "f64": np.float64}
TDT = {"f32": torch.float32, "f64": torch.float64}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _noalloc(d, plan, x, y, z, q):
    num = x.numel()
    out = [torch.full((num,), float("nan"), dtype=x.dtype, device="cuda") for _ in range(3)]
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    phi = torch.empty(plan.mesh_shape(), dtype=x.dtype, device="cuda")
    d.dks_poisson_solve_particles_noalloc(plan.handle, d._ptr(x), d._ptr(y), d._ptr(z), num, float(q),
                                          d._ptr(out[0]), d._ptr(out[1]), d._ptr(out[2]), d._ptr(phi),
                                          d._ptr(cnt), None)
    torch.cuda.synchronize()
    return np.stack([t.cpu().numpy() for t in out]).astype(np.float64), phi.cpu().numpy(), int(cnt.item())


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_noalloc_matches_solve_particles_two_calls(dt):
    from paper_1509_07685_amd import dks as d
    print(f"noalloc {dt}", flush=True)
    n = (64, 64, 64)
    plan = d.PoissonPlan(n, None, dt)
    big = 3_000_000 if dt == "f32" else 2_000_000
    need = d.dks_poisson_particle_scratch_bytes(plan.handle, big)
    assert need <= d.NOALLOC_SCRATCH_BYTES
    for num, seed in ((big, 501), (150_001, 502)):
        x, y, z = wl.halo_gaussian(num, 1e-3, 0.1, 5e-3, seed, NP_DT[dt])
        q = wl.TOTAL_CHARGE / num
        tx, ty, tz = (torch.from_numpy(a).cuda() for a in (x, y, z))
        got, phi_got, cnt = _noalloc(d, plan, tx, ty, tz, q)
        (Ex, Ey, Ez), phi, c0 = plan.solve_particles(tx, ty, tz, q, want_phi=True)
        torch.cuda.synchronize()
        want = np.stack([t.cpu().numpy() for t in (Ex, Ey, Ez)]).astype(np.float64)
        assert cnt == int(c0.item()) == 0
        assert rel_l2(got, want) <= TOL[dt], num
        assert rel_l2(phi_got, phi.cpu().numpy()) <= TOL[dt], num
        if num < 1_000_000:
            ref = orc.solve_particles(x, y, z, q, n, dtype=NP_DT[dt])
            assert rel_l2(got, ref["E"]) <= TOL[dt]


def test_noalloc_refuses_counts_beyond_its_scratch():
    from paper_1509_07685_amd import dks as d
    plan = d.PoissonPlan((32, 32, 32), None, "f32")
    num = 1
    while d.dks_poisson_particle_scratch_bytes(plan.handle, num) <= d.NOALLOC_SCRATCH_BYTES:
        num *= 2
    x = torch.zeros(num, dtype=torch.float32, device="cuda")
    out = torch.full((num,), 7.0, dtype=torch.float32, device="cuda")
    st = d._lib.dks_poisson_solve_particles_noalloc(plan.handle, d._ptr(x), d._ptr(x), d._ptr(x), num, 1e-15,
                                                    d._ptr(out), d._ptr(out), d._ptr(out), None, None, None)
    assert st == d.DKS_EWORKSPACE
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
