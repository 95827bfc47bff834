"""Parity with the FP64 oracle at the sizes the solver is built for, through
the C ABI, element by element:

  * mesh solves (rho -> phi, E) at 128^3 in FP64 and at 256^3 (the 512^3
    doubled grid of the benchmark) in FP32 and FP64, whole phi and E;
  * the request-stream meshes 96 x 96 x 192 (radix-3 doubled lengths 192 and
    384 on the runtime plans) and 128^3 as particle steps in both dtypes;
  * the benchmark's 1e8-particle step on the fitted 256^3 mesh in FP32 in the
    launch configuration the benchmark times: phi on every node and E at
    every particle.

Tolerances (relative L2 over the whole compared array): 1e-12 FP64, 2e-5 FP32.
Each test prints what it is about to run, so a failure names its case.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import poisson_oracle as orc  # noqa: E402
from paper_1509_07685_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-5, "f64": 1e-12}
NP_DT = {"f32": np.float32, "f64": np.float64}


def dks():
    from paper_1509_07685_amd import dks as mod
    return mod


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a.astype(NP_DT[dt]))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("n,h,dt", [
    ((128, 128, 128), (1e-4, 1e-4, 1e-4), "f64"),
    ((96, 96, 192), (1e-4, 1e-4, 2e-4), "f64"),
    ((96, 96, 192), (1e-4, 1e-4, 2e-4), "f32"),
    ((256, 256, 256), (1e-5, 1e-5, 1e-5), "f32"),
    ((256, 256, 256), (1e-5, 1e-5, 1e-5), "f64"),
])
def test_large_mesh_solve_whole_field(n, h, dt):
    """A white-noise density (every Fourier mode excited) on the whole mesh:
    phi and E everywhere against the oracle's doubled-grid convolution."""
    say(f"solve_rho {n} {dt}")
    g = np.random.default_rng(300 + n[0] + n[2])
    rho = g.standard_normal((n[2], n[1], n[0])).astype(NP_DT[dt])
    plan = dks().PoissonPlan(n, h, dt)
    phi, E = plan.solve_rho(dev(rho, dt))
    phi_d, E_d = host(phi), host(E)
    del phi, E, plan
    torch.cuda.empty_cache()
    phi_ref, E_ref = orc.solve_rho(rho.astype(np.float64), h)
    e_phi = rel_l2(phi_d, phi_ref[1:-1, 1:-1, 1:-1])
    e_E = rel_l2(E_d, E_ref)
    say(f"  rel-L2 phi {e_phi:.2e}  E {e_E:.2e}")
    assert e_phi <= TOL[dt] and e_E <= TOL[dt]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("n", [(96, 96, 192), (128, 128, 128)])
def test_request_stream_meshes_particle_step(n, dt):
    """The two largest meshes of the request stream, fitted to a bunch with
    independent random widths per axis (as a request draws them)."""
    say(f"particle step {n} {dt}")
    g = np.random.default_rng(n[2] + (1 if dt == "f32" else 2))
    sigma = tuple(float(s) for s in g.uniform(0.5e-3, 2e-3, 3))
    x, y, z = wl.gaussian_bunch(400_000, sigma, 410 + n[0], NP_DT[dt])
    q = wl.TOTAL_CHARGE / x.size
    plan = dks().PoissonPlan(n, None, dt)
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q, want_phi=True)
    ref = orc.solve_particles(x, y, z, q, n, dtype=NP_DT[dt])
    assert int(host(cnt)[0]) == ref["n_outside"] == 0
    assert plan.geometry()[0] == ref["h"]
    e_phi = rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1])
    e_E = rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"])
    say(f"  rel-L2 phi {e_phi:.2e}  E {e_E:.2e}")
    assert e_phi <= TOL[dt] and e_E <= TOL[dt]


def test_halo_gaussian_full_step_every_particle():
    """The 256^3 fitted mesh with 1e8 halo-Gaussian particles in FP32, one
    step as the benchmark runs it: phi on every node and E at every particle
    against the oracle's own deposit, convolution, field and gather."""
    cfg = wl.HALO_GAUSSIAN
    say(f"full step {cfg.name}: drawing particles")
    x, y, z = wl.particles_for(cfg, dtype="f32")
    q = cfg.charge_per_particle
    plan = dks().PoissonPlan(cfg.n, None, "f32")
    tx, ty, tz = dev(x, "f32"), dev(y, "f32"), dev(z, "f32")
    say("  device step")
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(tx, ty, tz, q, want_phi=True)
    n_out = int(host(cnt)[0])
    phi_d = host(phi)
    E_d = np.empty((3, x.size), dtype=np.float32)
    for d, t in enumerate((Ex, Ey, Ez)):
        torch.cuda.synchronize()
        E_d[d] = t.cpu().numpy()
    hg, og = plan.geometry()
    del Ex, Ey, Ez, phi, tx, ty, tz, plan
    torch.cuda.empty_cache()
    say(f"  oracle step ({orc.threads()} threads)")
    ref = orc.solve_particles(x, y, z, q, cfg.n, dtype=np.float32)
    assert hg == ref["h"] and og == ref["origin"]
    assert n_out == ref["n_outside"] == 0
    e_phi = rel_l2(phi_d, ref["phi_ext"][1:-1, 1:-1, 1:-1])
    del phi_d
    e_E = rel_l2(E_d, ref["E"])
    say(f"  rel-L2 phi {e_phi:.2e}  E {e_E:.2e}")
    assert e_phi <= TOL["f32"] and e_E <= TOL["f32"]
