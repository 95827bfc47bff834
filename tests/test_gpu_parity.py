"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Tolerances (relative L2 over the compared set): 1e-12 for the FP64 path and
2e-5 for the FP32 path, for phi and for E.  Integer results (out-of-mesh
counts) must match exactly; the fitted mesh geometry (FP64 on both sides,
same formula) must match to the last bit.  Inputs are seeded and synthetic;
FP32 runs feed the oracle the same FP32 values, and both sides take the
in/out-of-mesh decision in FP32.
"""

import functools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import poisson_oracle as orc  # noqa: E402
from paper_1509_07685_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-5, "f64": 1e-12}
NP_DT = {"f32": np.float32, "f64": np.float64}


def rho_tol(dt, n):
    """Tolerance for a deposited density compared alone (phi and E keep TOL).

    The FP32 path maps a position to its cell coordinate in FP32: the origin
    and 1/h are rounded (relative u = 2^-24 each), then the difference and the
    product (u each), so s = (x - x0)/h is off by at most u (|x0|/h + 3 s)
    <= 3.5 n u cells on a mesh of n nodes centred near the bunch.  The oracle
    takes the weights from the exact cell coordinate, so every weight of the
    device differs by up to that much.  Where few particles share a node the
    density's relative L2 error is of the order of the per-weight error, and
    on fine meshes (n of several hundred) it exceeds the 2e-5 that holds for
    phi and E, whose convolution averages the weight errors of many nodes.
    """
    if dt == "f64":
        return TOL[dt]
    return max(TOL[dt], 3.5 * max(n) * 2.0 ** -24)


def dks():
    from paper_1509_07685_amd import dks as mod
    return mod


def tdt(dt):
    return torch.float32 if dt == "f32" else torch.float64


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a.astype(NP_DT[dt]))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


# --------------------------------------------------------------------------
# mesh density -> potential and field
# --------------------------------------------------------------------------

RHO_CASES = [
    ((2, 2, 2), (1e-4, 1e-4, 1e-4)),      # smallest mesh
    ((3, 4, 6), (1.0, 2.0, 0.5)),         # odd, single-radix-3 x transform
    ((8, 8, 8), (1e-4, 1e-4, 1e-4)),
    ((12, 12, 12), (1e-4, 1e-4, 1e-4)),   # radix-3 passes
    ((6, 8, 9), (5e-5, 5e-5, 2e-4)),      # anisotropic cells
    ((32, 24, 18), (1e-4, 2e-4, 1.5e-4)),
    ((48, 36, 27), (1e-4, 1e-4, 1e-4)),   # several column tiles, ragged tails, 3^3 z
    ((64, 64, 64), (1e-4, 1e-4, 1e-4)),
    ((256, 9, 8), (1e-4, 2e-4, 1.5e-4)),  # rows of 256 (one wavefront per row in FP32), 110 rows
]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n,h", RHO_CASES)
def test_solve_rho_matches_oracle(n, h, dt):
    g = np.random.default_rng(100 + n[0] + 7 * n[1] + 13 * n[2])
    rho = g.standard_normal((n[2], n[1], n[0])).astype(NP_DT[dt])
    plan = dks().PoissonPlan(n, h, dt)
    phi, E = plan.solve_rho(dev(rho, dt))
    phi_ref, E_ref = orc.solve_rho(rho.astype(np.float64), h)
    assert rel_l2(host(phi), phi_ref[1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(host(E), E_ref) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_solve_rho_phi_only_and_field_only(dt):
    n, h = (16, 18, 24), (1e-4, 1e-4, 1e-4)
    rho = np.random.default_rng(5).random((24, 18, 16))
    plan = dks().PoissonPlan(n, h, dt)
    phi, E = plan.solve_rho(dev(rho, dt), want_phi=True, want_E=False)
    assert E is None
    phi2, E2 = plan.solve_rho(dev(rho, dt), want_phi=False, want_E=True)
    assert phi2 is None
    phi_ref, E_ref = orc.solve_rho(rho, h)
    assert rel_l2(host(phi), phi_ref[1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(host(E2), E_ref) <= TOL[dt]


def test_solve_rho_moved_origin_is_translation_invariant():
    n, h = (16, 16, 16), (1e-4, 1e-4, 1e-4)
    rho = np.random.default_rng(9).random((16, 16, 16))
    plan = dks().PoissonPlan(n, h, "f64")
    phi0, _ = plan.solve_rho(dev(rho, "f64"))
    plan.set_origin((1.0, -2.0, 3.0))
    phi1, _ = plan.solve_rho(dev(rho, "f64"))
    assert plan.geometry()[1] == (1.0, -2.0, 3.0)
    np.testing.assert_array_equal(host(phi0), host(phi1))


# --------------------------------------------------------------------------
# deposit and gather alone
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_deposit_matches_oracle_explicit_mesh(dt):
    cfg = wl.SMALL_GAUSSIAN
    x, y, z = wl.particles_for(cfg, dtype=dt)
    plan = dks().PoissonPlan(cfg.n, cfg.h, dt)
    rho, cnt = plan.deposit(dev(x, dt), dev(y, dt), dev(z, dt), cfg.charge_per_particle)
    origin = orc.centred_origin(cfg.n, cfg.h)
    Q, n_out = orc.deposit_cic(x, y, z, cfg.charge_per_particle, cfg.n, cfg.h, origin, NP_DT[dt])
    V = cfg.h[0] * cfg.h[1] * cfg.h[2]
    assert int(host(cnt)[0]) == n_out
    assert rel_l2(host(rho), Q / V) <= rho_tol(dt, cfg.n)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_deposit_matches_oracle_fitted_mesh(dt):
    cfg = wl.UNIFORM_SPHERE
    x, y, z = wl.particles_for(cfg, dtype=dt)
    plan = dks().PoissonPlan(cfg.n, None, dt)
    rho, cnt = plan.deposit(dev(x, dt), dev(y, dt), dev(z, dt), cfg.charge_per_particle)
    hc, origin = orc.fit_mesh(x, y, z, cfg.n)
    hg, og = plan.geometry()
    assert hg == (hc, hc, hc)
    assert og == origin
    Q, n_out = orc.deposit_cic(x, y, z, cfg.charge_per_particle, cfg.n, (hc,) * 3, origin, NP_DT[dt])
    assert n_out == 0 and int(host(cnt)[0]) == 0
    assert rel_l2(host(rho), Q / hc ** 3) <= rho_tol(dt, cfg.n)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_gather_matches_oracle(dt):
    n, h = (24, 18, 27), (1e-4, 1.2e-4, 0.8e-4)
    origin = orc.centred_origin(n, h)
    g = np.random.default_rng(21)
    E = g.standard_normal((3, n[2], n[1], n[0]))
    num = 50_000
    # include particles outside the mesh and exactly on the last node
    x = g.uniform(origin[0] - 2 * h[0], origin[0] + (n[0] + 1) * h[0], num)
    y = g.uniform(origin[1] - 2 * h[1], origin[1] + (n[1] + 1) * h[1], num)
    z = g.uniform(origin[2] - 2 * h[2], origin[2] + (n[2] + 1) * h[2], num)
    x[:3] = origin[0] + (n[0] - 1) * h[0]
    x, y, z = (a.astype(NP_DT[dt]) for a in (x, y, z))
    plan = dks().PoissonPlan(n, h, dt)
    out = plan.gather(dev(E, dt), dev(x, dt), dev(y, dt), dev(z, dt))
    ref = orc.gather_cic(E.astype(NP_DT[dt]).astype(np.float64), x, y, z, n, h, origin, NP_DT[dt])
    got = np.stack([host(t) for t in out])
    assert rel_l2(got, ref) <= TOL[dt]
    outside = ~orc.cic_stencil(x, y, z, n, h, origin, NP_DT[dt])[0]
    assert outside.sum() > 1000
    assert np.all(got[:, outside] == 0.0)


# --------------------------------------------------------------------------
# full particle step
# --------------------------------------------------------------------------

def _full_step(cfg, dt, num=None):
    x, y, z = wl.particles_for(cfg, dtype=dt, num=num)
    num = x.size
    q = wl.TOTAL_CHARGE / num
    plan = dks().PoissonPlan(cfg.n, cfg.h, dt)
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q, want_phi=True)
    ref = orc.solve_particles(x, y, z, q, cfg.n, cfg.h, dtype=NP_DT[dt])
    got_E = np.stack([host(Ex), host(Ey), host(Ez)])
    return plan, host(phi), got_E, int(host(cnt)[0]), ref


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_small_gaussian_full_step(dt):
    plan, phi, E, n_out, ref = _full_step(wl.SMALL_GAUSSIAN, dt)
    assert n_out == ref["n_outside"] > 0
    assert rel_l2(phi, ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(E, ref["E"]) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_uniform_sphere_full_step(dt):
    cfg = wl.UNIFORM_SPHERE
    plan, phi, E, n_out, ref = _full_step(cfg, dt)
    assert n_out == 0
    assert plan.geometry()[0] == ref["h"]
    assert rel_l2(phi, ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(E, ref["E"]) <= TOL[dt]
    # and against the analytic uniform sphere (shot-noise limited)
    R, Q = 2.5e-3, wl.TOTAL_CHARGE
    h = ref["h"][0]
    o = ref["origin"]
    c = [o[d] + np.arange(cfg.n[d]) * h for d in range(3)]
    Zg, Yg, Xg = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    r = np.sqrt(Xg ** 2 + Yg ** 2 + Zg ** 2)
    eps0 = 8.8541878128e-12
    rho0 = Q / (4.0 / 3.0 * math.pi * R ** 3)
    ana = np.where(r < R, rho0 * (3 * R * R - r * r) / (6 * eps0), Q / (4 * math.pi * eps0 * np.maximum(r, 1e-30)))
    assert rel_l2(phi, ana) < 3e-3


def test_elongated_bunch_full_step_f32():
    """128 x 128 x 256 mesh, anisotropic cells, 1e7 particles, FP32 bulk with the
    FP64-built Green's spectrum: the whole deposit-solve-gather step."""
    plan, phi, E, n_out, ref = _full_step(wl.ELONGATED, "f32")
    assert n_out == ref["n_outside"]
    assert 0.005 < n_out / wl.ELONGATED.num_particles < 0.03
    assert rel_l2(phi, ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL["f32"]
    assert rel_l2(E, ref["E"]) <= TOL["f32"]


def test_empty_and_single_particle():
    d = dks()
    plan = d.PoissonPlan((8, 8, 8), None, "f64")
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(empty, empty, empty, 1e-12, want_phi=True)
    assert host(phi).max() == 0.0 and host(phi).min() == 0.0
    assert int(host(cnt)[0]) == 0
    assert plan.geometry()[0] == (1.0, 1.0, 1.0)
    one = torch.tensor([1e-3], dtype=torch.float64, device="cuda")
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(one, one, one, 1e-12, want_phi=True)
    ref = orc.solve_particles(np.array([1e-3]), np.array([1e-3]), np.array([1e-3]), 1e-12, (8, 8, 8))
    assert rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= 1e-12
    # a lone particle on a node feels no field from itself
    assert abs(float(host(Ex)[0])) <= 1e-12 * np.abs(ref["E_mesh"]).max()


# --------------------------------------------------------------------------
# the 256^3 workload at full size
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def halo_full():
    cfg = wl.HALO_GAUSSIAN
    return cfg, wl.particles_for(cfg, dtype="f32")


def test_halo_gaussian_full_size_properties(halo_full):
    """1e8 particles on the fitted 256^3 mesh in FP32, in the launch
    configuration the benchmark times: mesh fit identical to the oracle's,
    nobody outside, charge conserved, and the total self-force of the bunch
    vanishes (CIC deposit/gather with a symmetric Green's function and
    antisymmetric central differences conserve momentum)."""
    cfg, (x, y, z) = halo_full
    q = cfg.charge_per_particle
    plan = dks().PoissonPlan(cfg.n, None, "f32")
    tx, ty, tz = dev(x, "f32"), dev(y, "f32"), dev(z, "f32")
    (Ex, Ey, Ez), _, cnt = plan.solve_particles(tx, ty, tz, q)
    hc, origin = orc.fit_mesh(x, y, z, cfg.n)
    hg, og = plan.geometry()
    assert hg == (hc, hc, hc) and og == origin
    assert int(host(cnt)[0]) == 0
    rho, _ = plan.deposit(tx, ty, tz, q)
    total = float(torch.sum(rho.double()).item()) * hc ** 3
    assert total == pytest.approx(wl.TOTAL_CHARGE, rel=2e-5)
    for comp in (Ex, Ey, Ez):
        c = comp.double()
        assert abs(float(c.sum())) <= 2e-5 * float(c.abs().sum())


def test_halo_gaussian_full_size_deposit(halo_full):
    """The 1e8-particle FP32 deposit at full size against the oracle: the whole
    deposited density on the fitted 256^3 mesh.  (Phi on every node and E at
    every particle of the same step are compared in test_gpu_targets.py.)"""
    cfg, (x, y, z) = halo_full
    q = cfg.charge_per_particle
    plan = dks().PoissonPlan(cfg.n, None, "f32")
    tx, ty, tz = dev(x, "f32"), dev(y, "f32"), dev(z, "f32")
    rho, cnt = plan.deposit(tx, ty, tz, q)
    hc, origin = orc.fit_mesh(x, y, z, cfg.n)
    Q, n_out = orc.deposit(x, y, z, q, cfg.n, (hc,) * 3, origin, np.float32)
    assert n_out == 0 and int(host(cnt)[0]) == 0
    assert rel_l2(host(rho), Q / hc ** 3) <= rho_tol("f32", cfg.n)


def test_full_size_mesh_solve_sampled_f32():
    """The 256^3 FP32 convolution (the benchmark's dominant kernels, same
    launch configuration) on a sparse random density: phi at sampled nodes,
    ghost nodes included, against the oracle's literal sum over the sources."""
    n, h = (256, 256, 256), (1e-5, 1e-5, 1e-5)
    g = np.random.default_rng(44)
    idx = g.integers(0, 256, (2000, 3))
    vals = g.standard_normal(2000)
    rho = np.zeros((256, 256, 256), dtype=np.float32)
    rho[idx[:, 2], idx[:, 1], idx[:, 0]] = vals.astype(np.float32)
    plan = dks().PoissonPlan(n, h, "f32")
    phi, E = plan.solve_rho(dev(rho, "f32"))
    phi_h = host(phi)
    src = np.argwhere(rho != 0)     # (k, j, i)
    w = rho[src[:, 0], src[:, 1], src[:, 2]].astype(np.float64)
    targets = np.concatenate([g.integers(0, 256, (48, 3)), [[0, 0, 0], [255, 255, 255], [0, 255, 128]]])
    got, want = [], []
    for (k, j, i) in targets:
        G = orc.igf_at(i - src[:, 2], j - src[:, 1], k - src[:, 0], h)
        want.append(orc.COULOMB_K * float(np.sum(w * G)))
        got.append(phi_h[k, j, i])
    assert rel_l2(got, want) <= TOL["f32"]


# --------------------------------------------------------------------------
# binned deposit/gather edge cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_dense_tile_spans_many_work_items(dt):
    """150k particles packed into one 16^3-cell tile of an explicit 48^3 mesh:
    the tile is split over many work items whose partial meshes are merged."""
    n, h = (48, 48, 48), (1e-4, 1e-4, 1e-4)
    origin = orc.centred_origin(n, h)
    g = np.random.default_rng(31)
    num = 150_000
    pos = [origin[d] + (17.0 + 14.0 * g.random(num)) * h[d] for d in range(3)]
    x, y, z = (a.astype(NP_DT[dt]) for a in pos)
    q = 1e-15
    plan = dks().PoissonPlan(n, h, dt)
    rho, cnt = plan.deposit(dev(x, dt), dev(y, dt), dev(z, dt), q)
    Q, n_out = orc.deposit_cic(x, y, z, q, n, h, origin, NP_DT[dt])
    assert int(host(cnt)[0]) == n_out == 0
    assert rel_l2(host(rho), Q / (h[0] * h[1] * h[2])) <= rho_tol(dt, n)
    (Ex, Ey, Ez), phi, _ = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q, want_phi=True)
    ref = orc.solve_particles(x, y, z, q, n, h, dtype=NP_DT[dt])
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_particles_on_tile_boundaries_and_mesh_edges(dt):
    """Particles exactly on nodes at tile boundaries (cell coordinate 16, 32),
    on the last node (n - 1), on the first node, and just outside."""
    n, h = (48, 36, 54), (1.0, 1.0, 1.0)
    origin = (0.0, 0.0, 0.0)
    g = np.random.default_rng(8)
    grid = np.array([0.0, 15.5, 16.0, 31.999, 32.0, 32.5])
    xs, ys, zs = np.meshgrid(np.r_[grid, 47.0, -0.001, 47.001], np.r_[grid, 35.0], np.r_[grid, 48.0, 53.0],
                             indexing="ij")
    x, y, z = (a.ravel().astype(NP_DT[dt]) for a in (xs, ys, zs))
    extra = [g.uniform(0, nd - 1, 5000) for nd in n]
    x, y, z = (np.concatenate([a, b.astype(NP_DT[dt])]) for a, b in zip((x, y, z), extra))
    plan = dks().PoissonPlan(n, h, dt)
    plan.set_origin(origin)
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), 1e-12, want_phi=True)
    ref = orc.solve_particles(x, y, z, 1e-12, n, h, origin=origin, dtype=NP_DT[dt])
    assert int(host(cnt)[0]) == ref["n_outside"] > 0
    assert rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]


def test_repeated_solves_reuse_state():
    """Ten solves in a row on one plan give the same answer each time (to FP32
    atomics reordering), with n_outside rewritten, not accumulated."""
    cfg = wl.SMALL_GAUSSIAN
    x, y, z = wl.particles_for(cfg, dtype="f32")
    plan = dks().PoissonPlan(cfg.n, cfg.h, "f32")
    tx, ty, tz = dev(x, "f32"), dev(y, "f32"), dev(z, "f32")
    first = None
    for _ in range(10):
        (Ex, Ey, Ez), _, cnt = plan.solve_particles(tx, ty, tz, cfg.charge_per_particle)
        e = np.stack([host(Ex), host(Ey), host(Ez)])
        if first is None:
            first, n0 = e, int(host(cnt)[0])
        assert int(host(cnt)[0]) == n0
        assert rel_l2(e, first) <= 1e-6


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("scheme,green,n", [("cic", "integrated", (32, 24, 36)), ("tsc", "integrated", (32, 24, 36)),
                                            ("ngp", "point", (32, 24, 36)),
                                            ("cic", "integrated", (256, 12, 8))])   # rows of 256: x inverse per wavefront
def test_batched_solve_matches_single_solves(dt, scheme, green, n):
    """One batched launch over elements with different particle counts and
    charges equals the elements solved one by one (and the oracle), for each
    assignment scheme and kernel."""
    d = dks()
    plan = d.PoissonPlan(n, None, dt, scheme=scheme, green=green)
    counts = [5000, 0, 12345, 1, 30000]
    charges = [1e-13, 2e-13, 5e-14, 1e-12, 3e-14]
    sig = [(1e-3, 1e-3, 1e-3), (1e-3, 1e-3, 1e-3), (0.5e-3, 1.5e-3, 1e-3), (1e-3, 1e-3, 1e-3), (2e-3, 1e-3, 1e-3)]
    parts = [wl.gaussian_bunch(c, s, 50 + i, NP_DT[dt]) for i, (c, s) in enumerate(zip(counts, sig))]
    max_np = max(counts)
    xs, ys, zs, outs = [], [], [], []
    for (x, y, z), c in zip(parts, counts):
        pad = lambda a: np.concatenate([a, np.full(max_np - c, 7.0, dtype=a.dtype)])   # beyond np: ignored
        xs.append(dev(pad(x), dt)); ys.append(dev(pad(y), dt)); zs.append(dev(pad(z), dt))
        outs.append(tuple(torch.full((max_np,), -1.0, dtype=tdt(dt), device="cuda") for _ in range(3)))
    cnt = torch.zeros(len(counts), dtype=torch.int64, device="cuda")
    table = d.particle_set_table([
        {"x": xs[b].data_ptr(), "y": ys[b].data_ptr(), "z": zs[b].data_ptr(), "Ex": outs[b][0].data_ptr(),
         "Ey": outs[b][1].data_ptr(), "Ez": outs[b][2].data_ptr(), "n_outside": cnt.data_ptr() + 8 * b,
         "np": counts[b], "q": charges[b]} for b in range(len(counts))])
    table_dev = torch.frombuffer(bytearray(table), dtype=torch.uint8).cuda()
    scratch = plan.batch_scratch(len(counts), max_np)
    plan.solve_particles_batched(table_dev, len(counts), max_np, scratch)
    cnts = host(cnt)
    for b, ((x, y, z), c, q) in enumerate(zip(parts, counts, charges)):
        got = np.stack([host(t)[:c] for t in outs[b]])
        assert np.all(host(outs[b][0])[c:] == -1.0)     # nothing written past np
        single = d.PoissonPlan(n, None, dt, scheme=scheme, green=green)
        (Ex, Ey, Ez), _, sc = single.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q)
        alone = np.stack([host(Ex), host(Ey), host(Ez)])
        assert int(cnts[b]) == int(host(sc)[0]) == 0
        if c > 1:
            assert rel_l2(got, alone) <= TOL[dt]
            ref = orc.solve_particles(x, y, z, q, n, dtype=NP_DT[dt], scheme=scheme, green=green)
            assert rel_l2(got, ref["E"]) <= TOL[dt]
        elif c == 1:
            assert np.allclose(got, alone, rtol=0, atol=1e-6 * (np.abs(alone).max() + 1e-30))


def test_batched_table_edge_elements():
    """Descriptor edge cases: an element with a NULL field pointer is empty and
    untouched; np above max_np is clamped to max_np; a negative np is empty."""
    d = dks()
    dt = "f32"
    n = (16, 16, 16)
    plan = d.PoissonPlan(n, None, dt)
    max_np = 3000
    x, y, z = wl.gaussian_bunch(5000, (1e-3, 1e-3, 1e-3), 71, np.float32)
    X, Y, Z = dev(x, dt), dev(y, dt), dev(z, dt)
    outs = [tuple(torch.full((5000,), -1.0, dtype=torch.float32, device="cuda") for _ in range(3))
            for _ in range(3)]
    cnt = torch.full((3,), -5, dtype=torch.int64, device="cuda")
    q = 1e-13
    ent = lambda b, npart, ez=True: {
        "x": X.data_ptr(), "y": Y.data_ptr(), "z": Z.data_ptr(), "Ex": outs[b][0].data_ptr(),
        "Ey": outs[b][1].data_ptr(), "Ez": outs[b][2].data_ptr() if ez else 0,
        "n_outside": cnt.data_ptr() + 8 * b, "np": npart, "q": q}
    table = d.particle_set_table([ent(0, 5000), ent(1, 100, ez=False), ent(2, -7)])
    table_dev = torch.frombuffer(bytearray(table), dtype=torch.uint8).cuda()
    plan.solve_particles_batched(table_dev, 3, max_np, plan.batch_scratch(3, max_np))
    got = np.stack([host(t) for t in outs[0]])
    assert np.all(got[:, max_np:] == -1.0)
    ref = orc.solve_particles(x[:max_np], y[:max_np], z[:max_np], q, n, dtype=np.float32)
    assert rel_l2(got[:, :max_np], ref["E"]) <= TOL[dt]
    for b in (1, 2):
        assert all(np.all(host(t) == -1.0) for t in outs[b])
    assert [int(v) for v in host(cnt)] == [0, 0, 0]


def test_deposit_with_global_tile_histogram():
    """A mesh with more than 8191 tiles of 16^3 cells: the binning keeps its
    per-tile histograms in device memory instead of LDS (512 x 256 x 256
    nodes -> 32 x 16 x 16 tiles)."""
    dt = "f32"
    n, h = (512, 256, 256), (2e-5, 2e-5, 2e-5)
    x, y, z = wl.gaussian_bunch(300_000, (2e-3, 1.2e-3, 1.2e-3), 81, np.float32)
    q = 1e-15
    plan = dks().PoissonPlan(n, h, dt)
    rho, cnt = plan.deposit(dev(x, dt), dev(y, dt), dev(z, dt), q)
    Q, n_out = orc.deposit_cic(x, y, z, q, n, h, orc.centred_origin(n, h), np.float32)
    assert int(host(cnt)[0]) == n_out
    assert rel_l2(host(rho), Q / (h[0] * h[1] * h[2])) <= rho_tol(dt, n)


@pytest.mark.parametrize("dt,num,tail", [("f32", 5 * 8192 * 256, 0), ("f32", 5 * 8192 * 256 + 4099, 4099),
                                         ("f64", 5 * 4096 * 256 + 17, 17)])
def test_pipelined_scatter_full_step(dt, num, tail):
    """Enough particles for the pipelined scatter (at least two whole chunks
    per CU: each workgroup loads its next chunk while storing the current
    one), with and without a partial last chunk, element by element against
    the oracle on a fitted 64^3 mesh."""
    x, y, z = wl.halo_gaussian(num, 1e-3, 0.1, 5e-3, 97, NP_DT[dt])
    q = 1e-16
    n = (64, 64, 64)
    plan = dks().PoissonPlan(n, None, dt)
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q, want_phi=True)
    ref = orc.solve_particles(x, y, z, q, n, dtype=NP_DT[dt])
    assert int(host(cnt)[0]) == ref["n_outside"] == 0
    assert rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]


@pytest.mark.parametrize("scheme", ["ngp", "tsc"])
def test_pipelined_scatter_schemes(scheme):
    """The pipelined scatter with the other assignment schemes (their tile of
    a particle is that of its lowest stencil node), at the smallest particle
    count that uses it plus a partial last chunk."""
    dt = "f32"
    num = 2 * 8192 * 256 + 5
    x, y, z = wl.halo_gaussian(num, 1e-3, 0.1, 5e-3, 98, NP_DT[dt])
    q = 1e-16
    n = (48, 48, 48)
    plan = dks().PoissonPlan(n, None, dt, scheme=scheme)
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q, want_phi=True)
    ref = orc.solve_particles(x, y, z, q, n, dtype=NP_DT[dt], scheme=scheme)
    assert int(host(cnt)[0]) == ref["n_outside"]
    assert rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]


def test_deposit_with_lds_histogram_without_staging():
    """6144 tiles (384 x 256 x 256 nodes): the FP32 tile histogram still fits
    in LDS, the chunk's records beside it do not, so the scatter stores each
    record straight from its lane instead of staging the chunk in LDS."""
    dt = "f32"
    n, h = (384, 256, 256), (2e-5, 2e-5, 2e-5)
    x, y, z = wl.gaussian_bunch(300_000, (1.6e-3, 1.2e-3, 1.2e-3), 83, np.float32)
    q = 1e-15
    plan = dks().PoissonPlan(n, h, dt)
    rho, cnt = plan.deposit(dev(x, dt), dev(y, dt), dev(z, dt), q)
    Q, n_out = orc.deposit_cic(x, y, z, q, n, h, orc.centred_origin(n, h), np.float32)
    assert int(host(cnt)[0]) == n_out
    assert rel_l2(host(rho), Q / (h[0] * h[1] * h[2])) <= rho_tol(dt, n)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_unaligned_particle_arrays_give_identical_results(dt):
    """Positions and field outputs that are not 16-byte aligned take the
    element-wise load/store paths.  Work-item sums are exact (fixed point), so
    the two runs differ only by the order in which the device atomics merge
    work items into shared mesh nodes: at the last bits."""
    d = dks()
    n = (48, 48, 48)
    num = 50_001
    x, y, z = wl.gaussian_bunch(num, (1e-3, 0.7e-3, 1.3e-3), 91, NP_DT[dt])
    q = 2e-14
    plan = d.PoissonPlan(n, None, dt)

    def run(offset):
        arrs = []
        for a in (x, y, z):
            buf = torch.zeros(num + 1, dtype=tdt(dt), device="cuda")
            buf[offset:offset + num] = dev(a, dt)
            arrs.append(buf[offset:offset + num])
        outs = [torch.zeros(num + 1, dtype=tdt(dt), device="cuda")[offset:offset + num] for _ in range(3)]
        c = torch.zeros(1, dtype=torch.int64, device="cuda")
        plan.solve_particles(*arrs, q, out=(outs[0], outs[1], outs[2], c))
        return np.stack([host(o) for o in outs]), int(host(c)[0])

    e0, c0 = run(0)
    e1, c1 = run(1)
    assert c0 == c1 == 0
    assert rel_l2(e1, e0) <= (1e-14 if dt == "f64" else 1e-6)
    ref = orc.solve_particles(x, y, z, q, n, dtype=NP_DT[dt])
    assert rel_l2(e0, ref["E"]) <= TOL[dt]


# --------------------------------------------------------------------------
# Assignment schemes (NGP, TSC) and the point kernel
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", ["ngp", "tsc"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_scheme_full_step_explicit_mesh(scheme, dt):
    """Explicit 32^3 mesh that leaves about a third of the bunch outside: the
    scheme's inside rule, deposit, solve and gather against the oracle."""
    cfg = wl.SMALL_GAUSSIAN
    x, y, z = wl.particles_for(cfg, dtype=dt)
    q = cfg.charge_per_particle
    plan = dks().PoissonPlan(cfg.n, cfg.h, dt, scheme=scheme)
    (Ex, Ey, Ez), phi, cnt = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q, want_phi=True)
    ref = orc.solve_particles(x, y, z, q, cfg.n, cfg.h, dtype=NP_DT[dt], scheme=scheme)
    assert int(host(cnt)[0]) == ref["n_outside"] > 0
    assert rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]


@pytest.mark.parametrize("scheme", ["ngp", "tsc"])
def test_scheme_fitted_mesh_tiles_and_deposit(scheme):
    """Fitted 48^3 mesh (three tiles per axis) with 2e5 particles: deposit and
    the full step against the oracle in FP64."""
    dt = "f64"
    n = (48, 48, 48)
    x, y, z = wl.gaussian_bunch(200_000, (1e-3, 0.8e-3, 1.3e-3), 61, np.float64)
    q = 1e-14
    plan = dks().PoissonPlan(n, None, dt, scheme=scheme)
    rho, cnt = plan.deposit(dev(x, dt), dev(y, dt), dev(z, dt), q)
    hc, origin = orc.fit_mesh(x, y, z, n)
    Q, n_out = orc.deposit(x, y, z, q, n, (hc,) * 3, origin, np.float64, scheme)
    assert n_out == 0 and int(host(cnt)[0]) == 0
    assert rel_l2(host(rho), Q / hc ** 3) <= TOL[dt]
    (Ex, Ey, Ez), _, _ = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q)
    ref = orc.solve_particles(x, y, z, q, n, dtype=np.float64, scheme=scheme)
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]


@pytest.mark.parametrize("scheme", ["ngp", "tsc"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_scheme_standalone_gather(scheme, dt):
    n, h = (24, 18, 27), (1e-4, 1.2e-4, 0.8e-4)
    origin = orc.centred_origin(n, h)
    g = np.random.default_rng(62)
    E = g.standard_normal((3, n[2], n[1], n[0]))
    x = (origin[0] + g.uniform(-1, n[0], 4000) * h[0]).astype(NP_DT[dt])
    y = (origin[1] + g.uniform(-1, n[1], 4000) * h[1]).astype(NP_DT[dt])
    z = (origin[2] + g.uniform(-1, n[2], 4000) * h[2]).astype(NP_DT[dt])
    plan = dks().PoissonPlan(n, h, dt, scheme=scheme)
    got = np.stack([host(t) for t in plan.gather(dev(E, dt), dev(x, dt), dev(y, dt), dev(z, dt))])
    ref = orc.gather(E, x, y, z, n, h, origin, NP_DT[dt], scheme)
    assert rel_l2(got, ref) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_point_kernel_solve_rho(dt):
    n, h = (24, 16, 18), (1e-4, 1.5e-4, 1e-4)
    rho = np.random.default_rng(63).standard_normal((n[2], n[1], n[0]))
    plan = dks().PoissonPlan(n, h, dt, green="point")
    phi, E = plan.solve_rho(dev(rho, dt))
    ref_phi, ref_E = orc.solve_rho(rho, h, green="point")
    assert rel_l2(host(phi), ref_phi[1:-1, 1:-1, 1:-1]) <= TOL[dt]
    assert rel_l2(host(E), ref_E) <= TOL[dt]
    # and it differs from the integrated kernel (a wrong switch would pass above only by accident)
    int_phi, _ = orc.solve_rho(rho, h)
    assert rel_l2(int_phi, ref_phi) > 1e-4


def test_point_kernel_fitted_particle_step_and_scheme_switch():
    """Point kernel on a fitted mesh (unit-spacing spectrum rescaled per
    solve) with TSC; then switching the same plan back to the integrated
    kernel requires a new prepare."""
    dt = "f64"
    n = (32, 32, 32)
    x, y, z = wl.gaussian_bunch(50_000, (1e-3, 1e-3, 1e-3), 64, np.float64)
    q = 2e-14
    d = dks()
    plan = d.PoissonPlan(n, None, dt, scheme="tsc", green="point")
    (Ex, Ey, Ez), _, _ = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q)
    ref = orc.solve_particles(x, y, z, q, n, dtype=np.float64, scheme="tsc", green="point")
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]
    d.dks_poisson_set_scheme(plan.handle, d.DKS_GREEN_INTEGRATED, d.DKS_ASSIGN_CIC)
    with pytest.raises(d.DKSError):
        plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q)
    plan.prepare()
    (Ex, Ey, Ez), _, _ = plan.solve_particles(dev(x, dt), dev(y, dt), dev(z, dt), q)
    ref = orc.solve_particles(x, y, z, q, n, dtype=np.float64)
    assert rel_l2(np.stack([host(Ex), host(Ey), host(Ez)]), ref["E"]) <= TOL[dt]


def test_particle_step_replays_from_a_captured_graph():
    """A full particle step captured into a HIP graph and replayed several
    times, with eager work between the replays, gives the eager result every
    time (to rounding: the deposit's merge uses float atomics)."""
    cfg = wl.UNIFORM_SPHERE
    x, y, z = wl.particles_for(cfg, dtype="f32", num=200_000)
    q = wl.TOTAL_CHARGE / x.size
    plan = dks().PoissonPlan(cfg.n, None, "f32")
    tx, ty, tz = dev(x, "f32"), dev(y, "f32"), dev(z, "f32")
    out = tuple(torch.empty(x.size, dtype=torch.float32, device="cuda") for _ in range(3))
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.solve_particles(tx, ty, tz, q, out=out + (cnt,))
    ref = np.stack([host(t) for t in out])
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        plan.solve_particles(tx, ty, tz, q, out=out + (cnt,))
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=cap):
        plan.solve_particles(tx, ty, tz, q, out=out + (cnt,))
    for rep in range(4):
        for t in out:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = np.stack([host(t) for t in out])
        assert rel_l2(got, ref) <= 1e-6, rep
        torch.randn(1 << 20, device="cuda").sum().item()    # unrelated eager work between replays
