"""The particle step with tile-ordered output (dks_poisson_solve_particles_sorted)
through the C ABI: the positions come back (in separate output arrays) as a
permutation of the input,
tile by tile of the step's mesh (particles outside the mesh last), the field
comes back in that order and equals the oracle's field of each particle, and
new_index maps every input index to its new place.  Tolerances: relative L2
2e-5 FP32, 1e-12 FP64."""

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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def tiles_of(x, y, z, n, h, origin, dtype):
    """16^3-cell tile of each particle's CIC cell (the oracle's stencil), K outside."""
    inside, (ix, iy, iz), _ = orc.cic_stencil(x, y, z, n, h, origin, dtype)
    tx, ty, tz = ((v + 15) // 16 for v in n)
    t = ((iz // 16) * ty + iy // 16) * tx + ix // 16
    return np.where(inside, t, tx * ty * tz)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("mesh", ["fitted", "explicit"])
def test_sorted_step_matches_oracle_and_orders_by_tile(dt, mesh):
    print(f"sorted step {dt} {mesh}", flush=True)
    n = (48, 36, 64)
    h = None if mesh == "fitted" else (8e-5, 8e-5, 8e-5)
    num = 300_001
    x, y, z = wl.halo_gaussian(num, 1e-3, 0.1, 5e-3, 120, NP_DT[dt])
    q = wl.TOTAL_CHARGE / num
    plan = dks().PoissonPlan(n, h, dt)
    gx, gy, gz = (torch.from_numpy(a.copy()).cuda() for a in (x, y, z))
    (tx, ty, tz), (Ex, Ey, Ez), phi, cnt, idx = plan.solve_particles_sorted(gx, gy, gz, q, want_phi=True,
                                                                           want_index=True)
    ni = host(idx).astype(np.int64)
    # new_index is a permutation, the positions moved with it exactly, and the
    # input arrays are untouched
    assert np.array_equal(np.sort(ni), np.arange(num))
    for before, after, inp in ((x, tx, gx), (y, ty, gy), (z, tz, gz)):
        a = host(after)
        assert np.array_equal(a[ni], before)
        assert np.array_equal(host(inp), before)
    ref = orc.solve_particles(x, y, z, q, n, h, dtype=NP_DT[dt])
    E = np.stack([host(t)[ni] for t in (Ex, Ey, Ez)])
    assert int(host(cnt)[0]) == ref["n_outside"]
    if mesh == "explicit":
        assert ref["n_outside"] > 0
    assert rel_l2(E, ref["E"]) <= TOL[dt]
    assert rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt]
    # binned order: tile indices never decrease along the arrays, outside last
    xs, ys, zs = host(tx), host(ty), host(tz)
    t = tiles_of(xs, ys, zs, n, ref["h"], ref["origin"], NP_DT[dt])
    assert np.all(np.diff(t) >= 0)
    # outside particles get no field
    out = t == t.max()
    if ref["n_outside"] > 0:
        assert np.all(host(Ex)[out] == 0) and np.all(host(Ez)[out] == 0)


def test_sorted_steps_in_a_row_and_the_regular_step_agree():
    """Three sorted steps in a row (each starting from the previous step's
    order) give every particle the field the regular step gives it."""
    dt = "f32"
    n = (64, 64, 64)
    num = 2 * 8192 * 256 + 777          # enough for the pipelined scatter, plus a partial chunk
    x, y, z = wl.halo_gaussian(num, 1e-3, 0.1, 5e-3, 121, np.float32)
    q = wl.TOTAL_CHARGE / num
    plan = dks().PoissonPlan(n, None, dt)
    gx, gy, gz = (torch.from_numpy(a).cuda() for a in (x, y, z))
    (Rx, Ry, Rz), _, _ = plan.solve_particles(gx, gy, gz, q)
    regular = np.stack([host(t) for t in (Rx, Ry, Rz)])
    cur = (gx.clone(), gy.clone(), gz.clone())
    other = tuple(torch.empty_like(t) for t in cur)
    where = np.arange(num)                 # current position of each original particle
    for step in range(3):
        # two sets of position arrays used in turn, as a resident caller would
        pos, (Ex, Ey, Ez), _, _, idx = plan.solve_particles_sorted(*cur, q, want_index=True, pos_out=other)
        cur, other = pos, cur
        where = host(idx).astype(np.int64)[where]
        E = np.stack([host(t)[where] for t in (Ex, Ey, Ez)])
        assert rel_l2(E, regular) <= 1e-6, step
        assert np.array_equal(host(cur[0])[where], x)


def test_sorted_step_full_size_against_the_regular_step():
    """The 1e8-particle halo-Gaussian bunch on the fitted 256^3 mesh, in the
    launch configuration of the benchmark: the sorted step's positions are the
    input permuted, and every particle's field equals the regular step's."""
    cfg = wl.HALO_GAUSSIAN
    print("sorted step full size", flush=True)
    x, y, z = wl.particles_for(cfg, dtype="f32")
    q = cfg.charge_per_particle
    plan = dks().PoissonPlan(cfg.n, None, "f32")
    gx, gy, gz = (torch.from_numpy(a).cuda() for a in (x, y, z))
    (Rx, Ry, Rz), _, rc = plan.solve_particles(gx, gy, gz, q)
    (tx, ty, tz), (Ex, Ey, Ez), _, sc, idx = plan.solve_particles_sorted(gx, gy, gz, q, want_index=True)
    torch.cuda.synchronize()
    assert int(rc.item()) == int(sc.item()) == 0
    ni = idx.long()
    assert bool(torch.equal(torch.sort(ni)[0], torch.arange(x.size, device="cuda")))
    for before, after in ((gx, tx), (gy, ty), (gz, tz)):
        assert bool(torch.equal(after[ni], before))
    num = 0.0
    den = 0.0
    for r, e in ((Rx, Ex), (Ry, Ey), (Rz, Ez)):
        d = e[ni].double() - r.double()
        num += float((d * d).sum())
        den += float((r.double() ** 2).sum())
    # both runs merge work items into the mesh with float atomics, in orders
    # that differ between runs: equal to FP32 rounding, held to the FP32 bar
    assert (num / den) ** 0.5 <= TOL["f32"]


def test_sorted_step_refuses_overlapping_outputs():
    d = dks()
    plan = d.PoissonPlan((16, 16, 16), None, "f32")
    x = torch.zeros(1000, dtype=torch.float32, device="cuda")
    e = [torch.zeros(1000, dtype=torch.float32, device="cuda") for _ in range(5)]
    plan.reserve_particles(1000)
    st = d._lib.dks_poisson_solve_particles_sorted(plan.handle, d._ptr(x), d._ptr(e[0]), d._ptr(e[1]), 1000, 1e-15,
                                                   d._ptr(x), d._ptr(e[2]), d._ptr(e[3]), d._ptr(e[4]),
                                                   d._ptr(e[4]), d._ptr(e[4]), None, None, None, None)
    assert st == d.DKS_EINVAL


def test_sorted_step_refuses_outputs_that_overlap_each_other():
    d = dks()
    plan = d.PoissonPlan((16, 16, 16), None, "f32")
    a = [torch.zeros(1000, dtype=torch.float32, device="cuda") for _ in range(8)]
    plan.reserve_particles(1000)
    p = [d._ptr(t) for t in a]
    st = d._lib.dks_poisson_solve_particles_sorted(plan.handle, p[0], p[1], p[2], 1000, 1e-15, p[3], p[4], p[5],
                                                   p[6], p[7], p[5], None, None, None, None)
    assert st == d.DKS_EINVAL


def test_sorted_step_refuses_index_that_overlaps_the_field():
    d = dks()
    plan = d.PoissonPlan((16, 16, 16), None, "f32")
    a = [torch.zeros(1000, dtype=torch.float32, device="cuda") for _ in range(9)]
    plan.reserve_particles(1000)
    p = [d._ptr(t) for t in a]
    st = d._lib.dks_poisson_solve_particles_sorted(plan.handle, p[0], p[1], p[2], 1000, 1e-15, p[3], p[4], p[5],
                                                   p[6], p[7], p[8], None, p[8], None, None)
    assert st == d.DKS_EINVAL


@pytest.mark.parametrize("scheme", ["cic", "ngp", "tsc"])
def test_sorted_step_schemes_from_random_and_from_binned_order(scheme):
    """FP32 sorted steps with each assignment scheme on a fitted 64^3 mesh
    (64 tiles) and an explicit mesh that leaves part of the bunch outside:
    from random order, and again from the first step's binned order (long
    runs of one tile): phi and E against the oracle both times."""
    dt = "f32"
    num = 700_001
    x, y, z = wl.halo_gaussian(num, 1e-3, 0.1, 5e-3, 122, np.float32)
    q = wl.TOTAL_CHARGE / num
    for n, h in (((64, 64, 64), None), ((36, 48, 54), (1.1e-4, 1.1e-4, 1.1e-4))):
        print(f"sorted step {scheme} {n}", flush=True)
        plan = dks().PoissonPlan(n, h, dt, scheme=scheme)
        ref = orc.solve_particles(x, y, z, q, n, h, dtype=np.float32, scheme=scheme)
        gx, gy, gz = (torch.from_numpy(a.copy()).cuda() for a in (x, y, z))
        pos, (Ex, Ey, Ez), phi, cnt, idx = plan.solve_particles_sorted(gx, gy, gz, q, want_phi=True, want_index=True)
        where = host(idx).astype(np.int64)
        for step in range(2):
            assert int(host(cnt)[0]) == ref["n_outside"]
            assert rel_l2(host(phi), ref["phi_ext"][1:-1, 1:-1, 1:-1]) <= TOL[dt], step
            E = np.stack([host(t)[where] for t in (Ex, Ey, Ez)])
            assert rel_l2(E, ref["E"]) <= TOL[dt], step
            if step == 0:
                pos, (Ex, Ey, Ez), phi, cnt, idx = plan.solve_particles_sorted(*pos, q, want_phi=True,
                                                                               want_index=True)
                where = host(idx).astype(np.int64)[where]
