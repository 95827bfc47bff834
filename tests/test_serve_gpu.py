"""The serving path on the GPU: HIP-graph replays of batched solves agree with
eager solves, and every request's result is the same alone and in the mix
(within the path's tolerance: 2e-5 FP32, 1e-12 FP64 relative L2)."""

import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1509_07685_amd import serve, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-5, "f64": 1e-12}


def rel_l2(a, b):
    a = a.double().cpu().numpy().ravel()
    b = b.double().cpu().numpy().ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_graph_replay_matches_eager():
    be = serve.GpuBackend(torch, max_batch=4, num_streams=2, max_np=20_000, use_graphs=True)
    key = ((32, 32, 32), "f32")
    ex = be.create_executor(key)
    eager_be = serve.GpuBackend(torch, max_batch=4, num_streams=1, max_np=20_000, use_graphs=False)
    ex_eager = eager_be.create_executor(key)
    for rep in range(4):
        # fresh request buffers every time: the replayed graph follows the table
        reqs = [wl.Request(i, 0.0, (32, 32, 32), 5000 + 3000 * i + 17 * rep, (1e-3, 1.2e-3, 0.8e-3), "f32",
                           77 + i + 10 * rep) for i in range(3 - rep % 2)]
        jobs = serve.make_jobs(torch, reqs)
        ref = serve.make_jobs(torch, reqs)
        t = be.launch(ex, jobs, rep % 2)
        while not be.done(t):
            pass
        t2 = eager_be.launch(ex_eager, ref, 0)
        while not eager_be.done(t2):
            pass
        torch.cuda.synchronize()
        # unrelated eager work between replays
        torch.randn(1 << 20, device="cuda").sum().item()
        for j, r in zip(jobs, ref):
            for d in range(3):
                assert rel_l2(j.payload[3][d], r.payload[3][d]) <= 1e-6
    assert sorted(ex.graphs) == [1, 2, 3, 4]


_ORACLE = {}


def _oracle_E(job):
    """The oracle's field at the request's particles (cached per request: both
    variants of the mix test serve the same requests)."""
    key = (job.rid, job.key)
    if key not in _ORACLE:
        from oracle import poisson_oracle as orc
        shape, dt = job.key
        x, y, z, _ = job.payload
        pos = [t.cpu().numpy() for t in (x, y, z)]
        ref = orc.solve_particles(*pos, job.charge, shape, dtype=np.float32 if dt == "f32" else np.float64)
        _ORACLE[key] = ref["E"]
    return _ORACLE[key]


@pytest.mark.parametrize("use_graphs", [True, False])
def test_each_result_is_the_same_alone_and_in_the_mix(use_graphs):
    """A burst over all five request-stream meshes (32^3, 48^3, 64^3,
    96 x 96 x 192, 128^3) in both dtypes: every served result equals the
    request solved alone on the device and the oracle's result."""
    from paper_1509_07685_amd import dks
    reqs = wl.serving_stream(30, rate_hz=20000.0, seed=9, min_log10=3.0, max_log10=4.5)
    assert {tuple(r.n) for r in reqs} == set(wl.SERVING_SHAPES)
    assert {r.dtype for r in reqs} == {"f32", "f64"}
    jobs = serve.make_jobs(torch, reqs)
    torch.cuda.synchronize()
    be = serve.GpuBackend(torch, max_batch=4, num_streams=3, max_np=40_000, use_graphs=use_graphs)
    stats = serve.Scheduler(be, budget_bytes=8 << 30).run(jobs)
    torch.cuda.synchronize()
    assert stats.completed == len(reqs) and stats.failed == 0 and stats.refused == 0
    assert max(stats.batch_hist) > 1
    plans = {}
    for j in jobs:
        shape, dt = j.key
        p = plans.get(j.key) or plans.setdefault(j.key, dks.PoissonPlan(shape, None, dt))
        x, y, z, outs = j.payload
        (Ex, Ey, Ez), _, _ = p.solve_particles(x, y, z, j.charge)
        torch.cuda.synchronize()
        for got, alone in zip(outs, (Ex, Ey, Ez)):
            assert rel_l2(got, alone) <= TOL[dt]
        got = np.stack([t.double().cpu().numpy() for t in outs])
        ref = _oracle_E(j)
        assert np.linalg.norm(got - ref) <= TOL[dt] * np.linalg.norm(ref), (j.rid, j.key)


def test_request_above_max_np_is_refused():
    reqs = wl.serving_stream(4, rate_hz=1e4, seed=4, min_log10=3.0, max_log10=3.2, shapes=((32, 32, 32),))
    reqs[2] = dataclasses.replace(reqs[2], num_particles=5000)
    jobs = serve.make_jobs(torch, reqs)
    be = serve.GpuBackend(torch, max_batch=2, num_streams=1, max_np=4000)
    stats = serve.Scheduler(be, budget_bytes=8 << 30).run(jobs)
    assert stats.refused == 1 and stats.completed == 3
    assert jobs[2].status == "refused"


def test_budget_too_small_refuses_everything_cleanly():
    reqs = wl.serving_stream(5, rate_hz=1e4, seed=3, min_log10=3.0, max_log10=3.5,
                             shapes=((32, 32, 32),))
    jobs = serve.make_jobs(torch, reqs)
    be = serve.GpuBackend(torch, max_batch=2, num_streams=1, max_np=10_000)
    stats = serve.Scheduler(be, budget_bytes=1 << 20).run(jobs)
    assert stats.refused == 5 and stats.completed == 0


@pytest.mark.parametrize("use_graphs", [True, False])
def test_host_resident_requests_match_device_solves(use_graphs):
    """Requests whose particles and fields live in page-locked host memory:
    uploaded into the executor's slots, solved in batches, downloaded; each
    result equals the request solved alone on the device."""
    from paper_1509_07685_amd import dks
    reqs = wl.serving_stream(16, rate_hz=20000.0, seed=12, min_log10=3.0, max_log10=4.3,
                             shapes=((32, 32, 32), (48, 48, 48)))
    jobs = serve.make_jobs(torch, reqs, host=True)
    be = serve.GpuBackend(torch, max_batch=4, num_streams=2, max_np=30_000, use_graphs=use_graphs, host_io=True)
    stats = serve.Scheduler(be, budget_bytes=8 << 30).run(jobs)
    torch.cuda.synchronize()
    assert stats.completed == len(reqs) and max(stats.batch_hist) > 1
    plans = {}
    for j in jobs:
        shape, dt = j.key
        p = plans.get(j.key) or plans.setdefault(j.key, dks.PoissonPlan(shape, None, dt))
        x, y, z, outs = j.payload
        assert outs[0].device.type == "cpu"
        (Ex, Ey, Ez), _, _ = p.solve_particles(x.cuda(), y.cuda(), z.cuda(), j.charge)
        torch.cuda.synchronize()
        for got, alone in zip(outs, (Ex, Ey, Ez)):
            assert rel_l2(got, alone) <= TOL[dt]
