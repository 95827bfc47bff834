"""Benchmark of the free-space PM Poisson step on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]

Workload (one "step" = the whole hot path once): the 256^3 particle-fitted
mesh (512^3 doubled grid) with 1e8 particles from a 3-D Gaussian plus a 10%
uniform halo out to 5 sigma, FP32 bulk path with the FP64-built Green's
spectrum: mesh fit, CIC deposit, the five pruned FFT passes with the fused
Green's multiply, central-difference field and CIC gather.  Inputs are
synthetic, seeded, resident in HBM before the clock starts.

Prints one JSON line: value = mesh points per second of the full step
(256^3 x steps / time).  It also carries the per-kernel breakdown measured
with HIP events on the library's stream (recorded around every kernel
launch over as many steps again, right after the timed ones: events
between the kernels would otherwise add to the timed steps), the roofline
of the 256^3 convolution from those durations, the mesh-only solve rates
in FP32 and FP64, the CPU oracle timed on a bounded sample of the same
workload, and the mixed-size request stream.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure


def algorithmic_bytes(n, num_particles, s, kernel, tile_order=False):
    """Bytes a kernel must move per launch in this design (its compulsory
    traffic: every array it reads and writes, once).  tile_order: the step
    that returns the particles in binned order (the scatter writes the binned
    positions into the caller's arrays and no inverse permutation, the gather
    reads them back and writes the field, and there is no unsort)."""
    nx, ny, nz = n
    c = 2 * s
    mesh = nx * ny * nz
    model = {
        "bbox": 3 * s * num_particles,
        "geometry": s * mesh,          # the fit and the zero fill of the deposit mesh
        "bin_count": 3 * s * num_particles,
        "bin_scan": 0,
        "bin_scatter": 3 * s * num_particles + 3 * s * num_particles + (0 if tile_order else 4 * num_particles),
        "deposit": 3 * s * num_particles + s * mesh,
        "fft_x_fwd": s * mesh + c * (nx + 1) * ny * nz,
        "fft_y_fwd": c * (nx + 1) * ny * nz + c * (nx + 1) * 2 * ny * nz,
        "fft_z_conv": (c * (nx + 1) * 2 * ny * nz + s * (nx + 1) * (ny + 1) * (nz + 1)
                       + c * (nx + 1) * 2 * ny * (nz + 2)),
        "fft_y_inv": c * (nx + 1) * 2 * ny * (nz + 2) + c * (nx + 1) * (ny + 2) * (nz + 2),
        "fft_x_inv": c * (nx + 1) * (ny + 2) * (nz + 2) + s * (nx + 2) * (ny + 2) * (nz + 2),
        "gradient": s * (nx + 2) * (ny + 2) * (nz + 2) + 3 * s * mesh,
        "gather": 6 * s * num_particles + s * (nx + 2) * (ny + 2) * (nz + 2),
        "unsort": 4 * num_particles + 3 * s * num_particles + 3 * s * num_particles,
    }
    return model[kernel]


def method_bytes(n, num_particles, s, kernel, tile_order=False):
    """Bytes the method itself must move per launch, by the per-step byte model
    of the path (mesh fit: positions read once; deposit: positions read, mesh
    written, plus one read and one write of the positions for binning; the
    five convolution passes; gather: positions read, field at the particles
    written in the caller's order, mesh read).  What a kernel moves beyond
    this (the count pass's second read of the positions, the permutation,
    the gather's sorted copy of the field and the unsort's re-read of it) is
    overhead of this design."""
    nx, ny, nz = n
    mesh = nx * ny * nz
    part = 3 * s * num_particles
    if kernel in ("fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv", "geometry", "bin_scan",
                  "gradient"):
        return algorithmic_bytes(n, num_particles, s, kernel)
    return {
        "bbox": part,
        "bin_count": 0,
        "bin_scatter": 2 * part,
        "deposit": part + s * mesh,
        "gather": (2 * part if tile_order else part) + s * (nx + 2) * (ny + 2) * (nz + 2),
        "unsort": part,
    }[kernel]


# Library timing names -> kernel symbols as rocprofv3 reports them (the
# 256^3 FP32 workload's instances).
KERNEL_SYMBOL = {
    "bbox": "k_bbox", "geometry": "k_geometry_zero", "bin_count": "k_bin_count",
    "bin_scan": "k_bin_scan", "bin_scatter": "k_bin_scatter_pipe", "deposit": "k_deposit_binned",
    "fft_x_fwd": "k_fft_x_fwd", "fft_y_fwd": "k_fft_y_fwd", "fft_z_conv": "k_fft_z_conv_pipe",
    "fft_y_inv": "k_fft_y_inv", "fft_x_inv": "k_fft_x_inv_wave", "gradient": "k_gradient",
    "gather": "k_gather_binned_field", "unsort": "k_unsort",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_halo_gaussian_256cubed_1e8_f32.json")


def measured_traffic(kernel, tile_order=False):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when there is none or the kernel's source file
    (or the shared internal header) has changed since it was taken."""
    import hashlib
    import json
    if not os.path.exists(TRAFFIC_FILE):
        return None
    doc = json.load(open(TRAFFIC_FILE))
    sym = KERNEL_SYMBOL.get(kernel, "")
    if kernel in ("bin_scatter", "deposit", "gather") and tile_order:
        sym += "_tile"          # the kernels' instances that work on the caller's arrays
    src = ("fft_kernels.hip" if sym.startswith("k_fft") else
           "particle_kernels.hip" if sym in ("k_bbox", "k_geometry_zero", "k_gradient") else "bin_kernels.hip")
    deps = (src, "dks_internal.h") + (("fft_engine.h",) if src == "fft_kernels.hip" else ())
    if src == "fft_kernels.hip" and not any(f.endswith("fft_engine.h") for f in doc["sources_sha256"]):
        return None
    for f, h in doc["sources_sha256"].items():
        if not f.endswith(deps):
            continue
        path = os.path.join(ROOT, f)
        if not os.path.exists(path) or hashlib.sha256(open(path, "rb").read()).hexdigest() != h:
            return None
    k = doc["kernels"].get(sym)
    if k is None:
        return None
    total = k["fetch_bytes"] + k["write_bytes"]
    # the scatter's whole chunks go through the pipelined kernel, a partial
    # last chunk through the one-chunk kernel launched after it
    part = sym.replace("k_bin_scatter_pipe", "k_bin_scatter")
    if sym.startswith("k_bin_scatter_pipe") and part in doc["kernels"]:
        t = doc["kernels"][part]
        total += t["fetch_bytes"] + t["write_bytes"]
    return total


def conv_bytes(n, s):
    return sum(algorithmic_bytes(n, 0, s, k) for k in
               ("fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv"))


def timed_and_kernels(torch, dks, fn, steps, warmup):
    """ms per call of fn over `steps` calls without the library's per-kernel
    timing, then {kernel: (launches, total_ms, min_ms, max_ms)} over as many
    calls with it (its events between the kernels are not in the first)."""
    ms = time_loop(torch, fn, steps, warmup)
    dks.dks_timing_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    kk = dks.dks_timing_read()
    dks.dks_timing_enable(False)
    return ms, kk


def time_loop(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def host_offload(torch, dks, n, dtype="f32", solves=20):
    """Host-resident solves at mesh n: rho from page-locked host memory, phi
    (and optionally E) back to host memory, transfer-inclusive.  One at a
    time (issue, wait: latency p50/p99) and pipelined (all issued back to
    back: throughput), next to the device-resident solve."""
    import numpy as np
    tdt = torch.float32 if dtype == "f32" else torch.float64
    plan = dks.PoissonPlan(n, (1e-5, 1e-5, 1e-5), dtype)
    shape = plan.mesh_shape()
    rhos = [torch.rand(shape, dtype=tdt).pin_memory() for _ in range(4)]
    phis = [torch.empty(shape, dtype=tdt).pin_memory() for _ in range(4)]
    Es = [torch.empty((3,) + shape, dtype=tdt).pin_memory() for _ in range(4)]
    out = {"mesh": list(n), "dtype": dtype, "solves": solves,
           "mesh_bytes": int(np.prod(n)) * (4 if dtype == "f32" else 8)}
    rho_d = rhos[0].cuda()
    out["device_resident_ms"] = time_loop(torch, lambda: plan.solve_rho(rho_d, want_E=False), 10, 2)
    for with_E in (False, True):
        tag = "phi_E" if with_E else "phi"
        for i in range(3):   # warm-up
            plan.host_wait(plan.solve_rho_host(rhos[i % 4], phis[i % 4], Es[i % 4] if with_E else None))
        lat = []
        for i in range(solves):
            t0 = time.perf_counter()
            plan.host_wait(plan.solve_rho_host(rhos[i % 4], phis[i % 4], Es[i % 4] if with_E else None))
            lat.append((time.perf_counter() - t0) * 1e3)
        t0 = time.perf_counter()
        last = None
        for i in range(solves):
            last = plan.solve_rho_host(rhos[i % 4], phis[i % 4], Es[i % 4] if with_E else None)
        plan.host_wait(last)
        pipe_ms = (time.perf_counter() - t0) * 1e3 / solves
        lat = np.array(lat)
        out[tag] = {"one_at_a_time_p50_ms": float(np.percentile(lat, 50)),
                    "one_at_a_time_p99_ms": float(np.percentile(lat, 99)),
                    "pipelined_ms_per_solve": pipe_ms, "pipelined_solves_per_s": 1e3 / pipe_ms,
                    "pipelined_mesh_pts_per_s": float(np.prod(n)) / (pipe_ms * 1e-3)}
    plan.close()
    return out


def raw_fft(torch, dks, n=(512, 512, 256)):
    """The raw 3-D FFT entry points at the paper's largest FFT size: C2C
    forward in place (FP32, FP64) and R2C forward (FP32), against three HBM
    round trips of the array (the pass structure's compulsory traffic);
    torch.fft (the platform FFT library) timed beside them for context."""
    out = {"mesh": list(n)}
    N = n[0] * n[1] * n[2]
    for dt, cdt in (("f32", torch.complex64), ("f64", torch.complex128)):
        plan = dks.FFTPlan(n, 1, "c2c", dt)
        buf = torch.randn((1, n[2], n[1], n[0]), dtype=cdt, device="cuda")
        ms = time_loop(torch, lambda: plan.forward(buf, out=buf), 10, 2)
        c = 8 if dt == "f32" else 16
        alg = 3 * 2 * c * N
        lib_ms = time_loop(torch, lambda: torch.fft.fftn(buf, dim=(-3, -2, -1)), 10, 2)
        out[f"c2c_{dt}"] = {"ms": ms, "alg_bytes": alg, "GB_s": alg / (ms * 1e-3) / 1e9,
                            "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "torch_fft_ms": lib_ms}
        del plan, buf
        torch.cuda.empty_cache()
    plan = dks.FFTPlan(n, 1, "r2c", "f32")
    x = torch.randn((1, n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
    H = torch.empty((1, n[2], n[1], n[0] // 2 + 1), dtype=torch.complex64, device="cuda")
    ms = time_loop(torch, lambda: plan.forward(x, out=H), 10, 2)
    nh = n[0] // 2 + 1
    alg = 4 * N + 8 * nh * n[1] * n[2] + 2 * 2 * 8 * nh * n[1] * n[2]
    lib_ms = time_loop(torch, lambda: torch.fft.rfftn(x, dim=(-3, -2, -1)), 10, 2)
    out["r2c_f32"] = {"ms": ms, "alg_bytes": alg, "GB_s": alg / (ms * 1e-3) / 1e9,
                      "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "torch_fft_ms": lib_ms}
    del plan, x, H
    torch.cuda.empty_cache()
    return out


def musr_fit(torch, dks):
    """chi-square and log-likelihood evaluations of 16 positron histograms of
    206 250 bins (the largest data set of the fitting table), FP64, data
    resident: device time per evaluation (back to back), the host round trip
    a minimiser sees per call (parameters in, one number back), and a
    133-set batch (a central-difference gradient of the 66 parameters)."""
    import numpy as np
    from paper_1509_07685_amd import workloads as wl
    cfg = wl.MUSR_LARGE
    d = wl.musr_histograms(cfg)
    p0 = wl.musr_start_params(cfg, d)
    nsets = 2 * p0.size + 1
    fit = dks.MusrFit(torch.from_numpy(d).cuda(), cfg.dt_us, max_sets=nsets)
    P = torch.from_numpy(np.tile(p0, (nsets, 1))).cuda()
    bins = cfg.n_det * cfg.n_bins
    out = {"detectors": cfg.n_det, "bins": bins, "dtype": "f64", "bytes_per_eval": 8 * bins}
    for stat in ("chisq", "mle"):
        dev_ms = time_loop(torch, lambda: fit.eval_async(stat, p0), 50, 5)
        lat = []
        for _ in range(50):
            t0 = time.perf_counter()
            fit(stat, p0)
            lat.append((time.perf_counter() - t0) * 1e3)
        batch_ms = time_loop(torch, lambda: fit.eval_batch(stat, P), 10, 2)
        out[stat] = {"device_ms_per_eval": dev_ms, "evals_per_s": 1e3 / dev_ms,
                     "bins_per_s": bins / (dev_ms * 1e-3),
                     "host_round_trip_p50_ms": float(np.percentile(lat, 50)),
                     "batch133_ms_per_eval": batch_ms / nsets,
                     "batch133_bins_per_s": bins * nsets / (batch_ms * 1e-3)}
    fit.close()
    return out


def cpu_baseline():
    """The oracle as it stands, timed on this host's cores.

    All threads (the oracle's chunk pool, FFT workers and Green's-function
    loops): one full particle step on the benchmark's own 256^3 fitted mesh
    with a 1e7-particle sample of the same halo-Gaussian bunch; the mesh part
    (Green's function, convolution, gradient) is timed alone and the per-step
    time for the 1e8 particles is the mesh part plus ten times the sample's
    particle part (deposit and gather are linear in the particle count).
    One thread: the same step on the workload scaled by 1/8 (128^3 mesh,
    1.25e7 particles), whose rate is reported as measured."""
    import numpy as np
    from oracle import poisson_oracle as orc
    from paper_1509_07685_amd import workloads as wl
    threads_all = len(os.sched_getaffinity(0))
    full = wl.HALO_GAUSSIAN
    n = full.n
    sample = 10_000_000
    x, y, z = wl.halo_gaussian(sample, 1e-3, 0.1, 5e-3, full.seed, np.float32)
    q = wl.TOTAL_CHARGE / sample
    orc.set_threads(threads_all)
    t0 = time.perf_counter()
    ref = orc.solve_particles(x, y, z, q, n, dtype=np.float32)
    t_step = time.perf_counter() - t0
    t0 = time.perf_counter()
    orc.solve_rho(ref["rho"], ref["h"])
    t_mesh = time.perf_counter() - t0
    del ref
    t_part = max(t_step - t_mesh, 0.0)
    t_full = t_mesh + t_part * full.num_particles / sample
    # one thread, the workload scaled by 1/8
    n8 = (128, 128, 128)
    x8, y8, z8 = wl.halo_gaussian(12_500_000, 1e-3, 0.1, 5e-3, full.seed, np.float32)
    orc.set_threads(1)
    t0 = time.perf_counter()
    orc.solve_particles(x8, y8, z8, wl.TOTAL_CHARGE / x8.size, n8, dtype=np.float32)
    t_one = time.perf_counter() - t0
    orc.set_threads(threads_all)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    mesh_pts = n[0] * n[1] * n[2]
    return {"value": mesh_pts / t_full, "unit": "mesh-pts/s", "cores": threads_all, "kind": "oracle",
            "host_cpu": model, "host_threads": threads_all,
            "sample": f"FP64 oracle (numpy, scipy.fft, the Green's function in 113-bit C), {threads_all} threads: "
                      f"one full particle step on the 256^3 fitted mesh with a 1e7-particle sample of the "
                      f"halo-Gaussian bunch; seconds per 1e8-particle step = mesh part + 10 x particle part",
            "seconds_per_step": t_full, "mesh_part_s": t_mesh, "particle_part_s_per_1e7": t_part,
            "single_thread": {"value": n8[0] * n8[1] * n8[2] / t_one, "unit": "mesh-pts/s", "cores": 1,
                              "sample": "one full particle step on a 128^3 fitted mesh with 1.25e7 particles "
                                        "(the workload scaled by 1/8), measured",
                              "seconds_per_step": t_one}}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--particles", type=int, default=100_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--order", choices=("tile", "input"), default="tile",
                    help="timed step: particles kept in the binned (tile) order, or field in the input order")
    ap.add_argument("--no-extra", action="store_true", help="skip the mesh-only and serving legs")
    ap.add_argument("--leg", choices=("raw_fft", "musr_fit", "host_offload"),
                    help="run only this secondary leg and print its JSON (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library has no "
              f"multi-GPU path; independent solves shard across GPUs by running one process per GPU.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1509_07685_amd import dks, workloads as wl
    torch.manual_seed(0)        # the inputs the secondary legs draw with torch

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.leg:
        legs = {"raw_fft": lambda: raw_fft(torch, dks), "musr_fit": lambda: musr_fit(torch, dks),
                "host_offload": lambda: host_offload(torch, dks, wl.HALO_GAUSSIAN.n)}
        print(json.dumps({args.leg: legs[args.leg]()}))
        return

    cfg = wl.HALO_GAUSSIAN
    n = cfg.n
    num = args.particles
    x, y, z = wl.particles_for(cfg, dtype="f32", num=num)
    tx, ty, tz = (torch.from_numpy(a).cuda() for a in (x, y, z))
    del x, y, z
    q = wl.TOTAL_CHARGE / num
    plan = dks.PoissonPlan(n, None, "f32")
    out = tuple(torch.empty(num, dtype=torch.float32, device="cuda") for _ in range(3))
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    bufs = out + (cnt,)

    # The timed step keeps the particles resident on the device in the order
    # the step bins them (each step rewrites the positions in its tile order
    # and returns the field in that order), as a particle code that keeps its
    # particles on the device does; the step that returns the field in the
    # caller's input order is timed beside it (input_order_step).
    tile_order = args.order == "tile"

    pos = [(tx, ty, tz), tuple(torch.empty_like(t) for t in (tx, ty, tz)) if tile_order else None]

    def step():
        if tile_order:
            # positions alternate between two sets of arrays, as a caller
            # keeping its particles resident does
            plan.solve_particles_sorted(*pos[0], q, pos_out=pos[1], out=bufs)
            pos.reverse()
        else:
            plan.solve_particles(tx, ty, tz, q, out=bufs)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps run without the library's per-kernel timing (its events
    # between the kernels would be part of the measured time) ...
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(args.steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms_per_step = a.elapsed_time(b) / args.steps
    progress(f"full step {ms_per_step:.3f} ms")
    # ... which the same number of steps then measures, kernel by kernel
    dks.dks_timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kt = dks.dks_timing_read()
    dks.dks_timing_enable(False)
    mesh_pts = n[0] * n[1] * n[2]
    # distribution of single steps (events around each step, outside the timed loop above)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    import numpy as np
    per = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    step_dist = {"p10": float(np.percentile(per, 10)), "p50": float(np.percentile(per, 50)),
                 "p90": float(np.percentile(per, 90)), "steps": len(per)}
    # the same step captured once as a HIP graph and replayed (one launch per step from the host)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        step()
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=cap):
        step()
    torch.cuda.synchronize()
    graph_ms = time_loop(torch, graph.replay, args.steps, 2)
    del graph
    # the Green's spectrum build of a fresh plan (FP64 kernel, cosine transforms, packing)
    gp = dks.PoissonPlan(n, None, "f32", prepare=False)
    gp.prepare()
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    gp.prepare()
    g1.record()
    torch.cuda.synchronize()
    green_ms = g0.elapsed_time(g1)
    gp.close()
    del gp
    value = mesh_pts / (ms_per_step * 1e-3)

    kernels = {}
    for name, (launches, total, mn, mx) in kt.items():
        avg = total / launches
        alg = algorithmic_bytes(n, num, 4, name, tile_order)
        mb = method_bytes(n, num, 4, name, tile_order)
        kernels[name] = {"launches": launches, "avg_ms": avg, "min_ms": mn, "max_ms": mx,
                         "alg_bytes": alg, "GB_s": alg / (avg * 1e-3) / 1e9 if alg else None,
                         "method_bytes": mb, "method_GB_s": mb / (avg * 1e-3) / 1e9 if mb else None}
    # a plain 1 GiB device-to-device copy on this GPU: the achievable streaming rate
    csrc = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    cdst = torch.empty_like(csrc)
    copy_ms = time_loop(torch, lambda: cdst.copy_(csrc), 10, 2)
    copy_gbs = 2 * csrc.numel() * 4 / (copy_ms * 1e-3) / 1e9
    del csrc, cdst
    # the roofline of the path's target: the five passes of the 256^3 FFT
    # convolution (512^3 doubled grid), their summed average launch durations
    # against the byte model of the pruned passes
    conv_names = ("fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv")
    conv_ms = sum(kernels[k]["avg_ms"] for k in conv_names if k in kernels)
    conv_alg = conv_bytes(n, 4)
    conv_traffic = [measured_traffic(k, tile_order) for k in conv_names]
    conv_gbs = conv_alg / (conv_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "convolution: " + " + ".join(KERNEL_SYMBOL[k] for k in conv_names),
                "achieved": conv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": conv_gbs / HBM_PEAK_GBS,
                "traffic": None if None in conv_traffic else sum(conv_traffic),
                "alg_bytes": conv_alg, "avg_ms": conv_ms,
                "per_kernel_ms": {KERNEL_SYMBOL[k]: kernels[k]["avg_ms"] for k in conv_names if k in kernels},
                "device_copy_GB_s": copy_gbs, "frac_of_device_copy": conv_gbs / copy_gbs}
    conv = {"ms": conv_ms, "alg_bytes": conv_alg, "GB_s": conv_gbs, "mesh_pts_per_s": mesh_pts / (conv_ms * 1e-3),
            "frac": conv_gbs / HBM_PEAK_GBS, "frac_of_device_copy": conv_gbs / copy_gbs}
    # the longest kernel of the step, by the method's bytes and by this design's
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    dk = kernels[dom]
    slowest = {"kernel": KERNEL_SYMBOL.get(dom, dom), "avg_ms": dk["avg_ms"], "method_bytes": dk["method_bytes"],
               "method_frac": (dk["method_GB_s"] or 0.0) / HBM_PEAK_GBS, "design_bytes": dk["alg_bytes"],
               "design_frac": (dk["GB_s"] or 0.0) / HBM_PEAK_GBS, "traffic": measured_traffic(dom, tile_order)}
    step_method = sum(k["method_bytes"] for k in kernels.values())
    step_design = sum(k["alg_bytes"] for k in kernels.values())
    step_bytes = {"method_bytes": step_method, "design_bytes": step_design,
                  "method_frac": step_method / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "design_frac": step_design / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS}

    extra = {}
    if tile_order:
        # the same step with the field returned in the caller's input order
        # (binning, then an unsort pass through the inverse permutation)
        io_ms, kk = timed_and_kernels(torch, dks, lambda: plan.solve_particles(*pos[0], q, out=bufs), args.steps, 2)
        io_k = {k: kk[k][1] / kk[k][0] for k in kk}
        extra["input_order_step"] = {
            "ms_per_step": io_ms, "mesh_pts_per_s": mesh_pts / (io_ms * 1e-3), "kernel_ms": io_k,
            "design_bytes": sum(algorithmic_bytes(n, num, 4, k) for k in kk)}
        progress(f"input-order step {io_ms:.3f} ms")
    # the same step with the order-independent deposit (integer node totals)
    plan.set_deterministic(True)
    det_ms, kk = timed_and_kernels(torch, dks, step, args.steps, 2)
    plan.set_deterministic(False)
    extra["deterministic_step"] = {
        "ms_per_step": det_ms, "mesh_pts_per_s": mesh_pts / (det_ms * 1e-3),
        "kernel_ms": {k: kk[k][1] / kk[k][0] for k in ("geometry", "deposit", "fixed_to_weights") if k in kk}}
    progress(f"order-independent deposit step {det_ms:.3f} ms")
    if not args.no_extra:
        # the same full step with the other assignment schemes and the point kernel
        variants = {}
        for green, scheme in (("integrated", "ngp"), ("integrated", "tsc"), ("point", "cic")):
            dks.dks_poisson_set_scheme(plan.handle, dks.GREENS[green], dks.SCHEMES[scheme])
            plan.prepare()
            ms, kk = timed_and_kernels(torch, dks, step, 10, 2)
            variants[f"{scheme}_{green}"] = {
                "ms_per_step": ms, "mesh_pts_per_s": mesh_pts / (ms * 1e-3),
                "kernel_ms": {k: kk[k][1] / kk[k][0] for k in ("bin_scatter", "deposit", "gather", "unsort")
                              if k in kk}}
        dks.dks_poisson_set_scheme(plan.handle, dks.DKS_GREEN_INTEGRATED, dks.DKS_ASSIGN_CIC)
        extra["variants"] = variants
        progress("scheme variants done")
        del tx, ty, tz, out, bufs, plan, pos
        torch.cuda.empty_cache()
        # mesh-only solves (rho -> phi and E) at 256^3 in FP32 and FP64
        for dt_name, tdt in (("f32", torch.float32), ("f64", torch.float64)):
            mp = dks.PoissonPlan(n, (1e-5, 1e-5, 1e-5), dt_name)
            rho = torch.rand((n[2], n[1], n[0]), dtype=tdt, device="cuda")
            phi = torch.empty_like(rho)
            ms, kk = timed_and_kernels(torch, dks, lambda: dks.dks_poisson_solve_rho(
                mp.handle, dks._ptr(rho), dks._ptr(phi), None, dks._stream_handle(None)), 10, 2)
            s = 4 if dt_name == "f32" else 8
            cms = sum(kk[k][1] / kk[k][0] for k in conv_names if k in kk)
            extra[f"solve_{dt_name}"] = {"ms": ms, "mesh_pts_per_s": mesh_pts / (ms * 1e-3), "conv_ms": cms,
                                         "conv_GB_s": conv_bytes(n, s) / (cms * 1e-3) / 1e9,
                                         "conv_frac": conv_bytes(n, s) / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            del mp, rho, phi
            torch.cuda.empty_cache()
        progress("mesh-only solves done")
        extra["host_offload"] = host_offload(torch, dks, n)
        progress("host-resident offload done")
        torch.cuda.empty_cache()
        extra["raw_fft"] = raw_fft(torch, dks)
        progress("raw FFT done")
        extra["musr_fit"] = musr_fit(torch, dks)
        progress("chi-square / likelihood done")
        torch.cuda.empty_cache()
        try:
            from paper_1509_07685_amd import serve
            extra["serving"] = serve.bench_stream(torch)
            progress("serving at 500/s done")
            torch.cuda.empty_cache()
            # the same stream at 8x the rate: requests queue, batches form
            extra["serving_4000_per_s"] = serve.bench_stream(torch, rate_hz=4000.0)
            torch.cuda.empty_cache()
            # transfer-inclusive: requests start and end in page-locked host memory
            extra["serving_host_io"] = serve.bench_stream(torch, num_requests=500, host_io=True)
            progress("serving with transfers done")
            torch.cuda.empty_cache()
            # capacity: the same 2000 requests all arriving at once, so each path
            # runs as fast as it can (served solves/s is then the path's capacity)
            extra["serving_capacity"] = serve.bench_stream(torch, rate_hz=None)
            progress("serving capacity done")
        except ImportError:
            extra["serving"] = None

    cpu = None if args.no_cpu else cpu_baseline()
    if cpu:
        progress("CPU oracle leg done")
    line = {
        "metric": "Poisson solve mesh-pts/s (FP32 vs FP64) + served solves/s at p50/p99 latency",
        "value": value,
        "unit": "mesh-pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "halo_gaussian_256cubed_1e8_f32: 256^3 fitted mesh (512^3 doubled), "
                               f"{num} particles (90% Gaussian sigma 1 mm + 10% uniform halo to 5 sigma), "
                               "full particle step per solve, Green's spectrum cached; "
                               + ("particles resident in the step's binned (tile) order, field returned in that "
                                  "order" if tile_order else "field returned in the input order"),
                   "mesh": list(n), "particles": num},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_ms": step_dist,
        "graph_ms_per_step": graph_ms,
        "green_build_ms": green_ms,
        "kernels": kernels,
        "convolution": conv,
        "slowest_kernel": slowest,
        "step_bytes": step_bytes,
        **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
