"""Seeded synthetic particle bunches and request streams.

Pure input generation: random numbers drawn with numpy's PCG64 generator, in
FP64, optionally rounded to FP32.  Nothing here performs any step of the
Poisson solve; both the library's tests/benchmark and the CPU checker read
the same arrays produced here.

The bunch shapes follow the beam-dynamics use the paper describes (a compact
charged bunch in free space, particle-fitted mesh).  The concrete workloads:

  small_gaussian   32^3 nodes, h = 1e-4 m, 1e4 particles, N(0, (1 mm)^2 I),
                   1 nC in total, FP64
  uniform_sphere   64^3 nodes fitted, 1e6 particles uniform in a ball of
                   radius 2.5 mm, 1 nC
  elongated        128x128x256 nodes, h = (5e-5, 5e-5, 2e-4) m, 1e7 particles
                   N(0, diag(1, 1, 100) mm^2), 1 nC
  halo_gaussian    256^3 nodes fitted, 1e8 particles: 90% N(0, (1 mm)^2 I)
                   plus 10% uniform in the ball of radius 5 mm, 1 nC
  serving stream   2000 requests, exponential inter-arrival (mean 2 ms),
                   mesh uniform over {32^3, 48^3, 64^3, 96x96x192, 128^3},
                   10^U(4,6) particles, sigma_d ~ U(0.5, 2) mm per axis,
                   FP32 with probability 0.7, 1 nC each
"""

import dataclasses

import numpy as np

TOTAL_CHARGE = 1e-9  # C


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _cast(arrs, dtype):
    return tuple(np.ascontiguousarray(a.astype(dtype)) for a in arrs)


def gaussian_bunch(num, sigma, seed, dtype=np.float64):
    """SoA (x, y, z) from N(0, diag(sigma^2)); sigma is a 3-tuple in metres."""
    g = rng(seed)
    pts = g.standard_normal((3, num))
    return _cast([pts[d] * sigma[d] for d in range(3)], dtype)


def uniform_ball(num, radius, seed, dtype=np.float64):
    """Uniform in a ball: Gaussian direction normalised, radius R * U^(1/3)."""
    g = rng(seed)
    v = g.standard_normal((3, num))
    v /= np.sqrt((v * v).sum(axis=0))
    r = radius * np.cbrt(g.random(num))
    return _cast([v[d] * r for d in range(3)], dtype)


def halo_gaussian(num, sigma, halo_frac, halo_radius, seed, dtype=np.float64):
    """(1 - halo_frac) Gaussian core plus halo_frac uniform in a ball."""
    g = rng(seed)
    n_halo = int(round(num * halo_frac))
    n_core = num - n_halo
    core = g.standard_normal((3, n_core)) * sigma
    v = g.standard_normal((3, n_halo))
    v /= np.sqrt((v * v).sum(axis=0))
    r = halo_radius * np.cbrt(g.random(n_halo))
    halo = v * r
    pts = np.concatenate([core, halo], axis=1)
    return _cast([pts[d] for d in range(3)], dtype)


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n: tuple            # (nx, ny, nz) mesh nodes
    h: object           # (hx, hy, hz) in metres, or None for the fitted cubic mesh
    num_particles: int
    dtype: str          # "f32" or "f64"
    seed: int

    @property
    def charge_per_particle(self):
        return TOTAL_CHARGE / self.num_particles


SMALL_GAUSSIAN = Config("gaussian_32cubed_1e4_f64", (32, 32, 32), (1e-4, 1e-4, 1e-4), 10_000, "f64", 1)
UNIFORM_SPHERE = Config("uniform_sphere_64cubed_1e6", (64, 64, 64), None, 1_000_000, "f32", 2)
ELONGATED = Config("elongated_128x128x256_1e7_f32", (128, 128, 256), (5e-5, 5e-5, 2e-4), 10_000_000, "f32", 3)
HALO_GAUSSIAN = Config("halo_gaussian_256cubed_1e8_f32", (256, 256, 256), None, 100_000_000, "f32", 4)


def particles_for(cfg, dtype=None, num=None):
    """The particle set of a named workload (optionally fewer particles)."""
    dt = np.float32 if (dtype or cfg.dtype) in ("f32", np.float32) else np.float64
    num = cfg.num_particles if num is None else num
    if cfg is SMALL_GAUSSIAN or cfg.name.startswith("gaussian_32"):
        return gaussian_bunch(num, (1e-3, 1e-3, 1e-3), cfg.seed, dt)
    if cfg.name.startswith("uniform_sphere"):
        return uniform_ball(num, 2.5e-3, cfg.seed, dt)
    if cfg.name.startswith("elongated"):
        return gaussian_bunch(num, (1e-3, 1e-3, 1e-2), cfg.seed, dt)
    if cfg.name.startswith("halo_gaussian"):
        return halo_gaussian(num, 1e-3, 0.1, 5e-3, cfg.seed, dt)
    raise ValueError(cfg.name)


# --------------------------------------------------------------------------
# Serving stream
# --------------------------------------------------------------------------

SERVING_SHAPES = ((32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 96, 192), (128, 128, 128))


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float     # scheduled arrival, seconds from stream start
    n: tuple
    num_particles: int
    sigma: tuple
    dtype: str
    seed: int

    @property
    def charge_per_particle(self):
        return TOTAL_CHARGE / self.num_particles


def serving_stream(num_requests=2000, rate_hz=500.0, seed=5,
                   shapes=SERVING_SHAPES, min_log10=4.0, max_log10=6.0, p_f32=0.7):
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_hz, num_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(num_requests):
        shape = shapes[int(g.integers(len(shapes)))]
        num = int(round(10.0 ** g.uniform(min_log10, max_log10)))
        sigma = tuple(float(s) for s in g.uniform(0.5e-3, 2e-3, 3))
        dt = "f32" if g.random() < p_f32 else "f64"
        out.append(Request(i, float(t[i]), shape, num, sigma, dt, int(1000 + i)))
    return out


def request_particles(req):
    dt = np.float32 if req.dtype == "f32" else np.float64
    return gaussian_bunch(req.num_particles, req.sigma, req.seed, dt)


def gaussian_bunch_torch(torch, num, sigma, seed, dtype, device="cuda"):
    """SoA Gaussian bunch drawn directly on the device with a seeded torch
    generator (used for the request stream, whose hundreds of millions of
    particles would take minutes to draw on the host)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    pts = torch.randn((3, num), generator=g, dtype=torch.float64, device=device)
    return tuple((pts[d] * sigma[d]).to(dtype).contiguous() for d in range(3))


# --------------------------------------------------------------------------
# Muon-spin-rotation positron histograms (the parameter-fitting workload)
# --------------------------------------------------------------------------
# Synthesised by simulating decays, not by evaluating the fit model: each
# muon decays after an exponential time with the muon lifetime, precesses at
# the Larmor frequency of the field it sees (the applied field plus a normal
# spread, which is what damps the signal), and its positron is counted by
# detector j with probability (1 + a_j cos(precession angle + phase_j)) / 2;
# uncorrelated background events fall uniformly over the bins.

MUON_LIFETIME_US = 2.1969811
MUON_GAMMA_MHZ_PER_G = 0.01355388094     # gamma_mu / 2 pi


@dataclasses.dataclass(frozen=True)
class MusrConfig:
    name: str
    n_det: int
    n_bins: int
    dt_us: float          # bin width
    decays_per_det: int   # simulated muon decays per detector (before acceptance)
    field_g: float        # applied field B (gauss)
    sigma_us: float       # field spread expressed as a depolarisation rate (1/us)
    background: float     # mean background counts per bin
    seed: int


# 16 detectors x 206 250 bins ~ 3.3e6 bins: the largest data set of the
# parameter-fitting table; 10 us of data.
MUSR_LARGE = MusrConfig("musr_16x206250", 16, 206_250, 10.0 / 206_250, 3_000_000, 100.0, 0.3, 0.5, 21)
MUSR_SMALL = MusrConfig("musr_16x4096", 16, 4096, 10.0 / 4096, 200_000, 100.0, 0.3, 0.5, 22)


def musr_truth(cfg):
    """The simulation's own settings per detector: (asymmetry a_j, phase_j)."""
    j = np.arange(cfg.n_det)
    return 0.25 + 0.01 * np.cos(j), 2.0 * np.pi * j / cfg.n_det


def musr_histograms(cfg, chunk=4_000_000):
    """Counts [n_det][n_bins] (float64 integers) of the simulated decays."""
    g = rng(cfg.seed)
    a, phase = musr_truth(cfg)
    spread_g = cfg.sigma_us / (2.0 * np.pi * MUON_GAMMA_MHZ_PER_G)
    out = np.zeros((cfg.n_det, cfg.n_bins), dtype=np.float64)
    t_end = cfg.n_bins * cfg.dt_us
    for j in range(cfg.n_det):
        left = cfg.decays_per_det
        while left > 0:
            m = min(chunk, left)
            left -= m
            t = g.exponential(MUON_LIFETIME_US, m)
            field = cfg.field_g + spread_g * g.standard_normal(m)
            angle = 2.0 * np.pi * MUON_GAMMA_MHZ_PER_G * field * t
            keep = (t < t_end) & (g.random(m) < 0.5 * (1.0 + a[j] * np.cos(angle + phase[j])))
            b = np.minimum((t[keep] / cfg.dt_us).astype(np.int64), cfg.n_bins - 1)
            out[j] += np.bincount(b, minlength=cfg.n_bins)
        out[j] += g.poisson(cfg.background, cfg.n_bins)
    return out


def musr_start_params(cfg, counts):
    """A plausible starting parameter vector [sigma, B, (N0, Nbkg, A0, phi) x n_det]
    from the simulation settings (N0 from the decay count per bin)."""
    a, phase = musr_truth(cfg)
    n0 = 0.5 * cfg.decays_per_det * cfg.dt_us / MUON_LIFETIME_US
    p = [cfg.sigma_us, cfg.field_g]
    for j in range(cfg.n_det):
        p += [n0, cfg.background, a[j], phase[j]]
    return np.array(p, dtype=np.float64)
