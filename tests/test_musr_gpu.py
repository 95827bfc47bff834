"""Parity of the muSR chi-square / log-likelihood evaluation with the FP64
oracle, through the C ABI.

Tolerance: relative 1e-12.  Every term is non-negative (a squared residual
over a positive weight; a Poisson deviance), so the relative error of the
sum is bounded by the terms' own relative errors (a few ulp from exp, cos
and log) plus the reduction's (at most ~25 additions deep here): both
below 1e-14.  Results must also be bitwise repeatable."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import musr_oracle as mo  # noqa: E402
from paper_1509_07685_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12


def dks():
    from paper_1509_07685_amd import dks as mod
    return mod


def rel(a, b):
    return abs(a - b) / abs(b)


def perturbed(p, seed, scale=0.05):
    g = np.random.default_rng(seed)
    return p * (1.0 + scale * g.standard_normal(p.shape))


@pytest.fixture(scope="module")
def small():
    cfg = wl.MUSR_SMALL
    d = wl.musr_histograms(cfg)
    return cfg, d, wl.musr_start_params(cfg, d)


@pytest.mark.parametrize("stat", ["chisq", "mle"])
def test_small_data_several_parameter_sets(small, stat):
    cfg, d, p0 = small
    fit = dks().MusrFit(torch.from_numpy(d).cuda(), cfg.dt_us)
    for s in range(4):
        p = p0 if s == 0 else perturbed(p0, s)
        assert rel(fit(stat, p), mo.evaluate(stat, d, p, cfg.dt_us)) <= TOL


@pytest.mark.parametrize("n_det,n_bins", [(1, 1), (1, 2047), (3, 2049), (5, 10000), (32, 777)])
@pytest.mark.parametrize("stat", ["chisq", "mle"])
def test_ragged_shapes_and_zero_counts(n_det, n_bins, stat):
    g = np.random.default_rng(n_det * 1000 + n_bins)
    d = g.poisson(3.0, (n_det, n_bins)).astype(np.float64)     # many zero bins
    dt = 7.0 / n_bins
    p = [0.4, 80.0]
    for j in range(n_det):
        p += [3.0 + g.random(), 0.2 * g.random(), 0.25, g.uniform(0, 6.28)]
    p = np.array(p)
    fit = dks().MusrFit(torch.from_numpy(d).cuda(), dt)
    assert rel(fit(stat, p), mo.evaluate(stat, d, p, dt)) <= TOL


def test_repeatable_and_counter_rearms(small):
    cfg, d, p0 = small
    fit = dks().MusrFit(torch.from_numpy(d).cuda(), cfg.dt_us)
    outs = torch.empty(60, dtype=torch.float64, device="cuda")
    for i in range(60):
        fit.eval_async("chisq" if i % 2 == 0 else "mle", p0, out=outs[i:i + 1])
    v = outs.cpu().numpy()
    assert np.all(v[0::2] == v[0]) and np.all(v[1::2] == v[1])
    assert rel(v[0], mo.chisq(d, p0, cfg.dt_us)) <= TOL and rel(v[1], mo.mle(d, p0, cfg.dt_us)) <= TOL


@pytest.mark.parametrize("stat", ["chisq", "mle"])
def test_batch_equals_single_evaluations(small, stat):
    """A central-difference gradient's 2 x 66 + 1 points in one launch."""
    cfg, d, p0 = small
    n = p0.size
    sets = [p0]
    for i in range(n):
        for sgn in (1, -1):
            q = p0.copy()
            q[i] += sgn * 1e-4 * max(abs(p0[i]), 1.0)
            sets.append(q)
    P = np.array(sets)
    fit = dks().MusrFit(torch.from_numpy(d).cuda(), cfg.dt_us, max_sets=len(sets))
    got = fit.eval_batch(stat, torch.from_numpy(P).cuda()).cpu().numpy()
    for k in (0, 1, 2, 77, len(sets) - 1):
        assert rel(got[k], fit(stat, P[k])) <= 1e-14
        assert rel(got[k], mo.evaluate(stat, d, P[k], cfg.dt_us)) <= TOL
    with pytest.raises(dks().DKSError):
        fit.eval_batch(stat, torch.from_numpy(np.vstack([P, P[:1]])).cuda())   # above max_sets


def test_full_size_16x206250():
    """The largest data set of the fitting table (about 3.3e6 bins)."""
    cfg = wl.MUSR_LARGE
    d = wl.musr_histograms(cfg)
    p0 = wl.musr_start_params(cfg, d)
    fit = dks().MusrFit(torch.from_numpy(d).cuda(), cfg.dt_us)
    for stat in ("chisq", "mle"):
        for p in (p0, perturbed(p0, 9, 0.01)):
            assert rel(fit(stat, p), mo.evaluate(stat, d, p, cfg.dt_us)) <= TOL
