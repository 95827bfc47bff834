"""Pins of the muon-spin-rotation oracle (oracle/musr_oracle.py): a literal
per-bin loop, the closed-form behaviour of the positron histogram (value at
t = 0, the lifetime decay, the Larmor period of the muon gyromagnetic ratio,
the Gaussian envelope), the chi-square of residuals of known size, and the
log-likelihood against the Poisson log-probabilities of scipy, its minimum
at N = d and its quadratic limit (the chi-square with errors sqrt(d))."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import musr_oracle as mo
from paper_1509_07685_amd import workloads as wl


def params_for(n_det, seed=0, sigma=0.3, B=100.0):
    g = np.random.default_rng(seed)
    p = [sigma, B]
    for j in range(n_det):
        p += [50.0 + 10 * g.random(), 0.5 + g.random(), 0.2 + 0.1 * g.random(), 2 * math.pi * g.random()]
    return np.array(p)


def test_literal_loop():
    n_det, n_bins, dt = 3, 7, 0.37
    p = params_for(n_det, 1)
    d = np.random.default_rng(2).poisson(30.0, (n_det, n_bins)).astype(float)
    d[0, 3] = 0.0
    chi = 0.0
    ml = 0.0
    for j in range(n_det):
        N0, Nb, A0, ph = p[2 + 4 * j: 6 + 4 * j]
        for n in range(n_bins):
            t = n * dt
            N = N0 * math.exp(-t / 2.1969811) * (
                1 + A0 * math.exp(-0.5 * (p[0] * t) ** 2) * math.cos(2 * math.pi * 0.01355388094 * p[1] * t + ph)) + Nb
            e2 = d[j, n] if d[j, n] > 0 else 1.0
            chi += (d[j, n] - N) ** 2 / e2
            ml += 2 * ((N - d[j, n]) + (d[j, n] * math.log(d[j, n] / N) if d[j, n] > 0 else 0.0))
    assert mo.chisq(d, p, dt) == pytest.approx(chi, rel=1e-13)
    assert mo.mle(d, p, dt) == pytest.approx(ml, rel=1e-13)


def test_histogram_closed_forms():
    n_det = 2
    p = params_for(n_det, 3)
    sigma, B = p[0], p[1]
    N = mo.model(p, n_det, 1, 0.1)
    for j in range(n_det):
        N0, Nb, A0, ph = p[2 + 4 * j: 6 + 4 * j]
        assert N[j, 0] == pytest.approx(N0 * (1 + A0 * math.cos(ph)) + Nb, rel=1e-15)
    # lifetime: without asymmetry or background the counts fall by e per tau
    q = p.copy()
    q[4::4] = 0.0     # A0
    q[3::4] = 0.0     # Nbkg
    tau = 2.1969811
    M = mo.model(q, n_det, 11, tau / 5)
    np.testing.assert_allclose(M[:, 5:] / M[:, :-5], math.exp(-1.0), rtol=1e-14)
    # Larmor period: B = 1 / 0.01355388094 G precesses at 1 MHz (period 1 us)
    r = params_for(1, 4, sigma=0.0, B=1.0 / 0.01355388094)
    r[3] = 0.0
    M = mo.model(r, 1, 41, 0.05)[0]
    osc = M / (r[2] * np.exp(-np.arange(41) * 0.05 / tau)) - 1.0
    np.testing.assert_allclose(osc[20:], osc[:21], atol=1e-12)
    np.testing.assert_allclose(osc[10], -osc[0], atol=1e-12)     # half a period later
    # Gaussian envelope: at the phase maxima the asymmetry is A0 exp(-(sigma t)^2 / 2)
    s = params_for(1, 5, sigma=0.7, B=1.0 / 0.01355388094)
    s[3] = 0.0
    s[5] = 0.0        # phi = 0: maxima at integer microseconds
    M = mo.model(s, 1, 5, 1.0)[0]
    t = np.arange(5.0)
    np.testing.assert_allclose(M / (s[2] * np.exp(-t / tau)) - 1.0, s[4] * np.exp(-0.5 * (0.7 * t) ** 2), rtol=1e-12)


def test_chisq_of_known_residuals():
    d = np.array([[4.0, 9.0, 0.0, 100.0, 1.0]])
    N = np.array([[2.0, 12.0, 0.5, 90.0, 1.0]])
    # residuals / errors: 2/2, -3/3, -0.5/1 (d = 0: unit error), 10/10, 0
    np.testing.assert_allclose(mo.chisq_terms(d, N)[0], [1.0, 1.0, 0.25, 1.0, 0.0], rtol=1e-15)


def test_mle_is_the_poisson_deviance():
    g = np.random.default_rng(6)
    d = g.poisson(7.0, 200).astype(float)
    N = g.uniform(0.5, 20.0, 200)
    dev = 2.0 * (stats.poisson.logpmf(d, d) - stats.poisson.logpmf(d, N))
    np.testing.assert_allclose(mo.mle_terms(d, N), dev, rtol=1e-10, atol=1e-12)
    assert np.all(mo.mle_terms(d, N) >= -1e-12)


def test_mle_minimum_and_quadratic_limit():
    d = np.array([25.0, 400.0, 3.0])
    assert np.all(mo.mle_terms(d, d) == 0.0)
    for eps in (1e-3, -1e-3):
        assert np.all(mo.mle_terms(d, d * (1 + eps)) > 0)
    # near N = d the deviance is the chi-square with Poisson errors to third order
    N = d + 0.01 * np.sqrt(d)
    np.testing.assert_allclose(mo.mle_terms(d, N), mo.chisq_terms(d, N), rtol=1e-2)
    # d <= 0: only the linear term
    assert mo.mle_terms(np.array([0.0]), np.array([3.5]))[0] == 7.0


def test_simulated_histograms_fit_the_model_statistically():
    """The decay simulation and the model agree: chi-square per bin near 1
    at the simulation's own settings (a check of the generator, through the
    oracle)."""
    cfg = wl.MUSR_SMALL
    d = wl.musr_histograms(cfg)
    p = wl.musr_start_params(cfg, d)
    # N0 from the decays per bin exactly: half the decays times the bin's decay probability
    p[2::4] = 0.5 * cfg.decays_per_det * (1.0 - math.exp(-cfg.dt_us / mo.TAU_MU_US))
    chi = mo.chisq(d, p, cfg.dt_us) / d.size
    assert 0.8 < chi < 1.3
