"""Oracle of the muon-spin-rotation chi-square and maximum-likelihood
evaluations -- test infrastructure only.

Only tests/, the smoke check and the benchmark's CPU leg import this module;
the library never does.

Written from the paper's section "Parameter Fitting with Minuit2":

  positron histogram equation:  N_j(t) = N0_j exp(-t/tau_mu) [1 + A_j(t)] + Nbkg_j,
  asymmetry equation:           A_j(t) = A0_j exp(-(sigma t)^2 / 2) cos(gamma_mu B t + phi_j),
  chi-square equation:          sum_j sum_n (d - N)^2 / d_err^2,  d_err = sqrt(d),
  log-likelihood equation:      2 sum_j sum_n [(N - d) + d log(d/N)]  (d > 0),  2 sum (N - d)  (d <= 0),

with t = n dt.  Readings: time in microseconds, B in gauss, sigma in 1/us;
tau_mu = 2.1969811 us and gamma_mu = 2 pi 0.01355388094 rad/(us G) (the
paper gives neither); d_err^2 := 1 where d <= 0 (sqrt(d) would divide by
zero); the log-likelihood expression is the Poisson deviance, which the fit
minimises.  Parameter vector [sigma, B, (N0, Nbkg, A0, phi) per detector].

All arithmetic FP64; the sums are exactly rounded (math.fsum).
"""

import math

import numpy as np

TAU_MU_US = 2.1969811
GAMMA_MU = 2.0 * math.pi * 0.01355388094     # rad / (us G)


def unpack(params, n_det):
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (2 + 4 * n_det,)
    det = p[2:].reshape(n_det, 4)
    return p[0], p[1], det[:, 0], det[:, 1], det[:, 2], det[:, 3]


def model(params, n_det, n_bins, dt):
    """Expected counts N_j(n dt), [n_det][n_bins]."""
    sigma, B, N0, Nbkg, A0, phi = unpack(params, n_det)
    t = np.arange(n_bins, dtype=np.float64) * dt
    asym = A0[:, None] * np.exp(-0.5 * (sigma * t[None, :]) ** 2) * np.cos(GAMMA_MU * B * t[None, :] + phi[:, None])
    return N0[:, None] * np.exp(-t[None, :] / TAU_MU_US) * (1.0 + asym) + Nbkg[:, None]


def chisq_terms(d, N):
    d = np.asarray(d, dtype=np.float64)
    e2 = np.where(d > 0, d, 1.0)
    return (d - N) ** 2 / e2


def mle_terms(d, N):
    d = np.asarray(d, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    out = N - d
    pos = d > 0
    out[pos] += d[pos] * np.log(d[pos] / N[pos])
    return 2.0 * out


def chisq(data, params, dt):
    n_det, n_bins = data.shape
    return math.fsum(chisq_terms(data, model(params, n_det, n_bins, dt)).ravel())


def mle(data, params, dt):
    n_det, n_bins = data.shape
    return math.fsum(mle_terms(data, model(params, n_det, n_bins, dt)).ravel())


def evaluate(stat, data, params, dt):
    return chisq(data, params, dt) if stat == "chisq" else mle(data, params, dt)
