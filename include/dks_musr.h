/*
 * dks_musr.h -- C ABI of the chi-square and maximum-likelihood evaluations of
 * muon-spin-rotation positron histograms (the paper's section "Parameter
 * Fitting with Minuit2": the minimiser runs on the host, the function it
 * minimises is evaluated on the device, the measured histograms stay on the
 * device, only the parameter set goes in and one number comes back).
 *
 * Model (positron histogram equation with the asymmetry equation): detector
 * j = 0 .. n_det-1, bin n = 0 .. n_bins-1, t = n dt (microseconds),
 *
 *   N_j(t) = N0_j exp(-t / tau_mu) [1 + A0_j exp(-(sigma t)^2 / 2) cos(gamma_mu B t + phi_j)] + Nbkg_j,
 *
 * tau_mu = 2.1969811 us (muon lifetime), gamma_mu = 2 pi x 0.01355388094
 * rad/(us G) (muon gyromagnetic ratio), sigma in 1/us, B in gauss, phi_j in
 * radians.  Parameter vector (2 + 4 n_det doubles, 66 for 16 detectors):
 *   [sigma, B, N0_0, Nbkg_0, A0_0, phi_0, N0_1, Nbkg_1, A0_1, phi_1, ...].
 *
 * Statistics over every bin of every detector, d = measured counts:
 *   DKS_MUSR_CHISQ : sum (d - N)^2 / e^2, e^2 = d for d > 0 and 1 otherwise
 *                    (chi-square equation with Poisson errors sqrt(d)),
 *   DKS_MUSR_MLE   : 2 sum [(N - d) + d log(d / N)] for d > 0, 2 sum (N - d)
 *                    for d <= 0 (log-likelihood equation; it is the Poisson
 *                    deviance, minimised by the fit).
 * Everything is FP64.  A result is deterministic: the same inputs give the
 * same bits (fixed-order reduction, no floating-point atomics).
 *
 * Status codes, dtypes and streams as in dks_poisson.h.  A plan's
 * evaluations share its workspace: issue them on one stream.
 */
#ifndef DKS_MUSR_H
#define DKS_MUSR_H

#include "dks_poisson.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { DKS_MUSR_CHISQ = 0, DKS_MUSR_MLE = 1 } dks_musr_stat;

typedef struct dks_musr_plan_s* dks_musr_plan_t;

/* Create a plan for n_det (1..32) histograms of n_bins (1..2^31-1) bins of
 * width dt > 0 microseconds, evaluating up to max_sets (1..1024) parameter
 * sets per batched call.  Host only. */
dks_status dks_musr_plan(int n_det, int64_t n_bins, double dt, int max_sets, dks_musr_plan_t* out);

/* Bytes of device workspace (per-set workgroup partials). */
dks_status dks_musr_workspace_bytes(dks_musr_plan_t plan, size_t* bytes);

/* Attach the caller-owned workspace (256-byte aligned); prepare must follow. */
dks_status dks_musr_set_workspace(dks_musr_plan_t plan, void* workspace, size_t bytes);

/* Mark the plan ready once its workspace is attached (nothing is enqueued). */
dks_status dks_musr_prepare(dks_musr_plan_t plan, dks_stream_t stream);

/* Attach the measured histograms: device FP64 [n_det][n_bins], caller-owned,
 * read by every later evaluation (the data stay resident on the device). */
dks_status dks_musr_set_data(dks_musr_plan_t plan, const double* data);

/* One evaluation.  params: host array of 2 + 4 n_det doubles, read before
 * the call returns (it travels as a kernel argument).  result: device
 * double, written on `stream`. */
dks_status dks_musr_eval(dks_musr_plan_t plan, dks_musr_stat stat, const double* params, double* result,
                         dks_stream_t stream);

/* nsets evaluations in one launch (e.g. the points of a numerical gradient).
 * params: device [nsets][2 + 4 n_det] doubles; results: device [nsets]. */
dks_status dks_musr_eval_batch(dks_musr_plan_t plan, dks_musr_stat stat, const double* params, int nsets,
                               double* results, dks_stream_t stream);

/* Release the plan's host state. */
dks_status dks_musr_destroy(dks_musr_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* DKS_MUSR_H */
