// Chi-square and maximum-likelihood evaluation of muon-spin-rotation positron
// histograms on the device (section "Parameter Fitting with Minuit2": the
// positron histogram and asymmetry equations give the model, the chi-square
// and log-likelihood equations the statistic).  The histograms stay resident;
// a call brings only the parameter vector and produces one FP64 number.
//
// One fused kernel per call: every workgroup takes 256 consecutive time
// bins of a group of detectors, evaluates the model (the time-only factors
// once per bin, shared by the group's detectors), accumulates the statistic
// in FP64, reduces it across the workgroup in a fixed order and stores a
// partial; a one-workgroup-per-set kernel then adds the partials in index
// order, so a result is bitwise reproducible.  (A last-workgroup-done
// counter in the first kernel would need an agent-scope release and
// acquire per workgroup, i.e. an L2 write-back and invalidate each, which
// measured slower than the second launch.)  Batched calls put the
// parameter set in the grid's z index.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include <hip/hip_runtime.h>

#include "dks_musr.h"

namespace dks {
namespace musr {

constexpr int kMaxDet = 32;
constexpr int kMaxSets = 1024;
constexpr int kThreads = 256;
constexpr int kChunk = 16;      // detector loads issued together
constexpr double kTauMu = 2.1969811;                         // muon lifetime, us
constexpr double kGammaMu = 6.283185307179586 * 0.01355388094;   // rad / (us G)

// Parameters of one evaluation, passed by value (kernel argument).
struct Params {
  double sigma, B;
  double det[kMaxDet][4];   // N0, Nbkg, A0, phi
};

// Sum over the workgroup in a fixed order: within each wavefront by xor
// shuffles, then the four wavefront sums in order.
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += lds[i];
  __syncthreads();
  return s;
}

template <int STAT>
__device__ __forceinline__ double term(double d, double N) {
  if constexpr (STAT == DKS_MUSR_CHISQ) {
    const double r = d - N;
    return d > 0.0 ? r * r / d : r * r;
  } else {
    return d > 0.0 ? (N - d) + d * log(d / N) : N - d;
  }
}

// grid: (time-bin blocks, detector groups, sets); partial: [sets][gx * gy].
// A thread owns one time bin t = n dt and every detector of its group: the
// decay exp(-t/tau), the damped decay exp(-t/tau - (sigma t)^2 / 2) and
// cos/sin of the precession angle gamma B t depend on t alone, so they are
// computed once per bin and the detectors' counts follow by
// cos(w t + phi_j) = cos(w t) cos(phi_j) - sin(w t) sin(phi_j).
template <int STAT, bool DEV>
__global__ __launch_bounds__(kThreads) void k_musr_eval(const double* __restrict__ data, long long n_bins,
                                                        double dt, Params prm, const double* __restrict__ dprm,
                                                        int nparam, int n_det, int dg,
                                                        double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  __shared__ double sN0[kMaxDet], sNb[kMaxDet], sAN[kMaxDet], sC[kMaxDet], sS[kMaxDet];
  const int set = blockIdx.z;
  const int j0 = blockIdx.y * dg;
  const int nj = min(dg, n_det - j0);
  const double* dp = DEV ? dprm + (size_t)set * nparam : nullptr;
  // the group's detector constants: lane t < nj takes detector j0 + t
  {
    const int t = (int)threadIdx.x;
    double N0 = 0.0, Nb = 0.0, A0 = 0.0, ph = 0.0;
    if constexpr (DEV) {
      if (t < nj) {
        const double* q = dp + 2 + 4 * (j0 + t);
        N0 = q[0];
        Nb = q[1];
        A0 = q[2];
        ph = q[3];
      }
    } else {
      for (int j = 0; j < nj; ++j)
        if (t == j) {
          N0 = prm.det[j0 + j][0];
          Nb = prm.det[j0 + j][1];
          A0 = prm.det[j0 + j][2];
          ph = prm.det[j0 + j][3];
        }
    }
    if (t < nj) {
      double sp, cp;
      sincos(ph, &sp, &cp);
      sN0[t] = N0;
      sNb[t] = Nb;
      sAN[t] = A0 * N0;
      sC[t] = cp;
      sS[t] = sp;
    }
  }
  __syncthreads();
  const double sigma = DEV ? dp[0] : prm.sigma;
  const double B = DEV ? dp[1] : prm.B;
  const long long n = (long long)blockIdx.x * kThreads + threadIdx.x;
  double acc = 0.0;
  if (n < n_bins) {
    const double t = (double)n * dt;
    const double a = -t / kTauMu;
    const double E = exp(a);
    const double EG = exp(a - 0.5 * (sigma * t) * (sigma * t));
    double sw, cw;
    sincos(kGammaMu * B * t, &sw, &cw);
    const double* col = data + (size_t)j0 * n_bins + n;
    // the detectors' counts of this bin in chunks of kChunk loads in flight
    for (int jb = 0; jb < nj; jb += kChunk) {
      double d[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) d[k] = jb + k < nj ? col[(size_t)(jb + k) * n_bins] : 0.0;
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        const int j = jb + k;
        if (j < nj) {
          const double N = sN0[j] * E + sAN[j] * EG * (cw * sC[j] - sw * sS[j]) + sNb[j];
          acc += term<STAT>(d[k], N);
        }
      }
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(size_t)set * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// One workgroup per set: the set's partials added in index order.
template <int STAT>
__global__ __launch_bounds__(kThreads) void k_musr_final(const double* __restrict__ partial, int nblk,
                                                         double* __restrict__ result) {
  __shared__ double red[kThreads / 64];
  const double* part = partial + (size_t)blockIdx.x * nblk;
  double v = 0.0;
  for (int i = (int)threadIdx.x; i < nblk; i += kThreads) v += part[i];
  const double tot = block_sum(v, red);
  if (threadIdx.x == 0) result[blockIdx.x] = STAT == DKS_MUSR_MLE ? 2.0 * tot : tot;
}

}  // namespace musr
}  // namespace dks

using namespace dks::musr;

struct dks_musr_plan_s {
  int n_det;
  long long n_bins;
  double dt;
  int max_sets;
  int bx;                 // time-bin workgroups
  int dg, gy;             // detectors per group, groups
  size_t ws_total;
  char* ws;
  const double* data;
  bool prepared;
};

namespace {

inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

template <int STAT, bool DEV>
hipError_t launch(const dks_musr_plan_s* p, const Params& prm, const double* dprm, int nsets, double* result,
                  hipStream_t st) {
  double* partial = reinterpret_cast<double*>(p->ws);
  hipLaunchKernelGGL((k_musr_eval<STAT, DEV>), dim3(p->bx, p->gy, nsets), dim3(kThreads), 0, st, p->data,
                     p->n_bins, p->dt, prm, dprm, 2 + 4 * p->n_det, p->n_det, p->dg, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_musr_final<STAT>), dim3(nsets), dim3(kThreads), 0, st, partial, p->bx * p->gy, result);
  return hipGetLastError();
}

dks_status run(const dks_musr_plan_s* p, dks_musr_stat stat, const Params& prm, const double* dprm, int nsets,
               double* result, hipStream_t st) {
  hipError_t e;
  if (stat == DKS_MUSR_CHISQ)
    e = dprm ? launch<DKS_MUSR_CHISQ, true>(p, prm, dprm, nsets, result, st)
             : launch<DKS_MUSR_CHISQ, false>(p, prm, dprm, nsets, result, st);
  else
    e = dprm ? launch<DKS_MUSR_MLE, true>(p, prm, dprm, nsets, result, st)
             : launch<DKS_MUSR_MLE, false>(p, prm, dprm, nsets, result, st);
  return e == hipSuccess ? DKS_OK : DKS_EHIP;
}

dks_status ready(const dks_musr_plan_s* p) {
  if (!p->ws) return DKS_EWORKSPACE;
  if (!p->prepared || !p->data) return DKS_ESTATE;
  return DKS_OK;
}

}  // namespace

extern "C" {

dks_status dks_musr_plan(int n_det, int64_t n_bins, double dt, int max_sets, dks_musr_plan_t* out) {
  if (!out) return DKS_EINVAL;
  *out = nullptr;
  if (n_det < 1 || n_det > kMaxDet || n_bins < 1 || n_bins > 0x7fffffffLL) return DKS_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt) || max_sets < 1 || max_sets > kMaxSets) return DKS_EINVAL;
  dks_musr_plan_s* p = new (std::nothrow) dks_musr_plan_s;
  if (!p) return DKS_ENOMEM;
  std::memset(p, 0, sizeof(*p));
  p->n_det = n_det;
  p->n_bins = n_bins;
  p->dt = dt;
  p->max_sets = max_sets;
  p->bx = (int)((n_bins + kThreads - 1) / kThreads);
  // share the per-bin transcendentals across as many detectors as possible
  // while keeping at least ~512 workgroups per set in flight
  const int groups = (int)std::min<long long>(n_det, std::max<long long>(1, (512 + p->bx - 1) / p->bx));
  p->dg = (n_det + groups - 1) / groups;
  p->gy = (n_det + p->dg - 1) / p->dg;
  p->ws_total = al256((size_t)max_sets * p->bx * p->gy * sizeof(double));
  *out = p;
  return DKS_OK;
}

dks_status dks_musr_workspace_bytes(dks_musr_plan_t p, size_t* bytes) {
  if (!p || !bytes) return DKS_EINVAL;
  *bytes = p->ws_total;
  return DKS_OK;
}

dks_status dks_musr_set_workspace(dks_musr_plan_t p, void* ws, size_t bytes) {
  if (!p) return DKS_EINVAL;
  if (!ws || bytes < p->ws_total || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DKS_EWORKSPACE;
  p->ws = static_cast<char*>(ws);
  p->prepared = false;
  return DKS_OK;
}

dks_status dks_musr_prepare(dks_musr_plan_t p, dks_stream_t stream) {
  (void)stream;
  if (!p) return DKS_EINVAL;
  if (!p->ws) return DKS_EWORKSPACE;
  p->prepared = true;   // the workspace holds only per-call partials: nothing to initialise
  return DKS_OK;
}

dks_status dks_musr_set_data(dks_musr_plan_t p, const double* data) {
  if (!p || !data) return DKS_EINVAL;
  p->data = data;
  return DKS_OK;
}

dks_status dks_musr_eval(dks_musr_plan_t p, dks_musr_stat stat, const double* params, double* result,
                         dks_stream_t stream) {
  if (!p || !params || !result || (stat != DKS_MUSR_CHISQ && stat != DKS_MUSR_MLE)) return DKS_EINVAL;
  const dks_status r = ready(p);
  if (r != DKS_OK) return r;
  Params prm;
  std::memset(&prm, 0, sizeof(prm));
  prm.sigma = params[0];
  prm.B = params[1];
  for (int j = 0; j < p->n_det; ++j)
    for (int q = 0; q < 4; ++q) prm.det[j][q] = params[2 + 4 * j + q];
  return run(p, stat, prm, nullptr, 1, result, static_cast<hipStream_t>(stream));
}

dks_status dks_musr_eval_batch(dks_musr_plan_t p, dks_musr_stat stat, const double* params, int nsets,
                               double* results, dks_stream_t stream) {
  if (!p || !params || !results || (stat != DKS_MUSR_CHISQ && stat != DKS_MUSR_MLE)) return DKS_EINVAL;
  if (nsets < 1 || nsets > p->max_sets) return DKS_EINVAL;
  const dks_status r = ready(p);
  if (r != DKS_OK) return r;
  Params prm;
  std::memset(&prm, 0, sizeof(prm));
  return run(p, stat, prm, params, nsets, results, static_cast<hipStream_t>(stream));
}

dks_status dks_musr_destroy(dks_musr_plan_t p) {
  if (!p) return DKS_EINVAL;
  delete p;
  return DKS_OK;
}

}  // extern "C"
