// Host-side checks of the invariants the Stockham pass kernels rely on.
//
// The pass kernels (fft_engine.h and the kernels built on it) assume, for
// every 1-D plan they are launched with:
//
//   V1  structure: 1 <= N <= max_length; npass <= max_pass, and npass = 0
//       only for N = 1 (a copy through the tile); every radix
//       is 2, 3, 4 or 8 and their product is N; Ns[0] = 1 and
//       Ns[p + 1] = Ns[p] R[p]; twiddle offsets tw_off[0] = tw_off[1] = 0 and
//       tw_off[p + 1] = tw_off[p] + Ns[p] (R[p] - 1)
//   V2  tile shape: W is a power of two, logW = log2 W, LD is W or W + 1
//   V3  butterfly coverage: a pass of radix R gives each thread
//       ceil(emax / R) butterfly slots, so W N / R <= ceil(emax / R) threads
//       for every pass (a pass that needs more would leave outputs unwritten)
//   V4  tile loads: a kernel that stages its whole tile through registers
//       first (the x passes: tile_elems values per row, tile_regs values per
//       thread) needs W tile_elems <= tile_regs threads
//   V5  LDS: the tile (N LD complex values) plus the kernel's extra LDS fits
//       the hardware's LDS per workgroup
//
// Barriers: every barrier of the pass kernels sits in workgroup-uniform
// control flow (pass loops over the plan, tile loops over the block's own
// range), which no plan value can change; that is a property of the code,
// not of a plan, and is not checked here.
//
// The function is plain C++ over any plan type with the fields of FFTPlan
// (N, npass, W, logW, LD, R[], Ns[], tw_off[]), so a host-only test can run
// it over every plan shape with the library's constants and with others.
#ifndef DKS_FFT_PLAN_CHECK_H
#define DKS_FFT_PLAN_CHECK_H

#include <stddef.h>

namespace dks {

// What the pass kernels were built with.
struct EngineLimits {
  int threads;       // lanes per workgroup of the pass kernels
  int emax;          // complex values of the tile per thread (sets butterfly slots per pass)
  int max_length;    // longest transform
  int max_pass;      // longest radix sequence
  size_t lds_hw;     // LDS per workgroup the hardware grants (bytes)
};

enum PlanViolation : int {
  kPlanOk = 0,
  kPlanStructure = 1,   // V1
  kPlanTileShape = 2,   // V2
  kPlanCoverage = 3,    // V3
  kPlanTileLoad = 4,    // V4
  kPlanLds = 5,         // V5
};

// csize: bytes per complex value.  tile_elems / tile_regs: V4's row length
// and per-thread register count (tile_regs = 0: the kernel does not stage
// its tile through registers).  extra_lds: LDS bytes the kernel uses beside
// the tile.
template <class Plan>
inline int fft_plan_violation(const Plan& P, const EngineLimits& L, size_t csize, int tile_elems, int tile_regs,
                              size_t extra_lds) {
  // V1
  if (P.N < 1 || P.N > L.max_length || P.npass < 0 || P.npass > L.max_pass) return kPlanStructure;
  if ((P.npass == 0) != (P.N == 1)) return kPlanStructure;
  long long prod = 1;
  int tw = 0;
  for (int p = 0; p < P.npass; ++p) {
    const int R = P.R[p];
    if (R != 2 && R != 3 && R != 4 && R != 8) return kPlanStructure;
    if (P.Ns[p] != prod) return kPlanStructure;
    if (P.tw_off[p] != tw) return kPlanStructure;
    if (p > 0) tw += P.Ns[p] * (R - 1);
    prod *= R;
  }
  if (prod != P.N) return kPlanStructure;
  // V2
  if (P.W < 1 || (P.W & (P.W - 1)) != 0 || (1 << P.logW) != P.W) return kPlanTileShape;
  if (P.LD != P.W && P.LD != P.W + 1) return kPlanTileShape;
  // V3
  for (int p = 0; p < P.npass; ++p) {
    const long long need = (long long)P.W * (P.N / P.R[p]);
    const long long have = (long long)((L.emax + P.R[p] - 1) / P.R[p]) * L.threads;
    if (need > have) return kPlanCoverage;
  }
  // V4
  if (tile_regs > 0 && (long long)P.W * tile_elems > (long long)tile_regs * L.threads) return kPlanTileLoad;
  // V5
  if ((size_t)P.N * (size_t)P.LD * csize + extra_lds > L.lds_hw) return kPlanLds;
  return kPlanOk;
}

}  // namespace dks

#endif  // DKS_FFT_PLAN_CHECK_H
