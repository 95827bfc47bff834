// Mixed-radix Stockham FFT engine shared by the convolution passes and the
// raw transform entry points: complex helpers, radix-2/3/4/8 butterflies, one
// pass over an LDS tile of W pencils ([element][pencil], pencil fastest), the
// pass loop with runtime plans, and compile-time plans for power-of-two
// lengths.  A transform of P passes reads its first pass from any source and
// hands its last pass to any sink, with P - 1 LDS round trips between.
#ifndef DKS_FFT_ENGINE_H
#define DKS_FFT_ENGINE_H

#include <type_traits>

#include "dks_internal.h"

namespace dks {

template <typename T> struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};
template <typename T> struct Cplx { using type = cpx<T>; };

// Register budget per thread: the tile holds at most kLdsBytes / sizeof(C)
// complex values spread over the block's threads (512 for FP32, 256 for
// FP64), i.e. 16 complex values per thread either way.
template <typename T> struct RegCfg {
  static constexpr int THREADS = sizeof(T) == 4 ? 512 : 256;
  static constexpr int EMAX = kLdsBytes / (2 * (int)sizeof(T)) / THREADS;
  static constexpr int ARR = EMAX + 2;     // ceil(EMAX / R) * R <= EMAX + 2 for R in {2,3,4,8}
};

// Real values per thread of an x-pass tile: a tile holds at most
// kLdsBytes / sizeof(complex) complex values, i.e. 16 per thread, and the
// forward x pass stages nx reals per row of nx complex slots.
constexpr int kTileReals = 16;

// Twiddle tables in device memory, addressed as global rather than generic
// memory: a generic (flat) load also counts in the LDS counter, so each
// pass's wait for its LDS writes before the barrier would wait for the
// twiddles' round trip to memory as well.
template <typename C> using GlobalPtr = const __attribute__((address_space(1))) C*;
template <typename C> __device__ __forceinline__ GlobalPtr<C> as_global(const void* p) {
  return (GlobalPtr<C>)p;
}

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }

// (x + iy) * (-i) in the forward direction, * (+i) in the inverse one.
template <bool INV, typename C> __device__ __forceinline__ C mul_mi(C a) {
  return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

template <bool INV, typename C> __device__ __forceinline__ void dft2(C* v) {
  const C a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4(C* v) {
  const C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  const C a2 = cadd(v[1], v[3]), a3 = mul_mi<INV>(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft8(C* v) {
  using T = decltype(C::x);
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  const T s = (T)0.70710678118654752440;   // cos(pi/4), rounded from the FP64 value
  // o[k] *= w8^k with w8 = exp(-+ i pi / 4)
  {
    const C a = o[1];
    o[1] = INV ? C{s * (a.x - a.y), s * (a.x + a.y)} : C{s * (a.x + a.y), s * (a.y - a.x)};
  }
  o[2] = mul_mi<INV>(o[2]);
  {
    const C a = o[3];
    o[3] = INV ? C{-s * (a.x + a.y), s * (a.x - a.y)} : C{s * (a.y - a.x), -s * (a.x + a.y)};
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

template <bool INV, typename C> __device__ __forceinline__ void dft3(C* v) {
  using T = decltype(C::x);
  const T sn = INV ? (T)0.86602540378443864676 : (T)-0.86602540378443864676;   // sin(-+2pi/3)
  const C t = cadd(v[1], v[2]);
  const C d = csub(v[1], v[2]);
  const C m = C{v[0].x - (T)0.5 * t.x, v[0].y - (T)0.5 * t.y};
  v[0] = cadd(v[0], t);
  const C si = C{-sn * d.y, sn * d.x};
  v[1] = cadd(m, si);
  v[2] = csub(m, si);
}

template <int R, bool INV, typename C> __device__ __forceinline__ void dft(C* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else dft8<INV>(v);
}

template <class F> __device__ __forceinline__ void radix_dispatch(int R, F&& f) {
  switch (R) {
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 3>{}); break;
  }
}

// One Stockham pass of radix R over the tile.  Every butterfly (pencil c,
// index j) this thread owns takes its R inputs j + r N/R from in(c, idx);
// after the optional barrier (needed when the pass reads and writes the LDS
// tile in place) the twiddles w^(r t), t = j mod Ns, and the radix-R DFT are
// applied and out(R, c, j, base, Ns, vals, k) receives the R outputs, whose
// positions are base + r Ns (k: the thread's butterfly slot).  pre(R, k, c, j)
// runs right after the inputs are requested, so loads it issues overlap the
// barrier.  The register array is local to this pass.
template <typename T, bool INV, int R, bool SYNC, class In, class Out, class Pre>
__device__ __forceinline__ void fft_pass(const FFTPlan* __restrict__ P, int p, In in, Out out, Pre pre) {
  using C = typename Cplx<T>::type;
  constexpr int TH = RegCfg<T>::THREADS;
  constexpr int K = (RegCfg<T>::EMAX + R - 1) / R;
  const int W = P->W, logW = P->logW, NR = P->N / R, nbf = W * NR, Ns = P->Ns[p];
  const GlobalPtr<C> tw = as_global<C>(P->tw) + P->tw_off[p];
  const unsigned magic = P->magic[p];
  C v[K * R];
  C w[K * (R - 1)];   // twiddles, fetched with the inputs so their latency hides under the barrier
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int b = (int)threadIdx.x + k * TH;
    if (b < nbf) {
      const int c = b & (W - 1), j = b >> logW;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k * R + r] = in(c, j + r * NR, k * R + r);
      pre(std::integral_constant<int, R>{}, k, c, j);
      if (Ns > 1) {
        const int q = (int)__umulhi((unsigned)j, magic);
        const GlobalPtr<C> wt = tw + (j - q * Ns) * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[k * (R - 1) + r - 1] = C{wt[r - 1].x, wt[r - 1].y};
      }
    }
  }
  if (SYNC) __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int b = (int)threadIdx.x + k * TH;
    if (b < nbf) {
      const int c = b & (W - 1), j = b >> logW;
      int base;
      if (Ns > 1) {
        const int q = (int)__umulhi((unsigned)j, magic);
        const int t = j - q * Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C wr = w[k * (R - 1) + r - 1];
          if (INV) wr.y = -wr.y;
          v[k * R + r] = cmul(v[k * R + r], wr);
        }
        base = q * Ns * R + t;
      } else {
        base = j * R;
      }
      dft<R, INV>(&v[k * R]);
      out(std::integral_constant<int, R>{}, c, j, base, Ns, &v[k * R], k);
    }
  }
}

// Runs passes [p0, npass) of plan P over the LDS tile.  Pass p0 reads
// first_in (the LDS tile itself when FIRST_LDS, so it synchronises before
// overwriting it); later passes read the tile.  The last pass hands its
// butterflies to last_out; earlier ones write the tile.  A barrier follows
// every pass that wrote the tile, except the last.
struct NoPre {
  template <class RC> __device__ __forceinline__ void operator()(RC, int, int, int) const {}
};

template <typename T, bool INV, bool FIRST_LDS, class FirstIn, class LastOut, class LastPre = NoPre>
__device__ __forceinline__ void run_fft(typename Cplx<T>::type* lds, const FFTPlan* __restrict__ P, int p0,
                                        FirstIn first_in, LastOut last_out, LastPre last_pre = LastPre{}) {
  using C = typename Cplx<T>::type;
  const int LD = P->LD;
  auto lds_in = [&](int c, int idx, int) { return lds[idx * LD + c]; };
  auto lds_out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
    for (int r = 0; r < RC.value; ++r) lds[(base + r * Ns) * LD + c] = vals[r];
  };
  const NoPre none;
  const int np = P->npass;
  for (int p = p0; p < np; ++p) {
    const bool first = p == p0, last = p == np - 1;
    radix_dispatch(P->R[p], [&](auto RC) {
      constexpr int R = RC.value;
      if (first && last) fft_pass<T, INV, R, FIRST_LDS>(P, p, first_in, last_out, last_pre);
      else if (first) fft_pass<T, INV, R, FIRST_LDS>(P, p, first_in, lds_out, none);
      else if (last) fft_pass<T, INV, R, true>(P, p, lds_in, last_out, last_pre);
      else fft_pass<T, INV, R, true>(P, p, lds_in, lds_out, none);
    });
    if (!last) __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Compile-time plans.  For the power-of-two lengths of common meshes the
// kernels are also instantiated with the whole plan known at compile time
// (length, tile width, LDS stride, radix order), so butterfly indexing,
// twiddle offsets and guards fold to constants; the runtime plan above
// serves every other shape.  A launcher uses a compile-time plan only when
// the host plan matches it exactly.
// ---------------------------------------------------------------------------
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

struct DynPlan {
  static constexpr bool is_static = false;
};

// Power-of-two length N: radix-8 passes, then one radix-4 or radix-2 pass
// (the host's order); REV reverses the order (the inverse z transform).
template <int N_, int W_, int LD_, bool REV_>
struct SPlan {
  static constexpr bool is_static = true;
  static constexpr int N = N_, W = W_, LD = LD_, logW = ilog2(W_);
  static constexpr int n8 = ilog2(N_) / 3, rem = ilog2(N_) % 3;
  static constexpr int npass = n8 + (rem ? 1 : 0);
  static constexpr int Rf(int p) { return p < n8 ? 8 : (rem == 2 ? 4 : 2); }
  static constexpr int R(int p) { return REV_ ? Rf(npass - 1 - p) : Rf(p); }
  static constexpr int Ns(int p) { return p == 0 ? 1 : Ns(p - 1) * R(p - 1); }
  static constexpr int tw_off(int p) { return p <= 1 ? 0 : tw_off(p - 1) + Ns(p - 1) * (R(p - 1) - 1); }
  using Reversed = SPlan<N_, W_, LD_, !REV_>;
};

// The inverse z plan of a forward plan: radices reversed.
template <class SP> struct InvPlan { using type = typename SP::Reversed; };
template <> struct InvPlan<DynPlan> { using type = DynPlan; };

// Element offsets inside one batch element's intermediate array: 32-bit with
// a compile-time plan (the launchers use those only when every offset fits),
// 64-bit otherwise.
template <class SP> using OffT = typename std::conditional<SP::is_static, unsigned, size_t>::type;

// Plan values a kernel needs, from the compile-time plan or the device copy.
template <class SP> __device__ __forceinline__ int plan_W(const FFTPlan* P) {
  if constexpr (SP::is_static) return SP::W;
  else return P->W;
}
template <class SP> __device__ __forceinline__ int plan_LD(const FFTPlan* P) {
  if constexpr (SP::is_static) return SP::LD;
  else return P->LD;
}
template <class SP> __device__ __forceinline__ int plan_N(const FFTPlan* P) {
  if constexpr (SP::is_static) return SP::N;
  else return P->N;
}
template <class SP> __device__ __forceinline__ int plan_npass(const FFTPlan* P) {
  if constexpr (SP::is_static) return SP::npass;
  else return P->npass;
}

// fft_pass with every plan value a constant.
// ZU: the transform's upper half inputs are zero (a zero-padded forward
// transform): inputs r >= R/2 of the first pass are not read.
// in(c, idx, slot): slot numbers the thread's inputs of the pass, k R + r
// (k (R / 2) + r with ZU), for callers that hold them in registers.
// TwP: pointer to the plan's twiddle table (global memory or an LDS copy).
template <typename T, bool INV, class SP, int p, bool SYNC, bool ZU, class TwP, class In, class Out, class Pre>
__device__ __forceinline__ void fft_pass_s(TwP twb, In in, Out out, Pre pre) {
  using C = typename Cplx<T>::type;
  constexpr int R = SP::R(p), Ns = SP::Ns(p), NR = SP::N / R, W = SP::W, logW = SP::logW;
  constexpr int TH = RegCfg<T>::THREADS, nbf = W * NR;
  constexpr int K = cmin((RegCfg<T>::EMAX + R - 1) / R, (nbf + TH - 1) / TH);
  constexpr bool guard = K * TH > nbf;
  const TwP tw = twb + SP::tw_off(p);
  C v[K * R];
  C w[K * (R - 1)];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int b = (int)threadIdx.x + k * TH;
    if (!guard || b < nbf) {
      const int c = b & (W - 1), j = b >> logW;
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[k * R + r] = (ZU && 2 * r >= R) ? C{0, 0} : in(c, j + r * NR, ZU ? k * (R / 2) + r : k * R + r);
      pre(std::integral_constant<int, R>{}, k, c, j);
      if constexpr (Ns > 1) {
        const TwP wt = tw + (j & (Ns - 1)) * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[k * (R - 1) + r - 1] = C{wt[r - 1].x, wt[r - 1].y};
      }
    }
  }
  if constexpr (SYNC) __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int b = (int)threadIdx.x + k * TH;
    if (!guard || b < nbf) {
      const int c = b & (W - 1), j = b >> logW;
      int base;
      if constexpr (Ns > 1) {
        const int t = j & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C wr = w[k * (R - 1) + r - 1];
          if (INV) wr.y = -wr.y;
          v[k * R + r] = cmul(v[k * R + r], wr);
        }
        base = (j - t) * R + t;
      } else {
        base = j * R;
      }
      dft<R, INV>(&v[k * R]);
      out(std::integral_constant<int, R>{}, c, j, base, Ns, &v[k * R], k);
    }
  }
}

template <typename T, bool INV, bool FIRST_LDS, class SP, int p, int p0, bool ZU>
struct RunStatic {
  template <class TwP, class FirstIn, class LastOut, class FirstPre, class LastPre>
  static __device__ __forceinline__ void go(typename Cplx<T>::type* lds, TwP tw,
                                            FirstIn& first_in, LastOut& last_out, FirstPre& first_pre,
                                            LastPre& last_pre) {
    using C = typename Cplx<T>::type;
    constexpr bool first = p == p0, last = p == SP::npass - 1;
    auto lds_in = [&](int c, int idx, int) { return lds[idx * SP::LD + c]; };
    auto lds_out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) lds[(base + r * Ns) * SP::LD + c] = vals[r];
    };
    const NoPre none;
    if constexpr (first && last) {
      auto both = [&](auto RC, int k, int c, int j) {
        first_pre(RC, k, c, j);
        last_pre(RC, k, c, j);
      };
      fft_pass_s<T, INV, SP, p, FIRST_LDS, ZU>(tw, first_in, last_out, both);
    } else if constexpr (first) {
      fft_pass_s<T, INV, SP, p, FIRST_LDS, ZU>(tw, first_in, lds_out, first_pre);
    } else if constexpr (last) {
      fft_pass_s<T, INV, SP, p, true, false>(tw, lds_in, last_out, last_pre);
    } else {
      fft_pass_s<T, INV, SP, p, true, false>(tw, lds_in, lds_out, none);
    }
    if constexpr (!last) {
      __syncthreads();
      RunStatic<T, INV, FIRST_LDS, SP, p + 1, p0, ZU>::go(lds, tw, first_in, last_out, first_pre, last_pre);
    }
  }
};

// Passes [P0, npass) with the compile-time plan SP, or with the device plan P.
// ZU (compile-time plans only): the first pass's upper-half inputs are zero.
template <typename T, bool INV, bool FIRST_LDS, class SP, int P0, bool ZU = false, class FirstIn, class LastOut,
          class LastPre = NoPre>
__device__ __forceinline__ void run_any(typename Cplx<T>::type* lds, const FFTPlan* __restrict__ P,
                                        FirstIn first_in, LastOut last_out, LastPre last_pre = LastPre{}) {
  if constexpr (SP::is_static) {
    NoPre none;
    RunStatic<T, INV, FIRST_LDS, SP, P0, P0, ZU>::go(lds, as_global<typename Cplx<T>::type>(P->tw), first_in, last_out,
                                                     none, last_pre);
  } else {
    run_fft<T, INV, FIRST_LDS>(lds, P, P0, first_in, last_out, last_pre);
  }
}

// Passes [P0, npass) of compile-time plan SP with its twiddle table at `tw`
// (for instance a copy in LDS, whose reads do not wait on vector memory).
template <typename T, bool INV, bool FIRST_LDS, class SP, int P0, bool ZU = false, class FirstIn, class LastOut,
          class LastPre = NoPre>
__device__ __forceinline__ void run_static_tw(typename Cplx<T>::type* lds, const typename Cplx<T>::type* tw,
                                              FirstIn first_in, LastOut last_out, LastPre last_pre = LastPre{}) {
  static_assert(SP::is_static, "compile-time plans only");
  NoPre none;
  RunStatic<T, INV, FIRST_LDS, SP, P0, P0, ZU>::go(lds, tw, first_in, last_out, none, last_pre);
}

// Complex twiddles in the table of compile-time plan SP.
template <class SP> constexpr int static_tw_count() { return SP::npass < 2 ? 0 : SP::tw_off(SP::npass); }

// ---------------------------------------------------------------------------
// Host helpers of the launchers
// ---------------------------------------------------------------------------
// ceil(2^32 / d): __umulhi(e, magic_of(d)) == e / d whenever e * d < 2^32.
static inline unsigned magic_of(int d) {
  return (unsigned)(((1ull << 32) + (unsigned long long)d - 1) / (unsigned long long)d);
}

template <typename T>
static inline size_t lds_bytes(const FFTPlan& P) {
  return (size_t)P.N * P.LD * sizeof(typename Cplx<T>::type);
}

template <class SP> static inline bool plan_matches(const FFTPlan& h) {
  if (h.N != SP::N || h.W != SP::W || h.LD != SP::LD || h.npass != SP::npass) return false;
  for (int p = 0; p < h.npass; ++p)
    if (h.R[p] != SP::R(p) || h.Ns[p] != SP::Ns(p) || h.tw_off[p] != SP::tw_off(p)) return false;
  return true;
}

}  // namespace dks

#endif  // DKS_FFT_ENGINE_H
