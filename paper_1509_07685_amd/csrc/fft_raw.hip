// Raw 3-D FFTs on device data (the FFT entry points of the paper's DKS usage
// example: data written to the device, a forward or inverse transform called
// on it, the result read back), on the same Stockham engine as the Poisson
// convolution: complex-to-complex forward and inverse, real-to-complex
// forward and complex-to-real inverse, every extent 2^a 3^b up to 4096,
// batched, unnormalised (inverse(forward(x)) = nx ny nz x).
//
// Layout: C-contiguous [batch][nz][ny][nx] (x fastest), interleaved complex.
// The real-to-complex transform keeps the nx/2 + 1 non-redundant x outputs
// per row ([batch][nz][ny][nx/2+1]); the complex-to-real inverse reads that
// layout.
//
// Passes: x is contiguous, so its tiles (W whole rows) are staged through LDS
// with linear, coalesced loads and stores.  y and z are strided: a tile is W
// adjacent x columns (128-byte row segments), its first radix pass reads
// straight from HBM and its last pass writes straight to HBM.  Every pass
// reads its whole tile before it writes any of it, so in-place transforms
// are safe.

#include <cstring>
#include <new>
#include <vector>

#include "dks_fft.h"
#include "fft_engine.h"
#include "fft_plan_check.h"

namespace dks {

template <typename T> hipError_t launch_twiddle_pass(void*, int, int, hipStream_t);
hipError_t launch_store_plans(const FFTPlan* four, FFTPlan* dev, hipStream_t s);

enum RowKind { kRowC2C = 0, kRowR2C = 1, kRowC2R = 2 };

// ---------------------------------------------------------------------------
// x: W rows per tile (row p of the tile holds element e at e / len, e mod len;
// the magic multipliers divide, len 1 aside).  kRowC2C: N complex in and out.  kRowR2C: N reals in
// (imaginary parts zero), the first N/2 + 1 outputs out.  kRowC2R: N/2 + 1
// complex in, completed to the full Hermitian row X[N - k] = conj X[k], the
// real parts of the inverse transform out.
// ---------------------------------------------------------------------------
template <typename T, class SP, bool INV, int KIND>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fftr_rows(const void* __restrict__ in,
                                                                 void* __restrict__ out, long long nrows,
                                                                 const FFTPlan* __restrict__ P, int in_len,
                                                                 int out_len, unsigned magic_in,
                                                                 unsigned magic_out) {
  using C = typename Cplx<T>::type;
  constexpr int TH = RegCfg<T>::THREADS;
  constexpr int KL = RegCfg<T>::EMAX;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int W = plan_W<SP>(P), LD = plan_LD<SP>(P), N = plan_N<SP>(P);
  const long long row0 = (long long)blockIdx.x * W;
  const int nvalid = (int)min((long long)W, nrows - row0);
  {
    const int total = nvalid * in_len;
    if constexpr (KIND == kRowR2C) {
      const T* src = static_cast<const T*>(in) + row0 * in_len;
      T v[KL];
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = (int)threadIdx.x + k * TH;
        v[k] = e < total ? src[e] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = (int)threadIdx.x + k * TH;
        if (e < total) {
          const int p = in_len == 1 ? e : (int)__umulhi((unsigned)e, magic_in);
          const int x = e - p * in_len;
          lds[x * LD + p] = C{v[k], (T)0};
        }
      }
    } else {
      const C* src = static_cast<const C*>(in) + row0 * in_len;
      C v[KL];
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = (int)threadIdx.x + k * TH;
        v[k] = e < total ? src[e] : C{0, 0};
      }
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = (int)threadIdx.x + k * TH;
        if (e < total) {
          const int p = in_len == 1 ? e : (int)__umulhi((unsigned)e, magic_in);
          const int x = e - p * in_len;
          lds[x * LD + p] = v[k];
          if constexpr (KIND == kRowC2R) {
            if (x >= 1 && N - x > x) lds[(N - x) * LD + p] = C{v[k].x, -v[k].y};
          }
        }
      }
    }
  }
  __syncthreads();
  {
    auto lin = [&](int c, int idx, int) { return lds[idx * LD + c]; };
    auto lout = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) lds[(base + r * Ns) * LD + c] = vals[r];
    };
    run_any<T, INV, true, SP, 0>(lds, P, lin, lout);
  }
  __syncthreads();
  const int total = nvalid * out_len;
  if constexpr (KIND == kRowC2R) {
    T* dst = static_cast<T*>(out) + row0 * out_len;
#pragma unroll 4
    for (int e = (int)threadIdx.x; e < total; e += TH) {
      const int p = out_len == 1 ? e : (int)__umulhi((unsigned)e, magic_out);
      const int x = e - p * out_len;
      dst[e] = lds[x * LD + p].x;
    }
  } else {
    C* dst = static_cast<C*>(out) + row0 * out_len;
#pragma unroll 4
    for (int e = (int)threadIdx.x; e < total; e += TH) {
      const int p = out_len == 1 ? e : (int)__umulhi((unsigned)e, magic_out);
      const int x = e - p * out_len;
      dst[e] = lds[x * LD + p];
    }
  }
}

// ---------------------------------------------------------------------------
// y or z: pencils of N elements S apart, W adjacent columns per tile.  Block
// b covers column tile b mod ntile of pencil group o = b / ntile, whose first
// element is (o / d1) s1 + (o mod d1) s2.
// ---------------------------------------------------------------------------
template <typename T, class SP, bool INV>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fftr_cols(const typename Cplx<T>::type* in,
                                                                 typename Cplx<T>::type* out, int ncols,
                                                                 int ntile, size_t S, int d1, size_t s1,
                                                                 size_t s2, const FFTPlan* __restrict__ P) {
  using C = typename Cplx<T>::type;
  using Off = OffT<SP>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int W = plan_W<SP>(P);
  const unsigned b = blockIdx.x;
  const unsigned o = b / (unsigned)ntile;
  const int tile = (int)(b - o * (unsigned)ntile);
  const unsigned o1 = o / (unsigned)d1, o2 = o - o1 * (unsigned)d1;
  const size_t base = (size_t)o1 * s1 + (size_t)o2 * s2 + (size_t)tile * W;
  const int ncol = min(W, ncols - tile * W);
  const C* src = in + base;
  C* dst = out + base;
  const Off st = (Off)S;
  auto rd = [&](int c, int idx, int) { return c < ncol ? src[(Off)idx * st + (Off)c] : C{0, 0}; };
  auto wr = [&](auto RC, int c, int, int bs, int Ns, C* vals, int) {
    if (c < ncol) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) dst[(Off)(bs + r * Ns) * st + (Off)c] = vals[r];
    }
  };
  run_any<T, INV, true, SP, 0>(lds, P, rd, wr);
}

// Tile width of an x (row) tile: the widest power of two <= w whose padded
// tile (N (W + 1) complex values) fits the LDS budget.
constexpr int row_width(int N, int c, int w) { return (w > 1 && N * (w + 1) * c > kLdsBytes) ? row_width(N, c, w / 2) : w; }

template <typename T, int N> using RowPlan =
    SPlan<N, row_width(N, 2 * (int)sizeof(T), 128 / (2 * (int)sizeof(T))),
          row_width(N, 2 * (int)sizeof(T), 128 / (2 * (int)sizeof(T))) + 1, false>;
template <typename T, int N> using ColPlan = SPlan<N, 128 / (2 * (int)sizeof(T)), 128 / (2 * (int)sizeof(T)), false>;

template <typename T, class F> static void with_row_plan(const FFTPlan& h, F&& f) {
  if (plan_matches<RowPlan<T, 512>>(h)) f(RowPlan<T, 512>{});
  else if (plan_matches<RowPlan<T, 256>>(h)) f(RowPlan<T, 256>{});
  else if (plan_matches<RowPlan<T, 128>>(h)) f(RowPlan<T, 128>{});
  else if (plan_matches<RowPlan<T, 64>>(h)) f(RowPlan<T, 64>{});
  else f(DynPlan{});
}

template <typename T, class F> static void with_col_plan(const FFTPlan& h, F&& f, bool off32) {
  if (!off32) f(DynPlan{});
  else if (plan_matches<ColPlan<T, 512>>(h)) f(ColPlan<T, 512>{});
  else if (plan_matches<ColPlan<T, 256>>(h)) f(ColPlan<T, 256>{});
  else if (plan_matches<ColPlan<T, 128>>(h)) f(ColPlan<T, 128>{});
  else if (plan_matches<ColPlan<T, 64>>(h)) f(ColPlan<T, 64>{});
  else f(DynPlan{});
}

template <typename T, bool INV, int KIND>
static hipError_t launch_rows(const void* in, void* out, long long nrows, const PlanRef& P, int in_len, int out_len,
                              hipStream_t s) {
  const long long nblk = (nrows + P.host.W - 1) / P.host.W;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  with_row_plan<T>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fftr_rows<T, decltype(sp), INV, KIND>), dim3((unsigned)nblk), dim3(RegCfg<T>::THREADS),
                       lds_bytes<T>(P.host), s, in, out, nrows, P.dev, in_len, out_len, magic_of(in_len),
                       magic_of(out_len));
  });
  return hipGetLastError();
}

template <typename T, bool INV>
static hipError_t launch_cols(const void* in, void* out, int ncols, size_t S, int nouter, int d1, size_t s1,
                              size_t s2, size_t elems, const PlanRef& P, hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int ntile = (ncols + P.host.W - 1) / P.host.W;
  const long long nblk = (long long)ntile * nouter;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  // 32-bit offsets inside a pencil tile when the whole array is addressable with them
  const bool off32 = elems < 0x7fffffffULL;
  with_col_plan<T>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fftr_cols<T, decltype(sp), INV>), dim3((unsigned)nblk), dim3(RegCfg<T>::THREADS),
                       lds_bytes<T>(P.host), s, (const C*)in, (C*)out, ncols, ntile, S, d1, s1, s2, P.dev);
  }, off32);
  return hipGetLastError();
}

}  // namespace dks

using namespace dks;

// A raw FFT plan: three axis plans (x rows, y and z columns), their twiddle
// tables and device copies in the caller's workspace, plus the complex
// scratch of the complex-to-real inverse.
struct dks_fft_plan_s {
  int n[3];
  int batch;
  dks_fft_kind kind;
  dks_dtype dtype;
  size_t csize;
  FFTPlanHost pl[3];
  size_t off_plans, off_tw[3], off_tmp, tmp_bytes, ws_total;
  char* ws;
  size_t ws_bytes;
  bool prepared;
};

namespace {

inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

bool is_23(int N) {
  if (N < 1) return false;
  while (N % 2 == 0) N /= 2;
  while (N % 3 == 0) N /= 3;
  return N == 1;
}

std::vector<int> radix_order(int N) {
  int a = 0, b = 0;
  while (N % 2 == 0) { N /= 2; ++a; }
  while (N % 3 == 0) { N /= 3; ++b; }
  std::vector<int> r;
  while (a >= 3) { r.push_back(8); a -= 3; }
  if (a == 2) r.push_back(4);
  if (a == 1) r.push_back(2);
  for (int i = 0; i < b; ++i) r.push_back(3);
  return r;
}

void make_axis(FFTPlanHost& P, int N, int W, int LD) {
  std::memset(&P, 0, sizeof(P));
  const std::vector<int> R = radix_order(N);
  P.dev.N = N;
  P.dev.npass = (int)R.size();
  P.dev.W = W;
  int lw = 0;
  while ((1 << lw) < W) ++lw;
  P.dev.logW = lw;
  P.dev.LD = LD;
  int Ns = 1, off = 0;
  for (size_t p = 0; p < R.size(); ++p) {
    P.dev.R[p] = R[p];
    P.dev.Ns[p] = Ns;
    P.dev.magic[p] = Ns >= 2 ? (unsigned)(((1ull << 32) + (unsigned long long)Ns - 1) / (unsigned long long)Ns) : 0u;
    P.dev.tw_off[p] = off;
    if (p > 0) off += Ns * (R[p] - 1);
    Ns *= R[p];
  }
  P.tw_count = off;
}

size_t row_len_complex(const dks_fft_plan_s* p) { return p->kind == DKS_FFT_R2C ? (size_t)(p->n[0] / 2 + 1) : (size_t)p->n[0]; }

PlanRef axis_ref(const dks_fft_plan_s* p, int a) {
  PlanRef r;
  r.host = p->pl[a].dev;
  r.host.tw = p->ws + p->off_tw[a];
  r.dev = reinterpret_cast<const FFTPlan*>(p->ws + p->off_plans) + a;
  return r;
}

// y then z column passes on the complex array `cur` (in place), or from
// `src` into `cur` for the first pass that runs.
template <typename T, bool INV>
dks_status run_cols(const dks_fft_plan_s* p, const void* src, void* cur, hipStream_t st) {
  const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const size_t L = row_len_complex(p);
  const size_t elems = L * ny * nz * p->batch;
  const void* from = src;
  if (ny > 1) {
    if (launch_cols<T, INV>(from, cur, (int)L, L, nz * p->batch, 1, L * ny, 0, elems, axis_ref(p, 1), st) !=
        hipSuccess)
      return DKS_EHIP;
    from = cur;
  }
  if (nz > 1) {
    if (launch_cols<T, INV>(from, cur, (int)L, L * ny, ny * p->batch, ny, L * ny * nz, L, elems, axis_ref(p, 2),
                            st) != hipSuccess)
      return DKS_EHIP;
    from = cur;
  }
  (void)nx;
  if (from != cur) {   // no column pass ran: move the data
    if (hipMemcpyAsync(cur, src, elems * p->csize, hipMemcpyDeviceToDevice, st) != hipSuccess) return DKS_EHIP;
  }
  return DKS_OK;
}

template <typename T>
dks_status execute(const dks_fft_plan_s* p, const void* in, void* out, bool inverse, hipStream_t st) {
  const long long rows = (long long)p->n[1] * p->n[2] * p->batch;
  const int nx = p->n[0];
  const int nh = nx / 2 + 1;
  if (p->kind == DKS_FFT_C2C) {
    const hipError_t e = inverse ? launch_rows<T, true, kRowC2C>(in, out, rows, axis_ref(p, 0), nx, nx, st)
                                 : launch_rows<T, false, kRowC2C>(in, out, rows, axis_ref(p, 0), nx, nx, st);
    if (e != hipSuccess) return DKS_EHIP;
    return inverse ? run_cols<T, true>(p, out, out, st) : run_cols<T, false>(p, out, out, st);
  }
  if (!inverse) {
    if (launch_rows<T, false, kRowR2C>(in, out, rows, axis_ref(p, 0), nx, nh, st) != hipSuccess) return DKS_EHIP;
    return run_cols<T, false>(p, out, out, st);
  }
  // complex-to-real: columns from the input into the scratch, then the rows
  const bool cols = p->n[1] > 1 || p->n[2] > 1;
  const void* rows_in = in;
  if (cols) {
    char* tmp = p->ws + p->off_tmp;
    const dks_status r = run_cols<T, true>(p, in, tmp, st);
    if (r != DKS_OK) return r;
    rows_in = tmp;
  }
  return launch_rows<T, true, kRowC2R>(rows_in, out, rows, axis_ref(p, 0), nh, nx, st) == hipSuccess ? DKS_OK
                                                                                                   : DKS_EHIP;
}

}  // namespace

extern "C" {

dks_status dks_fft_plan(int nx, int ny, int nz, int batch, dks_fft_kind kind, dks_dtype dtype,
                        dks_fft_plan_t* out) {
  if (!out) return DKS_EINVAL;
  *out = nullptr;
  if (dtype != DKS_F32 && dtype != DKS_F64) return DKS_EINVAL;
  if (kind != DKS_FFT_C2C && kind != DKS_FFT_R2C) return DKS_EINVAL;
  if (batch < 1 || nx < 1 || ny < 1 || nz < 1) return DKS_EINVAL;
  const int ns[3] = {nx, ny, nz};
  for (int n : ns)
    if (n > kMaxLength || !is_23(n)) return DKS_EUNSUPPORTED;
  // every pass's workgroup count must fit a 1-D grid (checked again at launch)
  if ((double)ny * nz * batch > 2147483647.0) return DKS_EINVAL;
  dks_fft_plan_s* p = new (std::nothrow) dks_fft_plan_s;
  if (!p) return DKS_ENOMEM;
  std::memset(p, 0, sizeof(*p));
  p->n[0] = nx;
  p->n[1] = ny;
  p->n[2] = nz;
  p->batch = batch;
  p->kind = kind;
  p->dtype = dtype;
  p->csize = dtype == DKS_F32 ? 8 : 16;
  const int c = (int)p->csize;
  const int wmax = 128 / c;
  // x: padded row tiles (unpadded single rows when even one padded row does not fit)
  const int Wx = row_width(nx, c, wmax);
  const bool padded = (size_t)nx * (Wx + 1) * c <= (size_t)kLdsBytes;
  make_axis(p->pl[0], nx, Wx, padded ? Wx + 1 : Wx);
  for (int a = 1; a < 3; ++a) {
    int W = wmax;
    while (W > 1 && (size_t)ns[a] * W * c > (size_t)kLdsBytes) W >>= 1;
    make_axis(p->pl[a], ns[a], W, W);
  }
  size_t off = 0;
  p->off_plans = off;
  off = al256(off + 4 * sizeof(FFTPlan));
  for (int a = 0; a < 3; ++a) {
    p->off_tw[a] = off;
    off = al256(off + (size_t)p->pl[a].tw_count * p->csize + 16);
  }
  // the pass kernels' invariants: rows staged through EMAX registers per
  // thread (N values per row at most), columns read straight from memory
  {
    EngineLimits L;
    L.threads = dtype == DKS_F32 ? RegCfg<float>::THREADS : RegCfg<double>::THREADS;
    L.emax = dtype == DKS_F32 ? RegCfg<float>::EMAX : RegCfg<double>::EMAX;
    L.max_length = kMaxLength;
    L.max_pass = kMaxPass;
    L.lds_hw = kLdsHardware;
    int v = fft_plan_violation(p->pl[0].dev, L, p->csize, nx, L.emax, 0);
    for (int a = 1; a < 3 && v == kPlanOk; ++a) v = fft_plan_violation(p->pl[a].dev, L, p->csize, 0, 0, 0);
    if (v != kPlanOk) {
      delete p;
      return DKS_EUNSUPPORTED;
    }
  }
  p->off_tmp = off;
  p->tmp_bytes = kind == DKS_FFT_R2C ? al256((size_t)(nx / 2 + 1) * ny * nz * batch * p->csize) : 0;
  p->ws_total = p->off_tmp + p->tmp_bytes;
  *out = p;
  return DKS_OK;
}

dks_status dks_fft_workspace_bytes(dks_fft_plan_t p, size_t* bytes) {
  if (!p || !bytes) return DKS_EINVAL;
  *bytes = p->ws_total;
  return DKS_OK;
}

dks_status dks_fft_set_workspace(dks_fft_plan_t p, void* ws, size_t bytes) {
  if (!p) return DKS_EINVAL;
  if (!ws || bytes < p->ws_total || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DKS_EWORKSPACE;
  p->ws = static_cast<char*>(ws);
  p->ws_bytes = bytes;
  p->prepared = false;
  return DKS_OK;
}

dks_status dks_fft_prepare(dks_fft_plan_t p, dks_stream_t stream) {
  if (!p) return DKS_EINVAL;
  if (!p->ws) return DKS_EWORKSPACE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  for (int a = 0; a < 3; ++a) {
    const FFTPlan& f = p->pl[a].dev;
    for (int q = 1; q < f.npass; ++q) {
      void* dst = p->ws + p->off_tw[a] + (size_t)f.tw_off[q] * p->csize;
      const hipError_t e = p->dtype == DKS_F32 ? launch_twiddle_pass<float>(dst, f.Ns[q], f.R[q], st)
                                               : launch_twiddle_pass<double>(dst, f.Ns[q], f.R[q], st);
      if (e != hipSuccess) return DKS_EHIP;
    }
  }
  FFTPlan four[4];
  for (int a = 0; a < 3; ++a) four[a] = axis_ref(p, a).host;
  four[3] = four[2];
  if (launch_store_plans(four, reinterpret_cast<FFTPlan*>(p->ws + p->off_plans), st) != hipSuccess) return DKS_EHIP;
  p->prepared = true;
  return DKS_OK;
}

static dks_status fft_exec(dks_fft_plan_t p, const void* in, void* out, bool inverse, dks_stream_t stream) {
  if (!p || !in || !out) return DKS_EINVAL;
  if (p->kind == DKS_FFT_R2C && in == out) return DKS_EINVAL;
  if (!p->ws) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  return p->dtype == DKS_F32 ? execute<float>(p, in, out, inverse, st) : execute<double>(p, in, out, inverse, st);
}

dks_status dks_fft_forward(dks_fft_plan_t p, const void* in, void* out, dks_stream_t stream) {
  return fft_exec(p, in, out, false, stream);
}

dks_status dks_fft_inverse(dks_fft_plan_t p, const void* in, void* out, dks_stream_t stream) {
  return fft_exec(p, in, out, true, stream);
}

dks_status dks_fft_destroy(dks_fft_plan_t p) {
  if (!p) return DKS_EINVAL;
  delete p;
  return DKS_OK;
}

}  // extern "C"
