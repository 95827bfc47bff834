// Pruned 3-D real-to-complex / complex-to-real FFT passes of the doubled-grid
// convolution (Hockney's open-boundary method, section "FFT Based
// Particle-Mesh Solver": phi = FT^-1{FT{rho} (Hadamard) FT{G}}, the Green's
// multiply fused between the forward and inverse z transforms).
//
// Every pass works on a tile of W pencils held in LDS as [element][pencil]
// (pencil index fastest).  A mixed-radix Stockham transform (radices 8, 4, 2,
// 3) runs over the tile: each pass loads its butterfly inputs from LDS into
// registers, synchronises, applies twiddles and the radix-R DFT and writes
// the outputs back in Stockham order.  The first pass of a transform can take
// its inputs straight from HBM (the y and z passes) and the last pass can
// hand its outputs straight to HBM, so a transform of P passes costs P - 1
// LDS round trips.  Lanes are mapped pencil-fastest so that a wavefront's 64
// lanes read and write W contiguous complex values per row: 128-byte HBM
// segments and conflict-free LDS rows.
//
// The two intermediates the z pass reads and writes (B after the y forward
// pass, C after the z pass) are z-blocked: element (z, ky, kx) sits in row
// ((z / 16) * 2ny + ky) * 16 + z % 16, so a z pencil spans 16-17 blocks of
// 16 adjacent rows instead of one row per plane, and a y pencil of one plane
// steps by 16 rows.
//
// Zero padding is never stored: the forward x transform reads the nx real
// values of a row, the forward y and z transforms read only the first half of
// their pencils, and the inverse transforms store only the outputs in
// [-1, n] per axis (the physical mesh plus one ghost node on each side).

#include "fft_engine.h"

namespace dks {

// ---------------------------------------------------------------------------
// x forward: real rows of nx values (zero-padded to 2 nx) -> nx + 1 complex.
// A length-2nx real transform is done as a length-nx complex transform of
// z[m] = x[2m] + i x[2m+1], then X[k] = (Z[k] + conj Z[nx-k]) / 2
// - i w^k (Z[k] - conj Z[nx-k]) / 2 with w = exp(-2 pi i / 2nx).
// ---------------------------------------------------------------------------
template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fft_x_fwd(const T* __restrict__ in, size_t in_stride,
                                                        typename Cplx<T>::type* __restrict__ out,
                                                        size_t out_stride, MeshDims m, const FFTPlan* __restrict__ P,
                                                        const typename Cplx<T>::type* __restrict__ post,
                                                        int nrows, unsigned magic_out, unsigned magic_nx) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const T* src = in + blockIdx.y * in_stride;
  C* dst = out + blockIdx.y * out_stride;
  const int Wt = plan_W<SP>(P), LDt = plan_LD<SP>(P);
  const int row0 = blockIdx.x * Wt;
  const int nvalid = min(Wt, nrows - row0);
  const int nx = m.nx, M = plan_N<SP>(P);
  {
    // The tile's rows are contiguous (nvalid * nx reals, at most kTileReals per
    // thread): every load of the thread is issued before the first LDS store.
    constexpr int TH = RegCfg<T>::THREADS;
    constexpr int KL = kTileReals;
    const T* tsrc = src + (size_t)row0 * nx;
    const int total = nvalid * nx;
    T v[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int e = (int)threadIdx.x + k * TH;
      v[k] = e < total ? tsrc[e] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int e = (int)threadIdx.x + k * TH;
      if (e < total) {
        const int p = (int)__umulhi((unsigned)e, magic_nx);
        const int x = e - p * nx;
        T* slot = reinterpret_cast<T*>(&lds[(x >> 1) * LDt + p]);
        slot[x & 1] = v[k];
        if ((x & 1) == 0 && x == nx - 1) slot[1] = (T)0;
      }
    }
  }
  // The nx + 1 post-twiddles go to LDS after the tile, so that the output
  // loop below has no global loads: a load there would make every iteration
  // wait for the previous iteration's store.
  C* lpost = lds + (size_t)M * LDt;
  for (int k = (int)threadIdx.x; k <= nx; k += RegCfg<T>::THREADS) lpost[k] = post[k];
  __syncthreads();
  {
    const int nnz = (nx + 1) >> 1;
    const int LD = LDt;
    auto in = [&](int c, int idx, int) { return idx < nnz ? lds[idx * LD + c] : C{0, 0}; };
    auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) lds[(base + r * Ns) * LD + c] = vals[r];
    };
    run_any<T, false, true, SP, 0, true>(lds, P, in, out);
  }
  __syncthreads();
  // outputs flattened over (row, column) so every lane has work: a row holds
  // nx + 1 values, which a row-per-lane-group split would leave ragged
  const int ncols = nx + 1;
  const int total = nvalid * ncols;
  for (int e = (int)threadIdx.x; e < total; e += RegCfg<T>::THREADS) {
    const int p = (int)__umulhi((unsigned)e, magic_out);
    const int k = e - p * ncols;
    const C zk = lds[(k == M ? 0 : k) * LDt + p];
    C zc = lds[(k == 0 ? 0 : M - k) * LDt + p];
    zc.y = -zc.y;
    const C s = cadd(zk, zc), d = csub(zk, zc);
    const C wd = cmul(lpost[k], d);
    dst[(size_t)(row0 + p) * m.cs + k] = C{(T)0.5 * (s.x + wd.y), (T)0.5 * (s.y - wd.x)};
  }
}

// ---------------------------------------------------------------------------
// y forward: pencils along y of the x-transformed rows.  Input A[z][y][kx]
// (y < ny), output B[z][ky][kx] (ky < 2 ny).  Grid: (column tiles, nz, batch).
// ---------------------------------------------------------------------------
template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fft_y_fwd(const typename Cplx<T>::type* __restrict__ A,
                                                        typename Cplx<T>::type* __restrict__ B,
                                                        size_t stride, MeshDims m, const FFTPlan* __restrict__ P) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int c0 = blockIdx.x * plan_W<SP>(P);
  const int ncol = min(plan_W<SP>(P), m.ncols - c0);
  const int z = blockIdx.y;
  const C* src = A + blockIdx.z * stride + (size_t)z * m.ny * m.cs + c0;
  C* dst = B + blockIdx.z * stride + ((size_t)(z >> 4) * m.Ny * 16 + (z & 15)) * m.cs + c0;
  const int ny = m.ny, cs = m.cs;
  const size_t ostep = (size_t)16 * cs;       // next ky row of this plane
  using Off = OffT<SP>;
  auto in = [&](int c, int idx, int) { return (idx < ny && c < ncol) ? src[(Off)idx * (Off)cs + (Off)c] : C{0, 0}; };
  auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
    if (c < ncol) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) dst[(Off)(base + r * Ns) * (Off)ostep + (Off)c] = vals[r];
    }
  };
  run_any<T, false, false, SP, 0, true>(lds, P, in, out);
}

// ---------------------------------------------------------------------------
// z: forward transform of each (kx, ky) pencil over its nz non-zero inputs,
// multiply by the real Green's spectrum times the solve's scale, inverse
// transform, keep z in [-1, nz].  Input B[z][ky][kx] (z < nz), output
// C[z + 1][ky][kx] for z in [-1, nz].  The inverse plan's radices are the
// forward's reversed, so the last forward pass and the first inverse pass
// share a butterfly layout and the multiply happens in registers between them.
//
// Rows ky and Ny - ky read the same Green's block (the spectrum is even in
// ky).  The 1-D grid (per batch element) is ordered so that the two
// workgroups of a pair are 8 apart: L = 16 A + 8 m + r, pair-tile index
// 8 A + r, member m.  Round-robin dispatch puts both on one XCD, one round
// apart, so the second finds the block in that XCD's L2.
// ---------------------------------------------------------------------------
template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fft_z_conv(
    const typename Cplx<T>::type* __restrict__ B, typename Cplx<T>::type* __restrict__ Cout,
    size_t stride, const T* __restrict__ G, const Geometry* __restrict__ geo, size_t geo_stride,
    MeshDims m, const FFTPlan* __restrict__ Pf, const FFTPlan* __restrict__ Pi) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int W = plan_W<SP>(Pf);
  const int ntile = (m.ncols + W - 1) / W;
  const unsigned L = blockIdx.x;
  const int pt = (int)(((L >> 4) << 3) | (L & 7u));    // pair-tile index
  const int pair = pt / ntile, tile = pt - pair * ntile;
  if (pair > m.Ny / 2) return;
  const bool second = (L >> 3) & 1u;
  if (second && (pair == 0 || 2 * pair == m.Ny)) return;   // rows 0 and Ny/2 pair with themselves
  const int ky = second ? m.Ny - pair : pair;
  const int c0 = tile * W;
  const int ncol = min(W, m.ncols - c0);
  const size_t zblock = (size_t)m.Ny * 16 * m.cs;   // one block of 16 z rows of B or C
  const C* src = B + blockIdx.y * stride + (size_t)ky * 16 * m.cs + c0;
  C* dst = Cout + blockIdx.y * stride + (size_t)ky * 16 * m.cs + c0;
  const Geometry* g = reinterpret_cast<const Geometry*>(reinterpret_cast<const char*>(geo) +
                                                        blockIdx.y * geo_stride);
  const T scale = Geo<T>::scale(g);
  const T* gblk = G + ((size_t)pair * (m.cs / W) + tile) * (m.nz + 1) * W;   // [kz][W]
  const int nz = m.nz, Nz = m.Nz, cs = m.cs, LD = plan_LD<SP>(Pf);
  using Off = OffT<SP>;
  auto zoff = [&](int z) { return (Off)(z >> 4) * (Off)zblock + (Off)(z & 15) * (Off)cs; };
  auto in = [&](int c, int idx, int) { return (idx < nz && c < ncol) ? src[zoff(idx) + (Off)c] : C{0, 0}; };
  // Final inverse outputs: keep z = -1 (index Nz - 1) and z = 0 .. nz as row z + 1.
  auto store_z = [&](int c, int idx, C val) {
    int zo = -1;
    if (idx <= nz) zo = idx + 1;
    else if (idx == Nz - 1) zo = 0;
    if (zo >= 0 && c < ncol) dst[zoff(zo) + (Off)c] = val;
  };
  using SPi = typename InvPlan<SP>::type;
  const bool inv_single = plan_npass<SPi>(Pi) == 1;
  // Last forward pass: its outputs sit at kz = j + r Ns, exactly the inputs of
  // the first inverse butterfly j (radix R, span 1, no twiddles).
  // The Green's values of each butterfly are requested with the last forward
  // pass's inputs (before its barrier); that pass writes kz = j + r * Nz / R.
  T gpre[RegCfg<T>::ARR];
  auto gload = [&](auto RC, int k, int c, int j) {
    constexpr int R = RC.value;
    const int span = Nz / R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int kz = j + r * span;
      const int kzr = min(kz, Nz - kz);
      gpre[k * R + r] = (c < ncol) ? gblk[kzr * W + c] : (T)0;
    }
  };
  auto mid = [&](auto RC, int c, int j, int, int, C* vals, int k) {
    constexpr int R = RC.value;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T gv = gpre[k * R + r] * scale;
      vals[r].x *= gv;
      vals[r].y *= gv;
    }
    dft<R, true>(vals);
    if (inv_single) {
#pragma unroll
      for (int r = 0; r < R; ++r) store_z(c, j * R + r, vals[r]);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(j * R + r) * LD + c] = vals[r];
    }
  };
  run_any<T, false, false, SP, 0, true>(lds, Pf, in, mid, gload);
  if (!inv_single) {
    __syncthreads();
    auto lds_in = [&](int c, int idx, int) { return lds[idx * LD + c]; };
    auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) store_z(c, base + r * Ns, vals[r]);
    };
    run_any<T, true, true, SPi, 1>(lds, Pi, lds_in, out);
  }
}

// ---------------------------------------------------------------------------
// y inverse: C[z'][ky][kx] -> D[z'][y + 1][kx] for y in [-1, ny].
// Grid: (column tiles, nz + 2, batch).
// ---------------------------------------------------------------------------
template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fft_y_inv(const typename Cplx<T>::type* __restrict__ Cin,
                                                        typename Cplx<T>::type* __restrict__ D,
                                                        size_t stride, MeshDims m, const FFTPlan* __restrict__ P) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int c0 = blockIdx.x * plan_W<SP>(P);
  const int ncol = min(plan_W<SP>(P), m.ncols - c0);
  const int zp = blockIdx.y;
  const C* src = Cin + blockIdx.z * stride + ((size_t)(zp >> 4) * m.Ny * 16 + (zp & 15)) * m.cs + c0;
  C* dst = D + blockIdx.z * stride + (size_t)zp * (m.ny + 2) * m.cs + c0;
  const int ny = m.ny, Ny = m.Ny, cs = m.cs;
  const size_t istep = (size_t)16 * cs;       // next ky row of this plane
  using Off = OffT<SP>;
  auto in = [&](int c, int idx, int) { return c < ncol ? src[(Off)idx * (Off)istep + (Off)c] : C{0, 0}; };
  auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
    for (int r = 0; r < RC.value; ++r) {
      const int idx = base + r * Ns;
      int yo = -1;
      if (idx <= ny) yo = idx + 1;
      else if (idx == Ny - 1) yo = 0;
      if (yo >= 0 && c < ncol) dst[(Off)yo * (Off)cs + (Off)c] = vals[r];
    }
  };
  run_any<T, true, false, SP, 0>(lds, P, in, out);
}

// ---------------------------------------------------------------------------
// x inverse: rows of nx + 1 complex (half spectrum of a real length-2nx row)
// -> real values at x in [-1, nx] (row of nx + 2, ghost nodes included).
// Z'[k] = (X[k] + conj X[nx-k]) + i w^-k (X[k] - conj X[nx-k]); the length-nx
// inverse transform of Z' gives 2nx * (x[2m] + i x[2m+1]) unnormalised; the
// normalisation is folded into the Green's spectrum.  Optionally also writes
// the physical part of phi to a [nz][ny][nx] array.
// ---------------------------------------------------------------------------
template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fft_x_inv(const typename Cplx<T>::type* __restrict__ D,
                                                        size_t in_stride, T* __restrict__ phi_ext,
                                                        size_t out_stride, ElemBatch phi_user,
                                                        MeshDims m, const FFTPlan* __restrict__ P,
                                                        const typename Cplx<T>::type* __restrict__ post,
                                                        int nrows, unsigned magic_out, unsigned magic_m) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const C* src = D + blockIdx.y * in_stride;
  T* dst = phi_ext + blockIdx.y * out_stride;
  T* user = reinterpret_cast<T*>(phi_user.at(blockIdx.y).phi);
  const int Wt = plan_W<SP>(P), LDt = plan_LD<SP>(P);
  const int row0 = blockIdx.x * Wt;
  const int nvalid = min(Wt, nrows - row0);
  const int nx = m.nx, M = plan_N<SP>(P);
  {
    // nvalid * M elements (at most kTileReals per thread), in two halves whose
    // loads are all issued before they are used.
    constexpr int TH = RegCfg<T>::THREADS;
    constexpr int KH = kTileReals / 2;
    const int total = nvalid * M;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      C xk[KH], xc[KH], w[KH];
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int e = (int)threadIdx.x + (h * KH + k) * TH;
        if (e < total) {
          const int p = (int)__umulhi((unsigned)e, magic_m);
          const int kk = e - p * M;
          const C* row = src + (size_t)(row0 + p) * m.cs;
          xk[k] = row[kk];
          xc[k] = row[M - kk];
          w[k] = post[kk];
        }
      }
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int e = (int)threadIdx.x + (h * KH + k) * TH;
        if (e < total) {
          const int p = (int)__umulhi((unsigned)e, magic_m);
          const int kk = e - p * M;
          C c = xc[k];
          c.y = -c.y;
          const C s = cadd(xk[k], c), d = csub(xk[k], c);
          C ww = w[k];
          ww.y = -ww.y;
          const C wd = cmul(ww, d);
          lds[kk * LDt + p] = C{s.x - wd.y, s.y + wd.x};
        }
      }
    }
  }
  __syncthreads();
  {
    const int LD = LDt;
    auto in = [&](int c, int idx, int) { return lds[idx * LD + c]; };
    auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) lds[(base + r * Ns) * LD + c] = vals[r];
    };
    run_any<T, true, true, SP, 0>(lds, P, in, out);
  }
  __syncthreads();
  // outputs flattened over (row, column) so every lane has work (rows of
  // nx + 2 values)
  const int nout = nx + 2;
  const int ny2 = m.ny + 2;
  const int total = nvalid * nout;
  for (int e = (int)threadIdx.x; e < total; e += RegCfg<T>::THREADS) {
    const int p = (int)__umulhi((unsigned)e, magic_out);
    const int xo = e - p * nout;
    const int r = row0 + p;          // row index z' * (ny + 2) + y'
    const int x = xo - 1;
    T val;
    if (x < 0) {
      val = lds[(M - 1) * LDt + p].y;
    } else {
      const C zv = lds[(x >> 1) * LDt + p];
      val = (x & 1) ? zv.y : zv.x;
    }
    dst[(size_t)r * nout + xo] = val;
    if (user && xo >= 1 && xo <= nx) {
      const int zp = r / ny2, yp = r - zp * ny2;
      if (zp >= 1 && zp <= m.nz && yp >= 1 && yp <= m.ny) user[((size_t)(zp - 1) * m.ny + (yp - 1)) * nx + xo - 1] = val;
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
// Every element offset the y and z passes form inside one batch element's
// intermediate arrays stays below (nz + 16) * Ny * cs.
static inline bool offsets_fit32(const MeshDims& m) {
  return (double)(m.nz + 16) * (double)m.Ny * (double)m.cs < 2147483648.0;
}

// Calls f with the compile-time plan equal to host plan h (tile width of 128
// bytes, LD = W + PAD), or with DynPlan when none is or when the kernel's
// element offsets may not fit 32 bits (!off32).
template <typename T, int PAD, class F> static void with_plan(const FFTPlan& h, F&& f, bool off32 = true) {
  constexpr int W = 128 / (2 * (int)sizeof(T));
  if (!off32) f(DynPlan{});
  else if (plan_matches<SPlan<512, W, W + PAD, false>>(h)) f(SPlan<512, W, W + PAD, false>{});
  else if (plan_matches<SPlan<256, W, W + PAD, false>>(h)) f(SPlan<256, W, W + PAD, false>{});
  else if (plan_matches<SPlan<128, W, W + PAD, false>>(h)) f(SPlan<128, W, W + PAD, false>{});
  else if (plan_matches<SPlan<64, W, W + PAD, false>>(h)) f(SPlan<64, W, W + PAD, false>{});
  else f(DynPlan{});
}

template <typename T>
hipError_t launch_fft_x_fwd(const void* in, size_t in_stride, void* out, size_t out_stride, const MeshDims& m,
                            const PlanRef& P, const void* post, int batch, hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int nrows = m.ny * m.nz;
  if ((size_t)P.host.W * m.nx > (size_t)kTileReals * RegCfg<T>::THREADS) return hipErrorInvalidValue;
  dim3 grid((nrows + P.host.W - 1) / P.host.W, batch);
  with_plan<T, 1>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fft_x_fwd<T, decltype(sp)>), grid, dim3(RegCfg<T>::THREADS),
                       lds_bytes<T>(P.host) + (size_t)(m.nx + 1) * sizeof(C), s,
                       (const T*)in, in_stride, (C*)out, out_stride, m, P.dev, (const C*)post, nrows, magic_of(m.nx + 1),
                       magic_of(m.nx));
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y_fwd(const void* A, void* B, size_t stride, const MeshDims& m, const PlanRef& P, int batch,
                            hipStream_t s) {
  using C = typename Cplx<T>::type;
  dim3 grid((m.ncols + P.host.W - 1) / P.host.W, m.nz, batch);
  with_plan<T, 0>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fft_y_fwd<T, decltype(sp)>), grid, dim3(RegCfg<T>::THREADS), lds_bytes<T>(P.host), s,
                       (const C*)A, (C*)B, stride, m, P.dev);
  }, offsets_fit32(m));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_z_conv(const void* B, void* Cout, size_t stride, const void* G, const Geometry* geo,
                             size_t geo_stride, const MeshDims& m, const PlanRef& Pf, const PlanRef& Pi, int batch,
                             hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int ntile = (m.ncols + Pf.host.W - 1) / Pf.host.W;
  const int npt = (m.Ny / 2 + 1) * ntile;                 // pair-tile indices
  dim3 grid((unsigned)((npt + 7) / 8 * 16), batch);
  with_plan<T, 0>(Pf.host, [&](auto sp) {
    using SP = decltype(sp);
    auto launch = [&](auto spl) {
      hipLaunchKernelGGL((k_fft_z_conv<T, decltype(spl)>), grid, dim3(RegCfg<T>::THREADS), lds_bytes<T>(Pf.host), s,
                         (const C*)B, (C*)Cout, stride, (const T*)G, geo, geo_stride, m, Pf.dev, Pi.dev);
    };
    if constexpr (SP::is_static) {
      if (plan_matches<typename SP::Reversed>(Pi.host)) launch(SP{});
      else launch(DynPlan{});
    } else {
      launch(DynPlan{});
    }
  }, offsets_fit32(m));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y_inv(const void* Cin, void* D, size_t stride, const MeshDims& m, const PlanRef& P, int batch,
                            hipStream_t s) {
  using C = typename Cplx<T>::type;
  dim3 grid((m.ncols + P.host.W - 1) / P.host.W, m.nz + 2, batch);
  with_plan<T, 0>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fft_y_inv<T, decltype(sp)>), grid, dim3(RegCfg<T>::THREADS), lds_bytes<T>(P.host), s,
                       (const C*)Cin, (C*)D, stride, m, P.dev);
  }, offsets_fit32(m));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_x_inv(const void* D, size_t in_stride, void* phi_ext, size_t out_stride,
                            const ElemBatch& phi_user, const MeshDims& m, const PlanRef& P, const void* post,
                            int batch, hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int nrows = (m.ny + 2) * (m.nz + 2);
  if ((size_t)P.host.W * P.host.N > (size_t)kTileReals * RegCfg<T>::THREADS) return hipErrorInvalidValue;
  dim3 grid((nrows + P.host.W - 1) / P.host.W, batch);
  with_plan<T, 1>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fft_x_inv<T, decltype(sp)>), grid, dim3(RegCfg<T>::THREADS), lds_bytes<T>(P.host), s,
                       (const C*)D, in_stride, (T*)phi_ext, out_stride, phi_user, m, P.dev, (const C*)post, nrows,
                       magic_of(m.nx + 2), magic_of(P.host.N));
  });
  return hipGetLastError();
}

// Copies the host-built plans into device memory (kernel arguments are
// copied at launch, so this is safe inside stream capture).
__global__ void k_store_plans(FFTPlan a, FFTPlan b, FFTPlan c, FFTPlan d, FFTPlan* out) {
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
    out[2] = c;
    out[3] = d;
  }
}

hipError_t launch_store_plans(const FFTPlan* four, FFTPlan* dev, hipStream_t s) {
  hipLaunchKernelGGL(k_store_plans, dim3(1), dim3(64), 0, s, four[0], four[1], four[2], four[3], dev);
  return hipGetLastError();
}

#define DKS_INSTANTIATE(T)                                                                                     \
  template hipError_t launch_fft_x_fwd<T>(const void*, size_t, void*, size_t, const MeshDims&, const PlanRef&, \
                                          const void*, int, hipStream_t);                                      \
  template hipError_t launch_fft_y_fwd<T>(const void*, void*, size_t, const MeshDims&, const PlanRef&, int,    \
                                          hipStream_t);                                                        \
  template hipError_t launch_fft_z_conv<T>(const void*, void*, size_t, const void*, const Geometry*, size_t,   \
                                           const MeshDims&, const PlanRef&, const PlanRef&, int, hipStream_t); \
  template hipError_t launch_fft_y_inv<T>(const void*, void*, size_t, const MeshDims&, const PlanRef&, int,    \
                                          hipStream_t);                                                        \
  template hipError_t launch_fft_x_inv<T>(const void*, size_t, void*, size_t, const ElemBatch&, const MeshDims&,\
                                          const PlanRef&, const void*, int, hipStream_t);
DKS_INSTANTIATE(float)
DKS_INSTANTIATE(double)
#undef DKS_INSTANTIATE

}  // namespace dks
