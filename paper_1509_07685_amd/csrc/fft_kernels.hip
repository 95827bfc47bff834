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
// pass, C after the z pass) are block-major: columns come in blocks of 128
// bytes, and a block's column segment of a (ky) row is contiguous over z, so
// a z pencil tile is one contiguous run of memory and a y pencil of one
// plane steps from block row to block row.
//
// Zero padding is never stored: the forward x transform reads the nx real
// values of a row, the forward y and z transforms read only the first half of
// their pencils, and the inverse transforms store only the outputs in
// [-1, n] per axis (the physical mesh plus one ghost node on each side).

#include <algorithm>

#include "fft_engine.h"

namespace dks {

// ---------------------------------------------------------------------------
// Column tiles.  The y and z passes work on tiles of W adjacent kx columns
// (128 bytes of a row); a mesh has ntile = ceil((nx + 1) / W) of them, the
// last one partly padding (columns nx + 1 .. cs - 1 of the padded row).
// Padding columns are transformed like the others and never read back by
// the x inverse pass, so no lane tests its column.
// ---------------------------------------------------------------------------
template <class SP> __device__ __forceinline__ int ntiles(const MeshDims& m, const FFTPlan* P) {
  const int W = plan_W<SP>(P);
  return (m.ncols + W - 1) / W;
}

// Columns per block of the tile-major intermediates: 128 bytes, the tile
// width of every compile-time plan (a runtime plan's tile may be narrower and
// then covers part of a block).
template <typename T> constexpr int kBlockCols = 128 / (2 * (int)sizeof(T));

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
  constexpr int TH = RegCfg<T>::THREADS;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const T* src = in + blockIdx.y * in_stride;
  C* dst = out + blockIdx.y * out_stride;
  const int Wt = plan_W<SP>(P), LDt = plan_LD<SP>(P);
  const int row0 = blockIdx.x * Wt;
  const int nvalid = min(Wt, nrows - row0);
  const int nx = m.nx, M = plan_N<SP>(P);
  C* lpost = lds + (size_t)M * LDt;
  if constexpr (SP::is_static) {
    // nx = N: each row is N reals = N/2 complex pairs z[m]; lane l of the
    // row's LPR lanes loads pairs l, l + LPR, ... (both halves of a pair in
    // one load) and puts pair m at tile element m.
    constexpr int N = SP::N, W = SP::W, LD = SP::LD, LPR = TH / W, NP = N / 2;
    static_assert(NP % LPR == 0, "rows of whole lane groups");
    const int p = (int)threadIdx.x / LPR, l = (int)threadIdx.x % LPR;
    if (p < nvalid) {
      const C* srow = reinterpret_cast<const C*>(src + (size_t)(row0 + p) * N);
      C v[NP / LPR];
#pragma unroll
      for (int i = 0; i < NP / LPR; ++i) v[i] = srow[l + LPR * i];
#pragma unroll
      for (int i = 0; i < NP / LPR; ++i) lds[(l + LPR * i) * LD + p] = v[i];
    }
    for (int k = (int)threadIdx.x; k <= N; k += TH) lpost[k] = post[k];
    __syncthreads();
    auto lin = [&](int c, int idx, int) { return lds[idx * LD + c]; };
    auto lout = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
      for (int r = 0; r < RC.value; ++r) lds[(base + r * Ns) * LD + c] = vals[r];
    };
    run_any<T, false, true, SP, 0, true>(lds, P, lin, lout);   // z[m] = 0 for m >= N/2: never read
    __syncthreads();
    if (p < nvalid) {
      C* drow = dst + (size_t)(row0 + p) * m.cs;
#pragma unroll
      for (int i = 0; i <= N / LPR; ++i) {
        const int k = l + LPR * i;
        if (i < N / LPR || k <= N) {
          const C zk = lds[(k & (N - 1)) * LD + p];
          C zc = lds[((N - k) & (N - 1)) * LD + p];
          zc.y = -zc.y;
          const C s = cadd(zk, zc), d = csub(zk, zc);
          const C wd = cmul(lpost[k], d);
          drow[k] = C{(T)0.5 * (s.x + wd.y), (T)0.5 * (s.y - wd.x)};
        }
      }
    }
    return;
  } else {
    {
      // The tile's rows are contiguous (nvalid * nx reals, at most kTileReals per
      // thread): every load of the thread is issued before the first LDS store.
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
    for (int k = (int)threadIdx.x; k <= nx; k += TH) lpost[k] = post[k];
    __syncthreads();
    {
      const int nnz = (nx + 1) >> 1;
      const int LD = LDt;
      auto lin = [&](int c, int idx, int) { return idx < nnz ? lds[idx * LD + c] : C{0, 0}; };
      auto lout = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
        for (int r = 0; r < RC.value; ++r) lds[(base + r * Ns) * LD + c] = vals[r];
      };
      run_any<T, false, true, SP, 0, true>(lds, P, lin, lout);
    }
    __syncthreads();
    // outputs flattened over (row, column) so every lane has work: a row holds
    // nx + 1 values, which a row-per-lane-group split would leave ragged
    const int ncols = nx + 1;
    const int total = nvalid * ncols;
    for (int e = (int)threadIdx.x; e < total; e += TH) {
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
}

// ---------------------------------------------------------------------------
// The z-pass intermediates are block-major: with WB = 128 bytes of columns
// and nb = cs / WB blocks per row, B (after the y forward pass) holds element
// (z, ky, kx) at ((ky nb + kx / WB) nz + z) WB + kx % WB, and C (after the z
// pass) holds z' = z + 1 in [0, nz + 2) at ((ky nb + kx / WB)(nz + 2) + z')
// WB + kx % WB.  A z pencil tile is then one contiguous block (nz WB
// complex), and a y pencil of one plane steps by nb nz WB (or nb (nz + 2) WB)
// elements.
// ---------------------------------------------------------------------------

// Stores of the last pass of an inverse transform of length N that keep only
// indices -1 .. n (n = N / 2) as output rows idx + 1, idx = N - 1 as row 0.
// With a compile-time plan the last pass has span Ns = N / R and butterfly
// base b in [0, Ns): outputs b + r Ns for r < R/2 are always kept, r = R/2
// only for b = 0 (index n), r = R - 1 only for b = Ns - 1 (index N - 1).
template <bool STATIC, int R, class St, class C>
__device__ __forceinline__ void keep_outputs(int base, int Ns, int N, const C* vals, St&& st) {
  if constexpr (STATIC) {
#pragma unroll
    for (int r = 0; r < R / 2; ++r) st(base + r * Ns + 1, vals[r]);
    if (base == 0) st(N / 2 + 1, vals[R / 2]);
    if (base == Ns - 1) st(0, vals[R - 1]);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int idx = base + r * Ns;
      if (idx <= N / 2) st(idx + 1, vals[r]);
      else if (idx == N - 1) st(0, vals[r]);
    }
  }
}

// ---------------------------------------------------------------------------
// y forward: pencils along y of the x-transformed rows.  Input A[z][y][kx]
// (y < ny), output B (ky < 2 ny, tile-major).  Grid: (column tiles, nz, batch):
// consecutive workgroups read adjacent segments of one A row (the loads are
// what a workgroup waits on; ordering by z instead, so that the stores to B
// are adjacent, measured slower).
// ---------------------------------------------------------------------------
template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fft_y_fwd(const typename Cplx<T>::type* __restrict__ A,
                                                        typename Cplx<T>::type* __restrict__ B,
                                                        size_t stride, MeshDims m, const FFTPlan* __restrict__ P,
                                                        int tile0) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  constexpr int WB = kBlockCols<T>;
  const int c0 = (tile0 + (int)blockIdx.x) * plan_W<SP>(P);
  const int z = blockIdx.y;
  using Off = OffT<SP>;
  const C* src = A + blockIdx.z * stride + (size_t)z * m.ny * m.cs + c0;
  C* dst = B + blockIdx.z * stride + ((size_t)(c0 / WB) * m.nz + z) * WB + c0 % WB;
  const int ny = m.ny, cs = m.cs;
  const Off kstep = (Off)(cs / WB) * (Off)m.nz * (Off)WB;   // next ky of this plane
  // compile-time plans: the first pass never reads its upper (zero) half, y < ny
  auto in = [&](int c, int idx, int) {
    return (SP::is_static || idx < ny) ? src[(Off)idx * (Off)cs + (Off)c] : C{0, 0};
  };
  auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
    for (int r = 0; r < RC.value; ++r) dst[(Off)(base + r * Ns) * kstep + (Off)c] = vals[r];
  };
  run_any<T, false, false, SP, 0, true>(lds, P, in, out);
}

// ---------------------------------------------------------------------------
// z: forward transform of each (kx, ky) pencil over its nz non-zero inputs,
// multiply by the real Green's spectrum times the solve's scale, inverse
// transform, keep z in [-1, nz].  Input B, output C (both tile-major, one
// contiguous block per pencil tile).  The inverse plan's radices are the
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
    MeshDims m, const FFTPlan* __restrict__ Pf, const FFTPlan* __restrict__ Pi, int tile0, int ntile) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  constexpr int WB = kBlockCols<T>;
  const int W = plan_W<SP>(Pf);
  const unsigned L = blockIdx.x;
  const int pt = (int)(((L >> 4) << 3) | (L & 7u));    // pair-tile index over the launch's ntile tiles
  const int pair = pt / ntile, tile = tile0 + pt - pair * ntile;
  if (pair > m.Ny / 2) return;
  const bool second = (L >> 3) & 1u;
  if (second && (pair == 0 || 2 * pair == m.Ny)) return;   // rows 0 and Ny/2 pair with themselves
  const int ky = second ? m.Ny - pair : pair;
  const int nz = m.nz, Nz = m.Nz, LD = plan_LD<SP>(Pf);
  using Off = OffT<SP>;
  const int c0 = tile * W;
  const size_t blk = (size_t)ky * (m.cs / WB) + c0 / WB;
  const C* src = B + blockIdx.y * stride + blk * nz * WB + c0 % WB;
  C* dst = Cout + blockIdx.y * stride + blk * (nz + 2) * WB + c0 % WB;
  const Geometry* g = reinterpret_cast<const Geometry*>(reinterpret_cast<const char*>(geo) +
                                                        blockIdx.y * geo_stride);
  const T scale = Geo<T>::scale(g);
  const T* gblk = G + ((size_t)pair * (m.cs / W) + tile) * (nz + 1) * W;   // [kz][W]
  auto in = [&](int c, int idx, int) {
    return (SP::is_static || idx < nz) ? src[(Off)idx * (Off)WB + (Off)c] : C{0, 0};
  };
  using SPi = typename InvPlan<SP>::type;
  const bool inv_single = plan_npass<SPi>(Pi) == 1;
  // Last forward pass: its outputs sit at kz = j + r Ns, exactly the inputs of
  // the first inverse butterfly j (radix R, span 1, no twiddles).
  // The Green's values of each butterfly are requested with the last forward
  // pass's inputs (before its barrier); that pass writes kz = j + r * Nz / R,
  // whose octant index is min(kz, Nz - kz): kz itself for r < R/2, and
  // (R - r) Nz / R - j for r >= R/2.
  T gpre[RegCfg<T>::ARR];
  auto gload = [&](auto RC, int k, int c, int j) {
    constexpr int R = RC.value;
    if constexpr (SP::is_static) {
      constexpr int span = SP::N / R;
      const int ia = j * W + c, ib = c - j * W;
#pragma unroll
      for (int r = 0; r < R; ++r) gpre[k * R + r] = r < R / 2 ? gblk[ia + r * span * W] : gblk[ib + (R - r) * span * W];
    } else {
      const int span = Nz / R;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int kz = j + r * span;
        const int kzr = min(kz, Nz - kz);
        gpre[k * R + r] = gblk[kzr * W + c];
      }
    }
  };
  auto store = [&](int c) {
    return [=](int zo, C val) { dst[(Off)zo * (Off)WB + (Off)c] = val; };
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
      keep_outputs<false, R>(j * R, 1, Nz, vals, store(c));
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
      keep_outputs<SPi::is_static, RC.value>(base, Ns, Nz, vals, store(c));
    };
    run_any<T, true, true, SPi, 1>(lds, Pi, lds_in, out);
  }
}

// Butterfly slots per thread of pass p of compile-time plan SP (as fft_pass_s
// assigns them): slot k of thread t is butterfly b = t + k TH, pencil
// b mod W, index b / W; slots with b >= W N / R are idle.
template <typename T, class SP, int p> struct PassSlots {
  static constexpr int R = SP::R(p), NR = SP::N / R, nbf = SP::W * NR, TH = RegCfg<T>::THREADS;
  static constexpr int K = cmin((RegCfg<T>::EMAX + R - 1) / R, (nbf + TH - 1) / TH);
  static constexpr bool guard = K * TH > nbf;
};

// Persistent z pass for compile-time plans and single solves: workgroup g
// takes the pair-tile indices L = g, g + G, g + 2G, ... of the one-shot
// kernel's grid (same order, so pair members are still dispatched together)
// and, while it transforms one pencil tile, has the loads of its next tile's
// inputs in flight, so each workgroup overlaps its own memory traffic with
// its arithmetic instead of relying on a second workgroup of the CU being in
// another phase.  Vector-memory loads complete in issue order, so nothing
// issued after the prefetch may be waited for before the next tile: the
// twiddle tables are copied to LDS once per workgroup, and a tile's Green's
// values are requested before the next tile's inputs.  Two workgroups per CU
// (the LDS tile bounds it): the register budget is held to what that
// occupancy allows.
template <typename T> struct PipeOcc {
  static constexpr int waves_per_simd = 2 * (RegCfg<T>::THREADS / 64) / 4;
};

template <class SP> struct PipeTw {
  using SPi = typename InvPlan<SP>::type;
  static constexpr int nf = static_tw_count<SP>(), ni = static_tw_count<SPi>();
  // a palindromic radix order gives the inverse plan the forward plan's table
  static constexpr bool shared = [] {
    for (int p = 0; p < SP::npass; ++p)
      if (SP::R(p) != SPi::R(p)) return false;
    return true;
  }();
  static constexpr int total = shared ? nf : nf + ni;
};

template <typename T, class SP>
static inline size_t z_pipe_lds_bytes(const FFTPlan& h) {
  return lds_bytes<T>(h) + (size_t)PipeTw<SP>::total * sizeof(typename Cplx<T>::type);
}

template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS, PipeOcc<T>::waves_per_simd) void k_fft_z_conv_pipe(
    const typename Cplx<T>::type* __restrict__ B, typename Cplx<T>::type* __restrict__ Cout,
    const T* __restrict__ G, const Geometry* __restrict__ geo, MeshDims m, const FFTPlan* __restrict__ Pf,
    const FFTPlan* __restrict__ Pi, int tile0, int ntile, int nL) {
  using C = typename Cplx<T>::type;
  static_assert(SP::is_static, "compile-time plans only");
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  constexpr int WB = kBlockCols<T>, W = SP::W, LD = SP::LD, N = SP::N, TH = RegCfg<T>::THREADS;
  using S0 = PassSlots<T, SP, 0>;
  using SL = PassSlots<T, SP, SP::npass - 1>;
  constexpr int R0 = S0::R, RL = SL::R;
  using SPi = typename InvPlan<SP>::type;
  using TW = PipeTw<SP>;
  // twiddle tables after the tile: forward, then (unless shared) inverse
  C* twf = lds + N * LD;
  C* twi = TW::shared ? twf : twf + TW::nf;
  {
    const C* gf = (const C*)Pf->tw;
    const C* gi = (const C*)Pi->tw;
    for (int i = (int)threadIdx.x; i < TW::nf; i += TH) twf[i] = gf[i];
    if constexpr (!TW::shared)
      for (int i = (int)threadIdx.x; i < TW::ni; i += TH) twi[i] = gi[i];
  }
  const int nz = m.nz, Nz = m.Nz, Ny = m.Ny;
  const T scale = Geo<T>::scale(geo);
  const size_t nb = (size_t)(m.cs / WB);
  // (pair, member) of index L; false when L names no tile
  auto decode = [&](int L, int& ky, int& tile, int& pair) {
    const int pt = ((L >> 4) << 3) | (L & 7);
    pair = pt / ntile;
    tile = tile0 + pt - pair * ntile;
    const bool second = (L >> 3) & 1;
    ky = second ? Ny - pair : pair;
    return pair <= Ny / 2 && !(second && (pair == 0 || 2 * pair == Ny));
  };
  // Every iteration issues the same loads (an index that names no tile, or
  // the end of the range, reads the first tile of the range instead), so the
  // compiler's wait counts are the same on every path: a wait for this tile's
  // Green's values never waits for the next tile's inputs, issued after them.
  C pf[S0::K * (R0 / 2)];
  auto prefetch = [&](int L) {
    int ky, tile, pair;
    if (L >= nL || !decode(L, ky, tile, pair)) {
      ky = 0;
      tile = tile0;
    }
    const int c0 = tile * W;
    const C* src = B + ((size_t)ky * nb + c0 / WB) * nz * WB + c0 % WB;
#pragma unroll
    for (int k = 0; k < S0::K; ++k) {
      const int b = (int)threadIdx.x + k * TH;
      if (!S0::guard || b < S0::nbf) {
        const int c = b & (W - 1), j = b >> SP::logW;
#pragma unroll
        for (int r = 0; r < R0 / 2; ++r) pf[k * (R0 / 2) + r] = src[(unsigned)((j + r * S0::NR) * WB + c)];
      }
    }
  };
  int L = blockIdx.x;
  prefetch(L);
  for (; L < nL; L += gridDim.x) {
    int ky, tile, pair;
    const bool valid = decode(L, ky, tile, pair);     // uniform over the workgroup
    C cur[S0::K * (R0 / 2)];
#pragma unroll
    for (int i = 0; i < S0::K * (R0 / 2); ++i) cur[i] = pf[i];
    // this tile's Green's values (kz = j + r Nz/R of the last forward pass;
    // octant index kz for r < R/2, (R - r) Nz/R - j above), before the prefetch
    T gcur[SL::K * RL];
    {
      const T* gblk = G + ((size_t)(valid ? pair : 0) * (m.cs / W) + (valid ? tile : tile0)) * (nz + 1) * W;
      constexpr int span = N / RL;
#pragma unroll
      for (int k = 0; k < SL::K; ++k) {
        const int b = (int)threadIdx.x + k * TH;
        if (!SL::guard || b < SL::nbf) {
          const int c = b & (W - 1), j = b >> SP::logW;
          const int ia = j * W + c, ib = c - j * W;
#pragma unroll
          for (int r = 0; r < RL; ++r)
            gcur[k * RL + r] = r < RL / 2 ? gblk[ia + r * span * W] : gblk[ib + (RL - r) * span * W];
        }
      }
    }
    prefetch(L + (int)gridDim.x);
    if (!valid) continue;
    const int c0 = tile * W;
    C* dst = Cout + ((size_t)ky * nb + c0 / WB) * (nz + 2) * WB + c0 % WB;
    __syncthreads();     // twiddles stored; the previous tile's last LDS reads are done
    auto in = [&](int, int, int slot) { return cur[slot]; };
    auto store = [&](int c) {
      return [=](int zo, C val) { dst[(unsigned)(zo * WB + c)] = val; };
    };
    auto mid = [&](auto RC, int c, int j, int, int, C* vals, int k) {
      constexpr int R = RC.value;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T gv = gcur[k * R + r] * scale;
        vals[r].x *= gv;
        vals[r].y *= gv;
      }
      dft<R, true>(vals);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(j * R + r) * LD + c] = vals[r];
    };
    run_static_tw<T, false, false, SP, 0, true>(lds, twf, in, mid);
    __syncthreads();
    auto lds_in = [&](int c, int idx, int) { return lds[idx * LD + c]; };
    auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
      keep_outputs<true, RC.value>(base, Ns, Nz, vals, store(c));
    };
    run_static_tw<T, true, true, SPi, 1>(lds, twi, lds_in, out);
  }
}

// ---------------------------------------------------------------------------
// y inverse: C (tile-major) -> D[z'][y + 1][kx] for y in [-1, ny].
// Grid: (nz + 2, column tiles, batch): consecutive workgroups read adjacent
// segments of each C row (one column block holds the rows of every z'), which
// measured faster than ordering by column tile, where the stores to D are the
// adjacent ones.
// ---------------------------------------------------------------------------
template <typename T, class SP>
__global__ __launch_bounds__(RegCfg<T>::THREADS) void k_fft_y_inv(const typename Cplx<T>::type* __restrict__ Cin,
                                                        typename Cplx<T>::type* __restrict__ D,
                                                        size_t stride, MeshDims m, const FFTPlan* __restrict__ P,
                                                        int tile0) {
  using C = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  constexpr int WB = kBlockCols<T>;
  const int c0 = (tile0 + (int)blockIdx.y) * plan_W<SP>(P);
  const int zp = blockIdx.x;
  using Off = OffT<SP>;
  const C* src = Cin + blockIdx.z * stride + ((size_t)(c0 / WB) * (m.nz + 2) + zp) * WB + c0 % WB;
  C* dst = D + blockIdx.z * stride + (size_t)zp * (m.ny + 2) * m.cs + c0;
  const int Ny = m.Ny, cs = m.cs;
  const Off kstep = (Off)(cs / WB) * (Off)(m.nz + 2) * (Off)WB;   // next ky of this plane
  auto in = [&](int c, int idx, int) { return src[(Off)idx * kstep + (Off)c]; };
  auto out = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
    keep_outputs<SP::is_static, RC.value>(base, Ns, Ny, vals,
                                          [&](int yo, C val) { dst[(Off)yo * (Off)cs + (Off)c] = val; });
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
  constexpr int TH = RegCfg<T>::THREADS;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const C* src = D + blockIdx.y * in_stride;
  T* dst = phi_ext + blockIdx.y * out_stride;
  T* user = reinterpret_cast<T*>(phi_user.at(blockIdx.y).phi);
  const int Wt = plan_W<SP>(P), LDt = plan_LD<SP>(P);
  const int row0 = blockIdx.x * Wt;
  const int nvalid = min(Wt, nrows - row0);
  const int nx = m.nx, M = plan_N<SP>(P);
  if constexpr (SP::is_static) {
    // nx = N.  Lane l of row p's LPR lanes forms Z'[k] for k = l, l + LPR, ...
    constexpr int N = SP::N, W = SP::W, LD = SP::LD, LPR = TH / W;
    static_assert(N % LPR == 0, "rows of whole lane groups");
    const int p = (int)threadIdx.x / LPR, l = (int)threadIdx.x % LPR;
    const int r = row0 + p;              // row z' (ny + 2) + y'
    if (p < nvalid) {
      const C* row = src + (size_t)r * m.cs;
      C xk[N / LPR], xc[N / LPR], w[N / LPR];
#pragma unroll
      for (int i = 0; i < N / LPR; ++i) {
        const int k = l + LPR * i;
        xk[i] = row[k];
        xc[i] = row[N - k];
        w[i] = post[k];
      }
#pragma unroll
      for (int i = 0; i < N / LPR; ++i) {
        C c = xc[i];
        c.y = -c.y;
        const C s = cadd(xk[i], c), d = csub(xk[i], c);
        C ww = w[i];
        ww.y = -ww.y;
        const C wd = cmul(ww, d);
        lds[(l + LPR * i) * LD + p] = C{s.x - wd.y, s.y + wd.x};
      }
    }
    __syncthreads();
    auto lin = [&](int c, int idx, int) { return lds[idx * LD + c]; };
    auto lout = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
      for (int q = 0; q < RC.value; ++q) lds[(base + q * Ns) * LD + c] = vals[q];
    };
    run_any<T, true, true, SP, 0>(lds, P, lin, lout);
    __syncthreads();
    if (p < nvalid) {
      // phi_ext row: x = -1 .. N as pairs (x = 2q - 1, 2q), q = 0 .. N/2;
      // x = 2q - 1 is the odd half of z[q - 1] (z[N - 1] for q = 0), x = 2q
      // the even half of z[q].
      C* orow = reinterpret_cast<C*>(dst + (size_t)r * (N + 2));
#pragma unroll
      for (int i = 0; i <= (N / 2) / LPR; ++i) {
        const int q = l + LPR * i;
        if (i < (N / 2) / LPR || q <= N / 2) {
          const T odd = lds[((q + N - 1) & (N - 1)) * LD + p].y;
          const T even = lds[q * LD + p].x;
          orow[q] = C{odd, even};
        }
      }
      if (user) {
        const int zq = r / (m.ny + 2);     // once per lane
        const int yq = r - zq * (m.ny + 2);
        if (zq >= 1 && zq <= m.nz && yq >= 1 && yq <= m.ny) {
          // physical x = 0 .. N - 1: pair (2q, 2q + 1) is z[q] itself
          T* urow = user + ((size_t)(zq - 1) * m.ny + (yq - 1)) * N;
          if ((reinterpret_cast<uintptr_t>(user) & (sizeof(C) - 1)) == 0) {
#pragma unroll
            for (int i = 0; i < (N / 2) / LPR; ++i) {
              const int q = l + LPR * i;
              reinterpret_cast<C*>(urow)[q] = lds[q * LD + p];
            }
          } else {
#pragma unroll
            for (int i = 0; i < (N / 2) / LPR; ++i) {
              const int q = l + LPR * i;
              const C v = lds[q * LD + p];
              urow[2 * q] = v.x;
              urow[2 * q + 1] = v.y;
            }
          }
        }
      }
    }
    return;
  } else {
    {
      // nvalid * M elements (at most kTileReals per thread), in two halves whose
      // loads are all issued before they are used.
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
      auto lin = [&](int c, int idx, int) { return lds[idx * LD + c]; };
      auto lout = [&](auto RC, int c, int, int base, int Ns, C* vals, int) {
#pragma unroll
        for (int q = 0; q < RC.value; ++q) lds[(base + q * Ns) * LD + c] = vals[q];
      };
      run_any<T, true, true, SP, 0>(lds, P, lin, lout);
    }
    __syncthreads();
    // outputs flattened over (row, column) so every lane has work (rows of
    // nx + 2 values)
    const int nout = nx + 2;
    const int ny2 = m.ny + 2;
    const int total = nvalid * nout;
    for (int e = (int)threadIdx.x; e < total; e += TH) {
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
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
// Every element offset the y and z passes form inside one batch element's
// intermediate arrays stays below (nz + 2) * Ny * cs (the size of C).
static inline bool offsets_fit32(const MeshDims& m) {
  return (double)(m.nz + 2) * (double)m.Ny * (double)m.cs < 2147483648.0;
}

// Calls f with the compile-time plan equal to host plan h (tile width of 128
// bytes, LD = W + PAD), or with DynPlan when none is or when the caller rules
// the compile-time kernels out (!allow: element offsets that may not fit 32
// bits, or input rows not aligned for paired loads).
template <typename T, int PAD, class F> static void with_plan(const FFTPlan& h, F&& f, bool allow = true) {
  constexpr int W = 128 / (2 * (int)sizeof(T));
  if (!allow) f(DynPlan{});
  else if (plan_matches<SPlan<512, W, W + PAD, false>>(h)) f(SPlan<512, W, W + PAD, false>{});
  else if (plan_matches<SPlan<256, W, W + PAD, false>>(h)) f(SPlan<256, W, W + PAD, false>{});
  else if (plan_matches<SPlan<128, W, W + PAD, false>>(h)) f(SPlan<128, W, W + PAD, false>{});
  else if (plan_matches<SPlan<64, W, W + PAD, false>>(h)) f(SPlan<64, W, W + PAD, false>{});
  else f(DynPlan{});
}

static int device_cus() {
  static const int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || cus <= 0)
      cus = 256;
    return cus;
  }();
  return n;
}

// Workgroups of the persistent z pass: four per CU (two are resident at a
// time, the LDS tile bounds it; the second round evens out the tiles left
// at the end of the first).  Measured at 256^3: two per CU 203 us, four 196 us
// (FP32); 303 and 300 us (FP64).
static int z_pipe_blocks() { return 4 * device_cus(); }

// The value held by lane (lane xor H) of the wavefront, H = 1, 2, ..., 32.
// Within a 16-lane row by DPP, one or two VALU operations: quad permutations
// (H = 1, 2) and row rotations (H = 8; H = 4 as two rotations, lane + 4
// written to banks 0 and 2 and lane - 4 to banks 1 and 3).  Across rows by
// the LDS crossbar (ds_bpermute), which costs no VALU work: gfx950's half-row
// and half-wavefront swaps do the same exchange but cost two copies, the swap
// and a select in VALU operations.
template <int H> __device__ __forceinline__ unsigned lane_xor_dpp_u32(unsigned v) {
  static_assert(H == 1 || H == 2 || H == 4 || H == 8, "xor distance within a 16-lane row");
  if constexpr (H == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);            // quad_perm [1, 0, 3, 2]
  } else if constexpr (H == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);            // quad_perm [2, 3, 0, 1]
  } else if constexpr (H == 4) {
    const unsigned t = __builtin_amdgcn_update_dpp(v, v, 0x12C, 0xF, 0x5, false);   // row_ror 12
    return __builtin_amdgcn_update_dpp(t, v, 0x124, 0xF, 0xA, false);               // row_ror 4
  } else {
    return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);           // row_ror 8
  }
}
template <int H> __device__ __forceinline__ unsigned lane_xor_u32(unsigned v, int lane) {
  if constexpr (H <= 8) return lane_xor_dpp_u32<H>(v);
  else return (unsigned)__builtin_amdgcn_ds_bpermute((lane ^ H) << 2, (int)v);
}
template <int H> __device__ __forceinline__ float lane_xor(float v, int lane) {
  return __uint_as_float(lane_xor_u32<H>(__float_as_uint(v), lane));
}
template <int H> __device__ __forceinline__ double lane_xor(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = lane_xor_u32<H>((unsigned)b, lane), hi = lane_xor_u32<H>((unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Six radix-2 decimation-in-frequency stages (spans h = 32, 16, ..., 1) of a
// length-64 transform over the lanes of a wavefront, applied to each of the
// P values per lane: of a lane pair (l, l xor h) the lower lane keeps a + b
// and the upper one (a - b) w^j, j = l mod h.  ws[st] is that lane's w^j for
// span 2^st (1 on lower lanes), sg[st] is -1 on upper lanes and +1 on lower
// ones.  Lane l ends with the output at index rev(l), rev the 6-bit reversal.
template <typename T, int P>
__device__ __forceinline__ void wave_dif64(typename Cplx<T>::type* v, const typename Cplx<T>::type* ws,
                                           const T* sg, int lane) {
  using C = typename Cplx<T>::type;
  auto stage = [&](auto STC) {
    constexpr int st = decltype(STC)::value, h = 1 << st;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const T px = lane_xor<h>(v[i].x, lane), py = lane_xor<h>(v[i].y, lane);
      const C t{sg[st] * v[i].x + px, sg[st] * v[i].y + py};
      v[i] = st == 0 ? t : cmul(t, ws[st]);    // span 1: every twiddle is 1
    }
  };
  stage(std::integral_constant<int, 5>{});
  stage(std::integral_constant<int, 4>{});
  stage(std::integral_constant<int, 3>{});
  stage(std::integral_constant<int, 2>{});
  stage(std::integral_constant<int, 1>{});
  stage(std::integral_constant<int, 0>{});
}

// ---------------------------------------------------------------------------
// x inverse with one wavefront per row, for nx = 64 P (P = 1, 2, 4, 8): no
// LDS tile and no barriers; the radix stages across lanes exchange values
// with wavefront shuffles.  Lane l holds Z'[k] (as in k_fft_x_inv) for
// k = l + 64 i, i < P, so its loads are row-contiguous.  With m = m1 + P m2
// the inverse transform z[m] = sum_k Z'[k] e^{+2 pi i k m / nx} splits into a
// length-P transform over i in registers, the twiddle e^{+2 pi i l m1 / nx},
// and for each m1 a length-64 transform over the lanes: six radix-2
// decimation-in-frequency stages (spans h = 32, 16, ..., 1) in which lane l
// takes its partner's value from lane l xor h (lane_xor).  That leaves
// z[m1 + P rev(l)] in lane l (rev the 6-bit reversal); the lanes write z to
// the wavefront's own LDS row at those places and read it back so that lane
// l forms the outputs l, l + 64, ...: both stores are lane-contiguous.  Every
// twiddle is an entry of the post table e^{-2 pi i k / (2 nx)}, k <= nx.
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__(256) void k_fft_x_inv_wave(const typename Cplx<T>::type* __restrict__ D,
                                                        size_t in_stride, T* __restrict__ phi_ext,
                                                        size_t out_stride, ElemBatch phi_user, MeshDims m,
                                                        const typename Cplx<T>::type* __restrict__ post, int nrows) {
  using C = typename Cplx<T>::type;
  constexpr int N = 64 * P;
  const int lane = (int)threadIdx.x & 63;
  const int rl = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);
  const C* src = D + blockIdx.y * in_stride;
  T* dst = phi_ext + blockIdx.y * out_stride;
  T* user = reinterpret_cast<T*>(phi_user.at(blockIdx.y).phi);
  const bool user_pairs = (reinterpret_cast<uintptr_t>(user) & (sizeof(C) - 1)) == 0;
  // the wavefront's row of z, for lane-contiguous stores (no barrier: only
  // this wavefront touches it, and its LDS operations complete in order)
  __shared__ C zrow[4][N];
  C* zb = zrow[threadIdx.x >> 6];
  // e^{+2 pi i t / N}, 0 <= t < N
  auto wpow = [&](int t) {
    const C w = 2 * t <= N ? post[2 * t] : C{-post[2 * t - N].x, -post[2 * t - N].y};
    return C{w.x, -w.y};
  };
  C wz[P], w2[P], ws[6];
  T sg[6];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const C w = post[lane + 64 * i];
    wz[i] = C{w.x, -w.y};
    w2[i] = wpow(lane * i);
  }
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int h = 1 << st;
    const bool upper = (lane & h) != 0;
    ws[st] = upper ? wpow((lane & (h - 1)) * (N / (2 * h))) : C{(T)1, (T)0};
    sg[st] = upper ? (T)-1 : (T)1;
  }
  // Rows r = wid, wid + nw, ... of this wavefront.  A row's inputs are used
  // up by the Z' formation at the start of its transform; the next row's
  // loads are issued into the same registers right after (a scheduling
  // barrier keeps them there), so they are in flight for the rest of the
  // transform.  A row past the end is loaded as row 0 and never used.
  const int wid = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int nw = (int)((gridDim.x * blockDim.x) >> 6);
  // byte offsets of the lane's elements in a row (the row base is uniform)
  const unsigned ok0 = (unsigned)(lane * (int)sizeof(C)), oc0 = (unsigned)((N - lane) * (int)sizeof(C));
  C xk[P], xc[P];
  auto load = [&](int r) {
    const char* row = reinterpret_cast<const char*>(src + (size_t)(r < nrows ? r : 0) * m.cs);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      xk[i] = *reinterpret_cast<const C*>(row + (ok0 + (unsigned)(64 * i * (int)sizeof(C))));
      xc[i] = *reinterpret_cast<const C*>(row + (oc0 - (unsigned)(64 * i * (int)sizeof(C))));
    }
  };
  load(wid);
  for (int r = wid; r < nrows; r += nw) {      // uniform over the wavefront
    C v[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const C c{xc[i].x, -xc[i].y};
      const C sm = cadd(xk[i], c), d = csub(xk[i], c);
      const C wd = cmul(wz[i], d);
      v[i] = C{sm.x - wd.y, sm.y + wd.x};
    }
    load(r + nw);
    __builtin_amdgcn_sched_barrier(0);   // keep the prefetch ahead of the transform
    if constexpr (P > 1) dft<P, true>(v);
#pragma unroll
    for (int i = 1; i < P; ++i) v[i] = cmul(v[i], w2[i]);
    wave_dif64<T, P>(v, ws, sg, lane);    // w = e^{+2 pi i / (2 h)}
    // lane l holds z[i + P rev(l)]
#pragma unroll
    for (int i = 0; i < P; ++i) zb[i + P * rl] = v[i];
    // pair q is (x = 2q - 1, x = 2q) = (z[q - 1].y, z[q].x), q = 0 .. N/2
    C* orow = reinterpret_cast<C*>(dst + (size_t)r * (N + 2));
#pragma unroll
    for (int j = 0; j <= (N / 2) / 64; ++j) {
      const int q = lane + 64 * j;
      if (j < (N / 2) / 64 || q <= N / 2) orow[q] = C{zb[(q + N - 1) & (N - 1)].y, zb[q].x};
    }
    if (user) {
      const int zq = r / (m.ny + 2), yq = r - zq * (m.ny + 2);
      if (zq >= 1 && zq <= m.nz && yq >= 1 && yq <= m.ny) {
        // physical x = 0 .. N - 1: pair (2q, 2q + 1) is z[q], q < N/2.  Global
        // (not generic) stores: a pending flat store would make the compiler
        // wait for every outstanding load, the prefetch included.
        using GT = __attribute__((address_space(1))) T;
        using GC = __attribute__((address_space(1))) C;
        GT* urow = (GT*)user + ((size_t)(zq - 1) * m.ny + (yq - 1)) * N;
#pragma unroll
        for (int j = 0; j < (N / 2 + 63) / 64; ++j) {
          const int q = lane + 64 * j;
          if (q < N / 2) {
            const C zv = zb[q];
            if (user_pairs) {
              GC* up = reinterpret_cast<GC*>(urow) + q;
              up->x = zv.x;
              up->y = zv.y;
            } else {
              urow[2 * q] = zv.x;
              urow[2 * q + 1] = zv.y;
            }
          }
        }
      }
    }
  }
}

template <typename T>
hipError_t launch_fft_x_fwd(const void* in, size_t in_stride, void* out, size_t out_stride, const MeshDims& m,
                            const PlanRef& P, const void* post, int batch, hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int nrows = m.ny * m.nz;
  if ((size_t)P.host.W * m.nx > (size_t)kTileReals * RegCfg<T>::THREADS) return hipErrorInvalidValue;
  dim3 grid((nrows + P.host.W - 1) / P.host.W, batch);
  // compile-time plans read pairs of reals as one complex value
  const bool pairs_aligned = (reinterpret_cast<uintptr_t>(in) % (2 * sizeof(T))) == 0 &&
                             (in_stride * sizeof(T)) % (2 * sizeof(T)) == 0;
  with_plan<T, 1>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fft_x_fwd<T, decltype(sp)>), grid, dim3(RegCfg<T>::THREADS),
                       lds_bytes<T>(P.host) + (size_t)(m.nx + 1) * sizeof(C), s,
                       (const T*)in, in_stride, (C*)out, out_stride, m, P.dev, (const C*)post, nrows, magic_of(m.nx + 1),
                       magic_of(m.nx));
  }, pairs_aligned);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y_fwd(const void* A, void* B, size_t stride, const MeshDims& m, const PlanRef& P, int batch,
                            int col0, int col1, hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int W = P.host.W, t0 = col0 / W;
  dim3 grid((col1 + W - 1) / W - t0, m.nz, batch);
  with_plan<T, 0>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fft_y_fwd<T, decltype(sp)>), grid, dim3(RegCfg<T>::THREADS), lds_bytes<T>(P.host), s,
                       (const C*)A, (C*)B, stride, m, P.dev, t0);
  }, offsets_fit32(m));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_z_conv(const void* B, void* Cout, size_t stride, const void* G, const Geometry* geo,
                             size_t geo_stride, const MeshDims& m, const PlanRef& Pf, const PlanRef& Pi, int batch,
                             int col0, int col1, hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int W = Pf.host.W, t0 = col0 / W;
  const int ntile = (col1 + W - 1) / W - t0;
  const int npt = (m.Ny / 2 + 1) * ntile;                 // pair-tile indices
  dim3 grid((unsigned)((npt + 7) / 8 * 16), batch);
  with_plan<T, 0>(Pf.host, [&](auto sp) {
    using SP = decltype(sp);
    auto launch = [&](auto spl) {
      hipLaunchKernelGGL((k_fft_z_conv<T, decltype(spl)>), grid, dim3(RegCfg<T>::THREADS), lds_bytes<T>(Pf.host), s,
                         (const C*)B, (C*)Cout, stride, (const T*)G, geo, geo_stride, m, Pf.dev, Pi.dev, t0, ntile);
    };
    if constexpr (SP::is_static) {
      if (!plan_matches<typename SP::Reversed>(Pi.host)) {
        launch(DynPlan{});
      } else if (batch == 1 && SP::npass >= 2) {
        const int nL = (int)grid.x;
        const int nwg = std::min(nL, z_pipe_blocks());
        const size_t lds = z_pipe_lds_bytes<T, SP>(Pf.host);
        hipLaunchKernelGGL((k_fft_z_conv_pipe<T, SP>), dim3(nwg), dim3(RegCfg<T>::THREADS), lds, s,
                           (const C*)B, (C*)Cout, (const T*)G, geo, m, Pf.dev, Pi.dev, t0, ntile, nL);
      } else {
        launch(SP{});
      }
    } else {
      launch(DynPlan{});
    }
  }, offsets_fit32(m));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y_inv(const void* Cin, void* D, size_t stride, const MeshDims& m, const PlanRef& P, int batch,
                            int col0, int col1, hipStream_t s) {
  using C = typename Cplx<T>::type;
  const int W = P.host.W, t0 = col0 / W;
  dim3 grid(m.nz + 2, (col1 + W - 1) / W - t0, batch);
  with_plan<T, 0>(P.host, [&](auto sp) {
    hipLaunchKernelGGL((k_fft_y_inv<T, decltype(sp)>), grid, dim3(RegCfg<T>::THREADS), lds_bytes<T>(P.host), s,
                       (const C*)Cin, (C*)D, stride, m, P.dev, t0);
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
  // FP32 rows of 256: one wavefront per row (four per workgroup, a few rows
  // each).  Measured at 256^3: 55 against 66 us for the LDS-tile kernel, 69
  // against 79 us when phi is also written; the LDS-tile kernel stays as
  // fast or faster in FP64 (111 against 110 us at 256^3, more registers per
  // lane) and for shorter rows (128^3, 64^3).
  if constexpr (sizeof(T) == 4) {
    if (m.nx == 256) {
      dim3 gw((unsigned)std::min((nrows + 3) / 4, 5 * device_cus()), batch);   // about the resident wavefronts
      hipLaunchKernelGGL((k_fft_x_inv_wave<T, 4>), gw, dim3(256), 0, s, (const C*)D, in_stride, (T*)phi_ext,
                         out_stride, phi_user, m, (const C*)post, nrows);
      return hipGetLastError();
    }
  }
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
                                          int, int, hipStream_t);                                              \
  template hipError_t launch_fft_z_conv<T>(const void*, void*, size_t, const void*, const Geometry*, size_t,   \
                                           const MeshDims&, const PlanRef&, const PlanRef&, int, int, int,     \
                                           hipStream_t);                                                       \
  template hipError_t launch_fft_y_inv<T>(const void*, void*, size_t, const MeshDims&, const PlanRef&, int,    \
                                          int, int, hipStream_t);                                              \
  template hipError_t launch_fft_x_inv<T>(const void*, size_t, void*, size_t, const ElemBatch&, const MeshDims&,\
                                          const PlanRef&, const void*, int, hipStream_t);
DKS_INSTANTIATE(float)
DKS_INSTANTIATE(double)
#undef DKS_INSTANTIATE

}  // namespace dks
