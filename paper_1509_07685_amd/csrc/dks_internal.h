// Internal declarations shared by the HIP translation units of libdks_poisson.
// Not part of the public ABI (include/dks_poisson.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dks_poisson.h"

namespace dks {

constexpr int kMaxPass = 12;        // radix passes per transform (N <= 4096)
constexpr int kMaxLength = 4096;    // longest transform length
constexpr int kLdsBytes = 65536;    // LDS budget per FFT workgroup
constexpr int kBboxBlocks = 1024;   // first-stage blocks of the bounding-box reduction
constexpr double kEps0 = 8.8541878128e-12;  // F/m (CODATA 2018)

// Per-solve geometry, written on the device by the geometry kernel and read
// by every later kernel of the same solve.  FP64 values, plus their roundings
// to float for the FP32 path.
struct alignas(256) Geometry {
  double h[3];
  double origin[3];
  double inv_h[3];
  double grad_coef[3];     // -1 / (2 h_d)
  double conv_scale;       // multiplier applied with the Green's spectrum
  double pad0;
  float origin_f[3];
  float inv_h_f[3];
  float grad_coef_f[3];
  float conv_scale_f;
  unsigned long long n_outside;   // internal out-of-mesh counter
};

template <typename T> struct Geo;
template <> struct Geo<float> {
  static __device__ __forceinline__ float origin(const Geometry* g, int d) { return g->origin_f[d]; }
  static __device__ __forceinline__ float inv_h(const Geometry* g, int d) { return g->inv_h_f[d]; }
  static __device__ __forceinline__ float grad(const Geometry* g, int d) { return g->grad_coef_f[d]; }
  static __device__ __forceinline__ float scale(const Geometry* g) { return g->conv_scale_f; }
};
template <> struct Geo<double> {
  static __device__ __forceinline__ double origin(const Geometry* g, int d) { return g->origin[d]; }
  static __device__ __forceinline__ double inv_h(const Geometry* g, int d) { return g->inv_h[d]; }
  static __device__ __forceinline__ double grad(const Geometry* g, int d) { return g->grad_coef[d]; }
  static __device__ __forceinline__ double scale(const Geometry* g) { return g->conv_scale; }
};

// One mixed-radix Stockham transform of length N, as the FFT kernels consume
// it.  Pass p has radix R[p] and span Ns[p] = R[0]*...*R[p-1]; its twiddles
// w^(r t) for t < Ns[p], r = 1..R[p]-1 start at tw + tw_off[p].
struct FFTPlan {
  int N;
  int npass;
  int W;        // pencils per workgroup tile (power of two)
  int logW;
  int LD;       // LDS row stride in elements (W, or W + 1 for the x passes)
  int R[kMaxPass];
  int Ns[kMaxPass];
  unsigned magic[kMaxPass];   // ceil(2^32 / Ns) for Ns >= 2
  int tw_off[kMaxPass];
  const void* tw;             // twiddle table base (dtype complex)
};

// A plan as the launchers need it: the host copy (grid and LDS sizes) and
// its device copy (what the kernels read, with uniform scalar loads).
struct PlanRef {
  FFTPlan host;
  const FFTPlan* dev;
};

// Host-side description of an FFTPlan before the workspace is attached.
struct FFTPlanHost {
  FFTPlan dev;
  int tw_count;   // complex twiddles in this plan's table
};

// Mesh extents and padded strides of the intermediate arrays of one solve.
struct MeshDims {
  int nx, ny, nz;
  int Nx, Ny, Nz;     // doubled extents
  int cs;             // padded complex row stride (>= nx + 1)
  int ncols;          // nx + 1 complex columns
};

constexpr int kMaxBatch = 16;
static_assert(sizeof(dks_particle_set) == 80, "dks_particle_set layout is part of the ABI");

// Per-element arguments of a particle solve: one element by value (single
// solves, solve_rho's phi) or a device table of elements read when the
// kernels run (batched solves).  Accessors return by value so no kernel
// argument is ever indexed at run time.  Counts are clamped to [0, max_np];
// an element without positions (or, when need_e, without field outputs) has
// no particles.
struct ElemBatch {
  dks_particle_set local;
  const dks_particle_set* dev;
  int64_t max_np;
  int need_e;
  __device__ __forceinline__ dks_particle_set at(int b) const { return dev ? dev[b] : local; }
  __device__ __forceinline__ int64_t n(const dks_particle_set& s) const {
    if (!s.x || !s.y || !s.z) return 0;
    if (need_e && (!s.Ex || !s.Ey || !s.Ez)) return 0;
    return s.np < 0 ? 0 : (s.np > max_np ? max_np : s.np);
  }
};

// Arguments of the per-solve geometry kernel.
struct GeoArgs {
  int n[3];
  int fitted;          // 1: cubic mesh fitted to the particles (bbox partials)
  int nblocks;         // bbox partial count per element
  int mode;            // 0: mesh density input, 1: particles
  double h[3];         // explicit cell sizes
  double origin[3];    // explicit origin
  size_t zero_off;     // slot offset of a uint32 array cleared by the kernel
  int zero_len;        // its length (0: none)
};

// Particle binning: 16^3-cell tiles, tile K collects out-of-mesh particles.
struct BinGeom {
  int tx, ty, tz;      // tiles per axis
  int K;               // tx * ty * tz
  int item;            // particles per deposit/gather work item
  int lds_hist;        // 1: per-block tile histograms fit in LDS
};

// Per-slot bin bookkeeping (uint32): count[K+1], offset[K+2], cursor[K+1],
// item_off[K+2], misc[4] (misc[0] = number of work items).
struct BinState {
  unsigned* count;
  unsigned* offset;
  unsigned* cursor;
  unsigned* item_off;
  unsigned* misc;
};

// Gauss-Legendre product rules of the Green's function bands: band i covers
// D in [lo[i], lo[i+1]), D = |cell centre| / largest cell side.
struct GLBands {
  int nb;
  double lo[6];
  int m[6];          // points per axis
  double t[6][12];   // nodes on [-1, 1]
  double w[6][12];   // weights
};

// Pointers to one solve's scratch (a "slot").
struct SlotPtrs {
  Geometry* geo;
  double* bbox;       // kBboxBlocks * 6 partial bounds
  void* R1;           // A, then C, then the interleaved E of the gather
  void* R2;           // B, then D
  void* R3;           // deposited weights, then phi with its ghost layer
};

}  // namespace dks
