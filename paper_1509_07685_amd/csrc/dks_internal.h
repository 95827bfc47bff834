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
constexpr size_t kLdsHardware = 163840;   // LDS per workgroup on gfx950 (160 KiB)
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

// 16-byte native vector of the dtype (4 floats or 2 doubles), and streaming
// (non-temporal) loads and stores of it: data read or written once bypasses
// the L2's normal retention so lines that are reused stay resident.
template <typename T> struct Vec16;
template <> struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <> struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
// The particle arrays come in through generic pointers; addressing them as
// global memory gives global (not flat) loads and stores, which do not share
// the LDS wait counter.
template <typename T> __device__ __forceinline__ typename Vec16<T>::type ld_stream(const T* p) {
  using V = typename Vec16<T>::type;
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) V*)p);
}
template <typename T> __device__ __forceinline__ void st_stream(T* p, typename Vec16<T>::type v) {
  using V = typename Vec16<T>::type;
  __builtin_nontemporal_store(v, (__attribute__((address_space(1))) V*)p);
}

__device__ __forceinline__ bool aligned16(const void* a, const void* b, const void* c) {
  return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) &
          15u) == 0;
}

// Contiguous share [start, end) of n particles for workgroup blk of nblk;
// shares start on multiples of 64 particles so vector loads stay aligned.
__device__ __forceinline__ void chunk_of(int64_t n, int blk, int nblk, int64_t* start, int64_t* end) {
  const int64_t ch = ((n + nblk - 1) / nblk + 63) & ~(int64_t)63;
  *start = min((int64_t)blk * ch, n);
  *end = min(*start + ch, n);
}

// Calls f(x, y, z, i) for every particle i of [start, end), the workgroup's
// threads sharing the range.  When the three arrays are 16-byte aligned at
// `start`, each lane reads two 16-byte vectors per array before using any
// of them (six loads in flight per lane); ragged ends go one element at a time.
template <typename T, typename F>
__device__ __forceinline__ void for_each_particle(const T* __restrict__ px, const T* __restrict__ py,
                                                  const T* __restrict__ pz, int64_t start, int64_t end, F&& f) {
  using V = typename Vec16<T>::type;
  constexpr int NV = Vec16<T>::n;
  int64_t i0 = start;
  if (end - start >= 2 * NV && aligned16(px + start, py + start, pz + start)) {
    const int64_t nv = (end - start) / NV;
    const int64_t step = 2 * (int64_t)blockDim.x;
    for (int64_t v = threadIdx.x; v < nv; v += step) {
      const int64_t v2 = v + blockDim.x;
      const bool two = v2 < nv;
      const V x0 = ld_stream(px + start + v * NV), y0 = ld_stream(py + start + v * NV),
              z0 = ld_stream(pz + start + v * NV);
      V x1 = x0, y1 = y0, z1 = z0;
      if (two) {
        x1 = ld_stream(px + start + v2 * NV);
        y1 = ld_stream(py + start + v2 * NV);
        z1 = ld_stream(pz + start + v2 * NV);
      }
#pragma unroll
      for (int k = 0; k < NV; ++k) f(x0[k], y0[k], z0[k], start + v * NV + k);
      if (two) {
#pragma unroll
        for (int k = 0; k < NV; ++k) f(x1[k], y1[k], z1[k], start + v2 * NV + k);
      }
    }
    i0 = start + nv * NV;
  }
  for (int64_t i = i0 + threadIdx.x; i < end; i += blockDim.x) f(px[i], py[i], pz[i], i);
}

// Assignment schemes: the weights that deposit charge on the mesh and
// interpolate the field back to the particles (the NGP / CIC / TSI
// interpolation box of the OPAL structure figure; the third is read as the
// second-order triangular-shaped cloud).
enum : int { kSchemeCIC = 0, kSchemeNGP = 1, kSchemeTSC = 2 };
template <int SCH> struct Scheme;
// width: stencil nodes per axis; lo: first stencil node relative to the node
// that files the particle into a tile.
template <> struct Scheme<kSchemeCIC> { static constexpr int width = 2, lo = 0; };
template <> struct Scheme<kSchemeNGP> { static constexpr int width = 1, lo = 0; };
template <> struct Scheme<kSchemeTSC> { static constexpr int width = 3, lo = -1; };

// One axis of a particle's stencil, for its cell coordinate s on n nodes.
// Returns false when the particle is outside on this axis: s outside
// [0, n - 1], or (TSC) a nearest node outside [1, n - 2].  node is the lower
// node of the cell (CIC, min(floor(s), n - 2)) or the nearest node
// floor(s + 1/2) (NGP, TSC); the stencil covers node + lo ...
// node + lo + width - 1 with weights w:
//   CIC  (1 - f, f),                     f = s - node
//   NGP  (1)
//   TSC  ((1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2),   d = s - node
// s + 1/2 and s - node are exact in the dtype for the node counts here.
template <typename T, int SCH>
__device__ __forceinline__ bool axis_stencil(T s, int n, int& node, T* w) {
  if (!(s >= (T)0 && s <= (T)(n - 1))) {
    node = 0;
#pragma unroll
    for (int k = 0; k < Scheme<SCH>::width; ++k) w[k] = (T)0;
    return false;
  }
  if constexpr (SCH == kSchemeCIC) {
    node = min((int)floor(s), n - 2);
    const T f = s - (T)node;
    w[0] = (T)1 - f;
    w[1] = f;
    return true;
  } else {
    node = (int)floor(s + (T)0.5);
    if constexpr (SCH == kSchemeNGP) {
      w[0] = (T)1;
      return true;
    } else {
      const T d = s - (T)node;
      const T a = (T)0.5 - d, c = (T)0.5 + d;
      w[0] = (T)0.5 * a * a;
      w[1] = (T)0.75 - d * d;
      w[2] = (T)0.5 * c * c;
      return node >= 1 && node <= n - 2;
    }
  }
}

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
  unsigned max_items;  // bound on the work-item count of one solve
  unsigned max_np;     // bound on binned particles per element (buffer size)
  int scheme;          // kSchemeCIC / kSchemeNGP / kSchemeTSC
};

// Binning counts and reserves per XCD group: the scatter's chunk c of batch
// element b belongs to group (b * nchunk + c) mod kXcd, which is the XCD that
// round-robin dispatch places its workgroup on.  Each tile's range is split
// into kXcd consecutive sub-ranges, one per group, so the partly written
// cache lines at the seams between chunks' segments are shared only by
// workgroups of one XCD and complete in that XCD's L2.  (The grouping is a
// pure function of the chunk index; results do not depend on the hardware's
// actual placement.)
constexpr int kXcd = 8;

// Per-slot bin bookkeeping (uint32), L = K + 1 tiles (tile K: outside):
// xcount[kXcd][L] (cleared by the geometry kernel), count[L], offset[L+1],
// xcursor[kXcd][L], item_off[L+1], misc[4] (misc[0] = number of work items).
struct BinState {
  unsigned* xcount;
  unsigned* count;
  unsigned* offset;
  unsigned* xcursor;
  unsigned* item_off;
  unsigned* misc;
};
// Total entries of that layout: 2 kXcd L + 3 L + 2 (the two L + 1 arrays) + 4.
__host__ __device__ constexpr int bins_entries(int K) { return (2 * kXcd + 3) * (K + 1) + 6; }

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
