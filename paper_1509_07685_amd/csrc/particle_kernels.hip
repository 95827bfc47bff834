// Particle <-> mesh kernels of the PM step: bounding box of the bunch (the
// particle-fitted mesh of the PM section), per-solve geometry in FP64,
// cloud-in-cell deposit and gather (the "NGP, CIC, TSI" interpolation of the
// OPAL structure figure), and the central-difference field (its D-operators).

#include <math.h>

#include <type_traits>

#include "dks_internal.h"

namespace dks {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Cell coordinate (x - x0) * (1/h) with two correctly rounded operations and
// no contraction, so the in/out and cell decisions are reproducible.
__device__ __forceinline__ float cell_coord(float x, float x0, float ih) {
  return __fmul_rn(__fsub_rn(x, x0), ih);
}
__device__ __forceinline__ double cell_coord(double x, double x0, double ih) {
  return __dmul_rn(__dsub_rn(x, x0), ih);
}

__device__ __forceinline__ const Geometry* geo_at(const Geometry* base, size_t stride, int b) {
  return reinterpret_cast<const Geometry*>(reinterpret_cast<const char*>(base) + (size_t)b * stride);
}

// ---------------------------------------------------------------------------
// Bounding box, stage 1: each block reduces a contiguous share of the
// particles of batch element blockIdx.y to (min x, min y, min z, max x, max y,
// max z) and writes it to its partial slot.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_bbox(ElemBatch eb, double* partial, size_t partial_stride) {
  const int b = blockIdx.y;
  const dks_particle_set e = eb.at(b);
  const T* p[3] = {(const T*)e.x, (const T*)e.y, (const T*)e.z};
  const int64_t n = eb.n(e);
  T lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = INFINITY;
    hi[d] = -INFINITY;
  }
  int64_t start, end;
  chunk_of(n, blockIdx.x, gridDim.x, &start, &end);
  for_each_particle<T>(p[0], p[1], p[2], start, end, [&](T x, T y, T z, int64_t) {
    lo[0] = fmin(lo[0], x);
    hi[0] = fmax(hi[0], x);
    lo[1] = fmin(lo[1], y);
    hi[1] = fmax(hi[1], y);
    lo[2] = fmin(lo[2], z);
    hi[2] = fmax(hi[2], z);
  });
  __shared__ T red[6][256];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    red[d][threadIdx.x] = lo[d];
    red[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
        red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6)
    partial[(size_t)b * partial_stride + (size_t)blockIdx.x * 6 + threadIdx.x] = (double)red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Geometry of each batch element (one block per element): reduce the bbox
// partials, fit h and the origin, and derive every FP64 factor of the solve.
// Thread 0 also clears the out-of-mesh counter.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void geometry_of(int b, const double* partial, size_t partial_stride, Geometry* geo,
                                            size_t geo_stride, const GeoArgs& a, const ElemBatch& eb) {
#pragma clang fp contract(off)
  const dks_particle_set e = eb.at(b);
  Geometry* g = reinterpret_cast<Geometry*>(reinterpret_cast<char*>(geo) + (size_t)b * geo_stride);
  if (a.zero_len > 0) {
    unsigned* z = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(g) + a.zero_off);
    for (int i = threadIdx.x; i < a.zero_len; i += blockDim.x) z[i] = 0u;
  }
  __shared__ double red[6][256];
  if (a.fitted) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const double* pp = partial + (size_t)b * partial_stride;
    for (int i = threadIdx.x; i < a.nblocks; i += blockDim.x) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(lo[d], pp[i * 6 + d]);
        hi[d] = fmax(hi[d], pp[i * 6 + 3 + d]);
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[d][threadIdx.x] = lo[d];
      red[3 + d][threadIdx.x] = hi[d];
    }
  }
  __syncthreads();
  if (a.fitted) {
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
          red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x != 0) return;
  double h[3], origin[3];
  if (a.fitted) {
    double lo[3], hi[3];
    const bool empty = eb.n(e) <= 0;
    for (int d = 0; d < 3; ++d) {
      lo[d] = empty ? 0.0 : red[d][0];
      hi[d] = empty ? 0.0 : red[3 + d][0];
    }
    double hc = 0.0;
    for (int d = 0; d < 3; ++d) hc = fmax(hc, (hi[d] - lo[d]) / (double)(a.n[d] - 3));
    if (!(hc > 0.0)) hc = 1.0;
    for (int d = 0; d < 3; ++d) {
      h[d] = hc;
      origin[d] = 0.5 * (lo[d] + hi[d]) - 0.5 * (double)(a.n[d] - 1) * hc;
    }
  } else {
    for (int d = 0; d < 3; ++d) {
      h[d] = a.h[d];
      origin[d] = a.origin[d];
    }
  }
  const double coulomb = 1.0 / (4.0 * M_PI * kEps0);
  double scale;
  if (a.mode == 0) scale = coulomb;                                   // rho given in C/m^3
  else if (a.fitted) scale = coulomb * e.q / h[0];                // spectrum built for h = 1 m
  else scale = coulomb * e.q / (h[0] * h[1] * h[2]);             // rho = q W / V
  for (int d = 0; d < 3; ++d) {
    g->h[d] = h[d];
    g->origin[d] = origin[d];
    g->inv_h[d] = 1.0 / h[d];
    g->grad_coef[d] = -1.0 / (2.0 * h[d]);
    g->origin_f[d] = (float)origin[d];
    g->inv_h_f[d] = (float)g->inv_h[d];
    g->grad_coef_f[d] = (float)g->grad_coef[d];
  }
  g->conv_scale = scale;
  g->conv_scale_f = (float)scale;
  g->n_outside = 0;
  if (e.n_outside) *e.n_outside = 0;
}

__global__ __launch_bounds__(256) void k_geometry(const double* partial, size_t partial_stride,
                                                  Geometry* geo, size_t geo_stride, GeoArgs a,
                                                  ElemBatch eb) {
  geometry_of(blockIdx.x, partial, partial_stride, geo, geo_stride, a, eb);
}

// The geometry of element blockIdx.y (by workgroup 0 of the row) and the
// zero fill of that element's deposit mesh (by every workgroup of the row):
// one launch for two steps that do not depend on each other.
__global__ __launch_bounds__(256) void k_geometry_zero(const double* partial, size_t partial_stride,
                                                       Geometry* geo, size_t geo_stride, GeoArgs a,
                                                       ElemBatch eb, void* zbase, size_t zstride, size_t zbytes) {
  if (blockIdx.x == 0) geometry_of(blockIdx.y, partial, partial_stride, geo, geo_stride, a, eb);
  char* p = reinterpret_cast<char*>(zbase) + (size_t)blockIdx.y * zstride;
  const size_t n16 = zbytes / 16;
  uint4* q = reinterpret_cast<uint4*>(p);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    q[i] = make_uint4(0, 0, 0, 0);
  const size_t tail = zbytes - n16 * 16;
  if (blockIdx.x == 0 && threadIdx.x < tail) p[n16 * 16 + threadIdx.x] = 0;
}

// rho = W * q / V for the deposit-only entry point (factor formed in FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_weights_to_density(const T* W, T* rho, size_t n, const Geometry* g,
                                                            double q) {
  const double f = q / (g->h[0] * g->h[1] * g->h[2]);
  const T ft = (T)f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    rho[i] = W[i] * ft;
}

// ---------------------------------------------------------------------------
// Central-difference field from phi with its ghost layer: E_d = -(phi(+e_d)
// - phi(-e_d)) / (2 h_d) on the physical nodes, written [3][nz][ny][nx].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gradient(const T* __restrict__ phi, T* __restrict__ out,
                                                  const Geometry* g, MeshDims m) {
  const int z = blockIdx.y;
  const int nx = m.nx, ny = m.ny, nz = m.nz;
  const int i2 = blockIdx.x * blockDim.x + threadIdx.x;    // y * nx + x within plane z
  if (i2 >= nx * ny) return;
  const int y = i2 / nx, x = i2 - y * nx;
  const T cx = Geo<T>::grad(g, 0), cy = Geo<T>::grad(g, 1), cz = Geo<T>::grad(g, 2);
  const size_t py = (size_t)nx + 2, pz = (size_t)(nx + 2) * (ny + 2);
  const size_t c = (size_t)(z + 1) * pz + (size_t)(y + 1) * py + (size_t)(x + 1);
  const size_t i = (size_t)z * nx * ny + i2;
  const size_t total = (size_t)nx * ny * nz;
  out[i] = cx * (phi[c + 1] - phi[c - 1]);
  out[total + i] = cy * (phi[c + py] - phi[c - py]);
  out[2 * total + i] = cz * (phi[c + pz] - phi[c - pz]);
}

// ---------------------------------------------------------------------------
// CIC gather of a [3][nz][ny][nx] mesh field at unsorted particles (the
// stand-alone gather entry point).  Outside particles receive 0.
// ---------------------------------------------------------------------------
template <typename T, int SCH>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ E, const T* __restrict__ px,
                                                const T* __restrict__ py, const T* __restrict__ pz,
                                                T* __restrict__ qx, T* __restrict__ qy, T* __restrict__ qz,
                                                int64_t n, const Geometry* g, MeshDims m) {
  constexpr int WD = Scheme<SCH>::width;
  const T ox = Geo<T>::origin(g, 0), oy = Geo<T>::origin(g, 1), oz = Geo<T>::origin(g, 2);
  const T ix = Geo<T>::inv_h(g, 0), iy = Geo<T>::inv_h(g, 1), iz = Geo<T>::inv_h(g, 2);
  const int nx = m.nx, ny = m.ny, nz = m.nz;
  const size_t total = (size_t)nx * ny * nz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    T wx[WD], wy[WD], wz[WD];
    int kx, ky, kz;
    // every axis is evaluated (its node and weights are set either way)
    const bool inx = axis_stencil<T, SCH>(cell_coord(px[i], ox, ix), nx, kx, wx);
    const bool iny = axis_stencil<T, SCH>(cell_coord(py[i], oy, iy), ny, ky, wy);
    const bool inz = axis_stencil<T, SCH>(cell_coord(pz[i], oz, iz), nz, kz, wz);
    const bool in = inx && iny && inz;
    T ax = 0, ay = 0, az = 0;
    if (in) {
      const int bx = kx + Scheme<SCH>::lo, by = ky + Scheme<SCH>::lo, bz = kz + Scheme<SCH>::lo;
#pragma unroll
      for (int cz = 0; cz < WD; ++cz)
#pragma unroll
        for (int cy = 0; cy < WD; ++cy)
#pragma unroll
          for (int cx = 0; cx < WD; ++cx) {
            const size_t node = ((size_t)(bz + cz) * ny + (by + cy)) * nx + (bx + cx);
            const T wgt = wz[cz] * wy[cy] * wx[cx];
            ax += wgt * E[node];
            ay += wgt * E[total + node];
            az += wgt * E[2 * total + node];
          }
    }
    qx[i] = ax;
    qy[i] = ay;
    qz[i] = az;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, unsigned cap) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

template <typename T>
hipError_t launch_bbox(const ElemBatch& eb, int batch, double* partial, size_t partial_stride, int* nblocks_out,
                       hipStream_t s) {
  const unsigned nb = grid_for(eb.max_np, kBboxBlocks);
  *nblocks_out = (int)nb;
  hipLaunchKernelGGL(k_bbox<T>, dim3(nb, batch), dim3(256), 0, s, eb, partial, partial_stride);
  return hipGetLastError();
}

hipError_t launch_geometry(const double* partial, size_t partial_stride, Geometry* geo, size_t geo_stride,
                           const GeoArgs& a, const ElemBatch& eb, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_geometry, dim3(batch), dim3(256), 0, s, partial, partial_stride, geo, geo_stride, a, eb);
  return hipGetLastError();
}

hipError_t launch_geometry_zero(const double* partial, size_t partial_stride, Geometry* geo, size_t geo_stride,
                                const GeoArgs& a, const ElemBatch& eb, int batch, void* zbase, size_t zstride,
                                size_t zbytes, hipStream_t s) {
  const unsigned nb = grid_for((int64_t)(zbytes / 16 + 1), 8192);
  hipLaunchKernelGGL(k_geometry_zero, dim3(nb, batch), dim3(256), 0, s, partial, partial_stride, geo, geo_stride, a,
                     eb, zbase, zstride, zbytes);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_weights_to_density(const void* W, void* rho, size_t n, const Geometry* g, double q,
                                     hipStream_t s) {
  hipLaunchKernelGGL(k_weights_to_density<T>, dim3(grid_for((int64_t)n, 8192)), dim3(256), 0, s, (const T*)W,
                     (T*)rho, n, g, q);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gradient(const void* phi, void* out, const Geometry* g, const MeshDims& m, hipStream_t s) {
  const unsigned gx = (unsigned)(((int64_t)m.nx * m.ny + 255) / 256);
  hipLaunchKernelGGL(k_gradient<T>, dim3(gx, m.nz), dim3(256), 0, s, (const T*)phi, (T*)out, g, m);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const void* E, const void* x, const void* y, const void* z, void* ex, void* ey, void* ez,
                         int64_t n, const Geometry* g, const MeshDims& m, int scheme, hipStream_t s) {
  if (n == 0) return hipSuccess;
  auto go = [&](auto sc) {
    hipLaunchKernelGGL((k_gather<T, decltype(sc)::value>), dim3(grid_for(n, 65535u * 4)), dim3(256), 0, s,
                       (const T*)E, (const T*)x, (const T*)y, (const T*)z, (T*)ex, (T*)ey, (T*)ez, n, g, m);
  };
  if (scheme == kSchemeNGP) go(std::integral_constant<int, kSchemeNGP>{});
  else if (scheme == kSchemeTSC) go(std::integral_constant<int, kSchemeTSC>{});
  else go(std::integral_constant<int, kSchemeCIC>{});
  return hipGetLastError();
}

#define DKS_INSTANTIATE(T)                                                                                   \
  template hipError_t launch_bbox<T>(const ElemBatch&, int, double*, size_t, int*, hipStream_t);           \
  template hipError_t launch_weights_to_density<T>(const void*, void*, size_t, const Geometry*, double,      \
                                                   hipStream_t);                                             \
  template hipError_t launch_gradient<T>(const void*, void*, const Geometry*, const MeshDims&, hipStream_t); \
  template hipError_t launch_gather<T>(const void*, const void*, const void*, const void*, void*, void*,     \
                                       void*, int64_t, const Geometry*, const MeshDims&, int, hipStream_t);
DKS_INSTANTIATE(float)
DKS_INSTANTIATE(double)
#undef DKS_INSTANTIATE

}  // namespace dks
