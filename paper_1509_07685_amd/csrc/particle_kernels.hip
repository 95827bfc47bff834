// Particle <-> mesh kernels of the PM step: bounding box of the bunch (the
// particle-fitted mesh of the PM section), per-solve geometry in FP64,
// cloud-in-cell deposit and gather (the "NGP, CIC, TSI" interpolation of the
// OPAL structure figure), and the central-difference field (its D-operators).

#include <math.h>

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
// Bounding box, stage 1: each block reduces a grid-stride share of the
// particles of batch element blockIdx.y to (min x, min y, min z, max x, max y,
// max z) and writes it to its partial slot.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_bbox(PtrBatch xs, PtrBatch ys, PtrBatch zs, BatchScalars bs,
                                              double* partial, size_t partial_stride) {
  const int b = blockIdx.y;
  const T* p[3] = {(const T*)xs.p[b], (const T*)ys.p[b], (const T*)zs.p[b]};
  const int64_t n = bs.np[b];
  T lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = INFINITY;
    hi[d] = -INFINITY;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T v = p[d][i];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  }
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
__global__ __launch_bounds__(256) void k_geometry(const double* partial, size_t partial_stride,
                                                  Geometry* geo, size_t geo_stride, GeoArgs a,
                                                  BatchScalars bs, PtrBatch counters) {
#pragma clang fp contract(off)
  const int b = blockIdx.x;
  Geometry* g = reinterpret_cast<Geometry*>(reinterpret_cast<char*>(geo) + (size_t)b * geo_stride);
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
    const bool empty = bs.np[b] <= 0;
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
  else if (a.fitted) scale = coulomb * bs.q[b] / h[0];                // spectrum built for h = 1 m
  else scale = coulomb * bs.q[b] / (h[0] * h[1] * h[2]);             // rho = q W / V
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
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counters.p[b]);
  if (cnt) *cnt = 0;
}

// Zero `count` elements of batch element blockIdx.y (vectorised, 16 B per store).
__global__ __launch_bounds__(256) void k_zero(void* base, size_t stride_bytes, size_t bytes) {
  char* p = reinterpret_cast<char*>(base) + (size_t)blockIdx.y * stride_bytes;
  const size_t n16 = bytes / 16;
  uint4* q = reinterpret_cast<uint4*>(p);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    q[i] = make_uint4(0, 0, 0, 0);
  const size_t tail = bytes - n16 * 16;
  if (blockIdx.x == 0 && threadIdx.x < tail) p[n16 * 16 + threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// CIC deposit of dimensionless weights W (charge = q W) with hardware
// floating-point atomics.  Out-of-mesh particles are counted per wavefront.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_deposit(PtrBatch xs, PtrBatch ys, PtrBatch zs, BatchScalars bs,
                                                 T* W, size_t w_stride, const Geometry* geo,
                                                 size_t geo_stride, MeshDims m, PtrBatch counters) {
  const int b = blockIdx.y;
  const T* px = (const T*)xs.p[b];
  const T* py = (const T*)ys.p[b];
  const T* pz = (const T*)zs.p[b];
  T* w = W + (size_t)b * w_stride;
  const Geometry* g = geo_at(geo, geo_stride, b);
  const T ox = Geo<T>::origin(g, 0), oy = Geo<T>::origin(g, 1), oz = Geo<T>::origin(g, 2);
  const T ix = Geo<T>::inv_h(g, 0), iy = Geo<T>::inv_h(g, 1), iz = Geo<T>::inv_h(g, 2);
  unsigned long long* cnt = counters.p[b] ? reinterpret_cast<unsigned long long*>(counters.p[b])
                                          : &const_cast<Geometry*>(g)->n_outside;
  const int64_t n = bs.np[b];
  const int nx = m.nx, ny = m.ny, nz = m.nz;
  const T ux = (T)(nx - 1), uy = (T)(ny - 1), uz = (T)(nz - 1);
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    bool outside = false;
    if (i < n) {
      const T sx = cell_coord(px[i], ox, ix);
      const T sy = cell_coord(py[i], oy, iy);
      const T sz = cell_coord(pz[i], oz, iz);
      if (sx >= (T)0 && sx <= ux && sy >= (T)0 && sy <= uy && sz >= (T)0 && sz <= uz) {
        const int jx = min((int)floor(sx), nx - 2);
        const int jy = min((int)floor(sy), ny - 2);
        const int jz = min((int)floor(sz), nz - 2);
        const T fx = sx - (T)jx, fy = sy - (T)jy, fz = sz - (T)jz;
        const T gx = (T)1 - fx, gy = (T)1 - fy, gz = (T)1 - fz;
        T* base = w + ((size_t)jz * ny + jy) * nx + jx;
        const size_t sy_ = nx, sz_ = (size_t)nx * ny;
        unsafeAtomicAdd(base, gz * gy * gx);
        unsafeAtomicAdd(base + 1, gz * gy * fx);
        unsafeAtomicAdd(base + sy_, gz * fy * gx);
        unsafeAtomicAdd(base + sy_ + 1, gz * fy * fx);
        unsafeAtomicAdd(base + sz_, fz * gy * gx);
        unsafeAtomicAdd(base + sz_ + 1, fz * gy * fx);
        unsafeAtomicAdd(base + sz_ + sy_, fz * fy * gx);
        unsafeAtomicAdd(base + sz_ + sy_ + 1, fz * fy * fx);
      } else {
        outside = true;
      }
    }
    const unsigned long long out_mask = __ballot(outside);
    if (out_mask != 0ull) {
      const unsigned long long active = __ballot(1);
      if ((int)(threadIdx.x & 63) == __ffsll((long long)active) - 1)
        atomicAdd(cnt, (unsigned long long)__popcll(out_mask));
    }
  }
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
// - phi(-e_d)) / (2 h_d) on the physical nodes.  INTERLEAVED writes
// [node][4] (x, y, z, 0) for the gather; otherwise [3][nz][ny][nx].
// ---------------------------------------------------------------------------
template <typename T, bool INTERLEAVED>
__global__ __launch_bounds__(256) void k_gradient(const T* __restrict__ phi, size_t phi_stride,
                                                  T* __restrict__ out, size_t out_stride,
                                                  const Geometry* geo, size_t geo_stride, MeshDims m) {
  const int b = blockIdx.z;
  const int z = blockIdx.y;
  const int nx = m.nx, ny = m.ny, nz = m.nz;
  const int i2 = blockIdx.x * blockDim.x + threadIdx.x;    // y * nx + x within plane z
  if (i2 >= nx * ny) return;
  const int y = i2 / nx, x = i2 - y * nx;
  const T* p = phi + (size_t)b * phi_stride;
  T* o = out + (size_t)b * out_stride;
  const Geometry* g = geo_at(geo, geo_stride, b);
  const T cx = Geo<T>::grad(g, 0), cy = Geo<T>::grad(g, 1), cz = Geo<T>::grad(g, 2);
  const size_t py = (size_t)nx + 2, pz = (size_t)(nx + 2) * (ny + 2);
  const size_t c = (size_t)(z + 1) * pz + (size_t)(y + 1) * py + (size_t)(x + 1);
  const T ex = cx * (p[c + 1] - p[c - 1]);
  const T ey = cy * (p[c + py] - p[c - py]);
  const T ez = cz * (p[c + pz] - p[c - pz]);
  const size_t i = (size_t)z * nx * ny + i2;
  if (INTERLEAVED) {
    typename Vec4<T>::type e;
    e.x = ex;
    e.y = ey;
    e.z = ez;
    e.w = (T)0;
    reinterpret_cast<typename Vec4<T>::type*>(o)[i] = e;
  } else {
    const size_t total = (size_t)nx * ny * nz;
    o[i] = ex;
    o[total + i] = ey;
    o[2 * total + i] = ez;
  }
}

// ---------------------------------------------------------------------------
// CIC gather with the deposit's weights.  INTERLEAVED reads [node][4];
// otherwise [3][nz][ny][nx].  Outside particles receive 0.
// ---------------------------------------------------------------------------
template <typename T, bool INTERLEAVED>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ E, size_t e_stride, PtrBatch xs,
                                                PtrBatch ys, PtrBatch zs, PtrBatch exs, PtrBatch eys,
                                                PtrBatch ezs, BatchScalars bs, const Geometry* geo,
                                                size_t geo_stride, MeshDims m) {
  const int b = blockIdx.y;
  const T* px = (const T*)xs.p[b];
  const T* py = (const T*)ys.p[b];
  const T* pz = (const T*)zs.p[b];
  T* qx = (T*)exs.p[b];
  T* qy = (T*)eys.p[b];
  T* qz = (T*)ezs.p[b];
  const T* e = E + (size_t)b * e_stride;
  const Geometry* g = geo_at(geo, geo_stride, b);
  const T ox = Geo<T>::origin(g, 0), oy = Geo<T>::origin(g, 1), oz = Geo<T>::origin(g, 2);
  const T ix = Geo<T>::inv_h(g, 0), iy = Geo<T>::inv_h(g, 1), iz = Geo<T>::inv_h(g, 2);
  const int64_t n = bs.np[b];
  const int nx = m.nx, ny = m.ny, nz = m.nz;
  const T ux = (T)(nx - 1), uy = (T)(ny - 1), uz = (T)(nz - 1);
  const size_t total = (size_t)nx * ny * nz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T sx = cell_coord(px[i], ox, ix);
    const T sy = cell_coord(py[i], oy, iy);
    const T sz = cell_coord(pz[i], oz, iz);
    T ax = 0, ay = 0, az = 0;
    if (sx >= (T)0 && sx <= ux && sy >= (T)0 && sy <= uy && sz >= (T)0 && sz <= uz) {
      const int jx = min((int)floor(sx), nx - 2);
      const int jy = min((int)floor(sy), ny - 2);
      const int jz = min((int)floor(sz), nz - 2);
      const T fx = sx - (T)jx, fy = sy - (T)jy, fz = sz - (T)jz;
      const T wx[2] = {(T)1 - fx, fx}, wy[2] = {(T)1 - fy, fy}, wz[2] = {(T)1 - fz, fz};
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const size_t node = ((size_t)(jz + cz) * ny + (jy + cy)) * nx + (jx + cx);
            const T wgt = wz[cz] * wy[cy] * wx[cx];
            if (INTERLEAVED) {
              const typename Vec4<T>::type v = reinterpret_cast<const typename Vec4<T>::type*>(e)[node];
              ax += wgt * v.x;
              ay += wgt * v.y;
              az += wgt * v.z;
            } else {
              ax += wgt * e[node];
              ay += wgt * e[total + node];
              az += wgt * e[2 * total + node];
            }
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
hipError_t launch_bbox(const PtrBatch& xs, const PtrBatch& ys, const PtrBatch& zs, const BatchScalars& bs,
                       int batch, double* partial, size_t partial_stride, int* nblocks_out, hipStream_t s) {
  int64_t maxn = 0;
  for (int b = 0; b < batch; ++b) maxn = std::max(maxn, bs.np[b]);
  const unsigned nb = grid_for(maxn, kBboxBlocks);
  *nblocks_out = (int)nb;
  hipLaunchKernelGGL(k_bbox<T>, dim3(nb, batch), dim3(256), 0, s, xs, ys, zs, bs, partial, partial_stride);
  return hipGetLastError();
}

hipError_t launch_geometry(const double* partial, size_t partial_stride, Geometry* geo, size_t geo_stride,
                           const GeoArgs& a, const BatchScalars& bs, const PtrBatch& counters, int batch,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_geometry, dim3(batch), dim3(256), 0, s, partial, partial_stride, geo, geo_stride, a, bs,
                     counters);
  return hipGetLastError();
}

hipError_t launch_zero(void* base, size_t stride_bytes, size_t bytes, int batch, hipStream_t s) {
  const unsigned nb = grid_for((int64_t)(bytes / 16 + 1), 8192);
  hipLaunchKernelGGL(k_zero, dim3(nb, batch), dim3(256), 0, s, base, stride_bytes, bytes);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_deposit(const PtrBatch& xs, const PtrBatch& ys, const PtrBatch& zs, const BatchScalars& bs,
                          int batch, void* W, size_t w_stride, const Geometry* geo, size_t geo_stride,
                          const MeshDims& m, const PtrBatch& counters, hipStream_t s) {
  int64_t maxn = 0;
  for (int b = 0; b < batch; ++b) maxn = std::max(maxn, bs.np[b]);
  if (maxn == 0) return hipSuccess;
  const unsigned nb = grid_for(maxn, 65535u * 4);
  hipLaunchKernelGGL(k_deposit<T>, dim3(nb, batch), dim3(256), 0, s, xs, ys, zs, bs, (T*)W, w_stride, geo,
                     geo_stride, m, counters);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_weights_to_density(const void* W, void* rho, size_t n, const Geometry* g, double q,
                                     hipStream_t s) {
  hipLaunchKernelGGL(k_weights_to_density<T>, dim3(grid_for((int64_t)n, 8192)), dim3(256), 0, s, (const T*)W,
                     (T*)rho, n, g, q);
  return hipGetLastError();
}

template <typename T, bool INTERLEAVED>
hipError_t launch_gradient(const void* phi, size_t phi_stride, void* out, size_t out_stride, const Geometry* geo,
                           size_t geo_stride, const MeshDims& m, int batch, hipStream_t s) {
  const unsigned gx = (unsigned)(((int64_t)m.nx * m.ny + 255) / 256);
  hipLaunchKernelGGL((k_gradient<T, INTERLEAVED>), dim3(gx, m.nz, batch), dim3(256), 0, s,
                     (const T*)phi, phi_stride, (T*)out, out_stride, geo, geo_stride, m);
  return hipGetLastError();
}

template <typename T, bool INTERLEAVED>
hipError_t launch_gather(const void* E, size_t e_stride, const PtrBatch& xs, const PtrBatch& ys,
                         const PtrBatch& zs, const PtrBatch& exs, const PtrBatch& eys, const PtrBatch& ezs,
                         const BatchScalars& bs, int batch, const Geometry* geo, size_t geo_stride,
                         const MeshDims& m, hipStream_t s) {
  int64_t maxn = 0;
  for (int b = 0; b < batch; ++b) maxn = std::max(maxn, bs.np[b]);
  if (maxn == 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather<T, INTERLEAVED>), dim3(grid_for(maxn, 65535u * 4), batch), dim3(256), 0, s,
                     (const T*)E, e_stride, xs, ys, zs, exs, eys, ezs, bs, geo, geo_stride, m);
  return hipGetLastError();
}

#define DKS_INSTANTIATE(T)                                                                                   \
  template hipError_t launch_bbox<T>(const PtrBatch&, const PtrBatch&, const PtrBatch&, const BatchScalars&, \
                                     int, double*, size_t, int*, hipStream_t);                               \
  template hipError_t launch_deposit<T>(const PtrBatch&, const PtrBatch&, const PtrBatch&,                   \
                                        const BatchScalars&, int, void*, size_t, const Geometry*, size_t,    \
                                        const MeshDims&, const PtrBatch&, hipStream_t);                      \
  template hipError_t launch_weights_to_density<T>(const void*, void*, size_t, const Geometry*, double,      \
                                                   hipStream_t);                                             \
  template hipError_t launch_gradient<T, true>(const void*, size_t, void*, size_t, const Geometry*, size_t,  \
                                               const MeshDims&, int, hipStream_t);                           \
  template hipError_t launch_gradient<T, false>(const void*, size_t, void*, size_t, const Geometry*, size_t, \
                                                const MeshDims&, int, hipStream_t);                          \
  template hipError_t launch_gather<T, true>(const void*, size_t, const PtrBatch&, const PtrBatch&,          \
                                             const PtrBatch&, const PtrBatch&, const PtrBatch&,              \
                                             const PtrBatch&, const BatchScalars&, int, const Geometry*,     \
                                             size_t, const MeshDims&, hipStream_t);                          \
  template hipError_t launch_gather<T, false>(const void*, size_t, const PtrBatch&, const PtrBatch&,         \
                                              const PtrBatch&, const PtrBatch&, const PtrBatch&,             \
                                              const PtrBatch&, const BatchScalars&, int, const Geometry*,    \
                                              size_t, const MeshDims&, hipStream_t);
DKS_INSTANTIATE(float)
DKS_INSTANTIATE(double)
#undef DKS_INSTANTIATE

}  // namespace dks
