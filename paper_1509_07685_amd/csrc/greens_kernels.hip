// Plan-time device work, all in FP64: twiddle tables (rounded to the dtype
// at the end), the cell-integrated Green's function on the octant of the
// doubled grid, and its spectrum.
//
// The paper computes the Green's function in a kernel of its own and FFTs it
// on a second stream, every solve (sequence diagram of the FFT Poisson solver).
// Here it is computed once per plan and kept resident.  G is the integral of
// 1/r over a mesh cell (the free-space kernel of the convolution-solution
// equation, integrated over the cell the charge of a node represents).  Near
// the origin it is the third mixed difference of a closed-form antiderivative
// over the cell corners; farther out that difference cancels catastrophically
// in FP64, so the cell integral is taken by a Gauss-Legendre product rule
// whose order is chosen by the distance (the integrand is analytic on the
// cell there), which reaches FP64 rounding.
//
// The doubled-grid kernel K[a] = G(min(a, 2n - a)) per axis is real and even,
// so its DFT is real and even and equals a type-I cosine transform of the
// octant: Ghat[k] = sum_{a=0..n} c_a G[a] cos(2 pi k a / 2n), c_0 = c_n = 1,
// c_a = 2 otherwise.  It is applied along x, y, z as three dense FP64
// contractions.

#include <math.h>

#include "dks_internal.h"

namespace dks {

template <typename T> struct alignas(2 * sizeof(T)) tw_cpx {
  T x, y;
};

// Per-pass Stockham twiddles: entry t * (R - 1) + (r - 1) = exp(-2 pi i r t / (Ns R)).
template <typename T>
__global__ void k_twiddle_pass(tw_cpx<T>* out, int Ns, int R) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Ns * (R - 1)) return;
  const int t = e / (R - 1), r = e - t * (R - 1) + 1;
  const long long den = (long long)Ns * R;
  const long long num = ((long long)r * t) % den;
  double s, c;
  sincospi(-2.0 * (double)num / (double)den, &s, &c);
  out[e] = tw_cpx<T>{(T)c, (T)s};
}

// exp(-2 pi i k / N), k < count.
template <typename T>
__global__ void k_twiddle_line(tw_cpx<T>* out, int N, int count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  double s, c;
  sincospi(-2.0 * (double)k / (double)N, &s, &c);
  out[k] = tw_cpx<T>{(T)c, (T)s};
}

// Antiderivative F with d^3 F / dx dy dz = 1 / r (no coordinate may be 0).
__device__ __forceinline__ double anti(double x, double y, double z) {
  const double r = sqrt(x * x + y * y + z * z);
  return y * z * log(x + r) + x * z * log(y + r) + x * y * log(z + r) - 0.5 * x * x * atan(y * z / (x * r)) -
         0.5 * y * y * atan(x * z / (y * r)) - 0.5 * z * z * atan(x * y / (z * r));
}

// G[c][b][a] for a <= nx, b <= ny, c <= nz (FP64).
__global__ __launch_bounds__(256) void k_igf_octant(double* G, int nx, int ny, int nz, double hx, double hy,
                                                    double hz, GLBands gl, int point) {
  const long long total = (long long)(nx + 1) * (ny + 1) * (nz + 1);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int a = (int)(e % (nx + 1));
  const long long rem = e / (nx + 1);
  const int b = (int)(rem % (ny + 1));
  const int c = (int)(rem / (ny + 1));
  const double hmax = fmax(hx, fmax(hy, hz));
  const double X = a * hx, Y = b * hy, Z = c * hz;
  if (point && (a | b | c)) {
    // point kernel of the brute-force convolution: the cell volume over r
    G[e] = hx * hy * hz / sqrt(X * X + Y * Y + Z * Z);
    return;
  }
  const double D = sqrt(X * X + Y * Y + Z * Z) / hmax;
  double g;
  if (D < gl.lo[0]) {
    g = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const double sgn = ((3 - dx - dy - dz) & 1) ? -1.0 : 1.0;
          g += sgn * anti((a - 0.5 + dx) * hx, (b - 0.5 + dy) * hy, (c - 0.5 + dz) * hz);
        }
  } else {
    int band = 0;
    for (int i = 1; i < gl.nb; ++i)
      if (D >= gl.lo[i]) band = i;
    const int m = gl.m[band];
    double acc = 0.0;
    for (int i = 0; i < m; ++i) {
      const double xi = (a + 0.5 * gl.t[band][i]) * hx;
      for (int j = 0; j < m; ++j) {
        const double yj = (b + 0.5 * gl.t[band][j]) * hy;
        const double wij = gl.w[band][i] * gl.w[band][j];
        double inner = 0.0;
        for (int k = 0; k < m; ++k) {
          const double zk = (c + 0.5 * gl.t[band][k]) * hz;
          inner += gl.w[band][k] / sqrt(xi * xi + yj * yj + zk * zk);
        }
        acc += wij * inner;
      }
    }
    g = acc * (hx * hy * hz / 8.0);
  }
  G[e] = g;
}

// Cosine matrix of one axis: M[k][a] = c_a cos(2 pi (k a mod N) / N), k, a <= n, N = 2n.
__global__ void k_cos_matrix(double* M, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = n + 1;
  if (e >= L * L) return;
  const int k = e / L, a = e - k * L;
  const long long N = 2LL * n;
  const long long num = ((long long)k * a) % N;
  const double c = (a == 0 || a == n) ? 1.0 : 2.0;
  M[e] = c * cospi(2.0 * (double)num / (double)N);
}

// out(r, k) = sum_a M[k][a] in(r, a) along one axis of an [n2+1][n1+1][n0+1]
// FP64 array: a dense (rows x L) by (L x L) product on the FP64 matrix cores.
// Row r = (rh, rl) with rl < Llo addresses rh * Shi + rl * Slo; the
// contracted index steps by Sa.  A workgroup of four wavefronts computes a
// 64 x 64 output tile, each wavefront a 32 x 32 quarter as 2 x 2 tiles of
// v_mfma_f64_16x16x4 (lane l holds A(l % 16, l / 16) and B(l / 16, l % 16)
// of the 16 x 4 and 4 x 16 operands, and D(4 e + l / 16, l % 16) in element
// e of the 16 x 16 result).  16-deep chunks of the contraction are staged in
// LDS, zero-filled past L.  Workgroup b runs on XCD b % 8 (round-robin
// dispatch); the k tiles of one row tile are consecutive on the same XCD, so
// its input rows come from that XCD's L2 after the first.
typedef double dks_dbl4 __attribute__((ext_vector_type(4)));
constexpr int kXcdGroups = 8;

template <bool AFAST>
__global__ __launch_bounds__(256) void k_apply_axis(const double* __restrict__ in, double* __restrict__ out,
                                                    const double* __restrict__ M, int L, long long nrows,
                                                    int Llo, long long Shi, long long Slo, long long Sa, int nrb,
                                                    int nkb) {
  __shared__ double sIn[16][64 + 1];
  __shared__ double sM[16][64 + 1];
  const int b = blockIdx.x;
  const int seq = b / kXcdGroups;
  const int rb = (seq / nkb) * kXcdGroups + b % kXcdGroups, kb = seq % nkb;
  if (rb >= nrb) return;
  const int tid = threadIdx.x;
  const long long r0 = (long long)rb * 64;
  const int k0 = kb * 64;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wk = (wave & 1) * 32;
  const int fi = lane & 15, fk = lane >> 4;
  // Staging map, fixed per thread: AFAST (contracted index contiguous in
  // memory) takes 16 consecutive a of four rows, otherwise 64 consecutive
  // rows of four a; the matrix always 16 consecutive a of four k.
  const int sa = AFAST ? (tid & 15) : (tid >> 6);
  const int sr = AFAST ? (tid >> 4) : (tid & 63);
  long long base[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long r = r0 + (AFAST ? sr + 16 * q : sr);
    const long long rh = r / Llo, rl = r - rh * Llo;
    base[q] = r < nrows ? rh * Shi + rl * Slo : -1;
  }
  const int ma = tid & 15, mk = tid >> 4;
  dks_dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dks_dbl4{0.0, 0.0, 0.0, 0.0};
  // chunk a0's operands are loaded into registers while chunk a0 - 16 is
  // multiplied
  double vIn[4], vM[4];
  auto load = [&](int a0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = a0 + (AFAST ? sa : sa + 4 * q);
      vIn[q] = (base[q] >= 0 && a < L) ? in[base[q] + a * Sa] : 0.0;
      const int k = k0 + mk + 16 * q, am = a0 + ma;
      vM[q] = (k < L && am < L) ? M[(long long)k * L + am] : 0.0;
    }
  };
  load(0);
  for (int a0 = 0; a0 < L; a0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sIn[AFAST ? sa : sa + 4 * q][AFAST ? sr + 16 * q : sr] = vIn[q];
      sM[ma][mk + 16 * q] = vM[q];
    }
    __syncthreads();
    if (a0 + 16 < L) load(a0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = sIn[kk + fk][wr + 16 * i + fi];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = sM[kk + fk][wk + 16 * j + fi];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long long r = r0 + wr + 16 * i + 4 * e + fk;
      if (r >= nrows) continue;
      const long long rh = r / Llo, rl = r - rh * Llo;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int k = k0 + wk + 16 * j + fi;
        if (k < L) out[rh * Shi + rl * Slo + (long long)k * Sa] = acc[i][j][e];
      }
    }
}

// Ghat (dtype) in the layout the z pass reads, times 1 / (Nx Ny Nz) formed
// in FP64: [ky][kx / W][kz][kx % W] for the z pass's tile width W, so the
// values one z-pass workgroup needs (one ky, W columns, every kz) are one
// contiguous block.  cs (a multiple of W) columns per ky.
template <typename T>
__global__ __launch_bounds__(256) void k_green_pack(const double* __restrict__ G64, T* __restrict__ out, int nx,
                                                    int ny, int nz, int cs, int W, double inv_ntot) {
  const long long total = (long long)(nx + 1) * (ny + 1) * (nz + 1);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int a = (int)(e % (nx + 1));
  const long long rem = e / (nx + 1);
  const int b = (int)(rem % (ny + 1));
  const int c = (int)(rem / (ny + 1));
  const long long tile = (long long)b * (cs / W) + a / W;
  out[(tile * (nz + 1) + c) * W + a % W] = (T)(G64[e] * inv_ntot);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_twiddle_pass(void* out, int Ns, int R, hipStream_t s) {
  const int n = Ns * (R - 1);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_twiddle_pass<T>, dim3((n + 255) / 256), dim3(256), 0, s, (tw_cpx<T>*)out, Ns, R);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_twiddle_line(void* out, int N, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddle_line<T>, dim3((count + 255) / 256), dim3(256), 0, s, (tw_cpx<T>*)out, N, count);
  return hipGetLastError();
}

hipError_t launch_igf_octant(double* G, const int n[3], const double h[3], const GLBands& gl, int point,
                             hipStream_t s) {
  const long long total = (long long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
  hipLaunchKernelGGL(k_igf_octant, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, G, n[0], n[1], n[2],
                     h[0], h[1], h[2], gl, point);
  return hipGetLastError();
}

hipError_t launch_cos_matrix(double* M, int n, hipStream_t s) {
  const int L = n + 1;
  hipLaunchKernelGGL(k_cos_matrix, dim3((L * L + 255) / 256), dim3(256), 0, s, M, n);
  return hipGetLastError();
}

// axis 0 = x, 1 = y, 2 = z of an [(n2+1)][(n1+1)][(n0+1)] array.
hipError_t launch_apply_axis(const double* in, double* out, const double* M, const int n[3], int axis,
                             hipStream_t s) {
  const long long L0 = n[0] + 1, L1 = n[1] + 1, L2 = n[2] + 1;
  long long nrows, Shi, Slo, Sa;
  int Llo, L;
  if (axis == 0) {          // rows (c, b): base (c * L1 + b) * L0
    L = (int)L0; nrows = L1 * L2; Llo = (int)L1; Shi = L0 * L1; Slo = L0; Sa = 1;
  } else if (axis == 1) {   // rows (c, a)
    L = (int)L1; nrows = L0 * L2; Llo = (int)L0; Shi = L0 * L1; Slo = 1; Sa = L0;
  } else {                  // rows (b, a)
    L = (int)L2; nrows = L0 * L1; Llo = (int)L0; Shi = L0; Slo = 1; Sa = L0 * L1;
  }
  const int nrb = (int)((nrows + 63) / 64), nkb = (L + 63) / 64;
  const long long blocks = (long long)(nrb + kXcdGroups - 1) / kXcdGroups * kXcdGroups * nkb;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (Sa == 1)
    hipLaunchKernelGGL(k_apply_axis<true>, dim3((unsigned)blocks), dim3(256), 0, s, in, out, M, L, nrows, Llo, Shi,
                       Slo, Sa, nrb, nkb);
  else
    hipLaunchKernelGGL(k_apply_axis<false>, dim3((unsigned)blocks), dim3(256), 0, s, in, out, M, L, nrows, Llo, Shi,
                       Slo, Sa, nrb, nkb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_green_pack(const double* G64, void* out, const int n[3], int cs, int W, double inv_ntot,
                             hipStream_t s) {
  if (W < 1 || cs % W != 0) return hipErrorInvalidValue;
  const long long total = (long long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
  hipLaunchKernelGGL(k_green_pack<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, G64, (T*)out, n[0],
                     n[1], n[2], cs, W, inv_ntot);
  return hipGetLastError();
}

template hipError_t launch_twiddle_pass<float>(void*, int, int, hipStream_t);
template hipError_t launch_twiddle_pass<double>(void*, int, int, hipStream_t);
template hipError_t launch_twiddle_line<float>(void*, int, int, hipStream_t);
template hipError_t launch_twiddle_line<double>(void*, int, int, hipStream_t);
template hipError_t launch_green_pack<float>(const double*, void*, const int*, int, int, double, hipStream_t);
template hipError_t launch_green_pack<double>(const double*, void*, const int*, int, int, double, hipStream_t);

}  // namespace dks
