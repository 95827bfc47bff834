/*
 * Integrated Green's function of the free-space kernel, evaluated in 113-bit
 * floating point.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; nothing in the
 * product path does.  It shares no code, table or constant with the HIP
 * library.
 *
 * Definition (paper, section "FFT-based Convolutions": the kernel 1/r of the
 * equation after the convolution solution, integrated over one mesh cell):
 *
 *   G_int(a,b,c) = integral over |u - a hx| <= hx/2, |v - b hy| <= hy/2,
 *                  |w - c hz| <= hz/2 of du dv dw / sqrt(u^2 + v^2 + w^2).
 *
 * It is written out exactly: with an antiderivative F whose mixed third
 * derivative is 1/r,
 *
 *   F(x,y,z) = yz ln(x + r) + xz ln(y + r) + xy ln(z + r)
 *              - x^2/2 atan(yz / (x r)) - y^2/2 atan(xz / (y r))
 *              - z^2/2 atan(xy / (z r)),        r = |(x, y, z)|,
 *
 * the integral over the cell is the alternating sum of F over the cell's
 * eight corners.  The sum cancels: at an offset of R cells, F is of order
 * R^2 ln R cell areas while G_int is of order 1/R, so about 3 log10(R) digits
 * are lost (9 at 256 cells).  FP64 would keep only 7 of its 16; this file
 * evaluates F and the sum in __float128 (34 digits), which keeps at least 24
 * digits at every offset below 10^4 cells, and rounds once to FP64.  No case
 * split, no quadrature, no table: the same expression at every offset.
 *
 * The corners are the half-integer lattice x = (a - 1/2) hx, a = 0 .. nx + 1
 * (same in y, z); no coordinate is 0 there.  F is continuous across the
 * coordinate planes (each atan that jumps there is multiplied by the square
 * of that coordinate), so the centre cell, which straddles them, needs no
 * special case.
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>

typedef __float128 q_t;

static q_t antiderivative(q_t x, q_t y, q_t z) {
  const q_t r = sqrtq(x * x + y * y + z * z);
  return y * z * logq(x + r) + x * z * logq(y + r) + x * y * logq(z + r) -
         0.5Q * x * x * atanq(y * z / (x * r)) - 0.5Q * y * y * atanq(x * z / (y * r)) -
         0.5Q * z * z * atanq(x * y / (z * r));
}

/* G_int at one integer offset (a, b, c) >= 0: the corner sum of F. */
static q_t cell_integral(int64_t a, int64_t b, int64_t c, q_t hx, q_t hy, q_t hz) {
  q_t total = 0.0Q;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const q_t x = ((q_t)a - 0.5Q + dx) * hx;
        const q_t y = ((q_t)b - 0.5Q + dy) * hy;
        const q_t z = ((q_t)c - 0.5Q + dz) * hz;
        const q_t f = antiderivative(x, y, z);
        /* sign (-1)^(3 - dx - dy - dz): + at the far corner (1, 1, 1) */
        if (((dx + dy + dz) & 1) == 1) total += f;
        else total -= f;
      }
  return total;
}

/* Number of OpenMP threads the loops below use. */
void oracle_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

/*
 * G_int on the octant a in [0, nx], b in [0, ny], c in [0, nz], written to
 * out[(c * (ny + 1) + b) * (nx + 1) + a].  F is evaluated once per lattice
 * corner; each cell then takes the same signed corner sum, in the same order,
 * as cell_integral (so both entry points give identical values).  Returns 0,
 * or -1 on bad arguments or allocation failure.
 */
int oracle_igf_octant(int nx, int ny, int nz, double hx, double hy, double hz, double* out) {
  if (nx < 0 || ny < 0 || nz < 0 || !(hx > 0) || !(hy > 0) || !(hz > 0) || !out) return -1;
  const int64_t Lx = nx + 2, Ly = ny + 2, Lz = nz + 2;
  q_t* F = (q_t*)malloc(sizeof(q_t) * (size_t)(Lx * Ly * Lz));
  if (!F) return -1;
  const q_t qx = hx, qy = hy, qz = hz;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < Lz; ++k)
    for (int64_t j = 0; j < Ly; ++j)
      for (int64_t i = 0; i < Lx; ++i)
        F[(k * Ly + j) * Lx + i] =
            antiderivative(((q_t)i - 0.5Q) * qx, ((q_t)j - 0.5Q) * qy, ((q_t)k - 0.5Q) * qz);
  const int64_t Ox = nx + 1, Oy = ny + 1, Oz = nz + 1;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < Oz; ++c)
    for (int64_t b = 0; b < Oy; ++b)
      for (int64_t a = 0; a < Ox; ++a) {
        q_t total = 0.0Q;
        for (int dz = 0; dz < 2; ++dz)
          for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
              const q_t f = F[((c + dz) * Ly + (b + dy)) * Lx + (a + dx)];
              if (((dx + dy + dz) & 1) == 1) total += f;
              else total -= f;
            }
        out[(c * Oy + b) * Ox + a] = (double)total;
      }
  free(F);
  return 0;
}

/*
 * G_int at m arbitrary integer offsets (a[i], b[i], c[i]); negative offsets
 * give the value at |offset| (the integral is even in each axis).  Returns 0,
 * or -1 on bad arguments.
 */
int oracle_igf_at(int64_t m, const int64_t* a, const int64_t* b, const int64_t* c, double hx, double hy, double hz,
                  double* out) {
  if (m < 0 || !(hx > 0) || !(hy > 0) || !(hz > 0) || (m > 0 && (!a || !b || !c || !out))) return -1;
  const q_t qx = hx, qy = hy, qz = hz;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const int64_t ai = a[i] < 0 ? -a[i] : a[i];
    const int64_t bi = b[i] < 0 ? -b[i] : b[i];
    const int64_t ci = c[i] < 0 ? -c[i] : c[i];
    out[i] = (double)cell_integral(ai, bi, ci, qx, qy, qz);
  }
  return 0;
}
