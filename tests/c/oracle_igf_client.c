/* Exercises the oracle's C part (oracle/igf_quad.c) for an AddressSanitizer
 * build: the octant table and the pointwise entry agree at every offset of
 * small, odd-shaped octants, and bad arguments are refused. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_igf_octant(int nx, int ny, int nz, double hx, double hy, double hz, double* out);
int oracle_igf_at(int64_t m, const int64_t* a, const int64_t* b, const int64_t* c, double hx, double hy, double hz,
                  double* out);
void oracle_set_threads(int n);

int main(void) {
  const int shapes[3][3] = {{0, 0, 0}, {3, 1, 2}, {6, 5, 4}};
  oracle_set_threads(2);
  for (int s = 0; s < 3; ++s) {
    const int nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2];
    const int64_t m = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    double* oct = malloc(sizeof(double) * (size_t)m);
    double* at = malloc(sizeof(double) * (size_t)m);
    int64_t* a = malloc(sizeof(int64_t) * (size_t)m);
    int64_t* b = malloc(sizeof(int64_t) * (size_t)m);
    int64_t* c = malloc(sizeof(int64_t) * (size_t)m);
    if (!oct || !at || !a || !b || !c) return 2;
    if (oracle_igf_octant(nx, ny, nz, 1.0, 1.5, 0.75, oct) != 0) return 3;
    for (int64_t e = 0; e < m; ++e) {
      a[e] = e % (nx + 1);
      b[e] = (e / (nx + 1)) % (ny + 1);
      c[e] = e / ((int64_t)(nx + 1) * (ny + 1));
      if (e % 2) a[e] = -a[e];      /* the integral is even in each axis */
    }
    if (oracle_igf_at(m, a, b, c, 1.0, 1.5, 0.75, at) != 0) return 4;
    for (int64_t e = 0; e < m; ++e)
      if (oct[e] != at[e]) {
        printf("mismatch %d %lld\n", s, (long long)e);
        return 5;
      }
    free(oct);
    free(at);
    free(a);
    free(b);
    free(c);
  }
  double v;
  if (oracle_igf_octant(-1, 0, 0, 1.0, 1.0, 1.0, &v) != -1) return 6;
  if (oracle_igf_at(1, NULL, NULL, NULL, 1.0, 1.0, 1.0, &v) != -1) return 7;
  printf("ok\n");
  return 0;
}
