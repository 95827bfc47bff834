// Host-only harness of the FFT plan invariant checker (csrc/fft_plan_check.h).
//
// It builds 1-D plans the way the library's plan code does (radix-8 passes,
// then one radix-4 or radix-2 pass, then radix-3 passes; the widest
// power-of-two tile of at most 128 bytes per row whose LDS tile fits the
// budget, x rows padded by one column), for every transform length the
// library accepts, and prints, for each set of engine constants and each
// role, how many plans break each invariant.  It also plants one mistake per
// invariant and prints the code the checker gives it.
//
//   g++ -std=c++17 -I paper_1509_07685_amd/csrc tests/c/plan_check.cpp -o plan_check
#include <cstdio>
#include <cstring>
#include <vector>

#include "fft_plan_check.h"

using namespace dks;

struct Plan {
  int N, npass, W, logW, LD;
  int R[12], Ns[12], tw_off[12];
};

static std::vector<int> radices(int N) {
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

static Plan make(int N, int W, bool padded) {
  Plan P;
  std::memset(&P, 0, sizeof(P));
  std::vector<int> r = radices(N);
  P.N = N;
  P.npass = (int)r.size();
  P.W = W;
  while ((1 << P.logW) < W) ++P.logW;
  P.LD = padded ? W + 1 : W;
  int Ns = 1, off = 0;
  for (size_t p = 0; p < r.size(); ++p) {
    P.R[p] = r[p];
    P.Ns[p] = Ns;
    P.tw_off[p] = off;
    if (p > 0) off += Ns * (r[p] - 1);
    Ns *= r[p];
  }
  return P;
}

static int width(int N, int csize, bool padded, int lds_budget) {
  int W = 128 / csize;
  while (W > 1 && (long long)N * (padded ? W + 1 : W) * csize > lds_budget) W >>= 1;
  return W;
}

static bool is23(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

struct Constants {
  const char* name;
  int lds_budget;
  int threads[2];   // FP32, FP64
  int tile_reals;
};

int main() {
  const Constants sets[2] = {{"committed", 65536, {512, 256}, 16}, {"variant_lds32k_t256", 32768, {256, 128}, 16}};
  for (const Constants& K : sets) {
    for (int dt = 0; dt < 2; ++dt) {
      const int csize = dt == 0 ? 8 : 16;
      EngineLimits L;
      L.threads = K.threads[dt];
      L.emax = K.lds_budget / csize / L.threads;
      L.max_length = 4096;
      L.max_pass = 12;
      L.lds_hw = 163840;
      int count[6][4] = {};   // [violation][role]: 0 x fwd, 1 x inv, 2 columns, 3 raw rows
      int plans = 0;
      for (int n = 1; n <= 4096; ++n) {
        if (!is23(n)) continue;
        ++plans;
        // Poisson x plan: length nx (complex pairs of a 2nx real row); mesh n = nx
        if (n >= 2 && n <= 2048 && is23(2 * n)) {
          const Plan px = make(n, width(n, csize, true, K.lds_budget), true);
          ++count[fft_plan_violation(px, L, csize, n, K.tile_reals, (size_t)(n + 1) * csize)][0];
          ++count[fft_plan_violation(px, L, csize, px.N, K.tile_reals, 0)][1];
        }
        // y / z pencils (length 2n of the Poisson solve, any length of the raw FFT)
        const Plan pc = make(n, width(n, csize, false, K.lds_budget), false);
        ++count[fft_plan_violation(pc, L, csize, 0, 0, 0)][2];
        // raw FFT rows: padded when one padded row fits, staged through emax registers
        int Wr = width(n, csize, true, K.lds_budget);
        const bool padded = (long long)n * (Wr + 1) * csize <= K.lds_budget;
        const Plan pr = make(n, Wr, padded);
        ++count[fft_plan_violation(pr, L, csize, n, L.emax, 0)][3];
      }
      printf("%s %s threads=%d emax=%d lengths=%d", K.name, dt == 0 ? "f32" : "f64", L.threads, L.emax, plans);
      const char* roles[4] = {"x_fwd", "x_inv", "cols", "raw_rows"};
      for (int r = 0; r < 4; ++r) {
        printf(" %s:", roles[r]);
        for (int v = 0; v < 6; ++v) printf("%s%d", v ? "/" : "", count[v][r]);
      }
      printf("\n");
    }
  }
  // planted mistakes, one per invariant (committed FP32 constants)
  EngineLimits L;
  L.threads = 512;
  L.emax = 16;
  L.max_length = 4096;
  L.max_pass = 12;
  L.lds_hw = 163840;
  Plan ok = make(512, 16, false);
  Plan bad = ok;
  bad.Ns[2] += 1;
  printf("planted structure %d\n", fft_plan_violation(bad, L, 8, 0, 0, 0));
  bad = ok;
  bad.LD = 18;
  printf("planted tile_shape %d\n", fft_plan_violation(bad, L, 8, 0, 0, 0));
  bad = make(512, 64, false);
  printf("planted coverage %d\n", fft_plan_violation(bad, L, 8, 0, 0, 0));
  bad = make(256, 16, true);
  printf("planted tile_load %d\n", fft_plan_violation(bad, L, 8, 1024, 16, 0));
  bad = make(4096, 4, false);
  L.emax = 64;
  printf("planted lds %d\n", fft_plan_violation(bad, L, 16, 0, 0, 0));
  printf("ok %d\n", fft_plan_violation(ok, L, 8, 0, 0, 0));
  return 0;
}
