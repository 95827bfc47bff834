/* A plain C client of the three headers: plans, workspace sizes and the
 * host-side argument checks, with no device work (runs without a GPU).
 * Prints "ok" and exits 0 when every check holds. */
#include <stdio.h>
#include <stdlib.h>

#include "dks_fft.h"
#include "dks_musr.h"
#include "dks_poisson.h"

#define CHECK(cond)                                               \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      return 1;                                                   \
    }                                                             \
  } while (0)

int main(void) {
  dks_poisson_plan_t p = NULL;
  size_t bytes = 0;
  CHECK(dks_poisson_plan(64, 64, 64, 1e-4, 1e-4, 1e-4, DKS_F32, &p) == DKS_OK && p != NULL);
  CHECK(dks_poisson_workspace_bytes(p, &bytes) == DKS_OK && bytes > 0);
  CHECK(dks_poisson_set_scheme(p, DKS_GREEN_POINT, DKS_ASSIGN_TSC) == DKS_OK);
  CHECK(dks_poisson_set_deterministic(p, 1) == DKS_OK && dks_poisson_set_deterministic(p, 2) == DKS_EINVAL);
  CHECK(dks_poisson_solve_rho(p, NULL, NULL, NULL, NULL) == DKS_EINVAL);
  CHECK(dks_poisson_host_staging_bytes(p, &bytes) == DKS_OK && bytes >= 10u * 64 * 64 * 64 * 4);
  CHECK(dks_poisson_destroy(p) == DKS_OK);
  CHECK(dks_poisson_plan(5, 8, 8, 1.0, 1.0, 1.0, DKS_F64, &p) == DKS_EUNSUPPORTED);

  /* runtime and compile-time plans of both dtypes, fitted and explicit: the
   * host-side layout, validation and scratch queries */
  {
    const int shapes[4][3] = {{96, 96, 192}, {48, 36, 64}, {256, 256, 256}, {4, 6, 9}};
    for (int s = 0; s < 4; ++s)
      for (int d = 0; d < 2; ++d)
        for (int f = 0; f < 2; ++f) {
          const double h = f ? 0.0 : 1e-4;
          p = NULL;
          CHECK(dks_poisson_plan(shapes[s][0], shapes[s][1], shapes[s][2], h, h, h, d ? DKS_F64 : DKS_F32, &p) ==
                    DKS_OK && p != NULL);
          CHECK(dks_poisson_workspace_bytes(p, &bytes) == DKS_OK && bytes > 0);
          CHECK(dks_poisson_particle_scratch_bytes(p, 1000000, &bytes) == DKS_OK && bytes >= 16000000u);
          CHECK(dks_poisson_batch_scratch_bytes(p, 3, 1000, &bytes) == DKS_OK && bytes > 0);
          CHECK(dks_poisson_set_origin(p, 0.0, 0.0, 0.0) == (f ? DKS_ESTATE : DKS_OK));
          CHECK(dks_poisson_set_scheme(p, DKS_GREEN_INTEGRATED, DKS_ASSIGN_NGP) == DKS_OK);
          CHECK(dks_poisson_set_deterministic(p, 1) == DKS_OK);
          CHECK(dks_poisson_solve_particles(p, NULL, NULL, NULL, 10, 1.0, NULL, NULL, NULL, NULL, NULL, NULL) ==
                DKS_EINVAL);
          CHECK(dks_poisson_destroy(p) == DKS_OK);
        }
  }
  for (int st = -8; st <= 0; ++st) CHECK(dks_status_string((dks_status)st) != NULL);

  dks_fft_plan_t f = NULL;
  CHECK(dks_fft_plan(512, 512, 256, 1, DKS_FFT_C2C, DKS_F32, &f) == DKS_OK);
  CHECK(dks_fft_workspace_bytes(f, &bytes) == DKS_OK && bytes > 0);
  CHECK(dks_fft_forward(f, NULL, NULL, NULL) == DKS_EINVAL);
  CHECK(dks_fft_destroy(f) == DKS_OK);

  dks_musr_plan_t m = NULL;
  CHECK(dks_musr_plan(16, 206250, 10.0 / 206250, 133, &m) == DKS_OK);
  CHECK(dks_musr_workspace_bytes(m, &bytes) == DKS_OK && bytes > 0);
  CHECK(dks_musr_eval(m, DKS_MUSR_CHISQ, NULL, NULL, NULL) == DKS_EINVAL);
  CHECK(dks_musr_destroy(m) == DKS_OK);

  printf("ok %s\n", dks_status_string(DKS_EWORKSPACE));
  return 0;
}
