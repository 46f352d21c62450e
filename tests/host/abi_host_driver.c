/* Host-only exercise of the C-ABI for the sanitizer build: every call here returns before any
 * device work (argument checks, host helpers, descriptor validation), so it runs without a GPU.
 * Exits 0 when every call returns the documented status. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/vbrdf.h"

static int failures = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                 \
    }                                                             \
  } while (0)

int main(void) {
  EXPECT(vbrdf_abi_version() == VBRDF_ABI_VERSION);
  double mu[128], al[128];
  for (int N = 1; N <= 128; N += 9) {
    EXPECT(vbrdf_gauss_nodes(N, mu, al) == VBRDF_OK);
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += al[i];
    EXPECT(s > 1.0 - 1e-13 && s < 1.0 + 1e-13);
  }
  EXPECT(vbrdf_gauss_nodes(0, mu, al) == VBRDF_E_INVALID);
  EXPECT(vbrdf_gauss_nodes(4, NULL, al) == VBRDF_E_INVALID);
  EXPECT(strlen(vbrdf_last_error()) > 0);

  int32_t N[3] = {8, 5, 3}, L[3] = {6, 9, 3}, M[3] = {4, 9, 3}, P[3] = {3, 4, 5};
  vbrdf_plan_desc d;
  memset(&d, 0, sizeof d);
  d.abi_version = VBRDF_ABI_VERSION;
  d.n_layers = 3;
  d.N = N;
  d.L = L;
  d.M = M;
  d.n_dphi = P;
  uint64_t bytes = 0;
  EXPECT(vbrdf_workspace_query(&d, &bytes) == VBRDF_OK && bytes > 0);
  d.flags = VBRDF_FLAG_SAVE_FOR_BACKWARD;
  uint64_t bytes_bwd = 0;
  EXPECT(vbrdf_workspace_query(&d, &bytes_bwd) == VBRDF_OK && bytes_bwd > bytes);
  d.flags = 0;

  vbrdf_plan* p = (vbrdf_plan*)0x1;
  vbrdf_plan_desc bad = d;
  bad.abi_version = 1;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_INVALID && p == NULL);
  bad = d;
  bad.n_layers = 0;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_INVALID);
  bad = d;
  bad.N = NULL;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_INVALID);
  bad = d;
  bad.precision = 9;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_UNSUPPORTED);
  bad = d;
  bad.flags = 1 << 10;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_UNSUPPORTED);
  bad = d;
  bad.qr_sweep_cap = -3;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_INVALID);
  bad = d;
  bad.workspace_cap_bytes = 64;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_NOMEM);
  bad = d;
  bad.workspace = (void*)0x1000;
  bad.workspace_bytes = 16;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_NOMEM);
  int32_t Mbad[3] = {4, 10, 3};
  bad = d;
  bad.M = Mbad;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_INVALID);
  int32_t below_bad[3] = {1, 2, 1}, below_ok[3] = {-1, -1, -1};
  bad = d;
  bad.below = below_bad;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_INVALID);
  bad = d;
  bad.below = below_ok;
  bad.base = 7;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_UNSUPPORTED);
  bad = d;
  bad.below = below_ok;
  bad.base = VBRDF_BASE_LAMBERTIAN;
  bad.flags = VBRDF_FLAG_EMIT_TRANSMISSION;
  EXPECT(vbrdf_plan_create(&bad, &p) == VBRDF_E_UNSUPPORTED);
  bad.flags = 0;
  uint64_t qb = 0;
  EXPECT(vbrdf_workspace_query(&bad, &qb) == VBRDF_OK && qb == bytes);
  EXPECT(vbrdf_plan_create(NULL, &p) == VBRDF_E_INVALID);
  EXPECT(vbrdf_plan_create(&d, NULL) == VBRDF_E_INVALID);

  EXPECT(vbrdf_plan_destroy(NULL) == VBRDF_OK);
  EXPECT(vbrdf_plan_output_bytes(NULL) == 0 && vbrdf_plan_workspace_bytes(NULL) == 0);
  EXPECT(vbrdf_solve(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == VBRDF_E_INVALID);
  EXPECT(vbrdf_solve_base(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == VBRDF_E_INVALID);
  EXPECT(vbrdf_plan_base_bytes(NULL) == 0);
  EXPECT(vbrdf_backward(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == VBRDF_E_INVALID);
  EXPECT(vbrdf_plan_inspect(NULL, 0, 0, NULL, NULL, NULL, NULL, NULL) == VBRDF_E_INVALID);
  double i0[4] = {1, 0, 0, 0};
  EXPECT(vbrdf_radiance(NULL, NULL, 0, 0, 0.0, i0, NULL, NULL) == VBRDF_E_INVALID);
  EXPECT(vbrdf_plan_stage_times(NULL, NULL, 0) == VBRDF_E_INVALID);
  vbrdf_tuning t = {0, 8};
  EXPECT(vbrdf_plan_get_tuning(NULL, &t) == VBRDF_E_INVALID);
  EXPECT(vbrdf_plan_set_tuning(NULL, &t) == VBRDF_E_INVALID);
  EXPECT(vbrdf_plan_autotune(NULL, NULL, NULL, NULL, NULL, NULL, NULL, &t) == VBRDF_E_INVALID);
  for (int i = -2; i < 20; ++i) {
    const char* s = vbrdf_stage_name(i);
    EXPECT((i >= 0 && i < 17) ? (s != NULL && strlen(s) > 0) : s == NULL);
  }
  double* fake = (double*)0x100000;
  int32_t* ifake = (int32_t*)0x100000;
  EXPECT(vbrdf_solve_noalloc(8, 4, 2, 8, NULL, fake, fake, fake, ifake, NULL) == VBRDF_E_INVALID);
  EXPECT(vbrdf_solve_noalloc(8, 4, 5, 8, fake, fake, fake, fake, ifake, NULL) == VBRDF_E_INVALID);
  EXPECT(vbrdf_solve_noalloc(129, 4, 2, 8, fake, fake, fake, fake, ifake, NULL) == VBRDF_E_UNSUPPORTED);
  EXPECT(vbrdf_solve_noalloc(128, 256, 256, 8, fake, fake, fake, fake, ifake, NULL) == VBRDF_E_NOMEM);
  if (failures) return 1;
  printf("abi host driver: all checks passed\n");
  return 0;
}
