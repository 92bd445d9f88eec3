/* Host-only exercise of the C ABI's argument checks, parameter validation
   and workspace carving, for a build with AddressSanitizer and
   UndefinedBehaviorSanitizer on the host code.  Nothing here reaches a
   device: every call either only computes sizes or is rejected before any
   HIP call.  Exit status 0 when every expectation holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "fracture.h"

static int failures = 0;

#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

static fracture_params tension(int nx, int ny) {
  fracture_params p;
  fracture_default_params(&p, nx, ny);
  p.ell = 4.0 / nx;
  return p;
}

static fracture_params thermal(int nx, int ny, int nz) {
  fracture_params p;
  fracture_default_params(&p, nx, ny);
  p.dim = 3;
  p.nz = nz;
  p.lz = 0.25;
  p.load_kind = FRACTURE_LOAD_THERMAL_3D;
  p.thermal_depth = 0.05;
  p.ell = 4.0 / nx;
  return p;
}

/* One invalid field per case: workspace_bytes is 0, create refuses it. */
static void invalid_cases(void) {
  void* fake = (void*)(uintptr_t)(1 << 20);   /* never dereferenced */
  for (int c = 0; c < 24; ++c) {
    fracture_params p = tension(64, 64);
    switch (c) {
      case 0: p.dim = 4; break;
      case 1: p.nx = 1; break;
      case 2: p.ly = 0.0; break;
      case 3: p.model = 3; break;
      case 4: p.nu = 0.5; break;
      case 5: p.ell = -1.0; break;
      case 6: p.k_ell = -1e-6; break;
      case 7: p.omega = 2.0; break;
      case 8: p.relax_mode = 5; break;
      case 9: p.load_kind = 7; break;
      case 10: p.precision = 2; break;
      case 11: p.max_am = 0; break;
      case 12: p.cheb_degree = 9; break;
      case 13: p.newton_vcycles = 3; break;
      case 14: p.pcg_reduction = 1.0; break;
      case 15: p.vi_reduction = -0.1; break;
      case 16: p.newton_stall = 0.0; break;
      case 17: p.deflate = 1; p.deflate_max_fragments = 99; break;
      case 18: p.E = NAN; break;
      case 19: p.nx = 65; p.ny = 65; break;                /* no coarse level fits */
      case 20: p.nx = 1 << 15; p.ny = 1 << 15; break;      /* above 2^29 nodes */
      case 21: p.load_kind = FRACTURE_LOAD_THERMAL_SHOCK_2D; p.thermal_dT = INFINITY; break;
      case 22: p.newton = 1; p.minres_rtol = 0.0; break;
      default: p.omega_auto = 2; break;
    }
    EXPECT(fracture_workspace_bytes(&p) == 0);
    fracture_t h = (fracture_t)fake;
    EXPECT(fracture_create(&p, NULL, fake, (size_t)1 << 30, NULL, &h) == FRACTURE_EINVAL);
    EXPECT(h == NULL);
  }
  fracture_params q = thermal(16, 16, 4);
  q.newton = 1;
  q.minres_rtol = -1.0;                          /* Newton needs a positive MINRES tolerance */
  EXPECT(fracture_workspace_bytes(&q) == 0);
}

static void workspace_and_create_checks(void) {
  void* fake = (void*)(uintptr_t)(1 << 20);
  const int shapes[][2] = {{8, 8}, {64, 64}, {96, 80}, {2048, 2048}, {1536, 1408}};
  for (int s = 0; s < 5; ++s) {
    for (int variant = 0; variant < 4; ++variant) {
      fracture_params p = tension(shapes[s][0], shapes[s][1]);
      p.newton = variant & 1;
      p.precision = (variant & 2) ? FRACTURE_MIXED : FRACTURE_FP64;
      const size_t ws = fracture_workspace_bytes(&p);
      int64_t nodes = 0, dofs = 0;
      EXPECT(fracture_sizes(&p, &nodes, &dofs) == FRACTURE_OK);
      EXPECT(nodes == (int64_t)(shapes[s][0] + 1) * (shapes[s][1] + 1));
      EXPECT(dofs == 2 * nodes);
      EXPECT(ws > (size_t)nodes * 8 * 20);
      fracture_t h = NULL;
      EXPECT(fracture_create(&p, NULL, fake, ws - 1, NULL, &h) == FRACTURE_ENOMEM);
      EXPECT(fracture_create(&p, NULL, (char*)fake + 8, ws, NULL, &h) == FRACTURE_EINVAL);
      EXPECT(fracture_create(&p, NULL, NULL, ws, NULL, &h) == FRACTURE_EINVAL);
      EXPECT(fracture_create(&p, NULL, fake, ws, NULL, NULL) == FRACTURE_EINVAL);
    }
  }
  fracture_params d = tension(512, 512), plain = tension(512, 512);
  d.deflate = 1;
  EXPECT(fracture_workspace_bytes(&d) > fracture_workspace_bytes(&plain));
  fracture_params t = thermal(128, 128, 32);
  int64_t nodes = 0, dofs = 0;
  EXPECT(fracture_workspace_bytes(&t) > 0);
  EXPECT(fracture_sizes(&t, &nodes, &dofs) == FRACTURE_OK);
  EXPECT(nodes == 129 * 129 * 33 && dofs == 3 * nodes);
  EXPECT(fracture_sizes(NULL, &nodes, &dofs) != FRACTURE_OK);
  EXPECT(fracture_workspace_bytes(NULL) == 0);
}

static void null_handle_checks(void) {
  double a = 0, b = 0, E[576];
  int n = 0, nx = 0, ny = 0, nz = 0;
  fracture_stats st;
  fracture_t none = NULL;
  int codes[1] = {0};
  EXPECT(fracture_set_load(NULL, 0.1) == FRACTURE_EINVAL);
  EXPECT(fracture_solve_step(NULL, &st) == FRACTURE_EINVAL);
  EXPECT(fracture_solve_steps(NULL, 1, &st, codes) == FRACTURE_EINVAL);
  EXPECT(fracture_solve_steps(&none, -1, &st, codes) == FRACTURE_EINVAL);
  EXPECT(fracture_set_monitor(NULL, NULL, NULL) == FRACTURE_EINVAL);
  EXPECT(fracture_energy(NULL, &a, &b) == FRACTURE_EINVAL);
  EXPECT(fracture_get_state(NULL, &a, &a, &a) == FRACTURE_EINVAL);
  EXPECT(fracture_set_state(NULL, &a, &a, &a) == FRACTURE_EINVAL);
  EXPECT(fracture_apply(NULL, FRACTURE_OP_ELASTICITY, 0, &a, &b) == FRACTURE_EINVAL);
  EXPECT(fracture_update_coefficients(NULL) == FRACTURE_EINVAL);
  EXPECT(fracture_gradient(NULL, &a, &b) == FRACTURE_EINVAL);
  EXPECT(fracture_levels(NULL, &n) == FRACTURE_EINVAL);
  EXPECT(fracture_level_shape(NULL, 0, &nx, &ny, &nz) == FRACTURE_EINVAL);
  EXPECT(fracture_time_kernel(NULL, 0, 1, &a, &b) == FRACTURE_EINVAL);
  EXPECT(fracture_kernel_timing(NULL, 1, 8) == FRACTURE_EINVAL);
  EXPECT(fracture_kernel_timing_read(NULL, &n, &a, &b) == FRACTURE_EINVAL);
  EXPECT(fracture_fragments(NULL, &n, NULL) == FRACTURE_EINVAL);
  EXPECT(fracture_deflation_matrix(NULL, &n, E) == FRACTURE_EINVAL);
  fracture_destroy(NULL);
}

static void noalloc_checks(void) {
  void* fake = (void*)(uintptr_t)(1 << 20);
  fracture_params p = tension(64, 64);
  EXPECT(fracture_energy_noalloc(&p, 0.1, NULL, fake, NULL, fake) == FRACTURE_EINVAL);
  EXPECT(fracture_energy_noalloc(&p, NAN, fake, fake, NULL, fake) == FRACTURE_EINVAL);
  EXPECT(fracture_energy_noalloc(NULL, 0.1, fake, fake, NULL, fake) == FRACTURE_EINVAL);
  fracture_params t = thermal(128, 128, 64);
  EXPECT(fracture_energy_noalloc(&t, 1.0, fake, fake, NULL, fake) == FRACTURE_ESCRATCH);
}

static void strerror_checks(void) {
  const int codes[] = {FRACTURE_OK, FRACTURE_EINVAL, FRACTURE_ENOMEM, FRACTURE_ENOTCONV,
                       FRACTURE_ENONFINITE, FRACTURE_EDEVICE, FRACTURE_ESCRATCH, -99, 17};
  for (size_t k = 0; k < sizeof(codes) / sizeof(codes[0]); ++k) {
    const char* s = fracture_strerror(codes[k]);
    EXPECT(s != NULL && strlen(s) > 0);
  }
}

int main(void) {
  invalid_cases();
  workspace_and_create_checks();
  null_handle_checks();
  noalloc_checks();
  strerror_checks();
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("host validation ok\n");
  return 0;
}
