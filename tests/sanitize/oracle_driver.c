/* oracle_driver.c -- standalone driver of the FP64 oracle for the host
 * sanitizer test (tests/test_sanitizers.py): it builds with the oracle's C
 * sources under AddressSanitizer and UndefinedBehaviorSanitizer and runs a
 * few steps of small boxes through every grid-level entry point (periodic
 * and walled, every equilibrium family, non-unit higher-order rates, a
 * window initialisation, the two-dimensional oracle).  Any sanitizer report
 * aborts the run with a nonzero status.  Test infrastructure only. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/cglbm_oracle.h"
#include "../../oracle/d2q9_oracle.h"

static int run3(int nx, int ny, int nz, unsigned walls, int model, int use_q, double omega_hi,
                int steps) {
  orc_params P;
  memset(&P, 0, sizeof(P));
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.walls = walls;
  P.model = model;
  P.use_q = use_q;
  P.rho0_r = 1.0;
  P.rho0_b = 0.1;
  P.alpha_r = 1.0 - (19.0 / 27.0) / 10.0;
  P.alpha_b = 8.0 / 27.0;
  P.nu_r = P.nu_b = 0.02;
  P.sigma = 0.01;
  P.beta = 0.7;
  for (int k = 0; k < 11; ++k) P.omega[k] = (k == 1 || k == 2) ? 1.0 : omega_hi;
  P.body_force[0] = 1e-6;
  P.gravity[2] = -1e-5;
  P.rho_ref = 0.5;
  const long n = (long)nx * ny * nz;
  double *rr = calloc(n, sizeof(double)), *rb = calloc(n, sizeof(double));
  double *u = calloc(3 * n, sizeof(double)), *f = calloc(2 * 27 * n, sizeof(double));
  double *fw = calloc(2 * 27 * n, sizeof(double)), *out = calloc(ORC_NFIELDS * n, sizeof(double));
  double *g = calloc(3 * n, sizeof(double));
  if (!rr || !rb || !u || !f || !fw || !out || !g) return 1;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long c = x + (long)nx * (y + (long)ny * z);
        const double d = sqrt((x - nx / 2.0) * (x - nx / 2.0) + (y - ny / 2.0) * (y - ny / 2.0) +
                              (z - nz / 2.0) * (z - nz / 2.0));
        rr[c] = d < 3.0 ? 1.0 : 0.0;
        rb[c] = d < 3.0 ? 0.0 : 0.1;
        u[c] = 0.02;
        u[n + c] = -0.01;
      }
  int rc = orc_init(&P, rr, rb, u, 7, 1e-5, 1, f);
  const int32_t gd[3] = {nx + 3, ny + 2, nz + 1}, go[3] = {2, 1, 5};
  rc |= orc_init_window(&P, rr, rb, u, 7, 1e-5, 1, gd, go, fw);
  rc |= orc_step(&P, f, steps);
  rc |= orc_fields(&P, f, out);
  rc |= orc_gradient(&P, out + 2 * n, g);
  for (long k = 0; k < ORC_NFIELDS * n; ++k)
    if (!isfinite(out[k])) rc = 2;
  free(rr);
  free(rb);
  free(u);
  free(f);
  free(fw);
  free(out);
  free(g);
  return rc;
}

static int run2(int nx, int ny, unsigned walls, int steps) {
  orc2_params P;
  memset(&P, 0, sizeof(P));
  P.nx = nx;
  P.ny = ny;
  P.walls = walls;
  P.use_q = 1;
  P.rho0_r = 10.0;
  P.rho0_b = 1.0;
  P.alpha_r = 1.0 - (5.0 / 9.0) / 10.0;
  P.alpha_b = 4.0 / 9.0;
  P.nu_r = P.nu_b = 0.1;
  P.sigma = 0.01;
  P.beta = 0.7;
  for (int k = 0; k < 5; ++k) P.omega[k] = 1.0;
  P.body_force[0] = 1e-6;
  const long n = (long)nx * ny;
  double *rr = calloc(n, sizeof(double)), *rb = calloc(n, sizeof(double));
  double *u = calloc(2 * n, sizeof(double)), *f = calloc(2 * 9 * n, sizeof(double));
  double *out = calloc(17 * n, sizeof(double));
  if (!rr || !rb || !u || !f || !out) return 1;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const long c = x + (long)nx * y;
      const double d = hypot(x - nx / 2.0, y - ny / 2.0);
      rr[c] = d < 4.0 ? 10.0 : 0.0;
      rb[c] = d < 4.0 ? 0.0 : 1.0;
      u[c] = 0.03;
    }
  int rc = orc2_init(&P, rr, rb, u, 3, 1e-5, 0, f);
  rc |= orc2_step(&P, f, steps);
  rc |= orc2_fields(&P, f, out);
  free(rr);
  free(rb);
  free(u);
  free(f);
  free(out);
  return rc;
}

int main(void) {
  int rc = 0;
  rc |= run3(9, 8, 7, 0, ORC_MODEL_D, 1, 1.0, 3);
  rc |= run3(7, 9, 8, 3, ORC_MODEL_D, 1, 1.0, 3);
  rc |= run3(6, 5, 7, 1, ORC_MODEL_A, 1, 1.0, 2);
  rc |= run3(6, 7, 5, 2, ORC_MODEL_B, 0, 1.0, 2);
  rc |= run3(5, 6, 6, 0, ORC_MODEL_C, 1, 1.3, 2);
  rc |= run3(1, 1, 1, 0, ORC_MODEL_D, 1, 1.0, 2);
  rc |= run2(13, 11, 0, 3);
  rc |= run2(9, 12, 1, 3);
  printf("oracle driver: %s\n", rc ? "FAILED" : "ok");
  return rc;
}
