/* abi_driver.c -- C driver of the host side of the C ABI for the host
 * sanitizer test (tests/test_sanitizers.py): parameter validation and
 * buffer sizes for every storage format and both lattices, and the error
 * path of every entry point that takes a handle (NULL handle), plus
 * cglbm_init's argument checks.  Run on a host without a GPU, where
 * cglbm_init must fail cleanly once the arguments are valid.  Exits nonzero
 * on an unexpected return code.  Test infrastructure only. */
#include <stdio.h>
#include <string.h>

#include "../../include/cglbm.h"

static int fails = 0;
#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                          \
    }                                                                   \
  } while (0)

static cglbm_box_params box(int nx, int ny, int nz, unsigned walls) {
  cglbm_box_params p;
  memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.walls = walls;
  p.red.rho0 = 1.0;
  p.red.alpha = 1.0 - (19.0 / 27.0) / 10.0;
  p.red.nu = 0.01;
  p.blue.rho0 = 0.1;
  p.blue.alpha = 8.0 / 27.0;
  p.blue.nu = 0.1;
  p.sigma = 0.01;
  p.beta = 0.7;
  p.omega_bulk = 1.0;
  for (int k = 0; k < 9; ++k) p.omega_hi[k] = 1.0;
  p.model = CGLBM_MODEL_D;
  p.q_correction = 1;
  return p;
}

int main(void) {
  size_t pop = 0, aux = 0;
  int64_t tot = 0;
  cglbm_box_params b[3] = {box(17, 13, 11, 0), box(24, 20, 9, 3), box(5, 7, 1, 1)};
  for (int st = 0; st <= 6; ++st) {
    EXPECT(cglbm_query_sizes(3, b, st, &pop, &aux, &tot) == CGLBM_OK);
    EXPECT(pop > 0 && aux > 0 && tot >= 17 * 13 * 11 + 24 * 20 * 9 + 35);
  }
  EXPECT(cglbm_query_sizes(3, b, 7, &pop, &aux, &tot) == CGLBM_EINVAL);
  EXPECT(cglbm_query_sizes(0, b, 0, &pop, &aux, &tot) == CGLBM_EINVAL);
  EXPECT(cglbm_query_sizes(1, NULL, 0, &pop, &aux, &tot) == CGLBM_EINVAL);
  EXPECT(strlen(cglbm_last_error()) > 0);
  cglbm_box_params bad = box(8, 8, 8, 0);
  bad.red.alpha = 1.0;
  EXPECT(cglbm_query_sizes(1, &bad, 0, &pop, &aux, &tot) == CGLBM_EINVAL);
  bad = box(8, 2, 8, 1);
  EXPECT(cglbm_query_sizes(1, &bad, 0, &pop, &aux, &tot) == CGLBM_EINVAL);
  bad = box(8, 8, 8, 4);
  EXPECT(cglbm_query_sizes(1, &bad, 0, &pop, &aux, &tot) == CGLBM_EINVAL);
  bad = box(8, 8, 8, 0);
  bad.omega_hi[3] = 2.5;
  EXPECT(cglbm_query_sizes(1, &bad, 0, &pop, &aux, &tot) == CGLBM_EINVAL);
  bad = box(1024, 1024, 512, 0);
  EXPECT(cglbm_query_sizes(1, &bad, 0, &pop, &aux, &tot) == CGLBM_EINVAL);
  cglbm_box_params b2[2] = {box(40, 30, 1, 0), box(33, 17, 1, 1)};
  for (int st = 0; st <= 4; ++st)
    EXPECT(cglbm_query_sizes_d2q9(2, b2, st, &pop, &aux, &tot) == CGLBM_OK);
  EXPECT(cglbm_query_sizes_d2q9(2, b2, 5, &pop, &aux, &tot) == CGLBM_EUNSUPPORTED);
  EXPECT(cglbm_query_sizes_d2q9(3, b, 0, &pop, &aux, &tot) == CGLBM_EINVAL);

  /* cglbm_init: argument checks, then no device on this host */
  cglbm_handle *h = (cglbm_handle *)0x1;
  float dummy[4];
  EXPECT(cglbm_init(NULL, 3, b, 0, dummy, dummy + 1, dummy, dummy, dummy, dummy, 0, 0.0, NULL) ==
         CGLBM_EINVAL);
  EXPECT(cglbm_init(&h, 3, b, 0, NULL, dummy, dummy, dummy, dummy, dummy, 0, 0.0, NULL) ==
         CGLBM_EINVAL);
  EXPECT(h == NULL);
  EXPECT(cglbm_init(&h, 3, b, 0, dummy, dummy, dummy, dummy, dummy, dummy, 0, 0.0, NULL) ==
         CGLBM_EINVAL);
  EXPECT(cglbm_init(&h, 3, b, 0, dummy, dummy + 1, NULL, dummy, dummy, dummy, 0, 0.0, NULL) ==
         CGLBM_EINVAL);
  EXPECT(cglbm_init(&h, 3, b, 0, dummy, dummy + 1, dummy, dummy, dummy, dummy, 0, -1.0, NULL) ==
         CGLBM_EINVAL);
  EXPECT(cglbm_init_d2q9(&h, 2, b2, 0, dummy, NULL, dummy, dummy, dummy, dummy, 0, 0.0, NULL) ==
         CGLBM_EUNSUPPORTED);
  const int rc = cglbm_init(&h, 3, b, 0, dummy, dummy + 1, dummy, dummy, dummy, dummy, 0, 0.0, NULL);
  EXPECT(rc == CGLBM_EHIP && h == NULL);

  /* every entry point that takes a handle, with a NULL handle */
  double d[16];
  int32_t info[4];
  int64_t l[8];
  EXPECT(cglbm_step(NULL, 1, NULL) == CGLBM_ESTATE);
  EXPECT(cglbm_moments(NULL, 0, 1u, (float *)d, NULL) == CGLBM_ESTATE);
  EXPECT(cglbm_reduce(NULL, NULL, d, 1, NULL) == CGLBM_ESTATE);
  EXPECT(cglbm_box_offset(NULL, 0) == -1);
  EXPECT(cglbm_state_buffer(NULL) == NULL);
  EXPECT(cglbm_load_state(NULL, d, NULL) == CGLBM_ESTATE);
  EXPECT(cglbm_set_schedule(NULL, 0) == CGLBM_ESTATE);
  EXPECT(cglbm_get_schedule(NULL) == -1);
  EXPECT(cglbm_compact_variant(NULL, info) == -1);
  EXPECT(cglbm_set_compact_variant(NULL, 0, NULL) == CGLBM_ESTATE);
  EXPECT(cglbm_set_graph(NULL, 1) == CGLBM_ESTATE);
  EXPECT(cglbm_set_variant(NULL, 0, NULL) == CGLBM_ESTATE);
  EXPECT(cglbm_get_variant(NULL) == -1);
  EXPECT(cglbm_autotune(NULL, 1, d, NULL) == CGLBM_ESTATE);
  EXPECT(cglbm_profile_begin(NULL, 4) == CGLBM_ESTATE);
  EXPECT(cglbm_profile_end(NULL, d, l, 4) == CGLBM_ESTATE);
  EXPECT(cglbm_lattice(NULL) == -1);
  cglbm_destroy(NULL);
  /* handle-free queries */
  EXPECT(cglbm_num_variants() > 0);
  for (int v = 0; v < cglbm_num_variants(); ++v) EXPECT(cglbm_variant_info(v, info) == CGLBM_OK);
  EXPECT(cglbm_variant_info(-1, info) == CGLBM_EINVAL);
  EXPECT(cglbm_variant_info(0, NULL) == CGLBM_EINVAL);
  EXPECT(cglbm_variant_info_d2q9(0, info) == CGLBM_OK);
  EXPECT(cglbm_variant_info_d2q9(99, info) == CGLBM_EINVAL);
  EXPECT(strlen(cglbm_version()) > 0);
  printf("abi driver: %s\n", fails ? "FAILED" : "ok");
  return fails ? 1 : 0;
}
