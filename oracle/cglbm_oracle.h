/*
 * cglbm_oracle.h -- FP64 CPU oracle for the two-colour D3Q27 colour-gradient
 * lattice Boltzmann step with generalized equilibria (Saito, Takada, Baba,
 * Someya, Ito, arXiv:2309.07801).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the HIP path.
 *
 * State convention: f[c][i][node], c = 0 red / 1 blue, i = 0..26 in the
 * velocity order of Eq. (1), node = x + nx*(y + ny*z).  The stored state is the
 * pre-collision (post-streaming) distribution f^k_i(x, t).
 */
#ifndef CGLBM_ORACLE_H
#define CGLBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Equilibrium families of Table I. */
enum { ORC_MODEL_A = 0, ORC_MODEL_B = 1, ORC_MODEL_C = 2, ORC_MODEL_D = 3 };

typedef struct {
  int32_t nx, ny, nz;
  uint32_t walls;          /* bit0: solid layers y=0,ny-1; bit1: solid layers z=0,nz-1 */
  int32_t model;           /* ORC_MODEL_* */
  int32_t use_q;           /* apply the correction term Q of Eq. (65) */
  double rho0_r, rho0_b;   /* reference densities of Eq. (14) */
  double alpha_r, alpha_b; /* rest fractions; (c_s^k)^2 = xi (1 - alpha_k) */
  double nu_r, nu_b;       /* kinematic viscosities, Eq. (21) */
  double sigma, beta;      /* Eq. (15), Eq. (19) */
  double omega[11];        /* omega_0..omega_10 of Eq. (25); omega[1] is ignored
                              (it follows from Eqs. (21)-(22) at every node) */
  double body_force[3];    /* constant force density added to F */
  double gravity[3];       /* g of the buoyancy force -(rho - rho_ref) g (Sec. IV.E) */
  double rho_ref;          /* reference density of the buoyancy force */
} orc_params;

/* ---- lattice and single-node pieces (exported for pin tests) ---- */
void orc_lattice(int32_t *c /* 27*3 */, double *w /* 27 */);
double orc_hermite(int32_t i, int32_t a, int32_t b, int32_t c);
double orc_isotropic_E(int32_t i);
void orc_feq(int32_t model, double rho, double p, const double *u, double *feq);
void orc_feq_standard_cg(double rho, double p, const double *u, double *feq);
void orc_feq_li_original(double rho, double p, const double *u, double *feq);
void orc_raw_moments(const double *f, double *m);
void orc_central_moments(const double *f, const double *u, double *k);
void orc_cm_to_f(const double *k, const double *u, double *f);
void orc_inverse_moment_matrix(double *minv /* 27*27 */);
void orc_moment_matrix(double *m /* 27*27 */);
void orc_collide(int32_t model, int32_t use_q, const double *f, double rho,
                 const double *u, double p, const double *F, const double *Q,
                 const double *omega, double *fstar);
void orc_recolour(const double *fstar, double rho_r, double rho_b, double p,
                  const double *n, double beta, double *fr, double *fb);
double orc_sound_speed2(double alpha);
uint64_t orc_splitmix64(uint64_t state);
double orc_noise(uint64_t seed, int32_t box, int64_t node, int32_t i, double amp);

/* ---- grid level ---- */
/* Isotropic gradient of Eq. (20) of a scalar field chi[N] -> out[3][N]. */
int orc_gradient(const orc_params *P, const double *chi, double *out);
/* Fields of the state f: 16 planes of N values:
 * rho_r, rho_b, phi, p, ux, uy, uz, nx, ny, nz, kappa, Fx, Fy, Fz, Qx, Qy, Qz
 * (17 planes; u includes F/2). */
#define ORC_NFIELDS 17
int orc_fields(const orc_params *P, const double *f, double *out);
int orc_init(const orc_params *P, const double *rho_r, const double *rho_b,
             const double *u /* [3][N] */, uint64_t seed, double amp, int32_t box,
             double *f);
int orc_init_window(const orc_params *P, const double *rho_r, const double *rho_b,
                    const double *u, uint64_t seed, double amp, int32_t box,
                    const int32_t *gdims, const int32_t *goff, double *f);
int orc_step(const orc_params *P, double *f, int32_t nsteps);
int orc_is_solid(const orc_params *P, int32_t x, int32_t y, int32_t z);
int orc_num_threads(void);
void orc_set_num_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
