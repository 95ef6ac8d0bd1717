/*
 * d2q9_oracle.h -- FP64 CPU oracle for the two-colour D2Q9 colour-gradient
 * lattice Boltzmann step with the two-dimensional generalized equilibrium of
 * App. A (Saito, Takada, Baba, Someya, Ito, arXiv:2309.07801).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the HIP path.
 *
 * State convention: f[c][i][node], c = 0 red / 1 blue, i = 0..8 in the
 * velocity order of Eq. (A1), node = x + nx*y.  The stored state is the
 * pre-collision (post-streaming) distribution f^k_i(x, t).
 */
#ifndef D2Q9_ORACLE_H
#define D2Q9_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nx, ny;
  uint32_t walls;          /* bit0: solid rows y = 0 and y = ny-1 */
  int32_t use_q;           /* apply the correction term Q (Eq. 65 in two dimensions) */
  double rho0_r, rho0_b;   /* reference densities of the order parameter (Eq. 14) */
  double alpha_r, alpha_b; /* rest fractions; (c_s^k)^2 = xi (1 - alpha_k), xi = 3/5 */
  double nu_r, nu_b;       /* kinematic viscosities, Eq. (21) */
  double sigma, beta;      /* Eq. (15), Eq. (19) */
  double omega[5];         /* rates of the two-dimensional Eq. (25): omega_0 (first
                              order), omega_1 (shear; ignored: it follows from
                              Eqs. (21)-(22) at every node), omega_2 (bulk),
                              omega_3 (third order), omega_4 (fourth order) */
  double body_force[2];    /* constant force density added to F */
} orc2_params;

/* ---- lattice and single-node pieces (exported for pin tests) ---- */
void orc2_lattice(int32_t *c /* 9*2 */, double *w /* 9 */);
double orc2_hermite(int32_t i, int32_t a, int32_t b);
double orc2_isotropic_E(int32_t i);
double orc2_xi(void);
void orc2_geq4(double rho, const double *u, double *g);
void orc2_feq(double rho, double p, const double *u, double *feq);
void orc2_central_moments(const double *f, const double *u, double *k);
void orc2_raw_moments(const double *f, double *m);
void orc2_cm_to_f(const double *k, const double *u, double *f);
void orc2_collide(int32_t use_q, const double *f, double rho, const double *u, double p,
                  const double *F, const double *Q, const double *omega, double *fstar);
void orc2_recolour(const double *fstar, double rho_r, double rho_b, double p,
                   const double *n, double beta, double *fr, double *fb);
double orc2_noise(uint64_t seed, int32_t box, int64_t node, int32_t i, double amp);

/* ---- grid level ---- */
/* Fields of the state f: 13 planes of N = nx*ny values:
 * rho_r, rho_b, phi, p, ux, uy, nx, ny, kappa, Fx, Fy, Qx, Qy (u includes F/2). */
#define ORC2_NFIELDS 13
int orc2_fields(const orc2_params *P, const double *f, double *out);
int orc2_init(const orc2_params *P, const double *rho_r, const double *rho_b,
              const double *u /* [2][N] */, uint64_t seed, double amp, int32_t box,
              double *f);
int orc2_init_window(const orc2_params *P, const double *rho_r, const double *rho_b,
                     const double *u, uint64_t seed, double amp, int32_t box,
                     const int32_t *gdims /* Nx, Ny */, const int32_t *goff, double *f);
int orc2_step(const orc2_params *P, double *f, int32_t nsteps);

#ifdef __cplusplus
}
#endif
#endif
