/*
 * cglbm_oracle.c -- plain FP64 CPU oracle for the two-colour D3Q27
 * colour-gradient lattice Boltzmann model with generalized equilibria
 * (Saito et al., arXiv:2309.07801).
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code with the HIP path: its lattice, Hermite tensors, equilibria and moment
 * transforms are written here from the paper's definitions.
 *
 * Everything follows the plain definitions, in the paper's order:
 *   - equilibria are evaluated in phase space by literal Hermite sums
 *     (Eqs. 26-29, 31, 39, 48, 56) and their central moments by brute-force
 *     sums (Eq. 30);
 *   - the collision is the general central-moment MRT of Eq. (25), with every
 *     relaxation rate taken from the parameters;
 *   - the back-transform goes central -> raw moments (binomial shift) -> f
 *     through the inverse of the 27x27 raw-moment matrix (Sec. II.B).
 * No blocking or fusion beyond the definitions.
 */
#include "cglbm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define NQ 27
static const double CS2 = 1.0 / 3.0;   /* c_s^2 of D3Q27 (Sec. II.A) */
static const double XI = 9.0 / 19.0;   /* xi of the D3Q27 lattice (Sec. II.A) */

/* Eq. (1): lattice velocities, columns of the printed 3x27 matrix. */
static const int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0,
                           0, 1, -1, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1};
static const int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1,
                           -1, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
static const int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1,
                           1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};

/* Eq. (9): weight by speed class |c_i|^2 = 0, 1, 2, 3. */
static double weight(int i) {
  int s = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
  switch (s) {
    case 0: return 8.0 / 27.0;
    case 1: return 2.0 / 27.0;
    case 2: return 1.0 / 54.0;
    default: return 1.0 / 216.0;
  }
}

static int opposite(int i) {
  for (int j = 0; j < NQ; ++j)
    if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
  return -1;
}

void orc_lattice(int32_t *c, double *w) {
  for (int i = 0; i < NQ; ++i) {
    c[3 * i + 0] = CX[i];
    c[3 * i + 1] = CY[i];
    c[3 * i + 2] = CZ[i];
    w[i] = weight(i);
  }
}

/* Appendix B: one-dimensional Hermite factors; every 3D tensor H_{i,abc} is
 * the product of the factors of orders a, b, c along x, y, z. */
static double herm1(int order, int c) {
  if (order == 0) return 1.0;
  if (order == 1) return (double)c;
  return (double)(c * c) - CS2;
}

double orc_hermite(int32_t i, int32_t a, int32_t b, int32_t c) {
  return herm1(a, CX[i]) * herm1(b, CY[i]) * herm1(c, CZ[i]);
}

/* The tensors and weights are constants of the lattice; they are tabulated
 * once when the library is loaded. */
static double g_herm[NQ][3][3][3];
static double g_w[NQ];
__attribute__((constructor)) static void tabulate_lattice(void) {
  for (int i = 0; i < NQ; ++i) {
    g_w[i] = weight(i);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) g_herm[i][a][b][c] = orc_hermite(i, a, b, c);
  }
}
#define H(i, a, b, c) g_herm[i][a][b][c]

/* Eq. (26): second-order single-phase equilibrium. */
static double geq2(int i, double rho, const double *u) {
  double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return rho * g_w[i] *
         (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Eq. (27): single-phase equilibrium from Hermite terms up to sixth order. */
static double geq6(int i, double rho, const double *u) {
  const double ux = u[0], uy = u[1], uz = u[2];
  const double c2 = CS2, c4 = CS2 * CS2, c6 = c4 * CS2, c8 = c6 * CS2,
               c10 = c8 * CS2, c12 = c10 * CS2;
  double s = 1.0;
  s += (ux * H(i, 1, 0, 0) + uy * H(i, 0, 1, 0) + uz * H(i, 0, 0, 1)) / c2;
  s += (ux * ux * H(i, 2, 0, 0) + uy * uy * H(i, 0, 2, 0) + uz * uz * H(i, 0, 0, 2) +
        2.0 * (ux * uy * H(i, 1, 1, 0) + uy * uz * H(i, 0, 1, 1) + ux * uz * H(i, 1, 0, 1))) /
       (2.0 * c4);
  s += (ux * ux * uy * H(i, 2, 1, 0) + ux * ux * uz * H(i, 2, 0, 1) +
        ux * uy * uy * H(i, 1, 2, 0) + ux * uz * uz * H(i, 1, 0, 2) +
        uy * uz * uz * H(i, 0, 1, 2) + uy * uy * uz * H(i, 0, 2, 1) +
        2.0 * ux * uy * uz * H(i, 1, 1, 1)) /
       (2.0 * c6);
  s += (ux * ux * uy * uy * H(i, 2, 2, 0) + ux * ux * uz * uz * H(i, 2, 0, 2) +
        uy * uy * uz * uz * H(i, 0, 2, 2) +
        2.0 * (ux * uy * uz * uz * H(i, 1, 1, 2) + ux * uy * uy * uz * H(i, 1, 2, 1) +
               ux * ux * uy * uz * H(i, 2, 1, 1))) /
       (4.0 * c8);
  s += (ux * ux * uy * uz * uz * H(i, 2, 1, 2) + ux * ux * uy * uy * uz * H(i, 2, 2, 1) +
        ux * uy * uy * uz * uz * H(i, 1, 2, 2)) /
       (4.0 * c10);
  s += ux * ux * uy * uy * uz * uz * H(i, 2, 2, 2) / (8.0 * c12);
  return rho * g_w[i] * s;
}

/* Eq. (29): isotropic operator E_i. */
double orc_isotropic_E(int32_t i) {
  const double c4 = CS2 * CS2, c6 = c4 * CS2, c8 = c6 * CS2;
  return g_w[i] * ((H(i, 2, 0, 0) + H(i, 0, 2, 0) + H(i, 0, 0, 2)) / (2.0 * c4) -
                      (H(i, 2, 2, 0) + H(i, 0, 2, 2) + H(i, 2, 0, 2)) / (4.0 * c6) +
                      H(i, 2, 2, 2) / (8.0 * c8));
}

/* Third-order part of the correction operator Phi_i, shared by Eq. (48)
 * (Model C) and the first line of Eq. (56) (Model D). */
static double phi3(int i, const double *u) {
  const double c6 = CS2 * CS2 * CS2;
  return g_w[i] *
         (u[0] * (H(i, 1, 2, 0) + H(i, 1, 0, 2)) + u[1] * (H(i, 2, 1, 0) + H(i, 0, 1, 2)) +
          u[2] * (H(i, 2, 0, 1) + H(i, 0, 2, 1))) /
         (2.0 * c6);
}

/* Eq. (56): correction operator Phi_i of the generalized equilibrium (Model D),
 * terms of Hermite order three to six. */
static double phi6(int i, const double *u) {
  const double ux = u[0], uy = u[1], uz = u[2];
  const double c2 = CS2, c8 = CS2 * CS2 * CS2 * CS2, c10 = c8 * CS2, c12 = c10 * CS2;
  double s = phi3(i, u) / g_w[i];
  s += ((ux * ux + uy * uy) * H(i, 2, 2, 0) + (uy * uy + uz * uz) * H(i, 0, 2, 2) +
        (ux * ux + uz * uz) * H(i, 2, 0, 2) +
        2.0 * (uy * uz * H(i, 2, 1, 1) + ux * uz * H(i, 1, 2, 1) + ux * uy * H(i, 1, 1, 2))) /
       (4.0 * c8);
  s += (ux * (uy * uy + uz * uz - c2) * H(i, 1, 2, 2) +
        uy * (ux * ux + uz * uz - c2) * H(i, 2, 1, 2) +
        uz * (ux * ux + uy * uy - c2) * H(i, 2, 2, 1)) /
       (4.0 * c10);
  s += (ux * ux * uy * uy + uy * uy * uz * uz + ux * ux * uz * uz -
        c2 * (ux * ux + uy * uy + uz * uz)) *
       H(i, 2, 2, 2) / (8.0 * c12);
  return g_w[i] * s;
}

/* Eq. (28) with the choices of Table I:
 *   A: g^{eq,2} + (p - rho c_s^2) E_i                     (Eq. 31)
 *   B: g^{eq,6} + (p - rho c_s^2) E_i                     (Eq. 39)
 *   C: g^{eq,6} + (p - rho c_s^2)(E_i + Phi_i, O(u^3))    (Eq. 48 with g^{eq,6})
 *   D: g^{eq,6} + (p - rho c_s^2)(E_i + Phi_i, O(u^6))    (Eq. 56) */
void orc_feq(int32_t model, double rho, double p, const double *u, double *feq) {
  const double dev = p - rho * CS2;
  for (int i = 0; i < NQ; ++i) {
    double g = (model == ORC_MODEL_A) ? geq2(i, rho, u) : geq6(i, rho, u);
    double corr = 0.0;
    if (model == ORC_MODEL_C) corr = phi3(i, u);
    if (model == ORC_MODEL_D) corr = phi6(i, u);
    feq[i] = g + dev * (orc_isotropic_E(i) + corr);
  }
}

/* Eqs. (7)-(8): the standard colour-gradient equilibrium with the
 * lattice-specific rest fraction varphi_i. */
void orc_feq_standard_cg(double rho, double p, const double *u, double *feq) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < NQ; ++i) {
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    int rest = (CX[i] == 0 && CY[i] == 0 && CZ[i] == 0);
    double vphi = rest ? 1.0 - p / (XI * rho) : g_w[i] * p / (rho * CS2);
    feq[i] = rho * (vphi + g_w[i] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)));
  }
}

/* Eq. (47): the original improved equilibrium of Li and co-workers, D = 3. */
void orc_feq_li_original(double rho, double p, const double *u, double *feq) {
  const double D = 3.0;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < NQ; ++i) {
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    double cc = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
    int rest = (cc == 0);
    double vphi = rest ? 1.0 - p / (XI * rho) : g_w[i] * p / (rho * CS2);
    feq[i] = rho * (vphi + g_w[i] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2) +
                                        cu / (2.0 * CS2) * (p / (rho * CS2) - 1.0) *
                                            (cc / CS2 - D - 2.0)));
  }
}

/* Moment index of (a, b, c), each in {0, 1, 2}. */
#define MI(a, b, c) ((a) + 3 * (b) + 9 * (c))

static double ipow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; ++k) r *= x;
  return r;
}

/* Eq. (23): raw moments m_abc = sum_i f_i cx^a cy^b cz^c. */
void orc_raw_moments(const double *f, double *m) {
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int i = 0; i < NQ; ++i) s += f[i] * ipow(CX[i], a) * ipow(CY[i], b) * ipow(CZ[i], c);
        m[MI(a, b, c)] = s;
      }
}

/* Eq. (24) (and Eq. 30 for f^eq): central moments by their definition. */
void orc_central_moments(const double *f, const double *u, double *k) {
  double px[NQ][3], py[NQ][3], pz[NQ][3];
  for (int i = 0; i < NQ; ++i)
    for (int a = 0; a < 3; ++a) {
      px[i][a] = ipow(CX[i] - u[0], a);
      py[i][a] = ipow(CY[i] - u[1], a);
      pz[i][a] = ipow(CZ[i] - u[2], a);
    }
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int i = 0; i < NQ; ++i) s += f[i] * px[i][a] * py[i][b] * pz[i][c];
        k[MI(a, b, c)] = s;
      }
}

/* The 27x27 matrix of Eq. (23): M[(abc), i] = cx^a cy^b cz^c. */
void orc_moment_matrix(double *M) {
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        for (int i = 0; i < NQ; ++i)
          M[MI(a, b, c) * NQ + i] = ipow(CX[i], a) * ipow(CY[i], b) * ipow(CZ[i], c);
}

/* Inverse of the raw-moment matrix by Gauss-Jordan elimination with partial
 * pivoting, computed once. */
static double g_minv[NQ * NQ];
static int g_minv_ready = 0;

void orc_inverse_moment_matrix(double *minv) {
  double A[NQ][2 * NQ];
  double M[NQ * NQ];
  orc_moment_matrix(M);
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < 2 * NQ; ++c) A[r][c] = (c < NQ) ? M[r * NQ + c] : (c - NQ == r ? 1.0 : 0.0);
  for (int col = 0; col < NQ; ++col) {
    int piv = col;
    for (int r = col + 1; r < NQ; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * NQ; ++c) {
        double t = A[col][c];
        A[col][c] = A[piv][c];
        A[piv][c] = t;
      }
    double d = A[col][col];
    for (int c = 0; c < 2 * NQ; ++c) A[col][c] /= d;
    for (int r = 0; r < NQ; ++r) {
      if (r == col) continue;
      double fct = A[r][col];
      if (fct == 0.0) continue;
      for (int c = 0; c < 2 * NQ; ++c) A[r][c] -= fct * A[col][c];
    }
  }
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) minv[r * NQ + c] = A[r][NQ + c];
}

static const double *minv_table(void) {
  if (!g_minv_ready) {
#pragma omp critical(orc_minv)
    {
      if (!g_minv_ready) {
        orc_inverse_moment_matrix(g_minv);
        g_minv_ready = 1;
      }
    }
  }
  return g_minv;
}

static double binom2(int n, int k) { return (n == 2 && k == 1) ? 2.0 : 1.0; }

/* Back-transform of Sec. II.B: central moments -> raw moments by expanding
 * c^a = ((c - u) + u)^a binomially, then raw moments -> f by the inverse of the
 * raw-moment matrix. */
void orc_cm_to_f(const double *k, const double *u, double *f) {
  double m[NQ];
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int c2 = 0; c2 <= c; ++c2)
          for (int b2 = 0; b2 <= b; ++b2)
            for (int a2 = 0; a2 <= a; ++a2)
              s += binom2(a, a2) * binom2(b, b2) * binom2(c, c2) * ipow(u[0], a - a2) *
                   ipow(u[1], b - b2) * ipow(u[2], c - c2) * k[MI(a2, b2, c2)];
        m[MI(a, b, c)] = s;
      }
  const double *Mi = minv_table();
  for (int i = 0; i < NQ; ++i) {
    double s = 0.0;
    for (int j = 0; j < NQ; ++j) s += Mi[i * NQ + j] * m[j];
    f[i] = s;
  }
}

/* Eq. (25): central-moment MRT collision with forcing.  omega[0..10] are the
 * rates omega_0..omega_10.  The moment combinations of Eq. (25) are relaxed
 * and then solved back for the individual moments.  k*_000 = rho. */
void orc_collide(int32_t model, int32_t use_q, const double *f, double rho, const double *u,
                 double p, const double *F, const double *Qin, const double *omega,
                 double *fstar) {
  double k[NQ], feq[NQ], ke[NQ], ks[NQ];
  double Q[3] = {0.0, 0.0, 0.0};
  if (use_q) {
    Q[0] = Qin[0];
    Q[1] = Qin[1];
    Q[2] = Qin[2];
  }
  const double w0 = omega[0], w1 = omega[1], w2 = omega[2], w3 = omega[3], w4 = omega[4],
               w5 = omega[5], w6 = omega[6], w7 = omega[7], w8 = omega[8], w9 = omega[9],
               w10 = omega[10];
  orc_central_moments(f, u, k);
  orc_feq(model, rho, p, u, feq);
  orc_central_moments(feq, u, ke);

  ks[MI(0, 0, 0)] = rho;
  /* first order */
  ks[MI(1, 0, 0)] = (1.0 - w0) * k[MI(1, 0, 0)] + (1.0 - w0 / 2.0) * F[0];
  ks[MI(0, 1, 0)] = (1.0 - w0) * k[MI(0, 1, 0)] + (1.0 - w0 / 2.0) * F[1];
  ks[MI(0, 0, 1)] = (1.0 - w0) * k[MI(0, 0, 1)] + (1.0 - w0 / 2.0) * F[2];
  /* second order, off-diagonal (as printed, k^eq of these moments is zero) */
  ks[MI(1, 1, 0)] = (1.0 - w1) * k[MI(1, 1, 0)];
  ks[MI(0, 1, 1)] = (1.0 - w1) * k[MI(0, 1, 1)];
  ks[MI(1, 0, 1)] = (1.0 - w1) * k[MI(1, 0, 1)];
  /* second order, diagonal combinations */
  {
    double kxx = k[MI(2, 0, 0)], kyy = k[MI(0, 2, 0)], kzz = k[MI(0, 0, 2)];
    double exx = ke[MI(2, 0, 0)], eyy = ke[MI(0, 2, 0)], ezz = ke[MI(0, 0, 2)];
    double A = (1.0 - w1) * (kxx - kyy) + w1 * (exx - eyy) + (1.0 - w1 / 2.0) * (Q[0] - Q[1]);
    double B = (1.0 - w1) * (kxx - kzz) + w1 * (exx - ezz) + (1.0 - w1 / 2.0) * (Q[0] - Q[2]);
    double T = (1.0 - w2) * (kxx + kyy + kzz) + w2 * (exx + eyy + ezz) +
               (1.0 - w2 / 2.0) * (Q[0] + Q[1] + Q[2]);
    /* A = k200-k020, B = k200-k002, T = k200+k020+k002 */
    ks[MI(2, 0, 0)] = (A + B + T) / 3.0;
    ks[MI(0, 2, 0)] = (T - 2.0 * A + B) / 3.0;
    ks[MI(0, 0, 2)] = (T + A - 2.0 * B) / 3.0;
  }
  /* third order: sums with omega_3 (+ forcing), differences with omega_4 */
  {
    /* pairs (k120, k102) with F_x; (k210, k012) with F_y; (k201, k021) with F_z */
    const int pa[3] = {MI(1, 2, 0), MI(2, 1, 0), MI(2, 0, 1)};
    const int pb[3] = {MI(1, 0, 2), MI(0, 1, 2), MI(0, 2, 1)};
    for (int d = 0; d < 3; ++d) {
      double S = (1.0 - w3) * (k[pa[d]] + k[pb[d]]) + w3 * (ke[pa[d]] + ke[pb[d]]) +
                 2.0 * (1.0 - w3 / 2.0) * F[d] * CS2;
      double D = (1.0 - w4) * (k[pa[d]] - k[pb[d]]) + w4 * (ke[pa[d]] - ke[pb[d]]);
      ks[pa[d]] = (S + D) / 2.0;
      ks[pb[d]] = (S - D) / 2.0;
    }
  }
  ks[MI(1, 1, 1)] = (1.0 - w5) * k[MI(1, 1, 1)] + w5 * ke[MI(1, 1, 1)];
  /* fourth order */
  {
    double a = k[MI(2, 2, 0)], b = k[MI(2, 0, 2)], c = k[MI(0, 2, 2)];
    double ea = ke[MI(2, 2, 0)], eb = ke[MI(2, 0, 2)], ec = ke[MI(0, 2, 2)];
    double X = (1.0 - w6) * (a - 2.0 * b + c) + w6 * (ea - 2.0 * eb + ec);
    double Y = (1.0 - w6) * (a + b - 2.0 * c) + w6 * (ea + eb - 2.0 * ec);
    double Z = (1.0 - w7) * (a + b + c) + w7 * (ea + eb + ec);
    ks[MI(2, 2, 0)] = (X + Y + Z) / 3.0;
    ks[MI(2, 0, 2)] = (Z - X) / 3.0;
    ks[MI(0, 2, 2)] = (Z - Y) / 3.0;
  }
  ks[MI(2, 1, 1)] = (1.0 - w8) * k[MI(2, 1, 1)] + w8 * ke[MI(2, 1, 1)];
  ks[MI(1, 2, 1)] = (1.0 - w8) * k[MI(1, 2, 1)] + w8 * ke[MI(1, 2, 1)];
  ks[MI(1, 1, 2)] = (1.0 - w8) * k[MI(1, 1, 2)] + w8 * ke[MI(1, 1, 2)];
  /* fifth order */
  ks[MI(1, 2, 2)] = (1.0 - w9) * k[MI(1, 2, 2)] + w9 * ke[MI(1, 2, 2)] +
                    (1.0 - w9 / 2.0) * F[0] * CS2 * CS2;
  ks[MI(2, 1, 2)] = (1.0 - w9) * k[MI(2, 1, 2)] + w9 * ke[MI(2, 1, 2)] +
                    (1.0 - w9 / 2.0) * F[1] * CS2 * CS2;
  ks[MI(2, 2, 1)] = (1.0 - w9) * k[MI(2, 2, 1)] + w9 * ke[MI(2, 2, 1)] +
                    (1.0 - w9 / 2.0) * F[2] * CS2 * CS2;
  /* sixth order */
  ks[MI(2, 2, 2)] = (1.0 - w10) * k[MI(2, 2, 2)] + w10 * ke[MI(2, 2, 2)];

  orc_cm_to_f(ks, u, fstar);
}

/* Eqs. (18)-(19): recolouring. */
void orc_recolour(const double *fstar, double rho_r, double rho_b, double p, const double *n,
                  double beta, double *fr, double *fb) {
  double rho = rho_r + rho_b;
  double R[3];
  for (int a = 0; a < 3; ++a) R[a] = beta * rho_r * rho_b / (rho * rho) * p * n[a];
  for (int i = 0; i < NQ; ++i) {
    double cR = CX[i] * R[0] + CY[i] * R[1] + CZ[i] * R[2];
    fr[i] = rho_r / rho * fstar[i] + g_w[i] / CS2 * cR;
    fb[i] = rho_b / rho * fstar[i] - g_w[i] / CS2 * cR;
  }
}

/* Eq. (13) with (c_s^k)^2 = xi (1 - alpha_k). */
double orc_sound_speed2(double alpha) { return XI * (1.0 - alpha); }

/* SplitMix64 (Steele, Lea, Flood 2014): output function applied to a state. */
uint64_t orc_splitmix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Counter-based noise: state = seed + golden * counter, counter packs
 * (box, node, i); 24-bit uniform in [0, 1) mapped to [-amp, amp). */
double orc_noise(uint64_t seed, int32_t box, int64_t node, int32_t i, double amp) {
  uint64_t ctr = ((uint64_t)(uint32_t)box << 48) ^ ((uint64_t)node << 5) ^ (uint64_t)i;
  uint64_t z = orc_splitmix64(seed + 0x9E3779B97F4A7C15ULL * ctr);
  double uni = (double)(z >> 40) * (1.0 / 16777216.0);
  return amp * (2.0 * uni - 1.0);
}

/* ---------------------------------------------------------------------- */
/* Grid level                                                              */
/* ---------------------------------------------------------------------- */

int orc_num_threads(void) { return omp_get_max_threads(); }

/* Threads of the parallel loops from now on (n >= 1). */
void orc_set_num_threads(int32_t n) {
  if (n >= 1) omp_set_num_threads(n);
}

int orc_is_solid(const orc_params *P, int32_t x, int32_t y, int32_t z) {
  (void)x;
  if ((P->walls & 1u) && (y == 0 || y == P->ny - 1)) return 1;
  if ((P->walls & 2u) && (z == 0 || z == P->nz - 1)) return 1;
  return 0;
}

static int64_t node_of(const orc_params *P, int x, int y, int z) {
  return (int64_t)x + (int64_t)P->nx * ((int64_t)y + (int64_t)P->ny * z);
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Eq. (20) at one fluid node: (1/c_s^2) sum_i w_i chi(x + c_i) c_i.  A
 * neighbour in a solid layer takes the value of the centre node. */
static void grad_at(const orc_params *P, const double *chi, int x, int y, int z, double *g) {
  int64_t c0 = node_of(P, x, y, z);
  g[0] = g[1] = g[2] = 0.0;
  for (int i = 0; i < NQ; ++i) {
    int xn = wrap(x + CX[i], P->nx), yn = wrap(y + CY[i], P->ny), zn = wrap(z + CZ[i], P->nz);
    double v = orc_is_solid(P, xn, yn, zn) ? chi[c0] : chi[node_of(P, xn, yn, zn)];
    g[0] += g_w[i] * v * CX[i];
    g[1] += g_w[i] * v * CY[i];
    g[2] += g_w[i] * v * CZ[i];
  }
  g[0] /= CS2;
  g[1] /= CS2;
  g[2] /= CS2;
}

int orc_gradient(const orc_params *P, const double *chi, double *out) {
  const int64_t N = (int64_t)P->nx * P->ny * P->nz;
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < P->nz; ++z)
    for (int y = 0; y < P->ny; ++y)
      for (int x = 0; x < P->nx; ++x) {
        int64_t c = node_of(P, x, y, z);
        double g[3] = {0.0, 0.0, 0.0};
        if (!orc_is_solid(P, x, y, z)) grad_at(P, chi, x, y, z, g);
        out[c] = g[0];
        out[N + c] = g[1];
        out[2 * N + c] = g[2];
      }
  return 0;
}

/* Work arrays of one step. */
typedef struct {
  double *rho_r, *rho_b, *rho, *p, *phi, *j;  /* j: [3][N] */
  double *gphi, *n, *kappa, *F, *u, *q, *Q;   /* [3][N] except kappa */
} fields_t;

static int fields_alloc(fields_t *W, int64_t N) {
  memset(W, 0, sizeof(*W));
  W->rho_r = malloc(sizeof(double) * N);
  W->rho_b = malloc(sizeof(double) * N);
  W->rho = malloc(sizeof(double) * N);
  W->p = malloc(sizeof(double) * N);
  W->phi = malloc(sizeof(double) * N);
  W->kappa = malloc(sizeof(double) * N);
  W->j = malloc(sizeof(double) * 3 * N);
  W->gphi = malloc(sizeof(double) * 3 * N);
  W->n = malloc(sizeof(double) * 3 * N);
  W->F = malloc(sizeof(double) * 3 * N);
  W->u = malloc(sizeof(double) * 3 * N);
  W->q = malloc(sizeof(double) * 3 * N);
  W->Q = malloc(sizeof(double) * 3 * N);
  return (W->rho_r && W->rho_b && W->rho && W->p && W->phi && W->kappa && W->j && W->gphi &&
          W->n && W->F && W->u && W->q && W->Q)
             ? 0
             : -1;
}

static void fields_free(fields_t *W) {
  free(W->rho_r); free(W->rho_b); free(W->rho); free(W->p); free(W->phi); free(W->kappa);
  free(W->j); free(W->gphi); free(W->n); free(W->F); free(W->u); free(W->q); free(W->Q);
}

/* Steps O1-O6: macroscopic and interface fields of the state f at time t. */
static void compute_fields(const orc_params *P, const double *f, fields_t *W) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const int64_t N = (int64_t)nx * ny * nz;
  const double cs2r = orc_sound_speed2(P->alpha_r), cs2b = orc_sound_speed2(P->alpha_b);

  /* Eqs. (10)-(14): colour densities, momentum sum, pressure, order parameter */
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    double rr = 0.0, rb = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < NQ; ++i) {
      double fr = f[(int64_t)i * N + c], fb = f[(int64_t)(NQ + i) * N + c];
      rr += fr;
      rb += fb;
      jx += (fr + fb) * CX[i];
      jy += (fr + fb) * CY[i];
      jz += (fr + fb) * CZ[i];
    }
    W->rho_r[c] = rr;
    W->rho_b[c] = rb;
    W->rho[c] = rr + rb;
    W->p[c] = rr * cs2r + rb * cs2b;
    W->phi[c] = (rr / P->rho0_r - rb / P->rho0_b) / (rr / P->rho0_r + rb / P->rho0_b);
    W->j[c] = jx;
    W->j[N + c] = jy;
    W->j[2 * N + c] = jz;
  }
  /* Eqs. (17), (20): gradient of phi and unit normal */
  orc_gradient(P, W->phi, W->gphi);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    double gx = W->gphi[c], gy = W->gphi[N + c], gz = W->gphi[2 * N + c];
    double mag = sqrt(gx * gx + gy * gy + gz * gz);
    if (mag > 1e-12) {
      W->n[c] = gx / mag;
      W->n[N + c] = gy / mag;
      W->n[2 * N + c] = gz / mag;
    } else {
      W->n[c] = W->n[N + c] = W->n[2 * N + c] = 0.0;
    }
  }
  /* Eqs. (15)-(16), (11): curvature from the gradient of each component of n,
   * CSF force, velocity including half the force */
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t c = node_of(P, x, y, z);
        double kap = 0.0, Fx = 0.0, Fy = 0.0, Fz = 0.0;
        if (!orc_is_solid(P, x, y, z)) {
          double dn[3][3]; /* dn[a][b] = d n_a / d x_b */
          for (int a = 0; a < 3; ++a) grad_at(P, W->n + a * N, x, y, z, dn[a]);
          double nv[3] = {W->n[c], W->n[N + c], W->n[2 * N + c]};
          /* kappa = -(I - n n) : grad n = -sum_a dn_a/dx_a + sum_ab n_a n_b dn_a/dx_b */
          double div = dn[0][0] + dn[1][1] + dn[2][2];
          double proj = 0.0;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) proj += nv[a] * nv[b] * dn[a][b];
          kap = -(div - proj);
          /* Eq. (15) plus the constant body force and the buoyancy force
           * -(rho - rho_ref) g of the Rayleigh-Taylor case (Sec. IV.E) */
          const double drho = W->rho[c] - P->rho_ref;
          Fx = 0.5 * P->sigma * kap * W->gphi[c] + P->body_force[0] - drho * P->gravity[0];
          Fy = 0.5 * P->sigma * kap * W->gphi[N + c] + P->body_force[1] - drho * P->gravity[1];
          Fz = 0.5 * P->sigma * kap * W->gphi[2 * N + c] + P->body_force[2] - drho * P->gravity[2];
        }
        W->kappa[c] = kap;
        W->F[c] = Fx;
        W->F[N + c] = Fy;
        W->F[2 * N + c] = Fz;
        W->u[c] = (W->j[c] + Fx / 2.0) / W->rho[c];
        W->u[N + c] = (W->j[N + c] + Fy / 2.0) / W->rho[c];
        W->u[2 * N + c] = (W->j[2 * N + c] + Fz / 2.0) / W->rho[c];
      }
  /* Eq. (65), component-wise: Q_a = -3 d/dx_a [(p - rho c_s^2) u_a] */
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c)
    for (int a = 0; a < 3; ++a) W->q[a * N + c] = (W->p[c] - W->rho[c] * CS2) * W->u[a * N + c];
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t c = node_of(P, x, y, z);
        for (int a = 0; a < 3; ++a) {
          double Qa = 0.0;
          if (!orc_is_solid(P, x, y, z)) {
            double g[3];
            grad_at(P, W->q + a * N, x, y, z, g);
            Qa = -3.0 * g[a];
          }
          W->Q[a * N + c] = Qa;
        }
      }
}

int orc_fields(const orc_params *P, const double *f, double *out) {
  const int64_t N = (int64_t)P->nx * P->ny * P->nz;
  fields_t W;
  if (fields_alloc(&W, N)) {
    fields_free(&W);
    return -1;
  }
  compute_fields(P, f, &W);
  memcpy(out + 0 * N, W.rho_r, sizeof(double) * N);
  memcpy(out + 1 * N, W.rho_b, sizeof(double) * N);
  memcpy(out + 2 * N, W.phi, sizeof(double) * N);
  memcpy(out + 3 * N, W.p, sizeof(double) * N);
  memcpy(out + 4 * N, W.u, sizeof(double) * 3 * N);
  memcpy(out + 7 * N, W.n, sizeof(double) * 3 * N);
  memcpy(out + 10 * N, W.kappa, sizeof(double) * N);
  memcpy(out + 11 * N, W.F, sizeof(double) * 3 * N);
  memcpy(out + 14 * N, W.Q, sizeof(double) * 3 * N);
  fields_free(&W);
  return 0;
}

/* One full step (O1-O12): fields, collision of the total distribution in
 * central-moment space, recolouring, streaming.  Solid nodes do not collide:
 * they reverse the populations that arrived (full-way bounce-back). */
int orc_step(const orc_params *P, double *f, int32_t nsteps) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const int64_t N = (int64_t)nx * ny * nz;
  double *post = malloc(sizeof(double) * 2 * NQ * N);
  fields_t W;
  if (!post || fields_alloc(&W, N)) {
    free(post);
    fields_free(&W);
    return -1;
  }
  int opp[NQ];
  for (int i = 0; i < NQ; ++i) opp[i] = opposite(i);
  (void)minv_table();

  for (int step = 0; step < nsteps; ++step) {
    compute_fields(P, f, &W);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          int64_t c = node_of(P, x, y, z);
          if (orc_is_solid(P, x, y, z)) {
            for (int i = 0; i < NQ; ++i) {
              post[(int64_t)opp[i] * N + c] = f[(int64_t)i * N + c];
              post[(int64_t)(NQ + opp[i]) * N + c] = f[(int64_t)(NQ + i) * N + c];
            }
            continue;
          }
          double ft[NQ], fs[NQ], fr[NQ], fb[NQ];
          for (int i = 0; i < NQ; ++i) ft[i] = f[(int64_t)i * N + c] + f[(int64_t)(NQ + i) * N + c];
          /* Eqs. (21)-(22): viscosity interpolation and relaxation time */
          double ph = W.phi[c];
          double nu = 0.5 * (1.0 + ph) * P->nu_r + 0.5 * (1.0 - ph) * P->nu_b;
          double tau = W.rho[c] * nu / W.p[c] + 0.5;
          double om[11];
          for (int r = 0; r < 11; ++r) om[r] = P->omega[r];
          om[1] = 1.0 / tau;
          double u[3] = {W.u[c], W.u[N + c], W.u[2 * N + c]};
          double F[3] = {W.F[c], W.F[N + c], W.F[2 * N + c]};
          double Q[3] = {W.Q[c], W.Q[N + c], W.Q[2 * N + c]};
          double n[3] = {W.n[c], W.n[N + c], W.n[2 * N + c]};
          orc_collide(P->model, P->use_q, ft, W.rho[c], u, W.p[c], F, Q, om, fs);
          orc_recolour(fs, W.rho_r[c], W.rho_b[c], W.p[c], n, P->beta, fr, fb);
          for (int i = 0; i < NQ; ++i) {
            post[(int64_t)i * N + c] = fr[i];
            post[(int64_t)(NQ + i) * N + c] = fb[i];
          }
        }
    /* Eq. (5): streaming of each colour, periodic wrap */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          int64_t c = node_of(P, x, y, z);
          for (int i = 0; i < NQ; ++i) {
            int64_t d = node_of(P, wrap(x + CX[i], nx), wrap(y + CY[i], ny), wrap(z + CZ[i], nz));
            f[(int64_t)i * N + d] = post[(int64_t)i * N + c];
            f[(int64_t)(NQ + i) * N + d] = post[(int64_t)(NQ + i) * N + c];
          }
        }
  }
  free(post);
  fields_free(&W);
  return 0;
}

/* Initial state: f = f^eq(rho, p, u) + noise, split by colour fraction
 * rho_k / rho so that pure phases stay pure. */
int orc_init(const orc_params *P, const double *rho_r, const double *rho_b, const double *u,
             uint64_t seed, double amp, int32_t box, double *f) {
  const int32_t dims[3] = {P->nx, P->ny, P->nz};
  const int32_t zero[3] = {0, 0, 0};
  return orc_init_window(P, rho_r, rho_b, u, seed, amp, box, dims, zero, f);
}

/* As orc_init for a window of a larger periodic box: node (x, y, z) of the
 * window is node ((x+ox) mod Nx, (y+oy) mod Ny, (z+oz) mod Nz) of the larger
 * box, whose index keys the noise. */
int orc_init_window(const orc_params *P, const double *rho_r, const double *rho_b,
                    const double *u, uint64_t seed, double amp, int32_t box,
                    const int32_t *gdims, const int32_t *goff, double *f) {
  const int64_t N = (int64_t)P->nx * P->ny * P->nz;
  const double cs2r = orc_sound_speed2(P->alpha_r), cs2b = orc_sound_speed2(P->alpha_b);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t c = 0; c < N; ++c) {
    double rho = rho_r[c] + rho_b[c];
    if (!(rho > 0.0)) {
      bad = 1;
      continue;
    }
    double p = rho_r[c] * cs2r + rho_b[c] * cs2b;
    double uu[3] = {u[c], u[N + c], u[2 * N + c]};
    double feq[NQ];
    orc_feq(P->model, rho, p, uu, feq);
    const int64_t x = c % P->nx, y = (c / P->nx) % P->ny, z = c / ((int64_t)P->nx * P->ny);
    const int64_t gnode = (int64_t)wrap((int)(x + goff[0]), gdims[0]) +
                          (int64_t)gdims[0] * ((int64_t)wrap((int)(y + goff[1]), gdims[1]) +
                                               (int64_t)gdims[1] * wrap((int)(z + goff[2]), gdims[2]));
    for (int i = 0; i < NQ; ++i) {
      double ft = feq[i] + (amp != 0.0 ? orc_noise(seed, box, gnode, i, amp) : 0.0);
      f[(int64_t)i * N + c] = rho_r[c] / rho * ft;
      f[(int64_t)(NQ + i) * N + c] = rho_b[c] / rho * ft;
    }
  }
  return bad ? -1 : 0;
}
