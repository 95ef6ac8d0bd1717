/*
 * d2q9_oracle.c -- plain FP64 CPU oracle for the two-colour D2Q9
 * colour-gradient lattice Boltzmann step with the two-dimensional generalized
 * equilibrium of App. A (Saito et al., arXiv:2309.07801).
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code with the HIP path.
 *
 * The model is the one of Sec. II with the D2Q9 lattice of App. A:
 *   - lattice velocities Eq. (A1), weights Eq. (A2), c_s^2 = 1/3;
 *   - equilibrium Eq. (A10): the fourth-order Hermite expansion Eq. (A3) plus
 *     (p - rho c_s^2) times the isotropic operator Eq. (A9) and its velocity
 *     terms, evaluated by literal Hermite sums (Eqs. A4-A8);
 *   - central moments by their definition (Eq. A11), back-transform through
 *     raw moments (binomial shift) and the inverse 9x9 raw-moment matrix;
 *   - collision: the two-dimensional form of the central-moment MRT of
 *     Eq. (25) (reading: first order omega_0; k_11 and k_20 - k_02 omega_1;
 *     k_20 + k_02 omega_2; k_21, k_12 omega_3 with the forcing moments
 *     c_s^2 F; k_22 omega_4), Q added to the diagonal second-order moments;
 *   - colour densities, pressure, order parameter, CSF force, curvature,
 *     isotropic gradients, viscosity interpolation and recolouring as in
 *     Eqs. (10)-(22) with the D2Q9 weights;
 *   - xi = 3/5: with phi_0 = 1 - p / (xi rho) and phi_i = w_i p / (rho c_s^2)
 *     (Eq. 8) the rest fractions sum to one only for xi = c_s^2 / (1 - w_0).
 * No blocking or fusion beyond the definitions.
 */
#include "d2q9_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define NQ 9
#define MI(a, b) ((a) + 3 * (b))
static const double CS2 = 1.0 / 3.0;

/* Eq. (A1): columns of the printed 2x9 matrix. */
static const int CX[NQ] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int CY[NQ] = {0, 0, 0, 1, -1, 1, -1, -1, 1};

/* Eq. (A2): weight by |c_i|^2 = 0, 1, 2. */
static double weight(int i) {
  switch (CX[i] * CX[i] + CY[i] * CY[i]) {
    case 0: return 4.0 / 9.0;
    case 1: return 1.0 / 9.0;
    default: return 1.0 / 36.0;
  }
}

static int opposite(int i) {
  for (int j = 0; j < NQ; ++j)
    if (CX[j] == -CX[i] && CY[j] == -CY[i]) return j;
  return -1;
}

double orc2_xi(void) { return CS2 / (1.0 - weight(0)); }

void orc2_lattice(int32_t *c, double *w) {
  for (int i = 0; i < NQ; ++i) {
    c[2 * i + 0] = CX[i];
    c[2 * i + 1] = CY[i];
    w[i] = weight(i);
  }
}

/* Eqs. (A4)-(A8): one-dimensional factors H_0 = 1, H_1 = c, H_2 = c^2 - c_s^2;
 * the mixed polynomials are their products (H_11 = H_10 H_01, H_12 = H_10 H_02,
 * H_21 = H_20 H_01, H_22 = H_20 H_02). */
static double h1(int order, int c) {
  if (order == 0) return 1.0;
  if (order == 1) return (double)c;
  return (double)(c * c) - CS2;
}

double orc2_hermite(int32_t i, int32_t a, int32_t b) { return h1(a, CX[i]) * h1(b, CY[i]); }

/* Eq. (A3): fourth-order Hermite equilibrium of the single-phase D2Q9 model. */
void orc2_geq4(double rho, const double *u, double *g) {
  const double ux = u[0], uy = u[1];
  for (int i = 0; i < NQ; ++i) {
    double s = 1.0;
    s += (ux * orc2_hermite(i, 1, 0) + uy * orc2_hermite(i, 0, 1)) / CS2;
    s += (ux * ux * orc2_hermite(i, 2, 0) + uy * uy * orc2_hermite(i, 0, 2) +
          2.0 * ux * uy * orc2_hermite(i, 1, 1)) /
         (2.0 * CS2 * CS2);
    s += (ux * ux * uy * orc2_hermite(i, 2, 1) + ux * uy * uy * orc2_hermite(i, 1, 2)) /
         (2.0 * CS2 * CS2 * CS2);
    s += ux * ux * uy * uy * orc2_hermite(i, 2, 2) / (4.0 * CS2 * CS2 * CS2 * CS2);
    g[i] = rho * weight(i) * s;
  }
}

/* Eq. (A9): isotropic operator of the D2Q9 lattice. */
double orc2_isotropic_E(int32_t i) {
  return weight(i) * ((orc2_hermite(i, 2, 0) + orc2_hermite(i, 0, 2)) / (2.0 * CS2 * CS2) -
                      orc2_hermite(i, 2, 2) / (4.0 * CS2 * CS2 * CS2));
}

/* Eq. (A10): generalized equilibrium for the D2Q9 lattice. */
void orc2_feq(double rho, double p, const double *u, double *feq) {
  const double ux = u[0], uy = u[1];
  double g[NQ];
  orc2_geq4(rho, u, g);
  for (int i = 0; i < NQ; ++i) {
    double v = (ux * orc2_hermite(i, 1, 2) + uy * orc2_hermite(i, 2, 1)) / (2.0 * CS2 * CS2 * CS2) +
               (ux * ux + uy * uy) * orc2_hermite(i, 2, 2) / (4.0 * CS2 * CS2 * CS2 * CS2);
    feq[i] = g[i] + (p - rho * CS2) * (orc2_isotropic_E(i) + weight(i) * v);
  }
}

static double ipow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; ++k) r *= x;
  return r;
}

/* Raw moments m_ab = sum_i f_i cx^a cy^b (two-dimensional Eq. 23). */
void orc2_raw_moments(const double *f, double *m) {
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int i = 0; i < NQ; ++i) s += f[i] * ipow(CX[i], a) * ipow(CY[i], b);
      m[MI(a, b)] = s;
    }
}

/* Eq. (A11): central moments by their definition. */
void orc2_central_moments(const double *f, const double *u, double *k) {
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int i = 0; i < NQ; ++i) s += f[i] * ipow(CX[i] - u[0], a) * ipow(CY[i] - u[1], b);
      k[MI(a, b)] = s;
    }
}

/* Inverse of the 9x9 raw-moment matrix M[(ab), i] = cx^a cy^b, by
 * Gauss-Jordan elimination with partial pivoting, computed once. */
static double g_minv[NQ * NQ];
static int g_minv_ready = 0;

static void invert_moment_matrix(void) {
  double A[NQ][2 * NQ];
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < NQ; ++i) {
        A[MI(a, b)][i] = ipow(CX[i], a) * ipow(CY[i], b);
        A[MI(a, b)][NQ + i] = (MI(a, b) == i) ? 1.0 : 0.0;
      }
  for (int col = 0; col < NQ; ++col) {
    int piv = col;
    for (int r = col + 1; r < NQ; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
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
      for (int c = 0; c < 2 * NQ; ++c) A[r][c] -= fct * A[col][c];
    }
  }
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) g_minv[r * NQ + c] = A[r][NQ + c];
}

static const double *minv_table(void) {
  if (!g_minv_ready) {
#pragma omp critical(orc2_minv)
    {
      if (!g_minv_ready) {
        invert_moment_matrix();
        g_minv_ready = 1;
      }
    }
  }
  return g_minv;
}

/* Central moments -> raw moments (binomial expansion of ((c - u) + u)^a) ->
 * f through the inverse raw-moment matrix. */
void orc2_cm_to_f(const double *k, const double *u, double *f) {
  static const double binom[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 2, 1}};
  double m[NQ];
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int b2 = 0; b2 <= b; ++b2)
        for (int a2 = 0; a2 <= a; ++a2)
          s += binom[a][a2] * binom[b][b2] * ipow(u[0], a - a2) * ipow(u[1], b - b2) *
               k[MI(a2, b2)];
      m[MI(a, b)] = s;
    }
  const double *Mi = minv_table();
  for (int i = 0; i < NQ; ++i) {
    double s = 0.0;
    for (int j = 0; j < NQ; ++j) s += Mi[i * NQ + j] * m[j];
    f[i] = s;
  }
}

/* Two-dimensional Eq. (25): central-moment MRT collision with forcing (first
 * order F, third order c_s^2 F) and the correction Q on the diagonal
 * second-order moments.  omega[0..4] as in orc2_params.  k*_00 = rho. */
void orc2_collide(int32_t use_q, const double *f, double rho, const double *u, double p,
                  const double *F, const double *Qin, const double *omega, double *fstar) {
  double k[NQ], feq[NQ], ke[NQ], ks[NQ];
  const double Qx = use_q ? Qin[0] : 0.0, Qy = use_q ? Qin[1] : 0.0;
  const double w0 = omega[0], w1 = omega[1], w2 = omega[2], w3 = omega[3], w4 = omega[4];
  orc2_central_moments(f, u, k);
  orc2_feq(rho, p, u, feq);
  orc2_central_moments(feq, u, ke);

  ks[MI(0, 0)] = rho;
  ks[MI(1, 0)] = (1.0 - w0) * k[MI(1, 0)] + (1.0 - w0 / 2.0) * F[0];
  ks[MI(0, 1)] = (1.0 - w0) * k[MI(0, 1)] + (1.0 - w0 / 2.0) * F[1];
  ks[MI(1, 1)] = (1.0 - w1) * k[MI(1, 1)] + w1 * ke[MI(1, 1)];
  {
    const double kxx = k[MI(2, 0)], kyy = k[MI(0, 2)], exx = ke[MI(2, 0)], eyy = ke[MI(0, 2)];
    const double D = (1.0 - w1) * (kxx - kyy) + w1 * (exx - eyy) + (1.0 - w1 / 2.0) * (Qx - Qy);
    const double T = (1.0 - w2) * (kxx + kyy) + w2 * (exx + eyy) + (1.0 - w2 / 2.0) * (Qx + Qy);
    ks[MI(2, 0)] = (T + D) / 2.0;
    ks[MI(0, 2)] = (T - D) / 2.0;
  }
  /* k_21 = sum f (cx-ux)^2 (cy-uy) carries F_y, k_12 carries F_x */
  ks[MI(2, 1)] = (1.0 - w3) * k[MI(2, 1)] + w3 * ke[MI(2, 1)] + (1.0 - w3 / 2.0) * F[1] * CS2;
  ks[MI(1, 2)] = (1.0 - w3) * k[MI(1, 2)] + w3 * ke[MI(1, 2)] + (1.0 - w3 / 2.0) * F[0] * CS2;
  ks[MI(2, 2)] = (1.0 - w4) * k[MI(2, 2)] + w4 * ke[MI(2, 2)];
  orc2_cm_to_f(ks, u, fstar);
}

/* Eqs. (18)-(19) with the D2Q9 weights. */
void orc2_recolour(const double *fstar, double rho_r, double rho_b, double p, const double *n,
                   double beta, double *fr, double *fb) {
  const double rho = rho_r + rho_b;
  const double Rx = beta * rho_r * rho_b / (rho * rho) * p * n[0];
  const double Ry = beta * rho_r * rho_b / (rho * rho) * p * n[1];
  for (int i = 0; i < NQ; ++i) {
    const double cR = CX[i] * Rx + CY[i] * Ry;
    fr[i] = rho_r / rho * fstar[i] + weight(i) / CS2 * cR;
    fb[i] = rho_b / rho * fstar[i] - weight(i) / CS2 * cR;
  }
}

/* SplitMix64 (Steele, Lea, Flood 2014), counter = (box, node, i) packed as
 * box << 48 ^ node << 5 ^ i; 24-bit uniform in [0, 1) mapped to [-amp, amp). */
static uint64_t splitmix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double orc2_noise(uint64_t seed, int32_t box, int64_t node, int32_t i, double amp) {
  uint64_t ctr = ((uint64_t)(uint32_t)box << 48) ^ ((uint64_t)node << 5) ^ (uint64_t)i;
  uint64_t z = splitmix64(seed + 0x9E3779B97F4A7C15ULL * ctr);
  double uni = (double)(z >> 40) * (1.0 / 16777216.0);
  return amp * (2.0 * uni - 1.0);
}

/* ---------------------------------------------------------------------- */
/* Grid level                                                              */
/* ---------------------------------------------------------------------- */

static int is_solid(const orc2_params *P, int y) {
  return (P->walls & 1u) && (y == 0 || y == P->ny - 1);
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Eq. (20) at one fluid node; a neighbour in a solid row takes the centre
 * node's value. */
static void grad_at(const orc2_params *P, const double *chi, int x, int y, double *g) {
  const int64_t c0 = (int64_t)x + (int64_t)P->nx * y;
  g[0] = g[1] = 0.0;
  for (int i = 0; i < NQ; ++i) {
    const int xn = wrap(x + CX[i], P->nx), yn = wrap(y + CY[i], P->ny);
    const double v = is_solid(P, yn) ? chi[c0] : chi[(int64_t)xn + (int64_t)P->nx * yn];
    g[0] += weight(i) * v * CX[i];
    g[1] += weight(i) * v * CY[i];
  }
  g[0] /= CS2;
  g[1] /= CS2;
}

typedef struct {
  double *rho_r, *rho_b, *rho, *p, *phi, *kappa;
  double *j, *gphi, *n, *F, *u, *q, *Q; /* [2][N] */
} fields_t;

static void fields_free(fields_t *W) {
  free(W->rho_r); free(W->rho_b); free(W->rho); free(W->p); free(W->phi); free(W->kappa);
  free(W->j); free(W->gphi); free(W->n); free(W->F); free(W->u); free(W->q); free(W->Q);
}

static int fields_alloc(fields_t *W, int64_t N) {
  memset(W, 0, sizeof(*W));
  double **one[] = {&W->rho_r, &W->rho_b, &W->rho, &W->p, &W->phi, &W->kappa};
  double **two[] = {&W->j, &W->gphi, &W->n, &W->F, &W->u, &W->q, &W->Q};
  int ok = 1;
  for (unsigned k = 0; k < sizeof(one) / sizeof(one[0]); ++k)
    ok &= (*one[k] = malloc(sizeof(double) * N)) != NULL;
  for (unsigned k = 0; k < sizeof(two) / sizeof(two[0]); ++k)
    ok &= (*two[k] = malloc(sizeof(double) * 2 * N)) != NULL;
  return ok ? 0 : -1;
}

/* Macroscopic and interface fields of the state f at time t. */
static void compute_fields(const orc2_params *P, const double *f, fields_t *W) {
  const int nx = P->nx, ny = P->ny;
  const int64_t N = (int64_t)nx * ny;
  const double xi = orc2_xi();
  const double cs2r = xi * (1.0 - P->alpha_r), cs2b = xi * (1.0 - P->alpha_b);

  /* Eqs. (10)-(14) */
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    double rr = 0.0, rb = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < NQ; ++i) {
      const double fr = f[(int64_t)i * N + c], fb = f[(int64_t)(NQ + i) * N + c];
      rr += fr;
      rb += fb;
      jx += (fr + fb) * CX[i];
      jy += (fr + fb) * CY[i];
    }
    W->rho_r[c] = rr;
    W->rho_b[c] = rb;
    W->rho[c] = rr + rb;
    W->p[c] = rr * cs2r + rb * cs2b;
    W->phi[c] = (rr / P->rho0_r - rb / P->rho0_b) / (rr / P->rho0_r + rb / P->rho0_b);
    W->j[c] = jx;
    W->j[N + c] = jy;
  }
  /* Eqs. (17), (20): gradient of phi and unit normal */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int64_t c = (int64_t)x + (int64_t)nx * y;
      double g[2] = {0.0, 0.0};
      if (!is_solid(P, y)) grad_at(P, W->phi, x, y, g);
      W->gphi[c] = g[0];
      W->gphi[N + c] = g[1];
      const double mag = sqrt(g[0] * g[0] + g[1] * g[1]);
      W->n[c] = mag > 1e-12 ? g[0] / mag : 0.0;
      W->n[N + c] = mag > 1e-12 ? g[1] / mag : 0.0;
    }
  /* Eqs. (15)-(16), (11): curvature -(I - n n) : grad n, CSF force, velocity */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int64_t c = (int64_t)x + (int64_t)nx * y;
      double kap = 0.0, Fx = 0.0, Fy = 0.0;
      if (!is_solid(P, y)) {
        double dn[2][2]; /* dn[a][b] = d n_a / d x_b */
        grad_at(P, W->n, x, y, dn[0]);
        grad_at(P, W->n + N, x, y, dn[1]);
        const double nv[2] = {W->n[c], W->n[N + c]};
        double proj = 0.0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) proj += nv[a] * nv[b] * dn[a][b];
        kap = -(dn[0][0] + dn[1][1] - proj);
        Fx = 0.5 * P->sigma * kap * W->gphi[c] + P->body_force[0];
        Fy = 0.5 * P->sigma * kap * W->gphi[N + c] + P->body_force[1];
      }
      W->kappa[c] = kap;
      W->F[c] = Fx;
      W->F[N + c] = Fy;
      W->u[c] = (W->j[c] + Fx / 2.0) / W->rho[c];
      W->u[N + c] = (W->j[N + c] + Fy / 2.0) / W->rho[c];
    }
  /* Eq. (65) in two dimensions, component-wise: Q_a = -3 d/dx_a [(p - rho c_s^2) u_a] */
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c)
    for (int a = 0; a < 2; ++a) W->q[a * N + c] = (W->p[c] - W->rho[c] * CS2) * W->u[a * N + c];
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int64_t c = (int64_t)x + (int64_t)nx * y;
      for (int a = 0; a < 2; ++a) {
        double Qa = 0.0;
        if (!is_solid(P, y)) {
          double g[2];
          grad_at(P, W->q + a * N, x, y, g);
          Qa = -3.0 * g[a];
        }
        W->Q[a * N + c] = Qa;
      }
    }
}

int orc2_fields(const orc2_params *P, const double *f, double *out) {
  const int64_t N = (int64_t)P->nx * P->ny;
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
  memcpy(out + 4 * N, W.u, sizeof(double) * 2 * N);
  memcpy(out + 6 * N, W.n, sizeof(double) * 2 * N);
  memcpy(out + 8 * N, W.kappa, sizeof(double) * N);
  memcpy(out + 9 * N, W.F, sizeof(double) * 2 * N);
  memcpy(out + 11 * N, W.Q, sizeof(double) * 2 * N);
  fields_free(&W);
  return 0;
}

/* One full step: fields, collision of the total distribution in
 * central-moment space, recolouring, streaming of each colour.  Solid nodes
 * reverse the populations that arrived (full-way bounce-back). */
int orc2_step(const orc2_params *P, double *f, int32_t nsteps) {
  const int nx = P->nx, ny = P->ny;
  const int64_t N = (int64_t)nx * ny;
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
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t c = (int64_t)x + (int64_t)nx * y;
        if (is_solid(P, y)) {
          for (int i = 0; i < NQ; ++i) {
            post[(int64_t)opp[i] * N + c] = f[(int64_t)i * N + c];
            post[(int64_t)(NQ + opp[i]) * N + c] = f[(int64_t)(NQ + i) * N + c];
          }
          continue;
        }
        double ft[NQ], fs[NQ], fr[NQ], fb[NQ];
        for (int i = 0; i < NQ; ++i) ft[i] = f[(int64_t)i * N + c] + f[(int64_t)(NQ + i) * N + c];
        /* Eqs. (21)-(22) */
        const double ph = W.phi[c];
        const double nu = 0.5 * (1.0 + ph) * P->nu_r + 0.5 * (1.0 - ph) * P->nu_b;
        const double tau = W.rho[c] * nu / W.p[c] + 0.5;
        double om[5];
        for (int r = 0; r < 5; ++r) om[r] = P->omega[r];
        om[1] = 1.0 / tau;
        const double u[2] = {W.u[c], W.u[N + c]};
        const double F[2] = {W.F[c], W.F[N + c]};
        const double Q[2] = {W.Q[c], W.Q[N + c]};
        const double n[2] = {W.n[c], W.n[N + c]};
        orc2_collide(P->use_q, ft, W.rho[c], u, W.p[c], F, Q, om, fs);
        orc2_recolour(fs, W.rho_r[c], W.rho_b[c], W.p[c], n, P->beta, fr, fb);
        for (int i = 0; i < NQ; ++i) {
          post[(int64_t)i * N + c] = fr[i];
          post[(int64_t)(NQ + i) * N + c] = fb[i];
        }
      }
    /* Eq. (5): streaming, periodic wrap */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t c = (int64_t)x + (int64_t)nx * y;
        for (int i = 0; i < NQ; ++i) {
          const int64_t d = (int64_t)wrap(x + CX[i], nx) + (int64_t)nx * wrap(y + CY[i], ny);
          f[(int64_t)i * N + d] = post[(int64_t)i * N + c];
          f[(int64_t)(NQ + i) * N + d] = post[(int64_t)(NQ + i) * N + c];
        }
      }
  }
  free(post);
  fields_free(&W);
  return 0;
}

/* Initial state: f = f^eq(rho, p, u) + noise, split by the colour fraction
 * rho_k / rho so that pure phases stay pure. */
int orc2_init(const orc2_params *P, const double *rho_r, const double *rho_b, const double *u,
              uint64_t seed, double amp, int32_t box, double *f) {
  const int32_t dims[2] = {P->nx, P->ny};
  const int32_t zero[2] = {0, 0};
  return orc2_init_window(P, rho_r, rho_b, u, seed, amp, box, dims, zero, f);
}

/* As orc2_init for a window of a larger periodic box: node (x, y) of the
 * window is node ((x+ox) mod Nx, (y+oy) mod Ny) of the larger box, whose
 * index keys the noise. */
int orc2_init_window(const orc2_params *P, const double *rho_r, const double *rho_b,
                     const double *u, uint64_t seed, double amp, int32_t box,
                     const int32_t *gdims, const int32_t *goff, double *f) {
  const int64_t N = (int64_t)P->nx * P->ny;
  const double xi = orc2_xi();
  const double cs2r = xi * (1.0 - P->alpha_r), cs2b = xi * (1.0 - P->alpha_b);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t c = 0; c < N; ++c) {
    const double rho = rho_r[c] + rho_b[c];
    if (!(rho > 0.0)) {
      bad = 1;
      continue;
    }
    const double p = rho_r[c] * cs2r + rho_b[c] * cs2b;
    const double uu[2] = {u[c], u[N + c]};
    double feq[NQ];
    orc2_feq(rho, p, uu, feq);
    const int64_t gnode = (int64_t)wrap((int)(c % P->nx + goff[0]), gdims[0]) +
                          (int64_t)gdims[0] * wrap((int)(c / P->nx + goff[1]), gdims[1]);
    for (int i = 0; i < NQ; ++i) {
      const double ft = feq[i] + (amp != 0.0 ? orc2_noise(seed, box, gnode, i, amp) : 0.0);
      f[(int64_t)i * N + c] = rho_r[c] / rho * ft;
      f[(int64_t)(NQ + i) * N + c] = rho_b[c] / rho * ft;
    }
  }
  return bad ? -1 : 0;
}
