// lattice.hpp -- D3Q27 constants and per-node building blocks of the HIP path.
//
// Velocity order: the columns of the matrix of Eq. (1) of Saito et al.,
// arXiv:2309.07801; opposite directions are the pairs (2k-1, 2k).  Weights:
// Eq. (9), i.e. the tensor product of the one-dimensional weights 2/3, 1/6.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cglbm {

constexpr int kQ = 27;

// Eq. (1).
constexpr int kCX[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0,
                         0, 1, -1, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int kCY[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1,
                         -1, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int kCZ[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1,
                         1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};

__host__ __device__ constexpr float w1d(int c) { return c == 0 ? 2.0f / 3.0f : 1.0f / 6.0f; }
__host__ __device__ constexpr float weight(int i) { return w1d(kCX[i]) * w1d(kCY[i]) * w1d(kCZ[i]); }

__host__ __device__ constexpr int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Direction index of the velocity (cx, cy, cz), each in {-1, 0, 1}.
__host__ __device__ constexpr int dir_of(int cx, int cy, int cz) {
  int r = -1;
  for (int i = 0; i < kQ; ++i)
    if (kCX[i] == cx && kCY[i] == cy && kCZ[i] == cz) r = i;
  return r;
}

constexpr float kCs2 = 1.0f / 3.0f;  // lattice c_s^2
constexpr float kCs4 = kCs2 * kCs2;

// ---------------------------------------------------------------------------
// Division by a runtime constant d >= 1 for n < 2^31 (round-up multiplier
// method of Granlund and Montgomery).
// ---------------------------------------------------------------------------
struct FastDiv {
  uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
  return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv &f) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t t = __umulhi(n, f.m);
#else
  uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
  return (t + n) >> f.s;
}

// ---------------------------------------------------------------------------
// Central moments -> populations, factorized over the three axes.
// D3Q27 is the tensor product of D1Q3, so the 27x27 transform of Sec. II.B
// splits into 1D maps applied along z, then y, then x.  One 1D map takes the
// central moments (m0, m1, m2) of a triplet about velocity u to its
// populations (f_-, f_0, f_+): first to raw moments M1 = m1 + u m0,
// M2 = m2 + 2u m1 + u^2 m0, then f_0 = m0 - M2, f_+- = (M2 +- M1)/2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cm_to_pop_1d(float m0, float m1, float m2, float u, float &fm,
                                             float &f0, float &fp) {
  const float M1 = fmaf(u, m0, m1);
  const float M2 = fmaf(u, fmaf(u, m0, 2.0f * m1), m2);
  f0 = m0 - M2;
  fp = 0.5f * (M2 + M1);
  fm = 0.5f * (M2 - M1);
}

// The same map with its two outer outputs doubled, (2 f_-, f_0, 2 f_+): the
// halvings are left out, so the results are those of cm_to_pop_1d times 1, 2
// exactly, in 7 operations instead of 9.  Applied along z and then y, it
// leaves 2^(|c_y| + |c_z|) on the nine values of each row, which the last
// (plain) x pass keeps and the recolouring divides out with its colour
// fractions scaled by the inverse power of two (exact).
__device__ __forceinline__ void cm_to_pop_1d_x2(float m0, float m1, float m2, float u, float &gm,
                                                float &f0, float &gp) {
  const float M1 = fmaf(u, m0, m1);
  const float M2 = fmaf(u, fmaf(u, m0, 2.0f * m1), m2);
  f0 = m0 - M2;
  gp = M2 + M1;
  gm = M2 - M1;
}

// k[a + 3b + 9c] (central moments of orders a, b, c along x, y, z) ->
// f[i] in the order of Eq. (1).
__device__ __forceinline__ void central_to_populations(const float (&k)[27], float ux, float uy,
                                                       float uz, float (&f)[27]) {
  // along z: g[a][b][cz]
  float g[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      cm_to_pop_1d(k[a + 3 * b], k[a + 3 * b + 9], k[a + 3 * b + 18], uz, g[a][b][0], g[a][b][1],
                   g[a][b][2]);
  // along y: h[a][cy][cz]
  float h[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
      cm_to_pop_1d(g[a][0][cz], g[a][1][cz], g[a][2][cz], uy, h[a][0][cz], h[a][1][cz],
                   h[a][2][cz]);
  // along x
#pragma unroll
  for (int cy = 0; cy < 3; ++cy)
#pragma unroll
    for (int cz = 0; cz < 3; ++cz) {
      float fm, f0, fp;
      cm_to_pop_1d(h[0][cy][cz], h[1][cy][cz], h[2][cy][cz], ux, fm, f0, fp);
      f[dir_of(-1, cy - 1, cz - 1)] = fm;
      f[dir_of(0, cy - 1, cz - 1)] = f0;
      f[dir_of(1, cy - 1, cz - 1)] = fp;
    }
}

// Post-collision (or equilibrium) central moments of the generalized
// equilibrium with unit higher-order rates (Eqs. 57-63 and 66-67): every
// moment above second order is fixed by p and F; the second-order ones are
// passed in.  k000 = rho, k100 = F/2.
__device__ __forceinline__ void model_d_moments(float rho, float p, float Fx, float Fy, float Fz,
                                                float kxx, float kyy, float kzz, float kxy,
                                                float kxz, float kyz, float (&k)[27]) {
#define K_(a, b, c) k[(a) + 3 * (b) + 9 * (c)]
  K_(0, 0, 0) = rho;
  K_(1, 0, 0) = 0.5f * Fx;
  K_(0, 1, 0) = 0.5f * Fy;
  K_(0, 0, 1) = 0.5f * Fz;
  K_(2, 0, 0) = kxx;
  K_(0, 2, 0) = kyy;
  K_(0, 0, 2) = kzz;
  K_(1, 1, 0) = kxy;
  K_(1, 0, 1) = kxz;
  K_(0, 1, 1) = kyz;
  K_(1, 2, 0) = K_(1, 0, 2) = 0.5f * kCs2 * Fx;
  K_(2, 1, 0) = K_(0, 1, 2) = 0.5f * kCs2 * Fy;
  K_(2, 0, 1) = K_(0, 2, 1) = 0.5f * kCs2 * Fz;
  K_(1, 1, 1) = 0.0f;
  K_(2, 2, 0) = K_(2, 0, 2) = K_(0, 2, 2) = p * kCs2;
  K_(2, 1, 1) = K_(1, 2, 1) = K_(1, 1, 2) = 0.0f;
  K_(1, 2, 2) = 0.5f * kCs4 * Fx;
  K_(2, 1, 2) = 0.5f * kCs4 * Fy;
  K_(2, 2, 1) = 0.5f * kCs4 * Fz;
  K_(2, 2, 2) = p * kCs4;
#undef K_
}

// Equilibrium families of Table I.
enum { MODEL_A = 0, MODEL_B = 1, MODEL_C = 2, MODEL_D = 3 };

// Post-collision central moments with unit higher-order rates for any of the
// four equilibria of Table I: the Model D moments and the forcing moments
// above, plus the velocity-dependent parts of the equilibrium moments of
// order three and higher of Models A (Eqs. 32-38), B (Eqs. 40-46) and C
// (Eqs. 49-55), with dev = p - rho c_s^2.  `model` is uniform per box.
__device__ __forceinline__ void model_moments(int model, float rho, float p, float ux, float uy,
                                              float uz, float Fx, float Fy, float Fz, float kxx,
                                              float kyy, float kzz, float kxy, float kxz,
                                              float kyz, float (&k)[27]) {
  model_d_moments(rho, p, Fx, Fy, Fz, kxx, kyy, kzz, kxy, kxz, kyz, k);
  if (model == MODEL_D) return;
#define K_(a, b, c) k[(a) + 3 * (b) + 9 * (c)]
  const float dev = p - rho * kCs2;
  const float x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
  const float s2 = x2 * y2 + x2 * z2 + y2 * z2, u2 = x2 + y2 + z2;
  if (model == MODEL_C) {
    // Eqs. 49-55: no third-order part; the others with the opposite sign
    K_(2, 2, 0) -= dev * (x2 + y2);
    K_(2, 0, 2) -= dev * (x2 + z2);
    K_(0, 2, 2) -= dev * (y2 + z2);
    K_(2, 1, 1) -= dev * uy * uz;
    K_(1, 2, 1) -= dev * ux * uz;
    K_(1, 1, 2) -= dev * ux * uy;
    K_(1, 2, 2) += dev * ux * (2.0f * (y2 + z2) + kCs2);
    K_(2, 1, 2) += dev * uy * (2.0f * (x2 + z2) + kCs2);
    K_(2, 2, 1) += dev * uz * (2.0f * (x2 + y2) + kCs2);
    K_(2, 2, 2) -= 3.0f * dev * (s2 + kCs2 * u2);
  } else {
    // Model B (Eqs. 40-46); Model A (Eqs. 32-38) adds the rho terms below
    K_(1, 2, 0) -= dev * ux;
    K_(1, 0, 2) -= dev * ux;
    K_(2, 1, 0) -= dev * uy;
    K_(0, 1, 2) -= dev * uy;
    K_(2, 0, 1) -= dev * uz;
    K_(0, 2, 1) -= dev * uz;
    K_(2, 2, 0) += dev * (x2 + y2);
    K_(2, 0, 2) += dev * (x2 + z2);
    K_(0, 2, 2) += dev * (y2 + z2);
    K_(2, 1, 1) += dev * uy * uz;
    K_(1, 2, 1) += dev * ux * uz;
    K_(1, 1, 2) += dev * ux * uy;
    K_(1, 2, 2) -= dev * ux * (y2 + z2 + kCs2);
    K_(2, 1, 2) -= dev * uy * (x2 + z2 + kCs2);
    K_(2, 2, 1) -= dev * uz * (x2 + y2 + kCs2);
    K_(2, 2, 2) += dev * (s2 + kCs2 * u2);
    if (model == MODEL_A) {
      K_(1, 2, 0) -= rho * ux * y2;
      K_(1, 0, 2) -= rho * ux * z2;
      K_(2, 1, 0) -= rho * x2 * uy;
      K_(0, 1, 2) -= rho * uy * z2;
      K_(2, 0, 1) -= rho * x2 * uz;
      K_(0, 2, 1) -= rho * y2 * uz;
      K_(1, 1, 1) -= rho * ux * uy * uz;
      K_(2, 2, 0) += 3.0f * rho * x2 * y2;
      K_(2, 0, 2) += 3.0f * rho * x2 * z2;
      K_(0, 2, 2) += 3.0f * rho * y2 * z2;
      K_(2, 1, 1) += 3.0f * rho * x2 * uy * uz;
      K_(1, 2, 1) += 3.0f * rho * ux * y2 * uz;
      K_(1, 1, 2) += 3.0f * rho * ux * uy * z2;
      K_(1, 2, 2) -= rho * ux * (6.0f * y2 * z2 + kCs2 * (y2 + z2));
      K_(2, 1, 2) -= rho * uy * (6.0f * x2 * z2 + kCs2 * (x2 + z2));
      K_(2, 2, 1) -= rho * uz * (6.0f * x2 * y2 + kCs2 * (x2 + y2));
      K_(2, 2, 2) += rho * (10.0f * x2 * y2 * z2 + 3.0f * kCs2 * s2);
    }
  }
#undef K_
}

// SplitMix64 output function (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t splitmix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Counter noise in [-amp, amp): 24-bit uniform of the hash of
// (seed, box, node, direction).
__host__ __device__ inline float counter_noise(uint64_t seed, uint32_t box, uint64_t node, int i,
                                               float amp) {
  const uint64_t ctr = ((uint64_t)box << 48) ^ (node << 5) ^ (uint64_t)i;
  const uint64_t z = splitmix64(seed + 0x9E3779B97F4A7C15ull * ctr);
  const float uni = (float)(uint32_t)(z >> 40) * (1.0f / 16777216.0f);
  return amp * (2.0f * uni - 1.0f);
}

}  // namespace cglbm
