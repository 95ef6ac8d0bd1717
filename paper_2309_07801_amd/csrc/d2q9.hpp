// d2q9.hpp -- HIP kernels (gfx950) of the two-dimensional (D2Q9, App. A)
// colour-gradient step with the generalized equilibrium of Eq. (A10).
//
// Storage: populations as colour-pair planes (red in the low half), pair
// plane i for direction i in the order of Eq. (A1): FP32 keeps all 9
// directions; the mass-exact formats (FP16 / BF16 shifted, FP32 exact) keep
// the 8 moving directions and the two rest populations in FP64 planes after
// them, as in three dimensions.  The aux planes keep the layout of the
// three-dimensional path (z components zero), so the field export and the
// diagnostics kernels serve both lattices.
//
// One step is one launch.  A block owns a TX x TY tile of a box: it pulls
// the populations of the tile and of a 3-node halo (Eq. 5) and forms the
// local moments in LDS, then evaluates the stencils of the interface in LDS
// (phase field and pressure, Eqs. 12 and 14; grad phi and n by the
// isotropic gradient of Eq. 20, halo 2; curvature, CSF force, velocity and
// q = (p - rho c_s^2) u, Eqs. 11, 15-17, halo 1; Q, Eq. 65), and collides
// and recolours the tile's own nodes (Eqs. 18-19, 21-22 and the unit-rate
// form of the two-dimensional Eq. 25 whose equilibrium moments are
// Eqs. A12-A16).  No moment or interface field leaves the chip between the
// pull and the collision.
#pragma once

#include "kernels.hpp"

namespace cglbm {
namespace d2q9 {

constexpr int kQ = 9;
// Eq. (A1)
constexpr int kCX[kQ] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int kCY[kQ] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
__host__ __device__ constexpr int opposite(int i) { return i == 0 ? 0 : (i & 1 ? i + 1 : i - 1); }
// Eq. (A2) by |c|^2 (0, 1, 2), and weight / c_s^2
__host__ __device__ constexpr float weight(int i) {
  return i == 0 ? 4.0f / 9.0f : (i < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
}
// 1 / c_s^2 times a weight: the coefficient of the isotropic gradient (Eq. 20)
__host__ __device__ constexpr float gw(int i) { return 3.0f * weight(i); }

// Views of one population buffer: pair planes, then (mass-exact formats)
// the FP64 rest populations of the two colours.
template <class S>
struct Pops2 {
  using W = typename S::W;
  static constexpr int kDirs = S::kExact ? kQ - 1 : kQ;
  W *pw;
  double *rest;
  int64_t plane;
  __device__ Pops2(void *base, int64_t plane_) : plane(plane_) {
    pw = (W *)base;
    rest = (double *)((char *)base + align256(kDirs * plane_ * (int64_t)sizeof(W)));
  }
  __device__ W *plane_of(int i) const { return pw + (int64_t)(S::kExact ? i - 1 : i) * plane; }
  __device__ double *restp(int c) const { return rest + (int64_t)c * plane; }
};

// Shift of direction i of colour c: the pure-phase rest equilibrium of the
// colour with the D2Q9 weight of i (host table by |c_i|^2), rounded to the
// format; zero for unshifted formats and the rest direction.
template <class S>
__device__ __forceinline__ float shift2(const BoxDev &B, int c, int i) {
  if (!S::kShift || i == 0) return 0.f;
  return S::dec(S::enc(B.shift[c][kCX[i] * kCX[i] + kCY[i] * kCY[i]]));
}

// Index of direction (cx, cy).
__host__ __device__ constexpr int dir_of(int cx, int cy) {
  return cy == 0 ? (cx == 0 ? 0 : (cx > 0 ? 1 : 2))
                 : (cx == 0 ? (cy > 0 ? 3 : 4)
                            : (cx == cy ? (cx > 0 ? 5 : 6) : (cx > 0 ? 7 : 8)));
}

__device__ __forceinline__ bool row_solid(const BoxDev &B, int y) {
  return (B.walls & 1u) && (y == 0 || y == B.ny - 1);
}

// Post-collision central moments k[a + 3b] -> populations f[i] (Eq. A1
// order): the 9x9 transform splits into the one-dimensional map along x for
// each order b, then along y for each cx.
__device__ __forceinline__ void central_to_pops(const float (&k)[9], float ux, float uy,
                                                float (&f)[kQ]) {
  float g[3][3];  // g[b][cx + 1]
#pragma unroll
  for (int b = 0; b < 3; ++b) cm_to_pop_1d(k[3 * b], k[3 * b + 1], k[3 * b + 2], ux, g[b][0], g[b][1], g[b][2]);
#pragma unroll
  for (int cx = 0; cx < 3; ++cx) {
    float fm, f0, fp;
    cm_to_pop_1d(g[0][cx], g[1][cx], g[2][cx], uy, fm, f0, fp);
    f[dir_of(cx - 1, -1)] = fm;
    f[dir_of(cx - 1, 0)] = f0;
    f[dir_of(cx - 1, 1)] = fp;
  }
}

// Equilibrium central moments of Eqs. (A12)-(A16) (velocity independent).
__device__ __forceinline__ void equilibrium_cms(float rho, float p, float (&k)[9]) {
  k[0] = rho;
  k[1] = k[3] = k[4] = k[5] = k[7] = 0.f;
  k[2] = k[6] = p;
  k[8] = p * (1.0f / 3.0f);
}

// Initial state: the equilibrium of Eq. (A10) at the given density and
// velocity (from its central moments) plus counter noise, split by colour
// fraction; stored un-streamed (direction i of node x at x - c_i), so that
// the first pull reproduces it at x.
template <class S>
__global__ __launch_bounds__(kBlock) void k2_init(const BoxDev *__restrict__ boxes,
                                                  const int32_t *__restrict__ blk_box,
                                                  const float *__restrict__ in_rr,
                                                  const float *__restrict__ in_rb,
                                                  const float *__restrict__ in_u,
                                                  void *__restrict__ dst_, int64_t plane,
                                                  uint64_t seed, float amp) {
  const int b = blk_box[blockIdx.x];
  const BoxDev B = boxes[b];
  const int64_t local = (int64_t)(blockIdx.x - B.blk0) * kBlock + threadIdx.x;
  if (local >= B.n) return;
  const uint32_t l = (uint32_t)local;
  const int y = (int)fdiv(l, B.fdx);
  const int x = (int)(l - (uint32_t)y * (uint32_t)B.nx);
  const uint32_t node = (uint32_t)(B.base + local);
  const float rr = in_rr[node], rb = in_rb[node];
  const float ux = in_u[node], uy = in_u[plane + node];
  const float rho = rr + rb;
  const float p = rr * B.cs2r + rb * B.cs2b;
  float k[9];
  equilibrium_cms(rho, p, k);
  float f[kQ];
  central_to_pops(k, ux, uy, f);
  const float cr = rr / rho, cb = rb / rho;
  const Pops2<S> dst(dst_, plane);
  double tr = 0.0, tb = 0.0, sr = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float ft = amp != 0.f ? f[i] + counter_noise(seed, (uint32_t)b, (uint64_t)local, i, amp)
                                : f[i];
    const float vr = cr * ft, vb = cb * ft;
    tr += (double)vr;
    tb += (double)vb;
    if (S::kExact && i == 0) continue;
    const int xd = wrap_once(x - kCX[i], B.nx), yd = wrap_once(y - kCY[i], B.ny);
    const uint32_t d = (uint32_t)B.base + (uint32_t)xd + (uint32_t)B.nx * (uint32_t)yd;
    const float shr = shift2<S>(B, 0, i), shb = shift2<S>(B, 1, i);
    const typename S::T er = S::enc(vr - shr), eb = S::enc(vb - shb);
    st(&at(dst.plane_of(i), d), S::pack(er, eb));
    sr += (double)(S::dec(er) + shr);
    sb += (double)(S::dec(eb) + shb);
  }
  // mass-exact formats: the rest populations close each colour's mass
  if (S::kExact) {
    st(&at(dst.restp(0), node), tr - sr);
    st(&at(dst.restp(1), node), tb - sb);
  }
}

// One time step (EXPORT = false) or the export of the fields of the stored
// state into aux (EXPORT = true: moments, n, F, Q, kappa; no populations
// written).  Grid: one block per tile (tile table tile_box, XCD-remapped,
// padded with idle blocks).
template <class S, int TX, int TY, int NT, bool EXPORT>
__global__ __launch_bounds__(NT) void k2_step(const BoxDev *__restrict__ boxes,
                                              const int32_t *__restrict__ tile_box,
                                              const void *__restrict__ src_,
                                              void *__restrict__ dst_, float *__restrict__ aux,
                                              int64_t plane) {
  using W = typename S::W;
  constexpr int i0 = S::kExact ? 1 : 0;  // first stored pair plane's direction
  constexpr int RW = TX + 6, RH = TY + 6;  // pulled region: halo 3
  constexpr int GW = TX + 4, GH = TY + 4;  // n, |grad phi|: halo 2
  constexpr int KW = TX + 2, KH = TY + 2;  // F, q: halo 1
  constexpr int ROWS = NT / TX;            // interior rows per pass
  constexpr int PER = TY / ROWS;           // interior nodes per thread
  static_assert(NT % TX == 0 && TY % ROWS == 0, "tile must split evenly over the block");
  // phi on the whole pulled region; densities and j where they are used
  // (halo 1: velocity and q, and the tile's own nodes)
  __shared__ float s_phi[RH][RW];
  __shared__ float s_nx[GH][GW], s_ny[GH][GW], s_mag[GH][GW];
  __shared__ float s_rr[KH][KW], s_rb[KH][KW], s_jx[KH][KW], s_jy[KH][KW];
  __shared__ float s_fx[KH][KW], s_fy[KH][KW], s_qx[KH][KW], s_qy[KH][KW];
  __shared__ int s_ry[RH];       // box row of each region row
  __shared__ uint8_t s_sol[RH];  // region row is a solid layer

  const uint32_t lb = xcd_block();
  const int b = tile_box[lb];
  if (b < 0) return;
  const BoxDev B = boxes[b];
  const uint32_t t = lb - (uint32_t)B.tile0;
  const int tyi = (int)fdiv(t, B.ftx);
  const int txi = (int)(t - (uint32_t)tyi * (uint32_t)B.tnx);
  const int x0 = txi * TX, y0 = tyi * TY;
  const int nx = B.nx, ny = B.ny;
  const int tid = threadIdx.x;
  const Pops2<S> src(const_cast<void *>(src_), plane), dst(dst_, plane);

  if (tid < RH) {
    const int gy = wrap_any(y0 - 3 + tid, ny);
    s_ry[tid] = gy;
    s_sol[tid] = row_solid(B, gy) ? 1 : 0;
  }
  __syncthreads();

  // ---- pull (Eq. 5) and local moments of one region node ----
  // Mass-exact formats sum each colour in FP64 (rest population included),
  // so that every tile holding a node as halo or as its own sees the same
  // densities; the FP64 sums of own nodes close the rest populations.
  auto pull = [&](int rx, int ry, bool own, float &pxx, float &pyy, float &pxy, double &drr,
                  double &drb) {
    const int gx = wrap_any(x0 - 3 + rx, nx), gy = s_ry[ry];
    const int xs[3] = {wrap_once(gx + 1, nx), gx, wrap_once(gx - 1, nx)};
    const int ys[3] = {wrap_once(gy + 1, ny), gy, wrap_once(gy - 1, ny)};
    const uint32_t node = (uint32_t)B.base + (uint32_t)gx + (uint32_t)nx * (uint32_t)gy;
    W gw_[kQ];
#pragma unroll
    for (int i = i0; i < kQ; ++i) {
      const uint32_t s = (uint32_t)B.base + (uint32_t)xs[kCX[i] + 1] +
                         (uint32_t)nx * (uint32_t)ys[kCY[i] + 1];
      gw_[i] = at(src.plane_of(i), s);
    }
    drr = drb = 0.0;
    if (S::kExact) {
      drr = at(src.restp(0), node);
      drb = at(src.restp(1), node);
    }
    float rr = 0.f, rb = 0.f, jx = 0.f, jy = 0.f;
    pxx = pyy = pxy = 0.f;
    if (s_sol[ry]) {
      // full-way bounce-back: reverse what arrived (the shift of a direction
      // equals its opposite's, so raw pairs are copied)
      if (own && !EXPORT) {
#pragma unroll
        for (int i = i0; i < kQ; ++i) st(&at(dst.plane_of(opposite(i)), node), gw_[i]);
        if (S::kExact) {
          st(&at(dst.restp(0), node), drr);
          st(&at(dst.restp(1), node), drb);
        }
      }
      drr = drb = 0.0;
    } else {
#pragma unroll
      for (int i = i0; i < kQ; ++i) {
        const float vr = S::dec(S::lo(gw_[i])) + shift2<S>(B, 0, i);
        const float vb = S::dec(S::hi(gw_[i])) + shift2<S>(B, 1, i);
        if (S::kExact) {
          drr += (double)vr;
          drb += (double)vb;
        } else {
          rr += vr;
          rb += vb;
        }
        const float f = vr + vb;
        if (kCX[i]) jx += kCX[i] > 0 ? f : -f;
        if (kCY[i]) jy += kCY[i] > 0 ? f : -f;
        if (kCX[i]) pxx += f;
        if (kCY[i]) pyy += f;
        if (kCX[i] * kCY[i]) pxy += kCX[i] * kCY[i] > 0 ? f : -f;
      }
      if (S::kExact) {
        rr = (float)drr;
        rb = (float)drb;
      }
    }
    if (rx >= 2 && rx < RW - 2 && ry >= 2 && ry < RH - 2) {
      s_rr[ry - 2][rx - 2] = rr;
      s_rb[ry - 2][rx - 2] = rb;
      s_jx[ry - 2][rx - 2] = jx;
      s_jy[ry - 2][rx - 2] = jy;
    }
    // Eq. (14); correctly rounded quotient: exactly +-1 in a pure phase
    const float sr = rr * B.ir0r, sb = rb * B.ir0b;
    s_phi[ry][rx] = (sr + sb) > 0.f ? (sr - sb) / (sr + sb) : 0.f;
  };

  const int ix = tid % TX, iy0 = tid / TX;
  float opxx[PER], opyy[PER], opxy[PER];
  double odrr[PER], odrb[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int ry = 3 + iy0 + k * ROWS;
    const bool in_box = x0 + ix < nx && y0 + iy0 + k * ROWS < ny;
    pull(3 + ix, ry, in_box, opxx[k], opyy[k], opxy[k], odrr[k], odrb[k]);
  }
  {
    // the halo ring: 3 rows above and below, 3 columns left and right
    constexpr int NH = 6 * RW + 6 * TY;
    for (int h = tid; h < NH; h += NT) {
      int rx, ry;
      if (h < 3 * RW) {
        rx = h % RW;
        ry = h / RW;
      } else if (h < 6 * RW) {
        rx = (h - 3 * RW) % RW;
        ry = RH - 3 + (h - 3 * RW) / RW;
      } else {
        const int s = h - 6 * RW;
        ry = 3 + s / 6;
        const int c = s % 6;
        rx = c < 3 ? c : RW - 6 + c;
      }
      float a, bb, c;
      double da, db;
      pull(rx, ry, false, a, bb, c, da, db);
    }
  }
  __syncthreads();

  // ---- grad phi and n on the halo-2 region (Eqs. 17, 20) ----
  for (int g = tid; g < GW * GH; g += NT) {
    const int gx = g % GW + 1, gy = g / GW + 1;  // region coordinates
    float nxv = 0.f, nyv = 0.f, mag = 0.f;
    if (!s_sol[gy]) {
      const float pc = s_phi[gy][gx];
      float ax = 0.f, ay = 0.f;
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const float v = s_sol[gy + kCY[i]] ? pc : s_phi[gy + kCY[i]][gx + kCX[i]];
        if (kCX[i]) ax = fmaf(gw(i) * (float)kCX[i], v, ax);
        if (kCY[i]) ay = fmaf(gw(i) * (float)kCY[i], v, ay);
      }
      const float m2 = ax * ax + ay * ay;
      if (m2 > 1e-24f) {
        const float r = rsq(m2);
        nxv = ax * r;
        nyv = ay * r;
        mag = m2 * r;
      }
    }
    s_nx[gy - 1][gx - 1] = nxv;
    s_ny[gy - 1][gx - 1] = nyv;
    s_mag[gy - 1][gx - 1] = mag;
  }
  __syncthreads();

  // ---- curvature, CSF force, velocity and q on the halo-1 region ----
  for (int g = tid; g < KW * KH; g += NT) {
    const int kx = g % KW, ky = g / KW;    // K coordinates
    const int ry = ky + 2;                 // region row
    const int cx = kx + 1, cy = ky + 1;    // G coordinates
    float Fx = 0.f, Fy = 0.f, qx = 0.f, qy = 0.f, kap = 0.f;
    if (!s_sol[ry]) {
      const float nxc = s_nx[cy][cx], nyc = s_ny[cy][cx];
      float dxx = 0.f, dxy = 0.f, dyx = 0.f, dyy = 0.f;  // d n_a / d x_b
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const bool sol = s_sol[ry + kCY[i]];
        const float vx = sol ? nxc : s_nx[cy + kCY[i]][cx + kCX[i]];
        const float vy = sol ? nyc : s_ny[cy + kCY[i]][cx + kCX[i]];
        if (kCX[i]) {
          dxx = fmaf(gw(i) * (float)kCX[i], vx, dxx);
          dyx = fmaf(gw(i) * (float)kCX[i], vy, dyx);
        }
        if (kCY[i]) {
          dxy = fmaf(gw(i) * (float)kCY[i], vx, dxy);
          dyy = fmaf(gw(i) * (float)kCY[i], vy, dyy);
        }
      }
      // Eq. (16): kappa = -(I - n n) : grad n
      const float proj = nxc * (nxc * dxx + nyc * dxy) + nyc * (nxc * dyx + nyc * dyy);
      kap = -(dxx + dyy - proj);
      // Eq. (15) with grad phi = |grad phi| n, plus the constant body force
      const float s = 0.5f * B.sigma * kap * s_mag[cy][cx];
      Fx = fmaf(s, nxc, B.Gx);
      Fy = fmaf(s, nyc, B.Gy);
      const float rr = s_rr[ky][kx], rb = s_rb[ky][kx];
      const float rho = rr + rb;
      const float p = rr * B.cs2r + rb * B.cs2b;
      const float irho = rcp(rho);
      const float ux = fmaf(0.5f, Fx, s_jx[ky][kx]) * irho;
      const float uy = fmaf(0.5f, Fy, s_jy[ky][kx]) * irho;
      const float e = fmaf(-rho, 1.0f / 3.0f, p);
      qx = e * ux;
      qy = e * uy;
    }
    s_fx[ky][kx] = Fx;
    s_fy[ky][kx] = Fy;
    s_qx[ky][kx] = qx;
    s_qy[ky][kx] = qy;
    if (EXPORT && kx >= 1 && kx <= TX && ky >= 1 && ky <= TY && x0 + kx - 1 < nx &&
        y0 + ky - 1 < ny) {
      const uint32_t node = (uint32_t)B.base + (uint32_t)(x0 + kx - 1) +
                            (uint32_t)nx * (uint32_t)(y0 + ky - 1);
      at(PL(aux, A_KAPPA), node) = kap;
      at(PL(aux, A_FX), node) = Fx;
      at(PL(aux, A_FY), node) = Fy;
      at(PL(aux, A_FZ), node) = 0.f;
      at(PL(aux, A_NX), node) = s_sol[ry] ? 0.f : s_nx[ky + 1][kx + 1];
      at(PL(aux, A_NY), node) = s_sol[ry] ? 0.f : s_ny[ky + 1][kx + 1];
      at(PL(aux, A_NZ), node) = 0.f;
    }
  }
  __syncthreads();

  // ---- correction term (Eq. 65), collision and recolouring of own nodes ----
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int ty = iy0 + k * ROWS;
    const int gx = x0 + ix, gy = y0 + ty;
    const int rx = ix + 3, ry = ty + 3;
    const int kx = ix + 1, ky = ty + 1;
    if (gx >= nx || gy >= ny || s_sol[ry]) {
      if (EXPORT && gx < nx && gy < ny) {
        const uint32_t node = (uint32_t)B.base + (uint32_t)gx + (uint32_t)nx * (uint32_t)gy;
#pragma unroll
        for (int a = 0; a <= A_PYZ; ++a) at(PL(aux, a), node) = 0.f;
        at(PL(aux, A_QX), node) = 0.f;
        at(PL(aux, A_QY), node) = 0.f;
        at(PL(aux, A_QZ), node) = 0.f;
        if (S::kExact) {
          double *r64 = aux_rho64(aux, plane);
          at(r64, node) = 0.0;
          at(r64 + plane, node) = 0.0;
        }
      }
      continue;
    }
    float Qx = 0.f, Qy = 0.f;
    if (B.qcorr) {
      const float qxc = s_qx[ky][kx], qyc = s_qy[ky][kx];
      float ax = 0.f, ay = 0.f;
#pragma unroll
      for (int i = 1; i < kQ; ++i) {
        const bool sol = s_sol[ry + kCY[i]];
        if (kCX[i]) ax = fmaf(gw(i) * (float)kCX[i], sol ? qxc : s_qx[ky + kCY[i]][kx + kCX[i]], ax);
        if (kCY[i]) ay = fmaf(gw(i) * (float)kCY[i], sol ? qyc : s_qy[ky + kCY[i]][kx + kCX[i]], ay);
      }
      Qx = -3.0f * ax;
      Qy = -3.0f * ay;
    }
    const float rr = s_rr[ky][kx], rb = s_rb[ky][kx];
    const float jx = s_jx[ky][kx], jy = s_jy[ky][kx];
    const float Fx = s_fx[ky][kx], Fy = s_fy[ky][kx];
    const uint32_t node = (uint32_t)B.base + (uint32_t)gx + (uint32_t)nx * (uint32_t)gy;
    if (EXPORT) {
      at(PL(aux, A_RR), node) = rr;
      at(PL(aux, A_RB), node) = rb;
      at(PL(aux, A_JX), node) = jx;
      at(PL(aux, A_JY), node) = jy;
      at(PL(aux, A_JZ), node) = 0.f;
      at(PL(aux, A_PXX), node) = opxx[k];
      at(PL(aux, A_PYY), node) = opyy[k];
      at(PL(aux, A_PZZ), node) = 0.f;
      at(PL(aux, A_PXY), node) = opxy[k];
      at(PL(aux, A_PXZ), node) = 0.f;
      at(PL(aux, A_PYZ), node) = 0.f;
      at(PL(aux, A_QX), node) = Qx;
      at(PL(aux, A_QY), node) = Qy;
      at(PL(aux, A_QZ), node) = 0.f;
      if (S::kExact) {
        double *r64 = aux_rho64(aux, plane);
        at(r64, node) = odrr[k];
        at(r64 + plane, node) = odrb[k];
      }
      continue;
    }
    const float rho = rr + rb;
    const float irho = rcp(rho);
    const float p = rr * B.cs2r + rb * B.cs2b;
    const float ux = div_refined(fmaf(0.5f, Fx, jx), rho, irho);
    const float uy = div_refined(fmaf(0.5f, Fy, jy), rho, irho);
    // Eqs. (21)-(22): omega_1 = 1 / tau, tau = rho nu / p + 1/2
    const float ph = s_phi[ry][rx];
    const float nu = 0.5f * ((1.f + ph) * B.nu_r + (1.f - ph) * B.nu_b);
    const float w1 = rcp(fmaf(rho * nu, rcp(p), 0.5f));
    const float w2 = B.omega2;
    // second-order central moments of the pulled state (j = rho u - F/2)
    const float k20 = fmaf(ux, Fx, fmaf(-rho * ux, ux, opxx[k]));
    const float k02 = fmaf(uy, Fy, fmaf(-rho * uy, uy, opyy[k]));
    const float k11 = fmaf(0.5f, fmaf(ux, Fy, uy * Fx), fmaf(-rho * ux, uy, opxy[k]));
    // two-dimensional Eq. (25), unit rates above second order and omega_0 = 1
    const float D = fmaf(1.f - w1, k20 - k02, (1.f - 0.5f * w1) * (Qx - Qy));
    const float T = fmaf(1.f - w2, k20 + k02, fmaf(2.f * w2, p, (1.f - 0.5f * w2) * (Qx + Qy)));
    float ks[9];
    ks[0] = rho;
    ks[1] = 0.5f * Fx;
    ks[3] = 0.5f * Fy;
    ks[4] = (1.f - w1) * k11;
    ks[2] = 0.5f * (T + D);
    ks[6] = 0.5f * (T - D);
    ks[5] = (1.0f / 6.0f) * Fy;  // k21 = c_s^2 F_y / 2
    ks[7] = (1.0f / 6.0f) * Fx;  // k12 = c_s^2 F_x / 2
    ks[8] = p * (1.0f / 3.0f);
    float f[kQ];
    central_to_pops(ks, ux, uy, f);
    // Eqs. (18)-(19)
    const float nxc = s_nx[ky + 1][kx + 1], nyc = s_ny[ky + 1][kx + 1];
    // colour fractions by correctly rounded division: exactly 0 and 1 in a
    // pure phase, so the reciprocal's rounding does not bias each colour's
    // mass step after step
    const float cr = rr / rho, cb = rb / rho;
    const float rs = B.beta * cr * cb * p;
    double sr = 0.0, sb = 0.0;
#pragma unroll
    for (int i = i0; i < kQ; ++i) {
      float cR = 0.f;
      if (kCX[i]) cR = fmaf((float)kCX[i], nxc, cR);
      if (kCY[i]) cR = fmaf((float)kCY[i], nyc, cR);
      const float d = gw(i) * rs * cR;
      const float shr = shift2<S>(B, 0, i), shb = shift2<S>(B, 1, i);
      const typename S::T er = S::enc(fmaf(cr, f[i], d) - shr), eb = S::enc(fmaf(cb, f[i], -d) - shb);
      st(&at(dst.plane_of(i), node), S::pack(er, eb));
      if (S::kExact) {
        sr += (double)(S::dec(er) + shr);
        sb += (double)(S::dec(eb) + shb);
      }
    }
    // mass-exact formats: the rest populations close each colour's mass on
    // the node's FP64 densities
    if (S::kExact) {
      st(&at(dst.restp(0), node), odrr[k] - sr);
      st(&at(dst.restp(1), node), odrb[k] - sb);
    }
  }
}

}  // namespace d2q9
}  // namespace cglbm
