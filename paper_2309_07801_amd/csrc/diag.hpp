// diag.hpp -- field export and the deterministic FP64 diagnostics of the
// colour-gradient LBM (the non-template kernels, compiled in the host unit
// only).
#pragma once

#include "kernels.hpp"

namespace cglbm {

// ---------------------------------------------------------------------------
// Field export of one box (after k_pull + k_interface).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_fields(const BoxDev *__restrict__ boxes, int box,
                                                   const float *__restrict__ aux, int64_t plane,
                                                   uint32_t mask, float *__restrict__ out) {
  const BoxDev B = boxes[box];
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= B.n) return;
  const uint32_t l = (uint32_t)local;
  const uint32_t yz = fdiv(l, B.fdx);
  const int z = (int)fdiv(yz, B.fdy);
  const int y = (int)(yz - (uint32_t)z * (uint32_t)B.ny);
  const uint32_t node = (uint32_t)(B.base + local);
  const bool solid = is_solid(B, y, z);
  const NodeIn in = load_node_in(aux, plane, node);
  const float rho = in.rr + in.rb;
  const float sr = in.rr * B.ir0r, sb = in.rb * B.ir0b;
  float v[17];
  v[0] = in.rr;
  v[1] = in.rb;
  v[2] = (sr + sb) > 0.f ? (sr - sb) / (sr + sb) : 0.f;
  v[3] = in.rr * B.cs2r + in.rb * B.cs2b;
  v[4] = solid ? 0.f : fmaf(0.5f, in.Fx, in.jx) / rho;
  v[5] = solid ? 0.f : fmaf(0.5f, in.Fy, in.jy) / rho;
  v[6] = solid ? 0.f : fmaf(0.5f, in.Fz, in.jz) / rho;
  v[7] = in.nx;
  v[8] = in.ny;
  v[9] = in.nz;
  v[10] = at(PL(aux, A_KAPPA), node);
  v[11] = in.Fx;
  v[12] = in.Fy;
  v[13] = in.Fz;
  v[14] = in.Qx;
  v[15] = in.Qy;
  v[16] = in.Qz;
  int slot = 0;
  for (int k = 0; k < 17; ++k) {
    if (mask & (1u << k)) {
      out[(int64_t)slot * B.n + local] = v[k];
      ++slot;
    }
  }
}

// ---------------------------------------------------------------------------
// Deterministic FP64 diagnostics.  Each box is cut into chunks of
// kRedChunk = kRedG x 256 consecutive nodes; a block of 256 threads sums one
// chunk (thread t adds nodes t, t + 256, ... in that order, then a fixed
// tree combines the 256 thread sums).  Pass 1 per chunk: sums of rho_r,
// rho_b, rho u, V = (1+phi)/2, red centroid offsets, kinetic energy,
// non-finite count.  Pass 2: inside / outside pressure sums given R_eff.
// The final passes sum the chunk partials of each box in chunk order: the
// order depends only on the box, never on the launch or the other boxes.
// ---------------------------------------------------------------------------
constexpr int kNPart = 16;  // doubles per partial and per box in diag
constexpr int kRedG = 64;
constexpr int64_t kRedChunk = (int64_t)kRedG * kBlock;

__device__ __forceinline__ float periodic_offset(float d, int n, bool periodic) {
  if (!periodic) return d;
  const float h = 0.5f * n;
  if (d > h) d -= n;
  if (d < -h) d += n;
  return d;
}

// Centre coordinate a of box b: the caller's (centre != NULL) or the box's.
__device__ __forceinline__ float centre_of(const BoxDev &B, const double *centre, int b, int a) {
  const int n = a == 0 ? B.nx : (a == 1 ? B.ny : B.nz);
  return centre ? (float)centre[3 * b + a] : (float)(0.5 * (n - 1));
}

template <int NV>
__device__ __forceinline__ void block_sum_f64(double (&v)[NV], double *part) {
  __shared__ double s[NV][kBlock];
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[k] = s[k][0];
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce1(const BoxDev *__restrict__ boxes,
                                                    const int32_t *__restrict__ rch_box,
                                                    const float *__restrict__ aux, int64_t plane,
                                                    const double *__restrict__ rho64,
                                                    const double *__restrict__ centre,
                                                    double *__restrict__ part) {
  const int b = rch_box[blockIdx.x];
  const BoxDev B = boxes[b];
  const float cx = centre_of(B, centre, b, 0), cy = centre_of(B, centre, b, 1),
              cz = centre_of(B, centre, b, 2);
  double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t first = (int64_t)(blockIdx.x - (uint32_t)B.rch0) * kRedChunk + threadIdx.x;
  for (int g = 0; g < kRedG; ++g) {
    const int64_t local = first + (int64_t)g * kBlock;
    if (local >= B.n) break;
    const uint32_t l = (uint32_t)local;
    const uint32_t yz = fdiv(l, B.fdx);
    const int x = (int)(l - yz * (uint32_t)B.nx);
    const int z = (int)fdiv(yz, B.fdy);
    const int y = (int)(yz - (uint32_t)z * (uint32_t)B.ny);
    if (is_solid(B, y, z)) continue;
    const uint32_t node = (uint32_t)(B.base + local);
    const NodeIn in = load_node_in(aux, plane, node);
    const bool finite = isfinite(in.rr) && isfinite(in.rb) && isfinite(in.jx) &&
                        isfinite(in.jy) && isfinite(in.jz) && isfinite(in.pxx) &&
                        isfinite(in.pyy) && isfinite(in.pzz) && isfinite(in.pxy) &&
                        isfinite(in.pxz) && isfinite(in.pyz);
    if (!finite) {
      v[10] += 1.0;
      continue;
    }
    // colour densities in FP64 where the storage carries them
    const double rr = rho64 ? at(rho64, node) : (double)in.rr;
    const double rb = rho64 ? at(rho64 + plane, node) : (double)in.rb;
    const double rho = rr + rb;
    const double jx = (double)in.jx + 0.5 * in.Fx, jy = (double)in.jy + 0.5 * in.Fy,
                 jz = (double)in.jz + 0.5 * in.Fz;
    const float sr = in.rr * B.ir0r, sb = in.rb * B.ir0b;
    const double phi = (sr + sb) > 0.f ? (double)((sr - sb) / (sr + sb)) : 0.0;
    const double dx = periodic_offset(x - cx, B.nx, true);
    const double dy = periodic_offset(y - cy, B.ny, !(B.walls & 1u));
    const double dz = periodic_offset(z - cz, B.nz, !(B.walls & 2u));
    v[0] += rr;
    v[1] += rb;
    v[2] += jx;
    v[3] += jy;
    v[4] += jz;
    v[5] += 0.5 * (1.0 + phi);
    v[6] += rr * dx;
    v[7] += rr * dy;
    v[8] += rr * dz;
    v[9] += 0.5 * (jx * jx + jy * jy + jz * jz) / rho;
  }
  block_sum_f64<11>(v, part + (int64_t)blockIdx.x * kNPart);
}

__global__ __launch_bounds__(kBlock) void k_reduce2(const BoxDev *__restrict__ boxes,
                                                    const int32_t *__restrict__ rch_box,
                                                    const float *__restrict__ aux, int64_t plane,
                                                    const double *__restrict__ centre,
                                                    const double *__restrict__ diag,
                                                    double *__restrict__ part) {
  const int b = rch_box[blockIdx.x];
  const BoxDev B = boxes[b];
  const float cx = centre_of(B, centre, b, 0), cy = centre_of(B, centre, b, 1),
              cz = centre_of(B, centre, b, 2);
  double v[4] = {0, 0, 0, 0};
  const double reff = diag[(int64_t)b * kNPart + 7];
  const int64_t first = (int64_t)(blockIdx.x - (uint32_t)B.rch0) * kRedChunk + threadIdx.x;
  for (int g = 0; g < kRedG; ++g) {
    const int64_t local = first + (int64_t)g * kBlock;
    if (local >= B.n) break;
    const uint32_t l = (uint32_t)local;
    const uint32_t yz = fdiv(l, B.fdx);
    const int x = (int)(l - yz * (uint32_t)B.nx);
    const int z = (int)fdiv(yz, B.fdy);
    const int y = (int)(yz - (uint32_t)z * (uint32_t)B.ny);
    if (is_solid(B, y, z)) continue;
    const uint32_t node = (uint32_t)(B.base + local);
    const double p = (double)(at(PL(aux, A_RR), node) * B.cs2r + at(PL(aux, A_RB), node) * B.cs2b);
    const double dx = periodic_offset(x - cx, B.nx, true);
    const double dy = periodic_offset(y - cy, B.ny, !(B.walls & 1u));
    const double dz = periodic_offset(z - cz, B.nz, !(B.walls & 2u));
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (isfinite(p)) {
      if (d < reff - 3.0) {
        v[0] += p;
        v[1] += 1.0;
      }
      if (d > reff + 5.0) {
        v[2] += p;
        v[3] += 1.0;
      }
    }
  }
  block_sum_f64<4>(v, part + (int64_t)blockIdx.x * kNPart);
}

// One block per box: fixed-order sum of the box's chunk partials.  Thread t
// sums the contiguous run [t*c, (t+1)*c) of partials in order, then a fixed
// tree combines the 256 thread sums; the order depends only on the box.
// pass 1 fills diag[0..4, 7 (R_eff), 8..10 (centroid), 11, 12]; pass 2 fills
// 5, 6 and, if out is not NULL, writes the box's CGLBM_NDIAG (13) values,
// diag[0..12], to out[13 b ...] (the packed layout of cglbm_reduce).
__global__ __launch_bounds__(kBlock) void k_reduce_final(const BoxDev *__restrict__ boxes,
                                                         const double *__restrict__ part, int pass,
                                                         double *__restrict__ diag,
                                                         double *__restrict__ out) {
  const int b = blockIdx.x;
  const BoxDev B = boxes[b];
  const int nch = (int)((B.n + kRedChunk - 1) / kRedChunk);
  const int chunk = (nch + kBlock - 1) / kBlock;
  const int k0 = min((int)threadIdx.x * chunk, nch), k1 = min(k0 + chunk, nch);
  double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int nv = pass == 1 ? 11 : 4;
  for (int k = k0; k < k1; ++k)
    for (int c = 0; c < nv; ++c) v[c] += part[(int64_t)(B.rch0 + k) * kNPart + c];
  __shared__ double tot[kNPart];
  {
    double w[11];
    for (int c = 0; c < 11; ++c) w[c] = v[c];
    block_sum_f64<11>(w, tot);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double *o = diag + (int64_t)b * kNPart;
  if (pass == 1) {
    o[0] = tot[0];
    o[1] = tot[1];
    o[2] = tot[2];
    o[3] = tot[3];
    o[4] = tot[4];
    // equivalent radius of the red volume (area in two dimensions)
    o[7] = B.d2q9 ? sqrt(tot[5] / 3.14159265358979323846)
                  : cbrt(3.0 * tot[5] / (4.0 * 3.14159265358979323846));
    o[8] = tot[0] > 0 ? tot[6] / tot[0] : 0.0;
    o[9] = tot[0] > 0 ? tot[7] / tot[0] : 0.0;
    o[10] = tot[0] > 0 ? tot[8] / tot[0] : 0.0;
    o[11] = tot[9];
    o[12] = tot[10];
  } else {
    o[5] = tot[1] > 0 ? tot[0] / tot[1] : 0.0;
    o[6] = tot[3] > 0 ? tot[2] / tot[3] : 0.0;
    if (out) {
      for (int k = 0; k < 13; ++k) out[(int64_t)b * 13 + k] = o[k];
    }
  }
}

}  // namespace cglbm
