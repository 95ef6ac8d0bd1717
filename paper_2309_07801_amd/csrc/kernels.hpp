// kernels.hpp -- HIP kernels (gfx950) of the colour-gradient LBM time step.
//
// Storage (all boxes concatenated, SoA planes of `plane` elements):
//   populations  FP32: pop[c*27 + i][node], c = 0 red, 1 blue, i in Eq. (1)
//                order; mass-exact formats: colour pairs of the 26 moving
//                directions, then the FP64 rest populations (see Pops)
//   aux          aux[k][node], float:
//     0 rho_r  1 rho_b  2..4 j = sum_i f_i c_i  5..10 Pi_xx,yy,zz,xy,xz,yz
//     11..13 n  14..16 F  17..19 Q  20 kappa (only written on request)
//
// One step = two launches (schedule 0):
//   k_pull     pull-stream (Eq. 5) + local moments; bounce-back at solid nodes
//   k_fused    z-marching interface stencils (Eqs. 11, 14-17, 20, 65) and
//              the collision with the generalized equilibrium (Eqs. 25,
//              57-63, 66-67) and recolouring (Eqs. 18-19), local store
// or three (schedule 1, and general models or rates):
//   k_pull, then k_interface (LDS-tiled stencils: phi, grad phi, n, kappa,
//   F, u, Q) and k_collide (collision, recolouring, local store)
// or, within one call of many steps (schedule 2, compact):
//   k_cpull    the moments after streaming, summed from the collided
//              populations the pull rebuilds from each node's 17-value
//              compact post-collision state
//   k_fused    as above, storing compact states instead of populations
//   (the call's first step runs k_pull, and k_emit stores the populations
//   at its end)
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <type_traits>

#include "lattice.hpp"

namespace cglbm {

enum AuxPlane {
  A_RR = 0, A_RB = 1, A_JX = 2, A_JY = 3, A_JZ = 4,
  A_PXX = 5, A_PYY = 6, A_PZZ = 7, A_PXY = 8, A_PXZ = 9, A_PYZ = 10,
  A_NX = 11, A_NY = 12, A_NZ = 13, A_FX = 14, A_FY = 15, A_FZ = 16,
  A_QX = 17, A_QY = 18, A_QZ = 19, A_KAPPA = 20, A_COUNT = 21
};

// Per-box constants, filled on the host.
struct BoxDev {
  int32_t nx, ny, nz;
  uint32_t walls;
  int64_t base;         // first node of the box in the concatenated arrays
  int64_t n;            // nx*ny*nz
  int32_t blk0;         // first 256-node block of the box (k_pull, k_collide)
  int32_t tile0;        // first tile of the box (k_interface)
  int32_t tnx, tny;     // tiles along x, y
  FastDiv fdx, fdy;     // division by nx, ny
  FastDiv ftx, fty;     // division by tnx, tny
  int32_t col0;         // unused (blocks carry their box and tile: TileEntry)
  int32_t ncx, ncy;     // columns along x, y
  FastDiv fcx, fcy;     // division by ncx, ncy
  float cs2r, cs2b;     // (c_s^k)^2 = xi (1 - alpha_k)
  float ir0r, ir0b;     // 1 / rho_k^0
  float nu_r, nu_b;
  float sigma, beta;
  float omega2;
  float Gx, Gy, Gz;
  float shift[2][4];    // storage shift by colour and speed class |c|^2
  float cdev[4];        // -3 w p_ref by speed class |c|^2, p_ref = min_k rho_k^0 (c_s^k)^2 (k_cpull)
  float pscale[2];      // colour-fraction formats: power-of-two scale of each colour's values
  float pinv[2];        // and its inverse
  float bgx, bgy, bgz;  // g of the buoyancy force -(rho - rho_ref) g
  float rho_ref;
  float omh[9];         // omega_0, omega_3..omega_10 of Eq. (25)
  int32_t full_rates;   // 1: some higher-order rate differs from 1
  int32_t model;        // equilibrium family of Table I (MODEL_A..MODEL_D)
  int32_t qcorr;        // 1: correction term Q of Eq. (65) in the collision
  int32_t d2q9;         // 1: two-dimensional box of the D2Q9 lattice (App. A)
  int32_t wbase, wn;    // wall-node slots of the box in the in-place stash
  int32_t wblk0;        // first block of the box in k_wall_copy
  int32_t ccol0;        // unused (see col0)
  int32_t rch0;         // first reduction chunk of the box (k_reduce1, k_reduce2)
  int32_t cncx, cncy;   // k_cpull columns along x, y
  FastDiv fccx, fccy;   // division by cncx, cncy
};

constexpr int kBlock = 256;

// One block of k_fused or k_cpull: a box, its xy column (x fastest) and the
// slabs [z0, z1) the block outputs; box < 0 for padding blocks.  Each launch
// gets its own list, so that a box's tiles can be split between launches:
// those whose stencils stay clear of solid layers run the kernel without
// wall logic, and the chunks next to a z wall are cut short so that few
// slabs need it.
struct TileEntry {
  int32_t box, xy, z0, z1;
};

// Plane p of a SoA array: a uniform (scalar) base pointer.  Node offsets are
// 32-bit (the host limits all boxes together to 2^30 nodes), so every access
// is a scalar base plus one 32-bit vector offset shared by all planes.
#define PL(ptr, p) ((ptr) + (int64_t)(p) * plane)

// Element idx of an array through a 32-bit byte offset (idx * sizeof(T) <
// 2^32): the address is a scalar base plus a zero-extended 32-bit vector
// offset, which the hardware addresses directly.
template <class T>
__device__ __forceinline__ T &at(T *base, uint32_t idx) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ const T &at(const T *base, uint32_t idx) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                      (uint32_t)(idx * (uint32_t)sizeof(T)));
}

// The value unchanged, but opaque to the optimizer: address arithmetic
// derived from it inside the z-march is not hoisted out of the loop, where
// the many plane base pointers would not fit in scalar registers.
__device__ __forceinline__ int64_t opaque_i64(int64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// Hardware reciprocal and reciprocal square root (about 1 ulp), in place of
// the correctly rounded division and square root sequences.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// The wall rule of the stencils (a solid neighbour takes the centre node's
// value).  The neighbour's value v is an argument, so its (in-bounds) LDS
// load is issued whatever the flag and the choice is one select: written as
// `solid ? centre : array[...]`, the conditional load had become a branch
// per stencil point in the walled kernels (450 branches in one of them).
__device__ __forceinline__ float wall_rule(bool solid, float centre, float v) {
  return solid ? centre : v;
}
// num / den from r, the hardware reciprocal of den, refined by one
// Newton-Raphson step on the residual num - den q (formed exactly by an
// FMA): within about half an ulp, exactly 1 for num == den and 0 for
// num == 0.  The colour fractions and the velocity use it: num * r alone
// carries the fixed relative error of r for a given den, which made the
// colour masses and momenta of uniform regions drift by the same fraction
// of an ulp at every step.
__device__ __forceinline__ float div_refined(float num, float den, float r) {
  const float q = num * r;
  return fmaf(r, fmaf(-den, q, num), q);
}

// Order parameter phi = (rr - rb) / (rr + rb) of the stencils (Eq. 14, the
// densities already divided by their reference densities): the refined
// quotient, exactly +-1 in a pure phase (num = +-den), so that the bulk
// gradient is exactly zero, at half the instructions of the correctly
// rounded division it replaced (measured 0.027 ms of the 0.48 ms compact
// fused kernel at 256^3, where it runs on 1.9x the column's points).
__device__ __forceinline__ float phase_field(float rr, float rb) {
  const float den = rr + rb;
  return den > 0.f ? div_refined(rr - rb, den, rcp(den)) : 0.f;
}

// Scalar buffer descriptor of plane p of an SoA array whose planes are
// plane_bytes apart.  The host keeps every plane below 4 GiB, so a lane
// addresses it with one 32-bit byte offset and no vector address arithmetic.
// The descriptor's extent is the plane itself: an access at kDrop lies
// beyond it, a store there is discarded and a load returns zero, which lets
// lanes without work issue the same memory instructions as the others.
constexpr uint32_t kDrop = 0xFFFFFFF0u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, int64_t plane_bytes,
                                                             int p) {
  return __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char *>(static_cast<const char *>(base)) + p * plane_bytes, 0,
      (int)(uint32_t)plane_bytes, 0x00020000);
}
// Population stores carry the non-temporal hint: the stored state is read
// only by the next step's pull, and keeping it out of the caches measured
// faster for both kernels of the step than plain stores.
constexpr int kNonTemporal = 2;  // cache policy bit of a streaming access
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float buf_ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ double buf_ld_f64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// A 4- or 8-byte word (a plane element of a population array).
template <class W>
__device__ __forceinline__ W buf_ld_w(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(W) == 8) {
    return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  } else {
    return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  }
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0,
                                        kNonTemporal);
}
__device__ __forceinline__ void buf_st(uint16_t v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)off, 0, kNonTemporal);
}
__device__ __forceinline__ void buf_st(uint32_t v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)off, 0, kNonTemporal);
}
__device__ __forceinline__ void buf_st(uint64_t v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0,
                                        kNonTemporal);
}
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0,
                                        kNonTemporal);
}
// The same, for values read once: the streaming hint keeps them from
// displacing the halo lines that neighbouring columns share in L2.
__device__ __forceinline__ float ldpl_nt(const float *base, int64_t plane, int p, uint32_t node) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                       plane_rsrc(base, plane * 4, p), (int)(node * 4u), 0, kNonTemporal));
}
__device__ __forceinline__ double buf_ld_f64_nt(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, kNonTemporal));
}
// Float plane p of an aux-like array at node.
__device__ __forceinline__ float ldpl(const float *base, int64_t plane, int p, uint32_t node) {
  return buf_ld_f32(plane_rsrc(base, plane * 4, p), node * 4u);
}
// Byte offset of node in a plane of T, or kDrop for a lane that must not
// access it.
template <class T>
__device__ __forceinline__ uint32_t boff(bool live, uint32_t node) {
  return live ? node * (uint32_t)sizeof(T) : kDrop;
}

// Workgroups are dispatched to the 8 XCDs in round-robin order.  Remap them
// so that each XCD, with its own L2, works through a contiguous range of
// logical blocks: neighbouring rows and columns then share cached halo lines.
// Grids using this are padded to a multiple of 8 with idle blocks.
__device__ __forceinline__ uint32_t xcd_block() {
  const uint32_t per = gridDim.x >> 3;
  return (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
}

__device__ __forceinline__ int wrap_once(int v, int n) {
  // v in [-n, 2n)
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

__device__ __forceinline__ int wrap_any(int v, int n) {
  while (v < 0) v += n;
  while (v >= n) v -= n;
  return v;
}

__device__ __forceinline__ bool is_solid(const BoxDev &B, int y, int z) {
  return ((B.walls & 1u) && (y == 0 || y == B.ny - 1)) ||
         ((B.walls & 2u) && (z == 0 || z == B.nz - 1));
}

// Slots of a box's solid nodes in the in-place wall stash (box-local; the
// box's slots start at B.wbase): first the z-wall planes (z = 0, then
// z = nz-1; slot z' nx ny + y nx + x), then the y-wall rows of the other
// layers (y = 0 and y = ny-1 alternating, layer by layer).  wall_node
// inverts the map.
__host__ __device__ inline uint32_t wall_slot(const BoxDev &B, int x, int y, int z) {
  const uint32_t nx = (uint32_t)B.nx, nxy = nx * (uint32_t)B.ny;
  const bool zw = (B.walls & 2u) != 0u;
  if (zw && (z == 0 || z == B.nz - 1))
    return (z == 0 ? 0u : nxy) + (uint32_t)y * nx + (uint32_t)x;
  const uint32_t zoff = zw ? 2u * nxy : 0u;
  const uint32_t layer = (uint32_t)(z - (zw ? 1 : 0));
  return zoff + (2u * layer + (y == 0 ? 0u : 1u)) * nx + (uint32_t)x;
}
__host__ __device__ inline void wall_node(const BoxDev &B, uint32_t slot, int &x, int &y, int &z) {
  const uint32_t nx = (uint32_t)B.nx, nxy = nx * (uint32_t)B.ny;
  const bool zw = (B.walls & 2u) != 0u;
  if (zw && slot < 2u * nxy) {
    z = slot < nxy ? 0 : B.nz - 1;
    const uint32_t r = slot < nxy ? slot : slot - nxy;
    y = (int)(r / nx);
    x = (int)(r - (uint32_t)y * nx);
    return;
  }
  const uint32_t r = slot - (zw ? 2u * nxy : 0u);
  const uint32_t row = r / nx;
  x = (int)(r - row * nx);
  z = (int)(row / 2u) + (zw ? 1 : 0);
  y = (row & 1u) ? B.ny - 1 : 0;
}

// ---------------------------------------------------------------------------
// Population storage formats.
//
// Plain FP32: 54 float planes, plane c*27 + i.
// Mass-exact formats: the 26 moving directions are stored in type T as
// colour pairs, pair plane i - 1, and the two rest populations in FP64
// planes after them.  The collision sets the rest population from the node's
// colour density (carried in FP64) minus the 26 stored moving populations
// as they will be read back, so each colour's mass is conserved to FP64
// rounding whatever the storage precision.  FP16/BF16 store each moving
// population minus the pure-phase rest equilibrium of its colour,
// s^k_i = w_i rho_k^0 (c_s^k)^2 / c_s^2, rounded to T (zero stays exact).
// ---------------------------------------------------------------------------
// A direction's red and blue populations stream from and to the same node,
// so the mass-exact formats store them as one pair word (red in the low
// half): one memory access moves both.  Plain FP32 keeps one plane per
// colour and direction: its collision kernel stores the populations faster
// that way, and its pull loses less than the collision gains (measured).
struct Split32 {
  using W = float;  // one plane element
  static constexpr bool kPaired = false;
  static constexpr bool kCShift = false;
};
struct Pair32 {
  using W = uint64_t;
  static constexpr bool kPaired = true;
  static constexpr bool kCShift = false;
  __device__ static W pack(float r, float b) {
    return (uint64_t)__builtin_bit_cast(uint32_t, r) | ((uint64_t)__builtin_bit_cast(uint32_t, b) << 32);
  }
  __device__ static float lo(W w) { return __builtin_bit_cast(float, (uint32_t)w); }
  __device__ static float hi(W w) { return __builtin_bit_cast(float, (uint32_t)(w >> 32)); }
};
struct Pair16 {
  using W = uint32_t;
  static constexpr bool kPaired = true;
  static constexpr bool kCShift = false;
  __device__ static W pack(uint16_t r, uint16_t b) { return (uint32_t)r | ((uint32_t)b << 16); }
  __device__ static uint16_t lo(W w) { return (uint16_t)w; }
  __device__ static uint16_t hi(W w) { return (uint16_t)(w >> 16); }
};
struct StoreF32 : Split32 {
  using T = float;
  static constexpr bool kExact = false, kShift = false;
  __device__ static T enc(float v) { return v; }
  __device__ static float dec(T g) { return g; }
};
// Plain FP32 in colour pairs: the same values as StoreF32, another layout
// (27 pair planes); faster where many small boxes leave tiles ragged.
struct StoreF32P : Pair32 {
  using T = float;
  static constexpr bool kExact = false, kShift = false;
  __device__ static T enc(float v) { return v; }
  __device__ static float dec(T g) { return g; }
};
struct StoreF32X : Pair32 {
  using T = float;
  static constexpr bool kExact = true, kShift = false;
  __device__ static T enc(float v) { return v; }
  __device__ static float dec(T g) { return g; }
};
struct StoreF16 : Pair16 {
  using T = uint16_t;
  static constexpr bool kExact = true, kShift = true;
  __device__ static T enc(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
  __device__ static float dec(T g) { return (float)__builtin_bit_cast(_Float16, g); }
};
struct StoreBF16 : Pair16 {
  using T = uint16_t;
  static constexpr bool kExact = true, kShift = true;
  // round to nearest even: one hardware conversion on gfx950 (the
  // integer-arithmetic rounding it replaces cost a branch and six
  // instructions per stored value)
  __device__ static T enc(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
  __device__ static float dec(T g) { return __builtin_bit_cast(float, (uint32_t)g << 16); }
};

// Colour-fraction-scaled shift (FP16 / BF16): each moving population is
// stored as f^k_i - c_k s^k_i, with s^k_i the pure-phase rest equilibrium of
// colour k as above (unrounded) and c_k the colour fraction rho_k / rho of
// the node that wrote it (red c_r, blue 1 - c_r), itself stored per node in
// the format's 16-bit type.  In a pure phase the stored values are the small
// deviations from equilibrium and the opposite colour stores exact zeros; at
// the interface, where the constant shift leaves a remainder of the order of
// s itself, each colour stores its deviation from its own share of the
// equilibrium.  A reader decodes a population with the fraction stored at
// its source node x - c_i.
struct StoreF16C : StoreF16 {
  static constexpr bool kCShift = true;
};
struct StoreBF16C : StoreBF16 {
  static constexpr bool kCShift = true;
};

__host__ __device__ inline int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

// Views of one population buffer.  Plain FP32: 54 float planes, plane
// c*27 + i (paired: 27 pair planes, plane i).  Mass-exact formats: 26 pair
// planes of the moving directions (plane i - 1), then the FP64 rest
// populations of the two colours.
template <class S>
struct Pops {
  using W = typename S::W;
  static constexpr int kDirs = S::kExact ? 26 : 27;  // stored directions per colour
  static constexpr int kPlanes = S::kPaired ? kDirs : 2 * kDirs;
  W *pw;
  double *rest;
  typename S::T *cfr;  // colour-fraction formats: the red fraction of each node
  int64_t plane;
  __device__ Pops(void *base, int64_t plane_) : plane(plane_) {
    pw = (W *)base;
    rest = (double *)((char *)base + align256(kPlanes * plane_ * (int64_t)sizeof(W)));
    cfr = (typename S::T *)(rest + 2 * plane_);
  }
  // plane of direction i (paired), or of direction i and colour c (split)
  __device__ static int slot(int i, int c = 0) {
    return (S::kExact ? i - 1 : i) + (S::kPaired ? 0 : c * kDirs);
  }
  __device__ W *plane_of(int i, int c = 0) const { return pw + (int64_t)slot(i, c) * plane; }
  __device__ double *restp(int c) const { return rest + (int64_t)c * plane; }
};

// FP64 colour densities (mass-exact formats), after the 21 float aux planes.
__device__ __forceinline__ double *aux_rho64(float *aux, int64_t plane) {
  return (double *)((char *)aux + align256((int64_t)A_COUNT * plane * 4));
}

// Shift of direction i of colour c (0 without shift): the constant shift
// rounded to the storage type, or, for the colour-fraction formats, the
// unrounded constant scaled by the writer's colour fraction (cr: its red
// fraction as stored; blue takes 1 - cr).  The stored value of a population
// f is enc(f - shift); it reads back as dec(stored) + shift, an expression
// every kernel evaluates the same way.
template <class S>
__device__ __forceinline__ float pop_shift(const BoxDev &B, int c, int i, float cr = 0.f) {
  if (!S::kShift || i == 0) return 0.f;
  const int cls = kCX[i] * kCX[i] + kCY[i] * kCY[i] + kCZ[i] * kCZ[i];
  if constexpr (S::kCShift) {
    const float frac = c == 0 ? cr : 1.0f - cr;
    return frac * B.shift[c][cls];
  } else {
    return S::dec(S::enc(B.shift[c][cls]));
  }
}
// Stored value of a population f of colour c whose shift is sh, and the
// value read back.  The colour-fraction formats store (f - sh) times the
// colour's power-of-two scale 2^(10 - e_c), e_c = floor(log2 rho_c^0): a
// colour's values at its reference density then sit near 2^10, far below
// half's largest finite value (65504), and its small values (the other
// phase's tail near an interface, the light phase at a density ratio of
// 1000) stay in half's normal range down to about 6e-8 rho_c^0 instead of
// becoming subnormals with an absolute step of 6e-8.  The scaling is exact.
template <class S>
__device__ __forceinline__ typename S::T encode_pop(const BoxDev &B, int c, float f, float sh) {
  if constexpr (S::kCShift) {
    return S::enc((f - sh) * B.pscale[c]);
  } else {
    return S::enc(f - sh);
  }
}
template <class S>
__device__ __forceinline__ float decode_pop(const BoxDev &B, int c, typename S::T g, float sh) {
  if constexpr (S::kCShift) {
    const float v = S::dec(g) * B.pinv[c];
    return v + sh;
  } else {
    return S::dec(g) + sh;
  }
}
// Red fraction rho_r / rho of a node as the colour-fraction formats store it
// (correctly rounded quotient: exactly 1 and 0 in the pure phases).
template <class S>
__device__ __forceinline__ typename S::T stored_fraction(float rr, float rb) {
  return S::enc(rr / (rr + rb));
}

template <class W>
__device__ __forceinline__ W ld(const W *p) {
  return __builtin_nontemporal_load(p);
}
template <class W>
__device__ __forceinline__ void st(W *p, W v) {
  __builtin_nontemporal_store(v, p);
}

// Both colours of direction i at node s, as stored (values of S::T).
template <class S>
__device__ __forceinline__ void ld_rb(const Pops<S> &p, int i, uint32_t s, typename S::T &r,
                                      typename S::T &b) {
  if constexpr (S::kPaired) {
    const typename S::W w = ld(&at(p.plane_of(i), s));
    r = S::lo(w);
    b = S::hi(w);
  } else {
    r = ld(&at(p.plane_of(i, 0), s));
    b = ld(&at(p.plane_of(i, 1), s));
  }
}
template <class S>
__device__ __forceinline__ void st_rb(const Pops<S> &p, int i, uint32_t d, typename S::T r,
                                      typename S::T b) {
  if constexpr (S::kPaired) {
    st(&at(p.plane_of(i), d), S::pack(r, b));
  } else {
    st(&at(p.plane_of(i, 0), d), r);
    st(&at(p.plane_of(i, 1), d), b);
  }
}

// A wall stash of the compact pull through one buffer descriptor over all
// its planes, with each access's plane in the lane offset (a stash holds
// solid nodes only; the host keeps it below 4 GiB).  The z march then holds
// one scalar descriptor per stash: with a pointer or a descriptor per plane
// the 54 plane addresses had been hoisted into scalar registers and spilled
// to vector lanes (627 v_readlane / v_writelane in one instantiation).
template <class S>
struct StashBuf {
  using W = typename S::W;
  __amdgpu_buffer_rsrc_t r;
  uint32_t pb;    // bytes per plane
  uint32_t rest;  // byte offset of the FP64 rest planes (mass-exact formats)
  __device__ StashBuf(const void *base, int64_t plane) {
    pb = (uint32_t)plane * (uint32_t)sizeof(W);
    rest = (uint32_t)align256(Pops<S>::kPlanes * plane * (int64_t)sizeof(W));
    const uint32_t bytes = rest + (S::kExact ? 16u * (uint32_t)plane : 0u);
    r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
  }
  __device__ uint32_t off(int i, int c, uint32_t s) const {
    return (uint32_t)Pops<S>::slot(i, c) * pb + s * (uint32_t)sizeof(W);
  }
  // both colours of direction i at slot s, as stored
  __device__ void ld(int i, uint32_t s, typename S::T &rv, typename S::T &bv) const {
    if constexpr (S::kPaired) {
      const W w = buf_ld_w<W>(r, off(i, 0, s));
      rv = S::lo(w);
      bv = S::hi(w);
    } else {
      rv = buf_ld_w<W>(r, off(i, 0, s));
      bv = buf_ld_w<W>(r, off(i, 1, s));
    }
  }
  __device__ void st(int i, uint32_t d, typename S::T rv, typename S::T bv) const {
    if constexpr (S::kPaired) {
      buf_st(S::pack(rv, bv), r, off(i, 0, d));
    } else {
      buf_st(rv, r, off(i, 0, d));
      buf_st(bv, r, off(i, 1, d));
    }
  }
  __device__ uint32_t rest_off(int c, uint32_t s) const {
    return rest + (uint32_t)c * (pb / (uint32_t)sizeof(W)) * 8u + s * 8u;
  }
};
// ---------------------------------------------------------------------------
// k_pull: f^k_i(x) = stored_i(x - c_i); local moments; bounce-back at solid
// nodes (the pulled populations are reversed and stored for the next step).
// In-place layouts (src == dst) pass a wall stash: the reversed populations
// of solid nodes go there (slot wall_slot, plane length wplane), because
// other nodes of this launch still read what the solid node holds;
// k_wall_copy moves them into place once the pull has completed.  STASH
// selects that path at compile time, so the two-buffer pull carries none of
// it (measured 4 % faster than one kernel with a run-time switch).  SS is
// the stash's format: the storage's own, or (the compact schedule of the
// 16-bit formats) the mass-exact FP32 one, into which the reversed
// populations go decoded.
// ---------------------------------------------------------------------------
template <class S, bool STASH, class SS = S>
__global__ __launch_bounds__(kBlock) void k_pull(const BoxDev *__restrict__ boxes,
                                                 const int32_t *__restrict__ blk_box,
                                                 void *__restrict__ src_, void *__restrict__ dst_,
                                                 float *__restrict__ aux, int64_t plane,
                                                 int bounce, void *__restrict__ stash_,
                                                 int64_t wplane) {
  const uint32_t lb = xcd_block();
  const int b = blk_box[lb];
  if (b < 0) return;
  const BoxDev B = boxes[b];
  const int64_t local = (int64_t)(lb - B.blk0) * kBlock + threadIdx.x;
  if (local >= B.n) return;
  const Pops<S> src(src_, plane), dst(dst_, plane);
  const uint32_t l = (uint32_t)local;
  const uint32_t yz = fdiv(l, B.fdx);
  const int x = (int)(l - yz * (uint32_t)B.nx);
  const int z = (int)fdiv(yz, B.fdy);
  const int y = (int)(yz - (uint32_t)z * (uint32_t)B.ny);
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  // source coordinates x - c: index 0 -> c = -1 (source x+1), 1 -> c = 0, 2 -> c = +1
  const int xs[3] = {wrap_once(x + 1, nx), x, wrap_once(x - 1, nx)};
  const int ys[3] = {wrap_once(y + 1, ny), y, wrap_once(y - 1, ny)};
  const int zs[3] = {wrap_once(z + 1, nz), z, wrap_once(z - 1, nz)};
  uint32_t row[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      row[a][c] = (uint32_t)B.base + (uint32_t)nx * ((uint32_t)ys[a] + (uint32_t)ny * (uint32_t)zs[c]);
  const uint32_t node = (uint32_t)(B.base + local);

  typename S::T gr[kQ], gb[kQ];
  constexpr int i0 = S::kExact ? 1 : 0;
#pragma unroll
  for (int i = i0; i < kQ; ++i) {
    const uint32_t s = row[kCY[i] + 1][kCZ[i] + 1] + (uint32_t)xs[kCX[i] + 1];
    ld_rb(src, i, s, gr[i], gb[i]);
  }
  // colour-fraction formats: the red fraction stored at each source node
  float csrc[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) csrc[i] = 0.f;
  if constexpr (S::kCShift) {
#pragma unroll
    for (int i = 1; i < kQ; ++i)
      csrc[i] = S::dec(ld(&at(src.cfr, row[kCY[i] + 1][kCZ[i] + 1] + (uint32_t)xs[kCX[i] + 1])));
  }
  double rr0 = 0.0, rb0 = 0.0;
  if (S::kExact) {
    rr0 = at(src.restp(0), node);
    rb0 = at(src.restp(1), node);
  }
  if (is_solid(B, y, z)) {
    if constexpr (!std::is_same<SS, S>::value) {
      // decoded into the mass-exact FP32 stash (rest populations as stored)
      static_assert(STASH && SS::kExact && S::kExact, "decoded stash of a mass-exact format");
      if (bounce) {
        const Pops<SS> out(stash_, wplane);
        const uint32_t at_ = (uint32_t)B.wbase + wall_slot(B, x, y, z);
#pragma unroll
        for (int i = 1; i < kQ; ++i)
          st_rb(out, opposite(i), at_, decode_pop<S>(B, 0, gr[i], pop_shift<S>(B, 0, i, csrc[i])),
                decode_pop<S>(B, 1, gb[i], pop_shift<S>(B, 1, i, csrc[i])));
        at(out.restp(0), at_) = rr0;
        at(out.restp(1), at_) = rb0;
      }
    } else if (bounce) {
      // the shift of direction i equals that of its opposite: copy raw pairs
      const Pops<S> out(STASH ? stash_ : dst_, STASH ? wplane : plane);
      const uint32_t at_ = STASH ? (uint32_t)B.wbase + wall_slot(B, x, y, z) : node;
      if constexpr (S::kCShift) {
        // the solid node takes the red fraction of its wall-normal fluid
        // neighbour and re-encodes each reversed population with it (one
        // more rounding of the bounced values; exact where the fluid next to
        // the wall is a pure phase and the decoded value less its shift is
        // the stored one)
        const int dy = (B.walls & 1u) ? (y == 0 ? -1 : (y == ny - 1 ? 1 : 0)) : 0;
        const int dz = (B.walls & 2u) ? (z == 0 ? -1 : (z == nz - 1 ? 1 : 0)) : 0;
        const uint32_t nb = (uint32_t)B.base + (uint32_t)x +
                            (uint32_t)nx * ((uint32_t)(y - dy) + (uint32_t)ny * (uint32_t)(z - dz));
        const typename S::T craw = ld(&at(src.cfr, nb));
        const float cown = S::dec(craw);
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
          const float fr = decode_pop<S>(B, 0, gr[i], pop_shift<S>(B, 0, i, csrc[i]));
          const float fb = decode_pop<S>(B, 1, gb[i], pop_shift<S>(B, 1, i, csrc[i]));
          st_rb(out, opposite(i), at_, encode_pop<S>(B, 0, fr, pop_shift<S>(B, 0, i, cown)),
                encode_pop<S>(B, 1, fb, pop_shift<S>(B, 1, i, cown)));
        }
        at(out.cfr, at_) = craw;
      } else {
#pragma unroll
        for (int i = i0; i < kQ; ++i) st_rb(out, opposite(i), at_, gr[i], gb[i]);
      }
      if (S::kExact) {
        at(out.restp(0), at_) = rr0;
        at(out.restp(1), at_) = rb0;
      }
    }
#pragma unroll
    for (int k = 0; k <= A_PYZ; ++k) at(PL(aux, k), node) = 0.0f;
    if (S::kExact) {
      double *r64 = aux_rho64(aux, plane);
      at(r64, node) = 0.0;
      at(r64 + plane, node) = 0.0;
    }
    return;
  }
  float rr = 0.f, rb = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
  float pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pxz = 0.f, pyz = 0.f;
  double drr = rr0, drb = rb0;
#pragma unroll
  for (int i = i0; i < kQ; ++i) {
    const float vr = decode_pop<S>(B, 0, gr[i], pop_shift<S>(B, 0, i, csrc[i]));
    const float vb = decode_pop<S>(B, 1, gb[i], pop_shift<S>(B, 1, i, csrc[i]));
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
    if (kCZ[i]) jz += kCZ[i] > 0 ? f : -f;
    if (kCX[i]) pxx += f;
    if (kCY[i]) pyy += f;
    if (kCZ[i]) pzz += f;
    if (kCX[i] * kCY[i]) pxy += kCX[i] * kCY[i] > 0 ? f : -f;
    if (kCX[i] * kCZ[i]) pxz += kCX[i] * kCZ[i] > 0 ? f : -f;
    if (kCY[i] * kCZ[i]) pyz += kCY[i] * kCZ[i] > 0 ? f : -f;
  }
  if (S::kExact) {
    rr = (float)drr;
    rb = (float)drb;
    double *r64 = aux_rho64(aux, plane);
    st(&at(r64, node), drr);
    st(&at(r64 + plane, node), drb);
  }
  // the moments stream to the next kernel: stores with the streaming hint
  // (measured faster for both kernels than plain stores)
  st(&at(PL(aux, A_RR), node), rr);
  st(&at(PL(aux, A_RB), node), rb);
  st(&at(PL(aux, A_JX), node), jx);
  st(&at(PL(aux, A_JY), node), jy);
  st(&at(PL(aux, A_JZ), node), jz);
  st(&at(PL(aux, A_PXX), node), pxx);
  st(&at(PL(aux, A_PYY), node), pyy);
  st(&at(PL(aux, A_PZZ), node), pzz);
  st(&at(PL(aux, A_PXY), node), pxy);
  st(&at(PL(aux, A_PXZ), node), pxz);
  st(&at(PL(aux, A_PYZ), node), pyz);
}

// Force density at a fluid node: the CSF force of Eq. (15) from the
// curvature, |grad phi| and the normal, the constant body force G, and the
// buoyancy force -(rho - rho_ref) g of the Rayleigh-Taylor case (Sec. IV.E).
__device__ __forceinline__ void interface_force(const BoxDev &B, float kap, float mag, float nxv,
                                                float nyv, float nzv, float rho, float &Fx,
                                                float &Fy, float &Fz) {
  const float hs = 0.5f * B.sigma * kap * mag;
  const float drho = rho - B.rho_ref;
  Fx = fmaf(-drho, B.bgx, fmaf(hs, nxv, B.Gx));
  Fy = fmaf(-drho, B.bgy, fmaf(hs, nyv, B.Gy));
  Fz = fmaf(-drho, B.bgz, fmaf(hs, nzv, B.Gz));
}

// ---------------------------------------------------------------------------
// k_interface: for a TX*TY*TZ tile, stage phi on the tile + 3 halo, grad phi
// and n on + 2, grad n, kappa, F, u, q on + 1, and Q on the tile.  Every
// stencil is Eq. (20): grad chi = 3 sum_i w_i chi(x + c_i) c_i; a neighbour in
// a solid layer takes the value of the stencil's centre node.
// ---------------------------------------------------------------------------
template <int TX, int TY, int TZ>
struct IfaceGeom {
  static constexpr int R3X = TX + 6, R3Y = TY + 6, R3Z = TZ + 6, R3 = R3X * R3Y * R3Z;
  static constexpr int R2X = TX + 4, R2Y = TY + 4, R2Z = TZ + 4, R2 = R2X * R2Y * R2Z;
  static constexpr int R1X = TX + 2, R1Y = TY + 2, R1Z = TZ + 2, R1 = R1X * R1Y * R1Z;
  static constexpr int T = TX * TY * TZ;
};

// 26-point isotropic gradient (Eq. 20) of a scalar field held in LDS with
// strides (1, SY, SZ).  Each component is summed over pairs of opposite
// neighbours as w * (chi(+) - chi(-)), so that a uniform field gives exactly
// zero.  solid(dy, dz) reports whether the neighbour row is solid; solid
// neighbours take the centre value.
template <int SY, int SZ, class Solid>
__device__ __forceinline__ void lds_gradient(const float *f, int c, Solid solid, float &gx,
                                             float &gy, float &gz) {
  const float vc = f[c];
  float v[3][3][3];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const bool s = solid(dy, dz);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx)
        v[dz + 1][dy + 1][dx + 1] = wall_rule(s, vc, f[c + dx + SY * dy + SZ * dz]);
    }
  // (1/c_s^2) w_i c_i = 3 * w(dx) w(dy) w(dz) * c_i; for the pair along one
  // axis the factor is 3 * (1/6) * w(.) w(.) = w(.) w(.) / 2.
  gx = gy = gz = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float w = 0.5f * w1d(a - 1) * w1d(b - 1);
      gx = fmaf(w, v[b][a][2] - v[b][a][0], gx);  // a: dy, b: dz
      gy = fmaf(w, v[b][2][a] - v[b][0][a], gy);  // a: dx, b: dz
      gz = fmaf(w, v[2][b][a] - v[0][b][a], gz);  // a: dx, b: dy
    }
}

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_interface(const BoxDev *__restrict__ boxes,
                                                      const int32_t *__restrict__ tile_box,
                                                      float *__restrict__ aux, int64_t plane,
                                                      int write_kappa) {
  using G = IfaceGeom<TX, TY, TZ>;
  __shared__ float s_phi[G::R3];
  __shared__ float s_n[4][G::R2];   // n_x, n_y, n_z, |grad phi|
  __shared__ float s_q[3][G::R1];
  __shared__ uint8_t s_sy[G::R3Y], s_sz[G::R3Z];

  const int b = tile_box[blockIdx.x];
  const BoxDev B = boxes[b];
  const uint32_t t = blockIdx.x - B.tile0;
  const uint32_t tyz = fdiv(t, B.ftx);
  const int tx = (int)(t - tyz * (uint32_t)B.tnx);
  const int tz = (int)fdiv(tyz, B.fty);
  const int ty = (int)(tyz - (uint32_t)tz * (uint32_t)B.tny);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int nx = B.nx, ny = B.ny, nz = B.nz;

  // solid flags of the halo rows
  for (int i = threadIdx.x; i < G::R3Y; i += kBlock) {
    const int gy = wrap_any(y0 + i - 3, ny);
    s_sy[i] = (B.walls & 1u) && (gy == 0 || gy == ny - 1);
  }
  for (int i = threadIdx.x; i < G::R3Z; i += kBlock) {
    const int gz = wrap_any(z0 + i - 3, nz);
    s_sz[i] = (B.walls & 2u) && (gz == 0 || gz == nz - 1);
  }
  // stage 1: phi on the tile + 3 (Eq. 14)
  for (int i = threadIdx.x; i < G::R3; i += kBlock) {
    const int lx = i % G::R3X, ly = (i / G::R3X) % G::R3Y, lz = i / (G::R3X * G::R3Y);
    const int gx = wrap_any(x0 + lx - 3, nx), gy = wrap_any(y0 + ly - 3, ny),
              gz = wrap_any(z0 + lz - 3, nz);
    const uint32_t node =
        (uint32_t)B.base + (uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz);
    const float rr = at(PL(aux, A_RR), node) * B.ir0r;
    const float rb = at(PL(aux, A_RB), node) * B.ir0b;
    s_phi[i] = phase_field(rr, rb);
  }
  __syncthreads();

  // stage 2: grad phi and n on the tile + 2 (Eqs. 17, 20)
  for (int i = threadIdx.x; i < G::R2; i += kBlock) {
    const int lx = i % G::R2X, ly = (i / G::R2X) % G::R2Y, lz = i / (G::R2X * G::R2Y);
    const int c3 = (lx + 1) + G::R3X * ((ly + 1) + G::R3Y * (lz + 1));
    float nxv = 0.f, nyv = 0.f, nzv = 0.f, mag = 0.f;
    if (!(s_sy[ly + 1] | s_sz[lz + 1])) {
      float gx, gy, gz;
      lds_gradient<G::R3X, G::R3X * G::R3Y>(
          s_phi, c3, [&](int dy, int dz) { return (bool)(s_sy[ly + 1 + dy] | s_sz[lz + 1 + dz]); },
          gx, gy, gz);
      const float g2 = gx * gx + gy * gy + gz * gz;
      if (g2 > 1e-24f) {  // |grad phi| > 1e-12
        const float inv = rsq(g2);
        mag = g2 * inv;
        nxv = gx * inv;
        nyv = gy * inv;
        nzv = gz * inv;
      }
    }
    s_n[0][i] = nxv;
    s_n[1][i] = nyv;
    s_n[2][i] = nzv;
    s_n[3][i] = mag;
  }
  __syncthreads();

  // stage 3: grad n, kappa, F, u, q on the tile + 1 (Eqs. 11, 15, 16, 65)
  for (int i = threadIdx.x; i < G::R1; i += kBlock) {
    const int lx = i % G::R1X, ly = (i / G::R1X) % G::R1Y, lz = i / (G::R1X * G::R1Y);
    const int c2 = (lx + 1) + G::R2X * ((ly + 1) + G::R2Y * (lz + 1));
    const int gx = wrap_any(x0 + lx - 1, nx), gy = wrap_any(y0 + ly - 1, ny),
              gz = wrap_any(z0 + lz - 1, nz);
    const uint32_t node =
        (uint32_t)B.base + (uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz);
    const bool solid = s_sy[ly + 2] | s_sz[lz + 2];
    float qx = 0.f, qy = 0.f, qz = 0.f;
    float kap = 0.f, Fx = 0.f, Fy = 0.f, Fz = 0.f;
    const float nxv = s_n[0][c2], nyv = s_n[1][c2], nzv = s_n[2][c2], mag = s_n[3][c2];
    if (!solid) {
      auto sol = [&](int dy, int dz) { return (bool)(s_sy[ly + 2 + dy] | s_sz[lz + 2 + dz]); };
      float dxx, dxy, dxz, dyx, dyy, dyz, dzx, dzy, dzz;  // d n_a / d x_b
      lds_gradient<G::R2X, G::R2X * G::R2Y>(s_n[0], c2, sol, dxx, dxy, dxz);
      lds_gradient<G::R2X, G::R2X * G::R2Y>(s_n[1], c2, sol, dyx, dyy, dyz);
      lds_gradient<G::R2X, G::R2X * G::R2Y>(s_n[2], c2, sol, dzx, dzy, dzz);
      // kappa = -(I - n n) : grad n
      const float div = dxx + dyy + dzz;
      const float proj = nxv * (nxv * dxx + nyv * dxy + nzv * dxz) +
                         nyv * (nxv * dyx + nyv * dyy + nzv * dyz) +
                         nzv * (nxv * dzx + nyv * dzy + nzv * dzz);
      kap = proj - div;
      const float rr = at(PL(aux, A_RR), node);
      const float rb = at(PL(aux, A_RB), node);
      const float rho = rr + rb;
      interface_force(B, kap, mag, nxv, nyv, nzv, rho, Fx, Fy, Fz);
      const float irho = rcp(rho);
      const float ux = fmaf(0.5f, Fx, at(PL(aux, A_JX), node)) * irho;
      const float uy = fmaf(0.5f, Fy, at(PL(aux, A_JY), node)) * irho;
      const float uz = fmaf(0.5f, Fz, at(PL(aux, A_JZ), node)) * irho;
      const float dev = rr * B.cs2r + rb * B.cs2b - rho * kCs2;
      qx = dev * ux;
      qy = dev * uy;
      qz = dev * uz;
    }
    s_q[0][i] = qx;
    s_q[1][i] = qy;
    s_q[2][i] = qz;
    // tile nodes: write n, F (and kappa)
    const int ox = lx - 1, oy = ly - 1, oz = lz - 1;
    if (ox >= 0 && ox < TX && oy >= 0 && oy < TY && oz >= 0 && oz < TZ && x0 + ox < nx &&
        y0 + oy < ny && z0 + oz < nz) {
      st(&at(PL(aux, A_NX), node), nxv);
      st(&at(PL(aux, A_NY), node), nyv);
      st(&at(PL(aux, A_NZ), node), nzv);
      st(&at(PL(aux, A_FX), node), Fx);
      st(&at(PL(aux, A_FY), node), Fy);
      st(&at(PL(aux, A_FZ), node), Fz);
      if (write_kappa) st(&at(PL(aux, A_KAPPA), node), kap);
    }
  }
  __syncthreads();

  // stage 4: Q on the tile (Eq. 65, component-wise)
  for (int i = threadIdx.x; i < G::T; i += kBlock) {
    const int ox = i % TX, oy = (i / TX) % TY, oz = i / (TX * TY);
    const int gx = x0 + ox, gy = y0 + oy, gz = z0 + oz;
    if (gx >= nx || gy >= ny || gz >= nz) continue;
    const uint32_t node =
        (uint32_t)B.base + (uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz);
    const int c1 = (ox + 1) + G::R1X * ((oy + 1) + G::R1Y * (oz + 1));
    float Qx = 0.f, Qy = 0.f, Qz = 0.f;
    if (!(s_sy[oy + 3] | s_sz[oz + 3])) {
      auto sol = [&](int dy, int dz) { return (bool)(s_sy[oy + 3 + dy] | s_sz[oz + 3 + dz]); };
      float a, bq, c;
      lds_gradient<G::R1X, G::R1X * G::R1Y>(s_q[0], c1, sol, a, bq, c);
      Qx = -3.0f * a;
      lds_gradient<G::R1X, G::R1X * G::R1Y>(s_q[1], c1, sol, a, bq, c);
      Qy = -3.0f * bq;
      lds_gradient<G::R1X, G::R1X * G::R1Y>(s_q[2], c1, sol, a, bq, c);
      Qz = -3.0f * c;
    }
    st(&at(PL(aux, A_QX), node), Qx);
    st(&at(PL(aux, A_QY), node), Qy);
    st(&at(PL(aux, A_QZ), node), Qz);
  }
}

// ---------------------------------------------------------------------------
// Node-local collision + recolouring.  Inputs: local moments (rho_r, rho_b, j,
// Pi) and interface fields (n, F, Q).  Output: f^{r*}, f^{b*} (Eqs. 18-19).
// ---------------------------------------------------------------------------
struct NodeIn {
  float rr, rb, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
  float nx, ny, nz, Fx, Fy, Fz, Qx, Qy, Qz;
};

// Back-transform of post-collision central moments k about u into
// populations (three passes of 1D triplet maps, z, y, x) with the
// recolouring of Eqs. (18)-(19) folded into the last pass: each direction's
// pair goes out through emit(i, f_r, f_b).
template <class Emit>
__device__ __forceinline__ void emit_recoloured(const BoxDev &B, const float (&k)[27], float ux,
                                                float uy, float uz, float cr, float cb,
                                                float p, float nx, float ny, float nz,
                                                Emit &&emit) {
  const float s = B.beta * cr * cb * p;
  const float Rx = s * nx, Ry = s * ny, Rz = s * nz;
  float g[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      cm_to_pop_1d_x2(k[a + 3 * b], k[a + 3 * b + 9], k[a + 3 * b + 18], uz, g[a][b][0],
                      g[a][b][1], g[a][b][2]);
  float h[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
      cm_to_pop_1d_x2(g[a][0][cz], g[a][1][cz], g[a][2][cz], uy, h[a][0][cz], h[a][1][cz],
                      h[a][2][cz]);
#pragma unroll
  for (int cz = 0; cz < 3; ++cz)
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) {
      // the z and y passes leave 2^(|c_y| + |c_z|) on this row: the colour
      // fractions take its inverse (exact), the x pass keeps plain outputs
      const float sc = 1.0f / (float)(1 << ((cy != 1) + (cz != 1)));
      const float crs = sc * cr, cbs = sc * cb;
      float fx[3];
      cm_to_pop_1d(h[0][cy][cz], h[1][cy][cz], h[2][cy][cz], ux, fx[0], fx[1], fx[2]);
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) {
        const int i = dir_of(cx - 1, cy - 1, cz - 1);
        const float cR = (kCX[i] ? (kCX[i] > 0 ? Rx : -Rx) : 0.f) +
                         (kCY[i] ? (kCY[i] > 0 ? Ry : -Ry) : 0.f) +
                         (kCZ[i] ? (kCZ[i] > 0 ? Rz : -Rz) : 0.f);
        const float d = 3.0f * weight(i) * cR;
        emit(i, fmaf(crs, fx[cx], d), fmaf(cbs, fx[cx], -d));
      }
    }
}


// Emits each direction's recoloured pair through emit(i, f_r, f_b) as soon as
// its x-triplet of the back-transform is done, so that the 54 outputs never
// have to be live at once.  GENERAL: the box's equilibrium family and
// correction switch apply; otherwise Model D with the correction Q.
struct NoHook {
  __device__ void operator()() const {}
};

// pre() runs after the central moments are built and before the first
// population is emitted (the fused kernel issues the next slab's loads there).
template <bool GENERAL = false, class Emit, class Pre = NoHook>
__device__ __forceinline__ void collide_node(const BoxDev &B, const NodeIn &in, Emit &&emit,
                                             Pre &&pre = Pre()) {
  const float rho = in.rr + in.rb;
  const float irho = rcp(rho);
  const float ux = div_refined(fmaf(0.5f, in.Fx, in.jx), rho, irho);  // Eq. (11)
  const float uy = div_refined(fmaf(0.5f, in.Fy, in.jy), rho, irho);
  const float uz = div_refined(fmaf(0.5f, in.Fz, in.jz), rho, irho);
  const float p = in.rr * B.cs2r + in.rb * B.cs2b;   // Eq. (12)
  // Eqs. (14), (21), (22): omega_1 from the interpolated viscosity
  const float sr = in.rr * B.ir0r, sb = in.rb * B.ir0b;
  const float phi = (sr - sb) * rcp(sr + sb);
  const float nu = 0.5f * ((1.0f + phi) * B.nu_r + (1.0f - phi) * B.nu_b);
  const float w1 = p * rcp(fmaf(rho, nu, 0.5f * p));  // 1 / (rho nu / p + 1/2)
  const float w2 = B.omega2;
  // second-order central moments from raw ones (Eqs. 23-24)
  const float kxx = in.pxx - 2.0f * ux * in.jx + rho * ux * ux;
  const float kyy = in.pyy - 2.0f * uy * in.jy + rho * uy * uy;
  const float kzz = in.pzz - 2.0f * uz * in.jz + rho * uz * uz;
  const float kxy = in.pxy - ux * in.jy - uy * in.jx + rho * ux * uy;
  const float kxz = in.pxz - ux * in.jz - uz * in.jx + rho * ux * uz;
  const float kyz = in.pyz - uy * in.jz - uz * in.jy + rho * uy * uz;
  // relaxation (Eq. 25 with omega_0 = omega_3..10 = 1 and k^eq of Eqs. 57-63)
  const bool use_q = !GENERAL || B.qcorr;
  const float Qx = use_q ? in.Qx : 0.f, Qy = use_q ? in.Qy : 0.f, Qz = use_q ? in.Qz : 0.f;
  const float r1 = 1.0f - w1, h1 = 1.0f - 0.5f * w1;
  const float A = r1 * (kxx - kyy) + h1 * (Qx - Qy);
  const float Bd = r1 * (kxx - kzz) + h1 * (Qx - Qz);
  const float T = (1.0f - w2) * (kxx + kyy + kzz) + 3.0f * w2 * p +
                  (1.0f - 0.5f * w2) * (Qx + Qy + Qz);
  const float third = 1.0f / 3.0f;
  const float sxx = (A + Bd + T) * third;
  const float syy = (T - 2.0f * A + Bd) * third;
  const float szz = (T + A - 2.0f * Bd) * third;
  float k[27];
  if (GENERAL)
    model_moments(B.model, rho, p, ux, uy, uz, in.Fx, in.Fy, in.Fz, sxx, syy, szz, r1 * kxy,
                  r1 * kxz, r1 * kyz, k);
  else
    model_d_moments(rho, p, in.Fx, in.Fy, in.Fz, sxx, syy, szz, r1 * kxy, r1 * kxz, r1 * kyz, k);
  pre();
  emit_recoloured(B, k, ux, uy, uz, div_refined(in.rr, rho, irho), div_refined(in.rb, rho, irho),
                  p, in.nx, in.ny, in.nz, emit);
}

// ---------------------------------------------------------------------------
// Compact post-collision state (unit higher rates, Model D with Q).  With
// every rate above second order equal to one, the collided populations of a
// node (Eqs. 66-67) and their recolouring (Eqs. 18-19) are a function of 17
// values: rho_r, rho_b, u, F, the six relaxed second-order central moments
// and n.  compact_of computes them from a node's moments and interface
// fields with the arithmetic of collide_node; emit_compact rebuilds the
// populations from them, bit for bit those collide_node emits.
// ---------------------------------------------------------------------------
constexpr int kCompact = 17;  // planes: rr rb ux uy uz Fx Fy Fz sxx syy szz sxy sxz syz nx ny nz
// FP64 colour densities of the compact state (mass-exact storage), after its
// 17 float planes.
__device__ __forceinline__ double *compact_rho64(void *cst, int64_t plane) {
  return (double *)((char *)cst + align256((int64_t)kCompact * plane * 4));
}

// GENERAL: the box's equilibrium family and correction switch (as
// collide_node<true>); the relaxed second moments have the same form.
template <bool GENERAL = false>
__device__ __forceinline__ void compact_of(const BoxDev &B, const NodeIn &in, float (&c)[kCompact]) {
  const float rho = in.rr + in.rb;
  const float irho = rcp(rho);
  const float ux = div_refined(fmaf(0.5f, in.Fx, in.jx), rho, irho);
  const float uy = div_refined(fmaf(0.5f, in.Fy, in.jy), rho, irho);
  const float uz = div_refined(fmaf(0.5f, in.Fz, in.jz), rho, irho);
  const float p = in.rr * B.cs2r + in.rb * B.cs2b;
  const float sr = in.rr * B.ir0r, sb = in.rb * B.ir0b;
  const float phi = (sr - sb) * rcp(sr + sb);
  const float nu = 0.5f * ((1.0f + phi) * B.nu_r + (1.0f - phi) * B.nu_b);
  const float w1 = p * rcp(fmaf(rho, nu, 0.5f * p));
  const float w2 = B.omega2;
  const float kxx = in.pxx - 2.0f * ux * in.jx + rho * ux * ux;
  const float kyy = in.pyy - 2.0f * uy * in.jy + rho * uy * uy;
  const float kzz = in.pzz - 2.0f * uz * in.jz + rho * uz * uz;
  const float kxy = in.pxy - ux * in.jy - uy * in.jx + rho * ux * uy;
  const float kxz = in.pxz - ux * in.jz - uz * in.jx + rho * ux * uz;
  const float kyz = in.pyz - uy * in.jz - uz * in.jy + rho * uy * uz;
  const float r1 = 1.0f - w1, h1 = 1.0f - 0.5f * w1;
  const bool use_q = !GENERAL || B.qcorr;
  const float Qx = use_q ? in.Qx : 0.f, Qy = use_q ? in.Qy : 0.f, Qz = use_q ? in.Qz : 0.f;
  const float A = r1 * (kxx - kyy) + h1 * (Qx - Qy);
  const float Bd = r1 * (kxx - kzz) + h1 * (Qx - Qz);
  const float T = (1.0f - w2) * (kxx + kyy + kzz) + 3.0f * w2 * p +
                  (1.0f - 0.5f * w2) * (Qx + Qy + Qz);
  const float third = 1.0f / 3.0f;
  c[0] = in.rr;
  c[1] = in.rb;
  c[2] = ux;
  c[3] = uy;
  c[4] = uz;
  c[5] = in.Fx;
  c[6] = in.Fy;
  c[7] = in.Fz;
  c[8] = (A + Bd + T) * third;
  c[9] = (T - 2.0f * A + Bd) * third;
  c[10] = (T + A - 2.0f * Bd) * third;
  c[11] = r1 * kxy;
  c[12] = r1 * kxz;
  c[13] = r1 * kyz;
  c[14] = in.nx;
  c[15] = in.ny;
  c[16] = in.nz;
}

// The central moments and recolouring inputs of a compact state: k (Eqs.
// 57-63 at unit higher rates), u, the colour fractions and R of Eq. (19).
struct CompactPost {
  float k[27];
  float ux, uy, uz, cr, cb, Rx, Ry, Rz;
};
template <bool GENERAL = false>
__device__ __forceinline__ void compact_post(const BoxDev &B, const float (&c)[kCompact],
                                             CompactPost &o) {
  const float rr = c[0], rb = c[1];
  const float rho = rr + rb;
  const float irho = rcp(rho);
  const float p = rr * B.cs2r + rb * B.cs2b;
  if (GENERAL)
    model_moments(B.model, rho, p, c[2], c[3], c[4], c[5], c[6], c[7], c[8], c[9], c[10], c[11],
                  c[12], c[13], o.k);
  else
    model_d_moments(rho, p, c[5], c[6], c[7], c[8], c[9], c[10], c[11], c[12], c[13], o.k);
  o.ux = c[2];
  o.uy = c[3];
  o.uz = c[4];
  o.cr = div_refined(rr, rho, irho);
  o.cb = div_refined(rb, rho, irho);
  const float s = B.beta * o.cr * o.cb * p;
  o.Rx = s * c[14];
  o.Ry = s * c[15];
  o.Rz = s * c[16];
}

// Populations -> central moments about u along one axis: (f_-, f_0, f_+) ->
// (k_0, k_1, k_2) = sum f (c - u)^n, n = 0, 1, 2 (Eq. 24 on D1Q3).
__device__ __forceinline__ void pop_to_cm_1d(float fm, float f0, float fp, float u, float &k0,
                                             float &k1, float &k2) {
  k0 = fm + f0 + fp;
  const float m1 = fp - fm, m2 = fp + fm;
  k1 = m1 - u * k0;
  k2 = m2 - 2.0f * u * m1 + u * u * k0;
}

// Collision with all relaxation rates of Eq. (25) (omega_0, omega_3..10 of
// the box, omega_1 from the viscosity, omega_2 the bulk rate): the 27
// central moments of the pulled total distribution f about u (x, y and z
// passes of pop_to_cm_1d), relaxed toward the equilibrium moments of the
// box's family with the forcing and correction terms, then back-transformed
// and recoloured.
template <class Emit>
__device__ __forceinline__ void collide_full(const BoxDev &B, const NodeIn &in,
                                             const float (&f)[27], Emit &&emit) {
  const float rho = in.rr + in.rb;
  const float irho = rcp(rho);
  const float ux = div_refined(fmaf(0.5f, in.Fx, in.jx), rho, irho);
  const float uy = div_refined(fmaf(0.5f, in.Fy, in.jy), rho, irho);
  const float uz = div_refined(fmaf(0.5f, in.Fz, in.jz), rho, irho);
  const float p = in.rr * B.cs2r + in.rb * B.cs2b;
  const float sr = in.rr * B.ir0r, sb = in.rb * B.ir0b;
  const float phi = (sr - sb) * rcp(sr + sb);
  const float nu = 0.5f * ((1.0f + phi) * B.nu_r + (1.0f - phi) * B.nu_b);
  const float w1 = p * rcp(fmaf(rho, nu, 0.5f * p));
  const float w2 = B.omega2;
  const float w0 = B.omh[0], w3 = B.omh[1], w4 = B.omh[2], w5 = B.omh[3], w6 = B.omh[4],
              w7 = B.omh[5], w8 = B.omh[6], w9 = B.omh[7], w10 = B.omh[8];
  const float Qx = B.qcorr ? in.Qx : 0.f, Qy = B.qcorr ? in.Qy : 0.f, Qz = B.qcorr ? in.Qz : 0.f;
  // central moments of f, k[a + 3b + 9c] = sum f (cx-ux)^a (cy-uy)^b (cz-uz)^c
  float g[3][3][3], h[3][3][3], k[27];
#pragma unroll
  for (int cy = 0; cy < 3; ++cy)
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
      pop_to_cm_1d(f[dir_of(-1, cy - 1, cz - 1)], f[dir_of(0, cy - 1, cz - 1)],
                   f[dir_of(1, cy - 1, cz - 1)], ux, g[0][cy][cz], g[1][cy][cz], g[2][cy][cz]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
      pop_to_cm_1d(g[a][0][cz], g[a][1][cz], g[a][2][cz], uy, h[a][0][cz], h[a][1][cz],
                   h[a][2][cz]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      pop_to_cm_1d(h[a][b][0], h[a][b][1], h[a][b][2], uz, k[a + 3 * b], k[a + 3 * b + 9],
                   k[a + 3 * b + 18]);
  float e[27];  // equilibrium central moments of the box's family
  model_moments(B.model, rho, p, ux, uy, uz, 0.f, 0.f, 0.f, p, p, p, 0.f, 0.f, 0.f, e);
#define K_(a, b, c) k[(a) + 3 * (b) + 9 * (c)]
#define E_(a, b, c) e[(a) + 3 * (b) + 9 * (c)]
#define S_(a, b, c) ks[(a) + 3 * (b) + 9 * (c)]
  float ks[27];
  S_(0, 0, 0) = rho;
  S_(1, 0, 0) = (1.0f - w0) * K_(1, 0, 0) + (1.0f - 0.5f * w0) * in.Fx;
  S_(0, 1, 0) = (1.0f - w0) * K_(0, 1, 0) + (1.0f - 0.5f * w0) * in.Fy;
  S_(0, 0, 1) = (1.0f - w0) * K_(0, 0, 1) + (1.0f - 0.5f * w0) * in.Fz;
  S_(1, 1, 0) = (1.0f - w1) * K_(1, 1, 0);
  S_(1, 0, 1) = (1.0f - w1) * K_(1, 0, 1);
  S_(0, 1, 1) = (1.0f - w1) * K_(0, 1, 1);
  {
    const float kxx = K_(2, 0, 0), kyy = K_(0, 2, 0), kzz = K_(0, 0, 2);
    const float exx = E_(2, 0, 0), eyy = E_(0, 2, 0), ezz = E_(0, 0, 2);
    const float A = (1.0f - w1) * (kxx - kyy) + w1 * (exx - eyy) + (1.0f - 0.5f * w1) * (Qx - Qy);
    const float Bd = (1.0f - w1) * (kxx - kzz) + w1 * (exx - ezz) + (1.0f - 0.5f * w1) * (Qx - Qz);
    const float T = (1.0f - w2) * (kxx + kyy + kzz) + w2 * (exx + eyy + ezz) +
                    (1.0f - 0.5f * w2) * (Qx + Qy + Qz);
    const float third = 1.0f / 3.0f;
    S_(2, 0, 0) = (A + Bd + T) * third;
    S_(0, 2, 0) = (T - 2.0f * A + Bd) * third;
    S_(0, 0, 2) = (T + A - 2.0f * Bd) * third;
  }
  {
    // third order: sums with omega_3 (and the force), differences with omega_4
    const int pa[3] = {1 + 3 * 2, 2 + 3 * 1, 2 + 9 * 1};  // k120, k210, k201
    const int pb[3] = {1 + 9 * 2, 3 * 1 + 9 * 2, 3 * 2 + 9 * 1};  // k102, k012, k021
    const float Fd[3] = {in.Fx, in.Fy, in.Fz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float S3 = (1.0f - w3) * (k[pa[d]] + k[pb[d]]) + w3 * (e[pa[d]] + e[pb[d]]) +
                       2.0f * (1.0f - 0.5f * w3) * Fd[d] * kCs2;
      const float D3 = (1.0f - w4) * (k[pa[d]] - k[pb[d]]) + w4 * (e[pa[d]] - e[pb[d]]);
      ks[pa[d]] = 0.5f * (S3 + D3);
      ks[pb[d]] = 0.5f * (S3 - D3);
    }
  }
  S_(1, 1, 1) = (1.0f - w5) * K_(1, 1, 1) + w5 * E_(1, 1, 1);
  {
    const float a = K_(2, 2, 0), b = K_(2, 0, 2), c = K_(0, 2, 2);
    const float ea = E_(2, 2, 0), eb = E_(2, 0, 2), ec = E_(0, 2, 2);
    const float X = (1.0f - w6) * (a - 2.0f * b + c) + w6 * (ea - 2.0f * eb + ec);
    const float Y = (1.0f - w6) * (a + b - 2.0f * c) + w6 * (ea + eb - 2.0f * ec);
    const float Z = (1.0f - w7) * (a + b + c) + w7 * (ea + eb + ec);
    const float third = 1.0f / 3.0f;
    S_(2, 2, 0) = (X + Y + Z) * third;
    S_(2, 0, 2) = (Z - X) * third;
    S_(0, 2, 2) = (Z - Y) * third;
  }
  S_(2, 1, 1) = (1.0f - w8) * K_(2, 1, 1) + w8 * E_(2, 1, 1);
  S_(1, 2, 1) = (1.0f - w8) * K_(1, 2, 1) + w8 * E_(1, 2, 1);
  S_(1, 1, 2) = (1.0f - w8) * K_(1, 1, 2) + w8 * E_(1, 1, 2);
  S_(1, 2, 2) = (1.0f - w9) * K_(1, 2, 2) + w9 * E_(1, 2, 2) + (1.0f - 0.5f * w9) * in.Fx * kCs4;
  S_(2, 1, 2) = (1.0f - w9) * K_(2, 1, 2) + w9 * E_(2, 1, 2) + (1.0f - 0.5f * w9) * in.Fy * kCs4;
  S_(2, 2, 1) = (1.0f - w9) * K_(2, 2, 1) + w9 * E_(2, 2, 1) + (1.0f - 0.5f * w9) * in.Fz * kCs4;
  S_(2, 2, 2) = (1.0f - w10) * K_(2, 2, 2) + w10 * E_(2, 2, 2);
#undef K_
#undef E_
#undef S_
  emit_recoloured(B, ks, ux, uy, uz, div_refined(in.rr, rho, irho), div_refined(in.rb, rho, irho),
                  p, in.nx, in.ny, in.nz, emit);
}

// Pulled total distribution f_i(x) = sum over colours of stored_i(x - c_i),
// decoded from storage format S (the rest populations of the mass-exact
// formats come from their FP64 planes at x).
template <class S>
__device__ __forceinline__ void pull_total(const BoxDev &B, const void *src_, int64_t plane, int x,
                                           int y, int z, uint32_t node, float (&f)[27]) {
  const Pops<S> src(const_cast<void *>(src_), plane);
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int xs[3] = {wrap_once(x + 1, nx), x, wrap_once(x - 1, nx)};
  const int ys[3] = {wrap_once(y + 1, ny), y, wrap_once(y - 1, ny)};
  const int zs[3] = {wrap_once(z + 1, nz), z, wrap_once(z - 1, nz)};
  constexpr int i0 = S::kExact ? 1 : 0;
#pragma unroll
  for (int i = i0; i < kQ; ++i) {
    const uint32_t s = (uint32_t)B.base + (uint32_t)xs[kCX[i] + 1] +
                       (uint32_t)nx * ((uint32_t)ys[kCY[i] + 1] + (uint32_t)ny * (uint32_t)zs[kCZ[i] + 1]);
    typename S::T r, b;
    ld_rb(src, i, s, r, b);
    const float cs = S::kCShift ? S::dec(ld(&at(src.cfr, s))) : 0.f;
    f[i] = decode_pop<S>(B, 0, r, pop_shift<S>(B, 0, i, cs)) +
           decode_pop<S>(B, 1, b, pop_shift<S>(B, 1, i, cs));
  }
  if (S::kExact) f[0] = (float)(at(src.restp(0), node) + at(src.restp(1), node));
}

__device__ __forceinline__ NodeIn load_node_in(const float *__restrict__ aux, int64_t plane,
                                               uint32_t node) {
  // every value is read once: streaming loads
  NodeIn in;
  in.rr = ld(&at(PL(aux, A_RR), node));
  in.rb = ld(&at(PL(aux, A_RB), node));
  in.jx = ld(&at(PL(aux, A_JX), node));
  in.jy = ld(&at(PL(aux, A_JY), node));
  in.jz = ld(&at(PL(aux, A_JZ), node));
  in.pxx = ld(&at(PL(aux, A_PXX), node));
  in.pyy = ld(&at(PL(aux, A_PYY), node));
  in.pzz = ld(&at(PL(aux, A_PZZ), node));
  in.pxy = ld(&at(PL(aux, A_PXY), node));
  in.pxz = ld(&at(PL(aux, A_PXZ), node));
  in.pyz = ld(&at(PL(aux, A_PYZ), node));
  in.nx = ld(&at(PL(aux, A_NX), node));
  in.ny = ld(&at(PL(aux, A_NY), node));
  in.nz = ld(&at(PL(aux, A_NZ), node));
  in.Fx = ld(&at(PL(aux, A_FX), node));
  in.Fy = ld(&at(PL(aux, A_FY), node));
  in.Fz = ld(&at(PL(aux, A_FZ), node));
  in.Qx = ld(&at(PL(aux, A_QX), node));
  in.Qy = ld(&at(PL(aux, A_QY), node));
  in.Qz = ld(&at(PL(aux, A_QZ), node));
  return in;
}

// Writes one node's collided, recoloured populations in storage format S.
// Mass-exact formats skip the rest population during the emission and close
// it at the end from the node's FP64 colour densities.
template <class S>
struct PopWriter {
  const Pops<S> &dst;
  const BoxDev &B;
  bool live;
  uint32_t node;
  double sr = 0.0, sb = 0.0;
  typename S::T craw{};  // colour-fraction formats: the node's red fraction as stored
  float cr = 0.f;        // and its value
  __device__ PopWriter(const Pops<S> &d, const BoxDev &b, uint32_t n, bool l = true)
      : dst(d), B(b), live(l), node(n) {}
  // the node's colour densities (colour-fraction formats; before the emission)
  __device__ __forceinline__ void set_fraction(float rr, float rb) {
    if constexpr (S::kCShift) {
      craw = stored_fraction<S>(rr, rb);
      cr = S::dec(craw);
    }
  }
  __device__ __forceinline__ void operator()(int i, float fr, float fb) {
    if (S::kExact && i == 0) return;
    const float shr = pop_shift<S>(B, 0, i, cr), shb = pop_shift<S>(B, 1, i, cr);
    const typename S::T er = encode_pop<S>(B, 0, fr, shr), eb = encode_pop<S>(B, 1, fb, shb);
    using W = typename S::W;
    const int64_t pb = dst.plane * (int64_t)sizeof(W);
    if constexpr (S::kPaired) {
      buf_st(S::pack(er, eb), plane_rsrc(dst.pw, pb, Pops<S>::slot(i)), boff<W>(live, node));
    } else {
      buf_st(er, plane_rsrc(dst.pw, pb, Pops<S>::slot(i, 0)), boff<W>(live, node));
      buf_st(eb, plane_rsrc(dst.pw, pb, Pops<S>::slot(i, 1)), boff<W>(live, node));
    }
    if (S::kExact) {
      sr += (double)decode_pop<S>(B, 0, er, shr);
      sb += (double)decode_pop<S>(B, 1, eb, shb);
    }
  }
  __device__ __forceinline__ void finish(double rho_r, double rho_b) {
    if (S::kExact) {
      const int64_t pb = dst.plane * 8;
      const uint32_t off = boff<double>(live, node);
      buf_st(rho_r - sr, plane_rsrc(dst.rest, pb, 0), off);
      buf_st(rho_b - sb, plane_rsrc(dst.rest, pb, 1), off);
    }
    if constexpr (S::kCShift)
      buf_st((uint16_t)craw, plane_rsrc(dst.cfr, dst.plane * 2, 0), boff<uint16_t>(live, node));
  }
};

// COMPACT: store the compact post-collision state (17 float planes of dst,
// see compact_of) instead of the populations; unit higher rates only.
template <class S, bool COMPACT = false>
__global__ __launch_bounds__(kBlock) void k_collide(const BoxDev *__restrict__ boxes,
                                                    const int32_t *__restrict__ blk_box,
                                                    float *__restrict__ aux,
                                                    const void *__restrict__ src_,
                                                    void *__restrict__ dst_, int64_t plane) {
  const uint32_t lb = xcd_block();
  const int b = blk_box[lb];
  if (b < 0) return;
  const BoxDev B = boxes[b];
  const int64_t local = (int64_t)(lb - B.blk0) * kBlock + threadIdx.x;
  if (local >= B.n) return;
  const uint32_t l = (uint32_t)local;
  const uint32_t yz = fdiv(l, B.fdx);
  const int z = (int)fdiv(yz, B.fdy);
  const int y = (int)(yz - (uint32_t)z * (uint32_t)B.ny);
  if (is_solid(B, y, z)) return;
  const uint32_t node = (uint32_t)(B.base + local);
  const NodeIn in = load_node_in(aux, plane, node);
  if (COMPACT) {
    float c[kCompact];
    compact_of<true>(B, in, c);
#pragma unroll
    for (int k = 0; k < kCompact; ++k) buf_st(c[k], plane_rsrc(dst_, plane * 4, k), node * 4u);
    return;
  }
  const Pops<S> dst(dst_, plane);
  PopWriter<S> w(dst, B, node);
  w.set_fraction(in.rr, in.rb);
  if (B.full_rates) {
    // non-unit higher-order rates need every central moment: pull again
    float f[27];
    const int x = (int)(l - yz * (uint32_t)B.nx);
    pull_total<S>(B, src_, plane, x, y, z, node, f);
    collide_full(B, in, f, w);
  } else {
    collide_node<true>(B, in, w);
  }
  if (S::kExact) {
    const double *r64 = aux_rho64(aux, plane);
    w.finish(at(r64, node), at(r64 + plane, node));
  }
}

// ---------------------------------------------------------------------------
// k_wall_copy: the solid nodes' reversed populations, stashed by k_pull of an
// in-place layout, into the population buffer (after the pull has
// completed; no other kernel of the step touches solid nodes).  One thread
// per wall slot; blocks per box from wblk_box.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(kBlock) void k_wall_copy(const BoxDev *__restrict__ boxes,
                                                      const int32_t *__restrict__ wblk_box,
                                                      const void *__restrict__ stash_,
                                                      void *__restrict__ pop_, int64_t plane,
                                                      int64_t wplane) {
  const int b = wblk_box[blockIdx.x];
  if (b < 0) return;
  const BoxDev B = boxes[b];
  const int32_t local = (int32_t)(blockIdx.x - (uint32_t)B.wblk0) * kBlock + (int32_t)threadIdx.x;
  if (local >= B.wn) return;
  int x, y, z;
  wall_node(B, (uint32_t)local, x, y, z);
  const uint32_t node = (uint32_t)B.base + (uint32_t)x +
                        (uint32_t)B.nx * ((uint32_t)y + (uint32_t)B.ny * (uint32_t)z);
  const uint32_t slot = (uint32_t)(B.wbase + local);
  const Pops<S> src(const_cast<void *>(stash_), wplane), dst(pop_, plane);
  constexpr int i0 = S::kExact ? 1 : 0;
#pragma unroll
  for (int i = i0; i < kQ; ++i) {
    typename S::T r, bl;
    ld_rb(src, i, slot, r, bl);
    st_rb(dst, i, node, r, bl);
  }
  if (S::kExact) {
    at(dst.restp(0), node) = at(src.restp(0), slot);
    at(dst.restp(1), node) = at(src.restp(1), slot);
  }
  if constexpr (S::kCShift) at(dst.cfr, node) = at(src.cfr, slot);
}

// The compact schedule of the 16-bit formats: the solid nodes' populations
// from a decoded (mass-exact FP32) wall stash, encoded into the stored
// format (after k_emit, whose red fractions of the fluid nodes the
// colour-fraction formats read: a solid node takes that of its wall-normal
// fluid neighbour, as the pull does).
template <class S>
__global__ __launch_bounds__(kBlock) void k_wall_encode(const BoxDev *__restrict__ boxes,
                                                        const int32_t *__restrict__ wblk_box,
                                                        const void *__restrict__ stash_,
                                                        void *__restrict__ pop_, int64_t plane,
                                                        int64_t wplane) {
  const int b = wblk_box[blockIdx.x];
  if (b < 0) return;
  const BoxDev B = boxes[b];
  const int32_t local = (int32_t)(blockIdx.x - (uint32_t)B.wblk0) * kBlock + (int32_t)threadIdx.x;
  if (local >= B.wn) return;
  int x, y, z;
  wall_node(B, (uint32_t)local, x, y, z);
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const uint32_t node = (uint32_t)B.base + (uint32_t)x +
                        (uint32_t)nx * ((uint32_t)y + (uint32_t)ny * (uint32_t)z);
  const uint32_t slot = (uint32_t)(B.wbase + local);
  const Pops<StoreF32X> src(const_cast<void *>(stash_), wplane);
  const Pops<S> dst(pop_, plane);
  float cown = 0.f;
  if constexpr (S::kCShift) {
    const int dy = (B.walls & 1u) ? (y == 0 ? -1 : (y == ny - 1 ? 1 : 0)) : 0;
    const int dz = (B.walls & 2u) ? (z == 0 ? -1 : (z == nz - 1 ? 1 : 0)) : 0;
    const uint32_t nb = (uint32_t)B.base + (uint32_t)x +
                        (uint32_t)nx * ((uint32_t)(y - dy) + (uint32_t)ny * (uint32_t)(z - dz));
    const typename S::T craw = ld(&at(dst.cfr, nb));
    cown = S::dec(craw);
    at(dst.cfr, node) = craw;
  }
#pragma unroll
  for (int i = 1; i < kQ; ++i) {
    float fr, fb;
    ld_rb(src, i, slot, fr, fb);
    st_rb(dst, i, node, encode_pop<S>(B, 0, fr, pop_shift<S>(B, 0, i, cown)),
          encode_pop<S>(B, 1, fb, pop_shift<S>(B, 1, i, cown)));
  }
  at(dst.restp(0), node) = at(src.restp(0), slot);
  at(dst.restp(1), node) = at(src.restp(1), slot);
}

// ---------------------------------------------------------------------------
// Initial state: f^k = (rho_k/rho)(f^eq + eta) with the Model D equilibrium
// built from its central moments (Eqs. 57-63), written un-streamed so that the
// first pull reproduces f(x, 0): stored_i(x - c_i) = f_i(x).  Mass-exact
// formats close the rest population on the FP64 sum of the node's values.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(kBlock) void k_init(const BoxDev *__restrict__ boxes,
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
  const Pops<S> dst(dst_, plane);
  const uint32_t l = (uint32_t)local;
  const uint32_t yz = fdiv(l, B.fdx);
  const int x = (int)(l - yz * (uint32_t)B.nx);
  const int z = (int)fdiv(yz, B.fdy);
  const int y = (int)(yz - (uint32_t)z * (uint32_t)B.ny);
  const uint32_t node = (uint32_t)(B.base + local);
  const float rr = in_rr[node], rb = in_rb[node];
  const float ux = in_u[node], uy = in_u[plane + node], uz = in_u[2 * plane + node];
  const float rho = rr + rb;
  const float p = rr * B.cs2r + rb * B.cs2b;
  float k[27];
  model_moments(B.model, rho, p, ux, uy, uz, 0.f, 0.f, 0.f, p, p, p, 0.f, 0.f, 0.f, k);
  float f[kQ];
  central_to_populations(k, ux, uy, uz, f);
  const float cr = rr / rho, cb = rb / rho;
  double tr = 0.0, tb = 0.0, sr = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float ft = amp != 0.f ? f[i] + counter_noise(seed, (uint32_t)b, (uint64_t)local, i, amp)
                                : f[i];
    const float vr = cr * ft, vb = cb * ft;
    tr += (double)vr;
    tb += (double)vb;
    if (S::kExact && i == 0) continue;
    const int xd = wrap_once(x - kCX[i], B.nx), yd = wrap_once(y - kCY[i], B.ny),
              zd = wrap_once(z - kCZ[i], B.nz);
    const uint32_t d = (uint32_t)B.base + (uint32_t)xd +
                       (uint32_t)B.nx * ((uint32_t)yd + (uint32_t)B.ny * (uint32_t)zd);
    // colour-fraction formats: the value is read back with the red fraction
    // the node d stores (written below by d's own thread)
    const float cd = S::kCShift ? S::dec(stored_fraction<S>(in_rr[d], in_rb[d])) : 0.f;
    const float shr = pop_shift<S>(B, 0, i, cd), shb = pop_shift<S>(B, 1, i, cd);
    const typename S::T er = encode_pop<S>(B, 0, vr, shr), eb = encode_pop<S>(B, 1, vb, shb);
    st_rb(dst, i, d, er, eb);
    sr += (double)decode_pop<S>(B, 0, er, shr);
    sb += (double)decode_pop<S>(B, 1, eb, shb);
  }
  if (S::kExact) {
    at(dst.restp(0), node) = tr - sr;
    at(dst.restp(1), node) = tb - sb;
  }
  if constexpr (S::kCShift) at(dst.cfr, node) = stored_fraction<S>(rr, rb);
}

// ---------------------------------------------------------------------------
// k_fused: interface stencils and collision in one pass.  A block owns a
// TX x TY column of the box and marches along z over ZC output slabs.  Slab
// s of the phase field enters a 3-slot LDS ring; n and |grad phi| of slab
// s-1, and q = (p - rho c_s^2) u of slab s-2 follow in their own rings; the
// correction term and the collision of slab s-3 complete the iteration.
// Halo widths in x, y: 3 for phi, 2 for n, 1 for q.
// ---------------------------------------------------------------------------
template <int TX, int TY>
struct FusedGeom {
  static constexpr int NT = TX * TY;
  static constexpr int R3X = TX + 6, R3Y = TY + 6, R3 = R3X * R3Y;
  static constexpr int R2X = TX + 4, R2Y = TY + 4, R2 = R2X * R2Y;
  static constexpr int R1X = TX + 2, R1Y = TY + 2, R1 = R1X * R1Y;
  static constexpr int A_PER = (R3 + NT - 1) / NT;
};

// COMPACT: store each node's compact post-collision state (17 float planes
// of dst, see compact_of) instead of its populations.
template <int TX, int TY, int ZC, int MINW, bool WALLS, class S, bool EXPORT, bool COMPACT = false>
__global__ __launch_bounds__(TX *TY, MINW) void k_fused(const BoxDev *__restrict__ boxes,
                                                  const TileEntry *__restrict__ tiles,
                                                  float *__restrict__ aux,
                                                  void *__restrict__ dst_, int64_t plane_arg) {
  using G = FusedGeom<TX, TY>;
  __shared__ float s_phi[3][G::R3];
  __shared__ float s_n[3][4][G::R2];
  __shared__ float s_q[3][3][G::R1];
  __shared__ uint8_t s_sy[G::R3Y];

  const int tid = threadIdx.x;
  const uint32_t lb = xcd_block();
  const TileEntry te = tiles[lb];
  if (te.box < 0) return;
  const int b = te.box;
  const BoxDev B = boxes[b];
  const uint32_t cyu = fdiv((uint32_t)te.xy, B.fcx);
  const int cx = (int)((uint32_t)te.xy - cyu * (uint32_t)B.ncx);
  const int cy = (int)cyu;
  const int x0 = cx * TX, y0 = cy * TY, z0 = te.z0;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int z1 = te.z1;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const bool zwalls = WALLS && (B.walls & 2u) != 0;

  for (int i = tid; i < G::R3Y; i += G::NT) {
    const int gy = wrap_any(y0 + i - 3, ny);
    s_sy[i] = WALLS && (B.walls & 1u) && (gy == 0 || gy == ny - 1);
  }
  // solid flag of an R3 row (always false without walls)
  auto sy = [&](int r) -> bool { return WALLS ? (bool)s_sy[r] : false; };
  // xy offsets of this thread's phase-field points (fixed over the march)
  int a_off[G::A_PER];
#pragma unroll
  for (int k = 0; k < G::A_PER; ++k) {
    const int i = tid + k * G::NT;
    a_off[k] = 0;
    if (i < G::R3) {
      const int lx = i % G::R3X, ly = i / G::R3X;
      a_off[k] = wrap_any(x0 + lx - 3, nx) + nx * wrap_any(y0 + ly - 3, ny);
    }
  }
  // R1 points of this thread: the tile point first, then the halo ring
  // (top and bottom rows, then the two side columns)
  auto r1_point = [&](int j, int &lx, int &ly) {
    if (j < G::NT) {
      lx = (j % TX) + 1;
      ly = (j / TX) + 1;
    } else {
      const int h = j - G::NT;
      if (h < 2 * G::R1X) {
        lx = h % G::R1X;
        ly = (h / G::R1X) * (G::R1Y - 1);
      } else {
        const int h2 = h - 2 * G::R1X;
        lx = (h2 & 1) * (G::R1X - 1);
        ly = (h2 >> 1) + 1;
      }
    }
  };
  constexpr int C_PER = (G::R1 + G::NT - 1) / G::NT;
  uint32_t c_off[C_PER];
#pragma unroll
  for (int kk = 0; kk < C_PER; ++kk) {
    const int j = tid + kk * G::NT;
    c_off[kk] = 0;
    if (j < G::R1) {
      int lx, ly;
      r1_point(j, lx, ly);
      c_off[kk] = (uint32_t)wrap_any(x0 + lx - 1, nx) + (uint32_t)nx * (uint32_t)wrap_any(y0 + ly - 1, ny);
    }
  }
  // tile point of this thread
  const int ox = tid % TX, oy = tid / TX;
  const int gxo = x0 + ox, gyo = y0 + oy;
  const bool in_xy = gxo < nx && gyo < ny;
  // the tile point clamped into the box: lanes outside it load valid
  // addresses and store nowhere
  const uint32_t oxy = (uint32_t)min(gxo, nx - 1) + (uint32_t)nx * (uint32_t)min(gyo, ny - 1);
  const bool solid_y_o = (B.walls & 1u) && (gyo == 0 || gyo == ny - 1);
  // interface values of the tile point, one slab behind the q ring
  float h_nx = 0.f, h_ny = 0.f, h_nz = 0.f, h_Fx = 0.f, h_Fy = 0.f, h_Fz = 0.f, h_k = 0.f;
  auto slab_solid = [&](int s) {
    if (!zwalls) return false;
    const int gz = wrap_any(s, nz);
    return gz == 0 || gz == nz - 1;
  };
  // Every vector memory access of the march is issued on every lane and in
  // every iteration (lanes and slabs without work use clamped addresses or
  // discarded stores), and the loads of stages A and C run one iteration
  // ahead, before the stores of the collision.  The waits for them then
  // never include those stores, which share the in-order vector memory
  // counter with the loads.
  // (except the loads of a wavefront's later points when none of its lanes
  // has one, e.g. the second R1 point in five of the eight wavefronts of a
  // 64x8 column: their values are set to zero instead)
  float a_rr[G::A_PER], a_rb[G::A_PER];
  float pc_[C_PER][5];
  const int wave0 = (int)__builtin_amdgcn_readfirstlane(tid);
  auto load_a = [&](int sl, int64_t pl) {
    const uint32_t zoff = (uint32_t)B.base + nxy * (uint32_t)wrap_any(sl, nz);
#pragma unroll
    for (int k = 0; k < G::A_PER; ++k) {
      if (k > 0 && wave0 + k * G::NT >= G::R3) {
        a_rr[k] = a_rb[k] = 0.f;
        continue;
      }
      const uint32_t node = zoff + (uint32_t)a_off[k];
      a_rr[k] = ldpl(aux, pl, A_RR, node);
      a_rb[k] = ldpl(aux, pl, A_RB, node);
    }
  };
  auto load_c = [&](int sl, int64_t pl) {
    const uint32_t zoff = (uint32_t)B.base + nxy * (uint32_t)wrap_any(sl, nz);
#pragma unroll
    for (int kk = 0; kk < C_PER; ++kk) {
      if (kk > 0 && wave0 + kk * G::NT >= G::R1) {
#pragma unroll
        for (int m = 0; m < 5; ++m) pc_[kk][m] = 0.f;
        continue;
      }
      const uint32_t node = zoff + c_off[kk];
      pc_[kk][0] = ldpl(aux, pl, A_RR, node);
      pc_[kk][1] = ldpl(aux, pl, A_RB, node);
      pc_[kk][2] = ldpl(aux, pl, A_JX, node);
      pc_[kk][3] = ldpl(aux, pl, A_JY, node);
      pc_[kk][4] = ldpl(aux, pl, A_JZ, node);
    }
  };
  // inputs of the collision at the (clamped) tile point.  With 16-bit
  // storage they are loaded one iteration ahead, inside the collision before
  // its first store (measured faster); with 32-bit storage at the top of the
  // iteration (the earlier issue measured slower there).
  constexpr bool kPipeD = sizeof(typename S::T) == 2;
  NodeIn din;
  double d_rr = 0.0, d_rb = 0.0;
  auto load_d = [&](int sl, int64_t pl) {
    if (EXPORT) return;
    const uint32_t node = (uint32_t)B.base + oxy + nxy * (uint32_t)wrap_any(sl, nz);
    // the second moments and FP64 densities are read by stage D only
    if (S::kExact) {
      const double *r64 = aux_rho64(aux, pl);
      d_rr = buf_ld_f64_nt(plane_rsrc(r64, pl * 8, 0), node * 8u);
      d_rb = buf_ld_f64_nt(plane_rsrc(r64, pl * 8, 1), node * 8u);
    }
    din.rr = ldpl(aux, pl, A_RR, node);
    din.rb = ldpl(aux, pl, A_RB, node);
    din.jx = ldpl(aux, pl, A_JX, node);
    din.jy = ldpl(aux, pl, A_JY, node);
    din.jz = ldpl(aux, pl, A_JZ, node);
    din.pxx = ldpl_nt(aux, pl, A_PXX, node);
    din.pyy = ldpl_nt(aux, pl, A_PYY, node);
    din.pzz = ldpl_nt(aux, pl, A_PZZ, node);
    din.pxy = ldpl_nt(aux, pl, A_PXY, node);
    din.pxz = ldpl_nt(aux, pl, A_PXZ, node);
    din.pyz = ldpl_nt(aux, pl, A_PYZ, node);
  };
  load_a(z0 - 3, plane_arg);
  load_c(z0 - 5, plane_arg);
  if (kPipeD) load_d(z0 - 6, plane_arg);
  // as many stores as stage D issues, all discarded: on entry to the march
  // the loads above are then followed by the same count of memory
  // instructions as in every later iteration, so the waits for them are
  // the same on both paths into the loop
  if (!EXPORT && COMPACT) {
#pragma unroll
    for (int k = 0; k < kCompact; ++k)
      buf_st(0.f, plane_rsrc(dst_, plane_arg * 4, k), kDrop);
    if (S::kExact) {
      double *r64 = compact_rho64(dst_, plane_arg);
      buf_st(0.0, plane_rsrc(r64, plane_arg * 8, 0), kDrop);
      buf_st(0.0, plane_rsrc(r64, plane_arg * 8, 1), kDrop);
    }
  } else if (!EXPORT) {
    const Pops<S> dst(dst_, plane_arg);
    PopWriter<S> w(dst, B, 0u, false);
#pragma unroll
    for (int i = 0; i < kQ; ++i) w(i, 0.f, 0.f);
    w.finish(0.0, 0.0);
  } else {
#pragma unroll
    for (int k = 0; k < 10; ++k) buf_st(0.f, plane_rsrc(aux, plane_arg * 4, A_NX + k), kDrop);
  }
  __syncthreads();

  for (int s = z0 - 3; s < z1 + 3; ++s) {
    const int64_t plane = opaque_i64(plane_arg);
    if (!kPipeD) load_d(s - 3, plane);
    // inputs of the collision of slab s-3 at the (clamped) tile point
    // ---- A: phase field of slab s (Eq. 14) ----
    {
      float *ph = s_phi[(s + 3) % 3];
#pragma unroll
      for (int k = 0; k < G::A_PER; ++k) {
        const int i = tid + k * G::NT;
        if (i < G::R3) {
          const float rr = a_rr[k] * B.ir0r;
          const float rb = a_rb[k] * B.ir0b;
          ph[i] = phase_field(rr, rb);
        }
      }
    }
    __syncthreads();
    // ---- B: grad phi and n of slab s-1 (Eqs. 17, 20) ----
    if (s - 1 >= z0 - 2) {
      const int sb = s - 1;
      const bool sz_m = slab_solid(sb - 1), sz_c = slab_solid(sb), sz_p = slab_solid(sb + 1);
      const float *pm = s_phi[(sb - 1 + 3) % 3];
      const float *pc = s_phi[(sb + 3) % 3];
      const float *pp = s_phi[(sb + 1 + 3) % 3];
      float(*nn)[G::R2] = s_n[(sb + 3) % 3];
      for (int i = tid; i < G::R2; i += G::NT) {
        const int lx = i % G::R2X, ly = i / G::R2X;
        const int c3 = (lx + 1) + G::R3X * (ly + 1);
        float nxv = 0.f, nyv = 0.f, nzv = 0.f, mag = 0.f;
        if (!(sy(ly + 1) | sz_c)) {
          const float vc = pc[c3];
          float v[3][3][3];
#pragma unroll
          for (int dz = -1; dz <= 1; ++dz) {
            const float *pl = dz < 0 ? pm : (dz > 0 ? pp : pc);
            const bool szd = dz < 0 ? sz_m : (dz > 0 ? sz_p : sz_c);
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
              const bool sd = szd | sy(ly + 1 + dy);
#pragma unroll
              for (int dx = -1; dx <= 1; ++dx)
                v[dz + 1][dy + 1][dx + 1] = wall_rule(sd, vc, pl[c3 + dx + G::R3X * dy]);
            }
          }
          float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
            for (int b2 = 0; b2 < 3; ++b2) {
              const float w = 0.5f * w1d(a2 - 1) * w1d(b2 - 1);
              gx = fmaf(w, v[b2][a2][2] - v[b2][a2][0], gx);
              gy = fmaf(w, v[b2][2][a2] - v[b2][0][a2], gy);
              gz = fmaf(w, v[2][b2][a2] - v[0][b2][a2], gz);
            }
          const float g2 = gx * gx + gy * gy + gz * gz;
          if (g2 > 1e-24f) {  // |grad phi| > 1e-12
            const float inv = rsq(g2);
            mag = g2 * inv;
            nxv = gx * inv;
            nyv = gy * inv;
            nzv = gz * inv;
          }
        }
        nn[0][i] = nxv;
        nn[1][i] = nyv;
        nn[2][i] = nzv;
        nn[3][i] = mag;
      }
    }
    __syncthreads();
    // ---- C: grad n, kappa, F, u, q of slab s-2 (Eqs. 11, 15, 16, 65) ----
    float f_nx = 0.f, f_ny = 0.f, f_nz = 0.f, f_Fx = 0.f, f_Fy = 0.f, f_Fz = 0.f, f_k = 0.f;
    if (s - 2 >= z0 - 1) {
      const int sc = s - 2;
      const bool sz_m = slab_solid(sc - 1), sz_c = slab_solid(sc), sz_p = slab_solid(sc + 1);
      float(*nm)[G::R2] = s_n[(sc - 1 + 3) % 3];
      float(*nc)[G::R2] = s_n[(sc + 3) % 3];
      float(*np)[G::R2] = s_n[(sc + 1 + 3) % 3];
      float(*qq)[G::R1] = s_q[(sc + 3) % 3];
      // first pass: the tile points in thread order, then the halo ring
#pragma unroll
      for (int kk = 0; kk < C_PER; ++kk) {
        const int j = tid + kk * G::NT;
        if (j >= G::R1) break;
        int lx, ly;
        r1_point(j, lx, ly);
        const int c2 = (lx + 1) + G::R2X * (ly + 1);
        const int ri = lx + G::R1X * ly;
        float qx = 0.f, qy = 0.f, qz = 0.f;
        float kap = 0.f, Fx = 0.f, Fy = 0.f, Fz = 0.f;
        const float nxv = nc[0][c2], nyv = nc[1][c2], nzv = nc[2][c2], mag = nc[3][c2];
        if (!(sy(ly + 2) | sz_c)) {
          float d[3][3];  // d[a][b] = d n_a / d x_b
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float vc = nc[a][c2];
            float v[3][3][3];
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
              const float *pl = dz < 0 ? nm[a] : (dz > 0 ? np[a] : nc[a]);
              const bool szd = dz < 0 ? sz_m : (dz > 0 ? sz_p : sz_c);
#pragma unroll
              for (int dy = -1; dy <= 1; ++dy) {
                const bool sd = szd | sy(ly + 2 + dy);
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                  v[dz + 1][dy + 1][dx + 1] = wall_rule(sd, vc, pl[c2 + dx + G::R2X * dy]);
              }
            }
            float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
            for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
              for (int b2 = 0; b2 < 3; ++b2) {
                const float w = 0.5f * w1d(a2 - 1) * w1d(b2 - 1);
                gx = fmaf(w, v[b2][a2][2] - v[b2][a2][0], gx);
                gy = fmaf(w, v[b2][2][a2] - v[b2][0][a2], gy);
                gz = fmaf(w, v[2][b2][a2] - v[0][b2][a2], gz);
              }
            d[a][0] = gx;
            d[a][1] = gy;
            d[a][2] = gz;
          }
          const float div = d[0][0] + d[1][1] + d[2][2];
          const float proj = nxv * (nxv * d[0][0] + nyv * d[0][1] + nzv * d[0][2]) +
                             nyv * (nxv * d[1][0] + nyv * d[1][1] + nzv * d[1][2]) +
                             nzv * (nxv * d[2][0] + nyv * d[2][1] + nzv * d[2][2]);
          kap = proj - div;
          const float rr = pc_[kk][0];
          const float rb = pc_[kk][1];
          const float rho = rr + rb;
          interface_force(B, kap, mag, nxv, nyv, nzv, rho, Fx, Fy, Fz);
          const float irho = rcp(rho);
          const float ux = fmaf(0.5f, Fx, pc_[kk][2]) * irho;
          const float uy = fmaf(0.5f, Fy, pc_[kk][3]) * irho;
          const float uz = fmaf(0.5f, Fz, pc_[kk][4]) * irho;
          const float dev = rr * B.cs2r + rb * B.cs2b - rho * kCs2;
          qx = dev * ux;
          qy = dev * uy;
          qz = dev * uz;
        }
        qq[0][ri] = qx;
        qq[1][ri] = qy;
        qq[2][ri] = qz;
        if (j < G::NT) {
          f_nx = nxv;
          f_ny = nyv;
          f_nz = nzv;
          f_Fx = Fx;
          f_Fy = Fy;
          f_Fz = Fz;
          f_k = kap;
        }
      }
    }
    __syncthreads();
    // loads of the next iteration, ahead of the stores below
    load_a(s + 1, plane);
    load_c(s - 1, plane);
    // ---- D: Q and the collision of slab s-3 (Eqs. 18-19, 25, 65-67) ----
    // Runs on every lane and in every iteration; only lanes of a fluid node
    // of the box in an output slab store.  The ring index keeps the slot
    // non-negative for the slabs before the first output slab.
    {
      const int sd = s - 3;
      const bool sz_m = slab_solid(sd - 1), sz_p = slab_solid(sd + 1);
      const bool fluid = in_xy && !(solid_y_o || slab_solid(sd));
      float(*qm)[G::R1] = s_q[(sd + 8) % 3];
      float(*qc)[G::R1] = s_q[(sd + 9) % 3];
      float(*qp)[G::R1] = s_q[(sd + 10) % 3];
      const int c1 = (ox + 1) + G::R1X * (oy + 1);
      // d q_x / dx: pairs along x over (dy, dz); likewise y and z
      float Qx = 0.f, Qy = 0.f, Qz = 0.f;
#pragma unroll
      for (int a2 = -1; a2 <= 1; ++a2)
#pragma unroll
        for (int b2 = -1; b2 <= 1; ++b2) {
          const float w = 0.5f * w1d(a2) * w1d(b2);
          {  // x: a2 = dy, b2 = dz
            const float *pl = b2 < 0 ? qm[0] : (b2 > 0 ? qp[0] : qc[0]);
            const bool sdd = (b2 < 0 ? sz_m : (b2 > 0 ? sz_p : false)) | sy(oy + 3 + a2);
            const float vc = qc[0][c1];
            const float vp = wall_rule(sdd, vc, pl[c1 + 1 + G::R1X * a2]);
            const float vm = wall_rule(sdd, vc, pl[c1 - 1 + G::R1X * a2]);
            Qx = fmaf(w, vp - vm, Qx);
          }
          {  // y: a2 = dx, b2 = dz
            const float *pl = b2 < 0 ? qm[1] : (b2 > 0 ? qp[1] : qc[1]);
            const bool szd = b2 < 0 ? sz_m : (b2 > 0 ? sz_p : false);
            const float vc = qc[1][c1];
            const float vp = wall_rule(szd | sy(oy + 4), vc, pl[c1 + a2 + G::R1X]);
            const float vm = wall_rule(szd | sy(oy + 2), vc, pl[c1 + a2 - G::R1X]);
            Qy = fmaf(w, vp - vm, Qy);
          }
          {  // z: a2 = dx, b2 = dy
            const bool syd = sy(oy + 3 + b2);
            const float vc = qc[2][c1];
            const float vp = wall_rule(sz_p | syd, vc, qp[2][c1 + a2 + G::R1X * b2]);
            const float vm = wall_rule(sz_m | syd, vc, qm[2][c1 + a2 + G::R1X * b2]);
            Qz = fmaf(w, vp - vm, Qz);
          }
        }
      Qx *= -3.0f;
      Qy *= -3.0f;
      Qz *= -3.0f;
      const uint32_t node = (uint32_t)B.base + oxy + nxy * (uint32_t)wrap_any(sd, nz);
      if (!EXPORT) {
        NodeIn in = din;
        in.nx = h_nx;
        in.ny = h_ny;
        in.nz = h_nz;
        in.Fx = h_Fx;
        in.Fy = h_Fy;
        in.Fz = h_Fz;
        in.Qx = Qx;
        in.Qy = Qy;
        in.Qz = Qz;
        if (COMPACT) {
          float c[kCompact];
          compact_of(B, in, c);
          const uint32_t off = boff<float>(fluid && sd >= z0, node);
#pragma unroll
          for (int k = 0; k < kCompact; ++k) buf_st(c[k], plane_rsrc(dst_, plane * 4, k), off);
          if (S::kExact) {
            // mass-exact storage: the FP64 colour densities travel with it
            double *r64 = compact_rho64(dst_, plane);
            const uint32_t off64 = boff<double>(fluid && sd >= z0, node);
            buf_st(d_rr, plane_rsrc(r64, plane * 8, 0), off64);
            buf_st(d_rb, plane_rsrc(r64, plane * 8, 1), off64);
          }
        } else {
          const double fr = d_rr, fb = d_rb;
          const Pops<S> dst(dst_, plane);
          PopWriter<S> w(dst, B, node, fluid && sd >= z0);
          w.set_fraction(in.rr, in.rb);
          collide_node(B, in, w, [&] {
            if (kPipeD) load_d(s - 2, plane);
          });
          w.finish(fr, fb);
        }
      } else {
        // interface fields of every node of the box (zero at solid nodes)
        const uint32_t off = boff<float>(in_xy && sd >= z0, node);
        const float v[10] = {h_nx, h_ny, h_nz, h_Fx, h_Fy, h_Fz, Qx, Qy, Qz, h_k};
#pragma unroll
        for (int k = 0; k < 10; ++k)
          buf_st(fluid ? v[k] : 0.f, plane_rsrc(aux, plane * 4, A_NX + k), off);
      }
    }
    // the interface values of slab s-2 become those of the next collision
    h_nx = f_nx;
    h_ny = f_ny;
    h_nz = f_nz;
    h_Fx = f_Fx;
    h_Fy = f_Fy;
    h_Fz = f_Fz;
    h_k = f_k;
  }
}

// ---------------------------------------------------------------------------
// k_cpull: the pull of the compact schedule.  The stored state is the
// compact post-collision state of every node (k_fused<..., COMPACT>); the
// moments of a node after streaming (Eq. 5) are sums of its neighbours'
// collided populations, f_i(x) = f*_i(x - c_i).  A block owns a TX x TY
// column and marches along z: for slab s it rebuilds the collided
// populations of the column and its one-node ring in registers (z and y
// passes of the back-transform), then, for each z component cz of the
// velocities in turn, finishes the x pass of those 9 directions, hands them
// through LDS, and every column node adds the 9 values arriving from its
// neighbours to the moments of slab s + cz.  Slab s - 1 is then complete
// (it received cz = +1 from s - 2, cz = 0 from s - 1 and cz = -1 from s, in
// that order) and its 11 moments go to aux.  Each thread rebuilds its own
// column node first (ring point k = 0), then one of the ring's halo points.
// WALLS: solid nodes keep populations (full-way bounce-back): a solid ring
// point emits what its slot of the wall stash wst_in holds (in storage
// format S), and what arrives at a solid column node is stored reversed in
// wst_out for the next step; its moments are zero.
// Mass-exact storage (S::kExact): the compact state carries each node's
// colour densities in FP64; a node's rest population is closed on them as
// rho_k minus the FP64 sum of the 26 moving values it emits (which its own
// thread computes as ring point k = 0), and the new colour densities are FP64
// sums of the arrivals and that rest, so each colour's mass is conserved to
// FP64 rounding; they go to the FP64 aux planes as well.
// ---------------------------------------------------------------------------
template <int TX, int TY>
struct CPullGeom {
  static constexpr int NT = TX * TY;
  static constexpr int R1X = TX + 2, R1Y = TY + 2, R1 = R1X * R1Y;
  static constexpr int CP = (R1 + NT - 1) / NT;  // ring points per thread
  // the halo fills whole wavefronts: those of the rows first, then one or
  // more of the columns
  static_assert(CP == 2 && NT % 64 == 0 && (2 * TX) % 64 == 0, "ring layout");
  // ring point j of the block: the column's own points first (thread j's
  // column node), then the halo: the rows below and above the tile (without
  // the corners), then the columns beside it (corners included); (lx, ly) in
  // the (TX + 2) x (TY + 2) ring
  __device__ static void point(int j, int &lx, int &ly) {
    if (j < NT) {
      lx = (j % TX) + 1;
      ly = (j / TX) + 1;
    } else {
      const int h = j - NT;
      if (h < 2 * TX) {
        lx = h % TX + 1;
        ly = (h / TX) * (R1Y - 1);
      } else {
        const int h2 = h - 2 * TX;
        lx = (h2 & 1) * (R1X - 1);
        ly = h2 >> 1;
      }
    }
  }
};

template <int TX, int TY, int ZC, bool WALLS = false, class S = StoreF32, bool GENERAL = false>
__global__ __launch_bounds__(TX *TY) void k_cpull(const BoxDev *__restrict__ boxes,
                                                  const TileEntry *__restrict__ tiles,
                                                  const float *__restrict__ cst,
                                                  float *__restrict__ aux, int64_t plane_arg,
                                                  const void *__restrict__ wst_in,
                                                  void *__restrict__ wst_out, int64_t wplane) {
  using G = CPullGeom<TX, TY>;
  constexpr bool EXACT = S::kExact;
  __shared__ float xb[18][G::R1];  // one z component: 9 directions x 2 colours
  const int tid = threadIdx.x;
  const uint32_t lb = xcd_block();
  const TileEntry te = tiles[lb];
  if (te.box < 0) return;
  const int b = te.box;
  const BoxDev B = boxes[b];
  const uint32_t cyu = fdiv((uint32_t)te.xy, B.fccx);
  const int cxi = (int)((uint32_t)te.xy - cyu * (uint32_t)B.cncx);
  const int cyi = (int)cyu;
  const int x0 = cxi * TX, y0 = cyi * TY, z0 = te.z0;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int z1 = te.z1;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  // ring points of this thread (its own column node first, then a halo
  // point or none) and their LDS slots (row-major in the ring); wavefronts
  // with no halo point skip the second pass, and the lanes past the ring in
  // the last halo wavefront read point 0 and write nothing
  uint32_t roff[G::CP];
  int rgx[G::CP], rgy[G::CP], rls[G::CP];
  // a halo point's one c_y row (above or below the tile) or c_x column
  // (beside it) that reaches the tile: c = +1 (true) or -1
  bool rfwd = false;
  // a wavefront of halo points holds rows only or columns only; the
  // wavefronts past the halo have no second point
  const int wave0 = (int)__builtin_amdgcn_readfirstlane(tid);
  const bool rowwave = wave0 < 2 * TX, halowave = wave0 + G::NT < G::R1;
#pragma unroll
  for (int k = 0; k < G::CP; ++k) {
    const int j = tid + k * G::NT;
    roff[k] = 0;
    rgx[k] = rgy[k] = rls[k] = 0;
    if (j < G::R1) {
      int lx, ly;
      G::point(j, lx, ly);
      if (k > 0) rfwd = rowwave ? ly == 0 : lx == 0;
      rls[k] = lx + G::R1X * ly;
      rgx[k] = wrap_any(x0 + lx - 1, nx);
      rgy[k] = wrap_any(y0 + ly - 1, ny);
      roff[k] = (uint32_t)rgx[k] + (uint32_t)nx * (uint32_t)rgy[k];
    }
  }
  const int ox = tid % TX, oy = tid / TX;
  const bool in_xy = x0 + ox < nx && y0 + oy < ny;
  const int gxo = min(x0 + ox, nx - 1), gyo = min(y0 + oy, ny - 1);
  const uint32_t oxy = (uint32_t)min(x0 + ox, nx - 1) + (uint32_t)nx * (uint32_t)min(y0 + oy, ny - 1);
  // moments of slabs s-1, s, s+1 at the column node
  float acc[3][11];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int m = 0; m < 11; ++m) acc[a][m] = 0.f;
  double acc64[3][2];  // mass-exact storage: the colour densities in FP64
#pragma unroll
  for (int a = 0; a < 3; ++a) acc64[a][0] = acc64[a][1] = 0.0;

  for (int s = z0 - 1; s <= z1; ++s) {
    const int64_t plane = opaque_i64(plane_arg);
    // the wall stashes (one descriptor each, rebuilt per slab from an
    // opaque plane length so that nothing of them is hoisted)
    const int64_t wpl = WALLS ? opaque_i64(wplane) : wplane;
    const StashBuf<S> win(wst_in, wpl), wout(wst_out, wpl);
    const int gz = wrap_any(s, nz);
    const uint32_t zoff = (uint32_t)B.base + nxy * (uint32_t)gz;
    bool rsolid[G::CP];
#pragma unroll
    for (int k = 0; k < G::CP; ++k)
      rsolid[k] = WALLS && tid + k * G::NT < G::R1 && is_solid(B, rgy[k], gz);
    // the column node's FP64 colour densities at slab s (its ring point k = 0)
    double own_r = 0.0, own_b = 0.0;
    if constexpr (EXACT) {
      const double *r64 = compact_rho64(const_cast<float *>(cst), plane);
      own_r = buf_ld_f64(plane_rsrc(r64, plane * 8, 0), (zoff + oxy) * 8u);
      own_b = buf_ld_f64(plane_rsrc(r64, plane * 8, 1), (zoff + oxy) * 8u);
    }
    float h[G::CP][3][3][3];
    float pux[G::CP], pcr[G::CP], pcb[G::CP], pRx[G::CP], pRy[G::CP], pRz[G::CP];
#pragma unroll
    for (int k = 0; k < G::CP; ++k) {
      if (k > 0 && !halowave) {
        // (defined values here keep the register use of the others down)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int cy = 0; cy < 3; ++cy)
#pragma unroll
            for (int cz = 0; cz < 3; ++cz) h[k][a][cy][cz] = 0.f;
        pux[k] = pcr[k] = pcb[k] = pRx[k] = pRy[k] = pRz[k] = 0.f;
        continue;
      }
      float c[kCompact];
#pragma unroll
      for (int m = 0; m < kCompact; ++m) c[m] = ldpl(cst, plane, m, zoff + roff[k]);
      CompactPost o;
      compact_post<GENERAL>(B, c, o);
      float g[3][3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
          cm_to_pop_1d(o.k[a + 3 * bb], o.k[a + 3 * bb + 9], o.k[a + 3 * bb + 18], o.uz,
                       g[a][bb][0], g[a][bb][1], g[a][bb][2]);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int cz = 0; cz < 3; ++cz)
          cm_to_pop_1d(g[a][0][cz], g[a][1][cz], g[a][2][cz], o.uy, h[k][a][0][cz],
                       h[k][a][1][cz], h[k][a][2][cz]);
      pux[k] = o.ux;
      pcr[k] = o.cr;
      pcb[k] = o.cb;
      pRx[k] = o.Rx;
      pRy[k] = o.Ry;
      pRz[k] = o.Rz;
    }
    // mass-exact storage: FP64 sums of the moving values the column node emits
    double emit_r = 0.0, emit_b = 0.0;
#pragma unroll
    for (int pz = 0; pz < 3; ++pz) {
      // the x pass and the recolouring (Eqs. 18-19) of the directions with
      // z component pz - 1, as emit_recoloured computes them
#pragma unroll
      for (int k = 0; k < G::CP; ++k) {
        const int j = tid + k * G::NT;
        if ((k == 0 || halowave) && j < G::R1) {
          // a solid ring point: what the bounce-back stored for these
          // directions, loaded before the emission so that the loads'
          // latency passes behind it
          typename S::T stv[9][2];
          if (WALLS && rsolid[k]) {
            const uint32_t wslot = (uint32_t)B.wbase + wall_slot(B, rgx[k], rgy[k], gz);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
              const int i = dir_of(q % 3 - 1, q / 3 - 1, pz - 1);
              if (EXACT && i == 0) {
                stv[q][0] = stv[q][1] = S::enc(0.f);
              } else {
                win.ld(i, wslot, stv[q][0], stv[q][1]);
              }
            }
          }
          const int slot = rls[k];
          if (k == 0) {
            // the column node: all nine directions
#pragma unroll
            for (int cy = 0; cy < 3; ++cy) {
              // (the plain maps here: the doubled ones of emit_recoloured
              // give the same bits but cost this kernel 8 VGPRs and an
              // occupancy step)
              float fx[3];
              cm_to_pop_1d(h[k][0][cy][pz], h[k][1][cy][pz], h[k][2][cy][pz], pux[k], fx[0], fx[1],
                           fx[2]);
#pragma unroll
              for (int cx = 0; cx < 3; ++cx) {
                const int i = dir_of(cx - 1, cy - 1, pz - 1);
                const float cR = (kCX[i] ? (kCX[i] > 0 ? pRx[k] : -pRx[k]) : 0.f) +
                                 (kCY[i] ? (kCY[i] > 0 ? pRy[k] : -pRy[k]) : 0.f) +
                                 (kCZ[i] ? (kCZ[i] > 0 ? pRz[k] : -pRz[k]) : 0.f);
                const float d = 3.0f * weight(i) * cR;
                const int q = 3 * cy + cx;
                const float vr = fmaf(pcr[k], fx[cx], d), vb = fmaf(pcb[k], fx[cx], -d);
                if (EXACT && i != 0) {
                  emit_r += (double)vr;
                  emit_b += (double)vb;
                }
                xb[2 * q][slot] = vr;
                xb[2 * q + 1][slot] = vb;
              }
            }
          } else if (rowwave) {
            // a halo point below (c_y = +1) or above (c_y = -1) the tile:
            // the three directions of that row, the same values as above
            const bool fw = rfwd;
            float fx[3];
            cm_to_pop_1d(fw ? h[k][0][2][pz] : h[k][0][0][pz], fw ? h[k][1][2][pz] : h[k][1][0][pz],
                         fw ? h[k][2][2][pz] : h[k][2][0][pz], pux[k], fx[0], fx[1], fx[2]);
            const float yR = fw ? pRy[k] : -pRy[k];
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) {
              const int i = dir_of(cx - 1, 1, pz - 1);  // |c|, c_x, c_z as in either row
              const float cR = (kCX[i] ? (kCX[i] > 0 ? pRx[k] : -pRx[k]) : 0.f) + yR +
                               (kCZ[i] ? (kCZ[i] > 0 ? pRz[k] : -pRz[k]) : 0.f);
              const float d = 3.0f * weight(i) * cR;
              const int q = (fw ? 6 : 0) + cx;
              xb[2 * q][slot] = fmaf(pcr[k], fx[cx], d);
              xb[2 * q + 1][slot] = fmaf(pcb[k], fx[cx], -d);
            }
          } else {
            // a halo point left (c_x = +1) or right (c_x = -1) of the tile:
            // the three directions of that column
            const bool fw = rfwd;
            const float xR = fw ? pRx[k] : -pRx[k];
#pragma unroll
            for (int cy = 0; cy < 3; ++cy) {
              float fx[3];
              cm_to_pop_1d(h[k][0][cy][pz], h[k][1][cy][pz], h[k][2][cy][pz], pux[k], fx[0], fx[1],
                           fx[2]);
              const float fv = fw ? fx[2] : fx[0];
              const int i = dir_of(1, cy - 1, pz - 1);  // |c|, c_y, c_z as in either column
              const float cR = xR + (kCY[i] ? (kCY[i] > 0 ? pRy[k] : -pRy[k]) : 0.f) +
                               (kCZ[i] ? (kCZ[i] > 0 ? pRz[k] : -pRz[k]) : 0.f);
              const float d = 3.0f * weight(i) * cR;
              const int q = 3 * cy + (fw ? 2 : 0);
              xb[2 * q][slot] = fmaf(pcr[k], fv, d);
              xb[2 * q + 1][slot] = fmaf(pcb[k], fv, -d);
            }
          }
          if (WALLS && rsolid[k]) {
            // A solid point emits what the bounce-back stored there instead
            // (its rest population, which only it receives, stays in the
            // stash): one branch per point and z component, after the
            // emission above.  (A solid column node's own sums above feed
            // only its own moments, which are stored as zero.)
#pragma unroll
            for (int q = 0; q < 9; ++q) {
              xb[2 * q][slot] = S::dec(stv[q][0]);
              xb[2 * q + 1][slot] = S::dec(stv[q][1]);
            }
          }
        }
      }
      __syncthreads();
      // what arrives at the column node from (x - c_x, y - c_y) of slab s:
      // the colour sums, then the moments of f = f_r + f_b over the 3 x 3
      // directions by an x pass (sum, difference, sum of the ends of each
      // row) and a y pass of the same kind
      {
        float fr[9], fb[9], f[9];
#pragma unroll
        for (int cy = 0; cy < 3; ++cy)
#pragma unroll
          for (int cx = 0; cx < 3; ++cx) {
            const int q = 3 * cy + cx;
            const int src = (ox + 2 - cx) + G::R1X * (oy + 2 - cy);
            fr[q] = xb[2 * q][src];
            fb[q] = xb[2 * q + 1][src];
            f[q] = fr[q] + fb[q];
          }
        float sr = fr[0], sb = fb[0];
#pragma unroll
        for (int q = 1; q < 9; ++q) {
          sr += fr[q];
          sb += fb[q];
        }
        if constexpr (EXACT) {
          // the arrivals in FP64; the node's own rest population is added
          // below, closed on its FP64 density
          double s64r = 0.0, s64b = 0.0;
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            if (pz == 1 && q == 4) continue;
            s64r += (double)fr[q];
            s64b += (double)fb[q];
          }
          acc64[pz][0] += s64r;
          acc64[pz][1] += s64b;
        }
        float r0[3], r1[3], r2[3];  // per row: sum, c_x-weighted, c_x^2-weighted
#pragma unroll
        for (int cy = 0; cy < 3; ++cy) {
          r2[cy] = f[3 * cy + 2] + f[3 * cy];
          r1[cy] = f[3 * cy + 2] - f[3 * cy];
          r0[cy] = r2[cy] + f[3 * cy + 1];
        }
        const float m02 = r0[2] + r0[0], m00 = m02 + r0[1];
        // c_y-weighted: differences of opposite directions first
        const float m01 = ((f[6] - f[0]) + (f[8] - f[2])) + (f[7] - f[1]);
        const float m11 = r1[2] - r1[0], m10 = (r1[2] + r1[0]) + r1[1];
        const float m20 = (r2[2] + r2[0]) + r2[1];
        // The z momentum of the node at slab d is what arrives from slab
        // d - 1 less what arrives from slab d + 1: two sums of nine
        // populations of order rho / 6 whose difference is of order rho u.
        // Rounded at the size of the large sums it carries an error of order
        // 1e-8 rho that repeats at every step of a steady flow (it drifted
        // the total momentum of droplets at rest).  Both are therefore summed
        // as deviations e_i = f_i - 3 w_i p_ref from the rest-state
        // populations at the box's reference pressure (the smaller of the two
        // pure phases' rest pressures, which the equilibria make equal when
        // the sound speeds follow the density ratio): the same float
        // constants enter both sums, so the reference cancels exactly and only
        // the deviations are rounded.  (The even moments keep the plain sums:
        // a reference added back as a constant would leave its own rounding
        // as a bias of order 1e-9 in every node's second moments.)
        float m00d = 0.f;
        if (pz != 1) {
          float e[9];
#pragma unroll
          for (int cy = 0; cy < 3; ++cy)
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) {
              const int q = 3 * cy + cx;
              e[q] = f[q] + B.cdev[(cx != 1) + (cy != 1) + 1];
            }
          m00d = (((e[0] + e[2]) + (e[6] + e[8])) + ((e[1] + e[7]) + (e[3] + e[5]))) + e[4];
        }
        if (WALLS) {
          // a solid column node keeps what arrives, reversed, for the next step
          const int d = s + pz - 1, gd = wrap_any(d, nz);
          if (in_xy && d >= z0 && d < z1 && is_solid(B, gyo, gd)) {
            const uint32_t slot = (uint32_t)B.wbase + wall_slot(B, gxo, gyo, gd);
#pragma unroll
            for (int cy = 0; cy < 3; ++cy)
#pragma unroll
              for (int cx = 0; cx < 3; ++cx) {
                const int q = 3 * cy + cx;
                const int i = dir_of(cx - 1, cy - 1, pz - 1);
                if (EXACT && i == 0) {
                  // mass-exact storage: the rest populations stay as stored
#pragma unroll
                  for (int c = 0; c < 2; ++c)
                    buf_st(buf_ld_f64(win.r, win.rest_off(c, slot)), wout.r, wout.rest_off(c, slot));
                } else {
                  wout.st(opposite(i), slot, S::enc(fr[q]), S::enc(fb[q]));
                }
              }
          }
        }
        float *a = acc[pz];
        a[0] += sr;
        a[1] += sb;
        a[2] += m10;
        a[3] += m01;
        a[5] += m20;
        a[6] += m02;
        a[8] += m11;
        if (pz != 1) {
          const bool up = pz == 2;
          a[4] += up ? m00d : -m00d;
          a[7] += m00;
          a[9] += up ? m10 : -m10;
          a[10] += up ? m01 : -m01;
        }
      }
      __syncthreads();
    }
    if constexpr (EXACT) {
      // the rest populations of the column node at slab s
      acc64[1][0] += own_r - emit_r;
      acc64[1][1] += own_b - emit_b;
    }
    // slab s - 1 is complete (solid nodes: zero moments)
    const int gzm = wrap_any(s - 1, nz);
    const uint32_t node = (uint32_t)B.base + oxy + nxy * (uint32_t)gzm;
    const uint32_t off = boff<float>(in_xy && s - 1 >= z0, node);
    const bool osolid = WALLS && is_solid(B, gyo, gzm);
    if constexpr (EXACT) {
      acc[0][0] = (float)acc64[0][0];
      acc[0][1] = (float)acc64[0][1];
      double *r64 = aux_rho64(aux, plane);
      const uint32_t off64 = boff<double>(in_xy && s - 1 >= z0, node);
      buf_st(osolid ? 0.0 : acc64[0][0], plane_rsrc(r64, plane * 8, 0), off64);
      buf_st(osolid ? 0.0 : acc64[0][1], plane_rsrc(r64, plane * 8, 1), off64);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        acc64[0][c] = acc64[1][c];
        acc64[1][c] = acc64[2][c];
        acc64[2][c] = 0.0;
      }
    }
#pragma unroll
    for (int m = 0; m < 11; ++m)
      buf_st(osolid ? 0.f : acc[0][m], plane_rsrc(aux, plane * 4, A_RR + m), off);
#pragma unroll
    for (int m = 0; m < 11; ++m) {
      acc[0][m] = acc[1][m];
      acc[1][m] = acc[2][m];
      acc[2][m] = 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// k_emit: the compact state back to stored populations in format S: each
// node's collided, recoloured populations (bit for bit those the fused
// kernel would have stored), the state the next pull reads.
// ---------------------------------------------------------------------------
template <class S, bool GENERAL = false>
__global__ __launch_bounds__(kBlock) void k_emit(const BoxDev *__restrict__ boxes,
                                                 const int32_t *__restrict__ blk_box,
                                                 const float *__restrict__ cst,
                                                 void *__restrict__ dst_, int64_t plane) {
  const uint32_t lb = xcd_block();
  const int b = blk_box[lb];
  if (b < 0) return;
  const BoxDev B = boxes[b];
  const int64_t local = (int64_t)(lb - B.blk0) * kBlock + threadIdx.x;
  if (local >= B.n) return;
  const uint32_t node = (uint32_t)(B.base + local);
  float c[kCompact];
#pragma unroll
  for (int m = 0; m < kCompact; ++m) c[m] = ldpl_nt(cst, plane, m, node);
  const float rho = c[0] + c[1];
  const float irho = rcp(rho);
  const float p = c[0] * B.cs2r + c[1] * B.cs2b;
  float k[27];
  if (GENERAL)
    model_moments(B.model, rho, p, c[2], c[3], c[4], c[5], c[6], c[7], c[8], c[9], c[10], c[11],
                  c[12], c[13], k);
  else
    model_d_moments(rho, p, c[5], c[6], c[7], c[8], c[9], c[10], c[11], c[12], c[13], k);
  const Pops<S> dst(dst_, plane);
  PopWriter<S> w(dst, B, node);
  w.set_fraction(c[0], c[1]);
  emit_recoloured(B, k, c[2], c[3], c[4], div_refined(c[0], rho, irho), div_refined(c[1], rho, irho),
                  p, c[14], c[15], c[16], w);
  if (S::kExact) {
    // mass-exact storage: the rest populations closed on the FP64 densities
    const double *r64 = compact_rho64(const_cast<float *>(cst), plane);
    w.finish(at(r64, node), at(r64 + plane, node));
  }
}

}  // namespace cglbm
