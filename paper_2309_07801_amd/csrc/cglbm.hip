// cglbm.hip -- host side of the C ABI declared in include/cglbm.h.
//
// Parameter validation, layout of the concatenated boxes, block and tile
// tables, launches on the caller's stream, FP64 diagnostics and per-kernel
// event timing.  All kernels live in kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cglbm.h"
#include "d2q9.hpp"
#include "diag.hpp"
#include "kernels.hpp"
#include "tables.hpp"

using namespace cglbm;

namespace {

thread_local std::string g_err;

// Scratch of cglbm_reduce_noalloc, a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends): the chunk
// partials of the two reduction passes (kNPart doubles per chunk, at most
// kScratchChunks chunks), then the per-box diagnostics (kNPart doubles per
// box, at most kScratchBoxes boxes): 8.5 MiB.  Host code never uses the
// array's name as an address: cglbm_init looks up its device address once
// per device (g_scratch) and only that address is passed to kernels.
constexpr size_t kScratchChunks = (size_t)1 << 16;
constexpr size_t kScratchBoxes = 4096;
constexpr size_t kScratchDoubles = (kScratchChunks + kScratchBoxes) * kNPart;
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(CGLBM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                                  \
  } while (0)

constexpr int kTX = 8, kTY = 8, kTZ = 8;   // interface tile (three-kernel schedule)

using EmitFn = void (*)(const BoxDev *, const int32_t *, const float *, void *, int64_t);
constexpr int kNumFused = kNumFusedVariants;
constexpr int kNumCPull = kNumCPullVariants;
constexpr int kNumV2 = kNumVariants2;
enum { LATTICE_D3Q27 = 0, LATTICE_D2Q9 = 1 };
constexpr int64_t kAlign = 64;             // node alignment of each box's base
// Limit of all boxes together: every plane of 8-byte values (with the plane
// length's padding of at most 2 * kAlign nodes) stays below 4 GiB, so that
// kernels address a plane with 32-bit byte offsets.
constexpr int64_t kMaxNodes = (1ll << 29) - (1ll << 20);
constexpr double kXi = 9.0 / 19.0;   // D3Q27 (Sec. II.A)
constexpr double kXi2 = 3.0 / 5.0;   // D2Q9: the rest fractions of Eq. (8) sum to one

// Kinds of timed launches: the pull of a step (k_pull, or k_cpull in the
// compact schedule), the interface and collide kernels of the three-kernel
// schedule, the fused kernel (the compact fused kernel in schedule 2), and
// the population pull that starts and the emission that ends a compact call.
enum {
  KIND_PULL = 0,
  KIND_IFACE = 1,
  KIND_COLLIDE = 2,
  KIND_FUSED = 3,
  KIND_PULL_FIRST = 4,
  KIND_EMIT = 5,
  KIND_N = 6
};

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Kernels by storage format (index = cglbm_storage).
using PullFn = void (*)(const BoxDev *, const int32_t *, void *, void *, float *, int64_t, int,
                        void *, int64_t);
using WallCopyFn = void (*)(const BoxDev *, const int32_t *, const void *, void *, int64_t,
                            int64_t);
using CollideFn = void (*)(const BoxDev *, const int32_t *, float *, const void *, void *,
                          int64_t);
// [stash][storage]: the in-place layout's pull writes solid nodes to the stash
const PullFn kPull[2][7] = {{k_pull<StoreF32, false>, k_pull<StoreF16, false>,
                             k_pull<StoreBF16, false>, k_pull<StoreF32X, false>,
                             k_pull<StoreF32P, false>, k_pull<StoreF16C, false>,
                             k_pull<StoreBF16C, false>},
                            {k_pull<StoreF32, true>, k_pull<StoreF16, true>,
                             k_pull<StoreBF16, true>, k_pull<StoreF32X, true>,
                             k_pull<StoreF32P, true>, k_pull<StoreF16C, true>,
                             k_pull<StoreBF16C, true>}};
const CollideFn kCollide[7] = {k_collide<StoreF32>,  k_collide<StoreF16>,  k_collide<StoreBF16>,
                               k_collide<StoreF32X>, k_collide<StoreF32P>, k_collide<StoreF16C>,
                               k_collide<StoreBF16C>};
const InitFn kInit[7] = {k_init<StoreF32>,  k_init<StoreF16>,  k_init<StoreBF16>, k_init<StoreF32X>,
                         k_init<StoreF32P>, k_init<StoreF16C>, k_init<StoreBF16C>};
// [FP32 pairs][general equilibrium family]
const EmitFn kEmit[2][2] = {{k_emit<StoreF32, false>, k_emit<StoreF32, true>},
                            {k_emit<StoreF32P, false>, k_emit<StoreF32P, true>}};
// the mass-exact storages (Model D with Q), by storage (none for the plain
// FP32 layouts)
const EmitFn kEmitX[7] = {nullptr,
                          k_emit<StoreF16, false>,
                          k_emit<StoreBF16, false>,
                          k_emit<StoreF32X, false>,
                          nullptr,
                          k_emit<StoreF16C, false>,
                          k_emit<StoreBF16C, false>};
// the compact schedule of the 16-bit formats: the first pull writes the
// solid nodes' reversed populations decoded into a mass-exact FP32 stash,
// and the call's end encodes the last stash into the stored format
const PullFn kPullDec[7] = {nullptr,
                            k_pull<StoreF16, true, StoreF32X>,
                            k_pull<StoreBF16, true, StoreF32X>,
                            nullptr,
                            nullptr,
                            k_pull<StoreF16C, true, StoreF32X>,
                            k_pull<StoreBF16C, true, StoreF32X>};
const WallCopyFn kWallEncode[7] = {nullptr,
                                   k_wall_encode<StoreF16>,
                                   k_wall_encode<StoreBF16>,
                                   nullptr,
                                   nullptr,
                                   k_wall_encode<StoreF16C>,
                                   k_wall_encode<StoreBF16C>};
// the three-kernel schedule's collision writing compact states
const CollideFn kCollideCompact = k_collide<StoreF32, true>;
const WallCopyFn kWallCopy[7] = {k_wall_copy<StoreF32>,  k_wall_copy<StoreF16>,
                                 k_wall_copy<StoreBF16>, k_wall_copy<StoreF32X>,
                                 k_wall_copy<StoreF32P>, k_wall_copy<StoreF16C>,
                                 k_wall_copy<StoreBF16C>};

// D2Q9 keeps FP32 in colour pairs in either FP32 format
int storage2_slot(int32_t st) { return st == CGLBM_FP32_PAIRS ? 0 : st; }
bool storage_exact(int32_t st) { return st != CGLBM_FP32 && st != CGLBM_FP32_PAIRS; }
bool storage_16bit(int32_t st) { return storage_exact(st) && st != CGLBM_FP32_EXACT; }
size_t storage_bytes(int32_t st) {
  return (st == CGLBM_FP16_SHIFT || st == CGLBM_BF16_SHIFT || st == CGLBM_FP16_CSHIFT ||
          st == CGLBM_BF16_CSHIFT)
             ? 2
             : 4;
}
// the colour-fraction-shifted formats keep one 16-bit fraction per node
bool storage_cshift(int32_t st) { return st == CGLBM_FP16_CSHIFT || st == CGLBM_BF16_CSHIFT; }

// Bytes of one population buffer and of the aux buffer for `total` nodes.
void buffer_sizes(int32_t st, int64_t total, size_t *pop, size_t *aux, int lattice = LATTICE_D3Q27) {
  if (lattice == LATTICE_D2Q9) {
    // pair planes (9, or 8 and the FP64 rest planes of the mass-exact formats)
    const int64_t word = 2 * (int64_t)storage_bytes(st);
    if (storage_exact(st))
      *pop = (size_t)align256(8 * total * word) + (size_t)(2 * total * 8);
    else
      *pop = (size_t)(d2q9::kQ * total * word);
    *aux = (size_t)align256((int64_t)A_COUNT * total * 4) + (storage_exact(st) ? (size_t)(2 * total * 8) : 0);
    return;
  }
  if (storage_exact(st))
    *pop = (size_t)align256(52 * total * (int64_t)storage_bytes(st)) + (size_t)(2 * total * 8) +
           (storage_cshift(st) ? (size_t)(2 * total) : 0);
  else
    *pop = (size_t)(54 * total * 4);
  *aux = (size_t)align256((int64_t)A_COUNT * total * 4) + (storage_exact(st) ? (size_t)(2 * total * 8) : 0);
}

struct Layout {
  std::vector<BoxDev> boxes;
  std::vector<int32_t> blk_box, tile_box, col_box;
  std::vector<int32_t> wblk_box;  // k_wall_copy blocks (in-place layouts with walls)
  std::vector<TileEntry> col_tiles;   // k_fused blocks (D3Q27)
  std::vector<TileEntry> ccol_tiles;  // k_cpull blocks
  std::vector<int32_t> rch_box;   // reduction chunks (kRedChunk nodes of one box each)
  int64_t wtotal = 0;             // wall-node slots of all boxes (stash plane length)
  int64_t total = 0;  // plane length (nodes, all boxes, aligned)
  int32_t nblk = 0, ntile = 0, ncol = 0, nblk_pad = 0;
  // D3Q27: col_tiles and ccol_tiles hold first the tiles that run the kernel
  // without wall logic (ncol_plain, nccol_plain entries, padded to a
  // multiple of 8), then those whose stencils or rings reach a solid layer
  int32_t ncol_plain = 0, nccol_plain = 0;
  // boxes with z walls: the slabs next to them form short chunks of their
  // own (else the first and last chunks of every column are near walls)
  bool zedge = true;
  bool walls = false;
  bool general = false;  // a box with Model A, B or C or without Q: three-kernel schedule
  bool full_rates = false;  // a box with a higher-order rate other than 1
  int lattice = LATTICE_D3Q27;
};

int validate(int32_t n_boxes, const cglbm_box_params *boxes, int32_t storage) {
  if (n_boxes <= 0 || !boxes) return fail(CGLBM_EINVAL, "n_boxes must be > 0 and boxes non-NULL");
  if (storage < CGLBM_FP32 || storage > CGLBM_BF16_CSHIFT)
    return fail(CGLBM_EINVAL, "unknown storage format %d", storage);
  int64_t total = 0;
  for (int b = 0; b < n_boxes; ++b) {
    const cglbm_box_params &P = boxes[b];
    if (P.nx < 1 || P.ny < 1 || P.nz < 1)
      return fail(CGLBM_EINVAL, "box %d: extents must be >= 1", b);
    total += align_up((int64_t)P.nx * P.ny * P.nz, kAlign);
    if (total > kMaxNodes)
      return fail(CGLBM_EINVAL, "all boxes together exceed %lld nodes", (long long)kMaxNodes);
    if ((int64_t)P.nx * P.ny * P.nz > kMaxNodes)
      return fail(CGLBM_EINVAL, "box %d: more than %lld nodes", b, (long long)kMaxNodes);
    if (P.walls & ~3u) return fail(CGLBM_EINVAL, "box %d: unknown wall bits 0x%x", b, P.walls);
    if ((P.walls & 1u) && P.ny < 3) return fail(CGLBM_EINVAL, "box %d: y walls need ny >= 3", b);
    if ((P.walls & 2u) && P.nz < 3) return fail(CGLBM_EINVAL, "box %d: z walls need nz >= 3", b);
    const cglbm_phase *ph[2] = {&P.red, &P.blue};
    for (int c = 0; c < 2; ++c) {
      if (!(ph[c]->rho0 > 0.0) || !std::isfinite(ph[c]->rho0))
        return fail(CGLBM_EINVAL, "box %d: rho0 of colour %d must be > 0", b, c);
      if (!(ph[c]->alpha >= 0.0 && ph[c]->alpha < 1.0))
        return fail(CGLBM_EINVAL, "box %d: alpha of colour %d must lie in [0, 1)", b, c);
      if (!(ph[c]->nu >= 0.0) || !std::isfinite(ph[c]->nu))
        return fail(CGLBM_EINVAL, "box %d: nu of colour %d must be >= 0", b, c);
    }
    if (!std::isfinite(P.sigma) || P.sigma < 0.0)
      return fail(CGLBM_EINVAL, "box %d: sigma must be finite and >= 0", b);
    if (!std::isfinite(P.beta) || P.beta < 0.0)
      return fail(CGLBM_EINVAL, "box %d: beta must be finite and >= 0", b);
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(P.gravity[a]) || !std::isfinite(P.body_force[a]))
        return fail(CGLBM_EINVAL, "box %d: body force and gravity must be finite", b);
    if (!std::isfinite(P.rho_ref)) return fail(CGLBM_EINVAL, "box %d: rho_ref must be finite", b);
    if (P.model < CGLBM_MODEL_A || P.model > CGLBM_MODEL_D)
      return fail(CGLBM_EINVAL, "box %d: unknown equilibrium model %d", b, P.model);
    if (P.q_correction != 0 && P.q_correction != 1)
      return fail(CGLBM_EINVAL, "box %d: q_correction must be 0 or 1", b);
    if (!(P.omega_bulk > 0.0 && P.omega_bulk < 2.0))
      return fail(CGLBM_EINVAL, "box %d: omega_bulk must lie in (0, 2)", b);
    for (int k = 0; k < 9; ++k)
      if (!(P.omega_hi[k] > 0.0 && P.omega_hi[k] <= 2.0))
        return fail(CGLBM_EINVAL, "box %d: omega_hi[%d] = %g must lie in (0, 2]", b, k,
                    P.omega_hi[k]);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(P.body_force[k]))
        return fail(CGLBM_EINVAL, "box %d: body force must be finite", b);
  }
  return CGLBM_OK;
}

// The D2Q9 lattice of App. A: one-layer boxes, the generalized equilibrium
// of Eq. (A10) with unit rates above second order.
int validate_d2q9(int32_t n_boxes, const cglbm_box_params *boxes, int32_t storage) {
  int rc = validate(n_boxes, boxes, storage);
  if (rc) return rc;
  for (int b = 0; b < n_boxes; ++b) {
    const cglbm_box_params &P = boxes[b];
    if (P.nz != 1) return fail(CGLBM_EINVAL, "box %d: a D2Q9 box has nz = 1", b);
    if (storage_cshift(storage))
      return fail(CGLBM_EUNSUPPORTED, "the colour-fraction-shifted formats are built for D3Q27 only");
    if (P.walls & 2u) return fail(CGLBM_EINVAL, "box %d: a D2Q9 box has no z walls", b);
    if (P.model != CGLBM_MODEL_D)
      return fail(CGLBM_EUNSUPPORTED, "box %d: D2Q9 implements the equilibrium of Eq. (A10) only", b);
    for (int k = 0; k < 9; ++k)
      if (P.omega_hi[k] != 1.0)
        return fail(CGLBM_EUNSUPPORTED, "box %d: D2Q9 relaxes the higher moments at rate 1", b);
    for (int a = 0; a < 3; ++a)
      if (P.gravity[a] != 0.0) return fail(CGLBM_EUNSUPPORTED, "box %d: no buoyancy force in D2Q9", b);
  }
  return CGLBM_OK;
}

void build_layout(int32_t n_boxes, const cglbm_box_params *boxes, Layout &L,
                  int lattice = LATTICE_D3Q27) {
  L = Layout();
  L.lattice = lattice;
  const double xi = lattice == LATTICE_D2Q9 ? kXi2 : kXi;
  int64_t off = 0;
  int32_t blk = 0, tile = 0;
  for (int b = 0; b < n_boxes; ++b) {
    const cglbm_box_params &P = boxes[b];
    BoxDev B;
    std::memset(&B, 0, sizeof(B));
    B.nx = P.nx;
    B.ny = P.ny;
    B.nz = P.nz;
    B.walls = P.walls;
    B.n = (int64_t)P.nx * P.ny * P.nz;
    B.base = off;
    off = align_up(off + B.n, kAlign);
    B.blk0 = blk;
    const int32_t nb = (int32_t)((B.n + kBlock - 1) / kBlock);
    for (int32_t k = 0; k < nb; ++k) L.blk_box.push_back(b);
    blk += nb;
    B.rch0 = (int32_t)L.rch_box.size();
    for (int64_t k = 0; k < (B.n + kRedChunk - 1) / kRedChunk; ++k) L.rch_box.push_back(b);
    B.tile0 = tile;
    B.tnx = (P.nx + kTX - 1) / kTX;
    B.tny = (P.ny + kTY - 1) / kTY;
    const int32_t tnz = (P.nz + kTZ - 1) / kTZ;
    const int32_t nt = B.tnx * B.tny * tnz;
    for (int32_t k = 0; k < nt; ++k) L.tile_box.push_back(b);
    tile += nt;
    B.fdx = make_fastdiv((uint32_t)P.nx);
    B.fdy = make_fastdiv((uint32_t)P.ny);
    B.ftx = make_fastdiv((uint32_t)B.tnx);
    B.fty = make_fastdiv((uint32_t)B.tny);
    B.cs2r = (float)(xi * (1.0 - P.red.alpha));
    B.cs2b = (float)(xi * (1.0 - P.blue.alpha));
    B.d2q9 = lattice == LATTICE_D2Q9 ? 1 : 0;
    B.ir0r = (float)(1.0 / P.red.rho0);
    B.ir0b = (float)(1.0 / P.blue.rho0);
    B.nu_r = (float)P.red.nu;
    B.nu_b = (float)P.blue.nu;
    B.sigma = (float)P.sigma;
    B.beta = (float)P.beta;
    B.omega2 = (float)P.omega_bulk;
    B.Gx = (float)P.body_force[0];
    B.Gy = (float)P.body_force[1];
    B.Gz = (float)P.body_force[2];
    B.bgx = (float)P.gravity[0];
    B.bgy = (float)P.gravity[1];
    B.bgz = (float)P.gravity[2];
    B.rho_ref = (float)P.rho_ref;
    B.model = P.model;
    B.qcorr = P.q_correction;
    B.full_rates = 0;
    for (int k = 0; k < 9; ++k) {
      B.omh[k] = (float)P.omega_hi[k];
      if (P.omega_hi[k] != 1.0) B.full_rates = 1;
    }
    if (P.model != CGLBM_MODEL_D || !P.q_correction || B.full_rates) L.general = true;
    if (B.full_rates) L.full_rates = true;
    {
      // pure-phase rest equilibrium of each colour: w_i rho_k^0 (c_s^k)^2 / c_s^2,
      // by speed class |c_i|^2 (D3Q27 weights, or the D2Q9 ones of Eq. A2)
      const double w3[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
      const double w2[4] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 0.0};
      const double *w = lattice == LATTICE_D2Q9 ? w2 : w3;
      const double p0[2] = {P.red.rho0 * xi * (1.0 - P.red.alpha),
                            P.blue.rho0 * xi * (1.0 - P.blue.alpha)};
      for (int c = 0; c < 2; ++c)
        for (int k = 0; k < 4; ++k) B.shift[c][k] = (float)(w[k] * p0[c] * 3.0);
      // k_cpull's reference for the z momentum: the rest-state populations
      // 3 w_i p_ref (D3Q27 weights)
      const double pref = std::min(p0[0], p0[1]);
      for (int k = 0; k < 4; ++k) B.cdev[k] = (float)(-3.0 * w3[k] * pref);
      // power-of-two scale of each colour's stored values (colour-fraction
      // formats): 2^(10 - floor(log2 rho_k^0))
      const double r0[2] = {P.red.rho0, P.blue.rho0};
      for (int c = 0; c < 2; ++c) {
        const int e = std::max(-60, std::min(60, std::ilogb(r0[c]))) - 10;
        B.pscale[c] = (float)std::ldexp(1.0, -e);
        B.pinv[c] = (float)std::ldexp(1.0, e);
      }
    }
    // solid nodes: the z-wall planes, then the y-wall rows of the other layers
    {
      const int64_t nzw = (P.walls & 2u) ? 2 : 0;
      const int64_t wn = nzw * P.nx * P.ny + ((P.walls & 1u) ? 2 * (int64_t)P.nx * (P.nz - nzw) : 0);
      B.wbase = (int32_t)L.wtotal;
      B.wn = (int32_t)wn;
      B.wblk0 = (int32_t)L.wblk_box.size();
      for (int64_t k = 0; k < (wn + kBlock - 1) / kBlock; ++k) L.wblk_box.push_back(b);
      L.wtotal = align_up(L.wtotal + wn, kAlign);
    }
    L.boxes.push_back(B);
    if (P.walls) L.walls = true;
  }
  // Plane length: an odd multiple of kAlign nodes, so that consecutive
  // planes of 4-byte words start an odd number of 256-byte units apart and
  // one wave's accesses to the 27 planes spread over more memory channels
  // (16-bit storage measured 1-3 % faster than with power-of-two planes).
  L.total = std::max<int64_t>(off, kAlign);
  if ((L.total / kAlign) % 2 == 0) L.total += kAlign;
  L.nblk = blk;
  L.ntile = tile;
  // grids remapped across XCDs are padded to a multiple of 8 idle blocks
  L.nblk_pad = (int32_t)align_up(blk, 8);
  while ((int32_t)L.blk_box.size() < L.nblk_pad) L.blk_box.push_back(-1);
}

// Split of a box's tiles between the launch without wall logic and the one
// with it: a tile goes to the latter if the y rows or z slabs it reads
// (its extent widened by `halo`) come within one node of a solid layer.
bool tile_near_walls(const BoxDev &B, int y0, int ty, int z0, int z1, int halo) {
  const bool yw = (B.walls & 1u) && !(y0 - halo - 1 >= 1 && y0 + ty + halo <= B.ny - 2);
  const bool zw = (B.walls & 2u) && !(z0 - halo - 1 >= 1 && z1 + halo <= B.nz - 2);
  return yw || zw;
}

// Plain tiles first, then the tiles near walls, each list padded to a
// multiple of 8 (the XCD remap); returns the length of the first list.
int32_t pack_tiles(std::vector<TileEntry> &out, std::vector<TileEntry> &plain,
                   std::vector<TileEntry> &near) {
  const TileEntry pad = {-1, 0, 0, 0};
  while (plain.size() % 8) plain.push_back(pad);
  while (near.size() % 8) near.push_back(pad);
  out = plain;
  out.insert(out.end(), near.begin(), near.end());
  return (int32_t)plain.size();
}

// z chunks [z0, z1) of a box: zc slabs each, except that a box with z walls
// gets a chunk of `edge` slabs at each wall, so that the chunks between them
// (whose stencils then stay clear of the walls) run without wall logic.
std::vector<std::pair<int, int>> z_chunks(const BoxDev &B, int zc, int edge) {
  std::vector<std::pair<int, int>> out;
  int lo = 0, hi = B.nz;
  if (edge > 0 && (B.walls & 2u) && B.nz > 2 * edge + zc) {
    out.push_back({0, edge});
    lo = edge;
    hi = B.nz - edge;
  }
  for (int z = lo; z < hi; z += zc) out.push_back({z, std::min(z + zc, hi)});
  if (hi < B.nz) out.push_back({hi, B.nz});
  return out;
}

// Tile lists of one kernel geometry: every (chunk, column) of every box,
// split by tile_near_walls with the kernel's reach `halo`; `edge` slabs form
// the chunks at z walls.
void build_tiles(Layout &L, int tx, int ty, int zc, int halo, int edge,
                 std::vector<TileEntry> &out, int32_t &nplain, bool cpull) {
  std::vector<TileEntry> plain, near;
  for (size_t b = 0; b < L.boxes.size(); ++b) {
    BoxDev &B = L.boxes[b];
    const int32_t ncx = (B.nx + tx - 1) / tx, ncy = (B.ny + ty - 1) / ty;
    if (cpull) {
      B.ccol0 = 0;
      B.cncx = ncx;
      B.cncy = ncy;
      B.fccx = make_fastdiv((uint32_t)ncx);
      B.fccy = make_fastdiv((uint32_t)ncy);
    } else {
      B.col0 = 0;
      B.ncx = ncx;
      B.ncy = ncy;
      B.fcx = make_fastdiv((uint32_t)ncx);
      B.fcy = make_fastdiv((uint32_t)ncy);
    }
    for (const auto &zr : z_chunks(B, zc, edge))
      for (int32_t cy = 0; cy < ncy; ++cy)
        for (int32_t cx = 0; cx < ncx; ++cx) {
          const TileEntry e = {(int32_t)b, cx + ncx * cy, zr.first, zr.second};
          (tile_near_walls(B, cy * ty, ty, zr.first, zr.second, halo) ? near : plain).push_back(e);
        }
  }
  nplain = pack_tiles(out, plain, near);
}

// Column table of k_cpull variant v.  Its ring reaches one node around the
// column and one slab beyond the chunk.
void build_ccolumns(Layout &L, int v) {
  const CPullVariant &C = cpull_variant(v);
  build_tiles(L, C.tx, C.ty, C.zc, 1, L.zedge ? 3 : 0, L.ccol_tiles, L.nccol_plain, true);
}

// Column table of fused variant v.  Its stencils reach three nodes around
// the column, and its march three slabs beyond the chunk, plus the slabs its
// loads run ahead (five below the chunk).
void build_columns(Layout &L, int v) {
  const FusedVariant &F = fused_variant(v);
  build_tiles(L, F.tx, F.ty, F.zc, 4, L.zedge ? 6 : 0, L.col_tiles, L.ncol_plain, false);
  L.ncol = (int32_t)L.col_tiles.size();
}

// Tile table of the D2Q9 step kernel for variant v (kept in the column
// table's place): per box tile0, tnx, tny, ftx.
void build_tiles2(Layout &L, int v) {
  const Variant2 &V = variant2(v);
  L.col_box.clear();
  int32_t tile = 0;
  for (size_t b = 0; b < L.boxes.size(); ++b) {
    BoxDev &B = L.boxes[b];
    B.tile0 = tile;
    B.tnx = (B.nx + V.tx - 1) / V.tx;
    B.tny = (B.ny + V.ty - 1) / V.ty;
    B.ftx = make_fastdiv((uint32_t)B.tnx);
    const int32_t nt = B.tnx * B.tny;
    for (int32_t k = 0; k < nt; ++k) L.col_box.push_back((int32_t)b);
    tile += nt;
  }
  L.ncol = (int32_t)align_up(tile, 8);
  while ((int32_t)L.col_box.size() < L.ncol) L.col_box.push_back(-1);
}

// Host check of the division helper on the values a box can produce.
bool fastdiv_ok(uint32_t d, uint32_t nmax) {
  FastDiv f = make_fastdiv(d);
  const uint32_t probes[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, nmax / 2, nmax - 1, nmax};
  for (uint32_t n : probes)
    if (n <= nmax && fdiv(n, f) != n / d) return false;
  for (uint32_t k = 0; k < 4096; ++k) {
    uint32_t n = (uint32_t)(((uint64_t)k * 2654435761u) % ((uint64_t)nmax + 1));
    if (fdiv(n, f) != n / d) return false;
  }
  return true;
}

}  // namespace

struct cglbm_handle {
  int32_t n_boxes = 0;
  std::vector<cglbm_box_params> params;
  Layout L;
  int32_t storage = CGLBM_FP32;
  void *pop[2] = {nullptr, nullptr};
  float *aux = nullptr;
  int cur = 0;  // buffer holding the stored (post-collision) state
  bool inplace = false;          // pop[0] == pop[1]: one population buffer
  void *stash = nullptr;         // in-place layouts with walls: solid nodes' populations
  int32_t *d_wblk_box = nullptr;
  TileEntry *d_ccol_tiles = nullptr;  // k_cpull blocks
  void *cstash[2] = {nullptr, nullptr};  // compact schedule with walls: solid nodes' populations
  size_t ccol_cap = 0;             // capacity of d_ccol_tiles (entries)
  int32_t cvariant = 0;            // k_cpull geometry
  int device = 0;
  BoxDev *d_boxes = nullptr;
  int32_t *d_blk_box = nullptr;
  int32_t *d_tile_box = nullptr;
  int32_t *d_col_box = nullptr;       // D2Q9 tiles
  TileEntry *d_col_tiles = nullptr;    // D3Q27 k_fused blocks
  size_t col_tiles_cap = 0;            // capacity of d_col_tiles (entries)
  int32_t schedule = 0;        // 0 fused, 1 three kernels (D3Q27)
  int32_t lattice = LATTICE_D3Q27;
  int32_t variant = 0;         // fused launch geometry (its column table is loaded)
  int32_t fvar_pop = 0;        // fused geometry for schedules 0 and 1
  int32_t fvar_compact = 0;    // fused geometry for schedule 2
  // wall mode (boxes with walls): bit 0 short z-edge chunks (Layout::zedge),
  // bit 1 the launches over tiles near walls on the side stream; the current
  // one and the autotuner's choices per schedule
  int32_t wmode = 3, wmode_pop = 3, wmode_compact = 3;
  size_t col_cap = 0;          // capacity of d_col_box (entries)
  int32_t *d_rch_box = nullptr;  // reduction chunk -> box
  double *d_part = nullptr;    // chunk partials of the reduction (kNPart doubles each)
  double *d_diag = nullptr;    // per box kNPart doubles
  double *d_centre = nullptr;  // per box 3 doubles
  double *d_out = nullptr;     // per box CGLBM_NDIAG doubles (host-output reduce)
  // time steps as a captured graph: two steps from each buffer parity
  int32_t use_graph = 1;
  hipStream_t cap_stream = nullptr;
  // the launch over the tiles near walls runs on `side`, beside the one over
  // the other tiles on the caller's stream (fork and join by events)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t graphc[2] = {nullptr, nullptr};  // compact schedule: two inner steps
  // compact schedule with the state resident between calls
  // (cglbm_set_resident): clive is set while the other population buffer
  // holds the compact state of the last step and the state buffer is stale;
  // cwi is the wall stash that step wrote, cstream the stream it ran on
  bool resident = false, clive = false;
  int32_t cwi = 0;
  hipStream_t cstream = nullptr;
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
};

namespace {

// The pull (bounce != 0: with the bounce-back writes of a time step).  In
// place, the solid nodes' reversed populations go to the stash and
// k_wall_copy moves them into the buffer after the pull has completed.
int launch_pull(cglbm_handle *h, hipStream_t s, int bounce) {
  void *stash = bounce && h->stash ? h->stash : nullptr;
  hipLaunchKernelGGL(kPull[stash ? 1 : 0][h->storage], dim3(h->L.nblk_pad), dim3(kBlock), 0, s,
                     h->d_boxes,
                     h->d_blk_box, h->pop[h->cur], h->pop[1 - h->cur], h->aux, h->L.total,
                     bounce, stash, h->L.wtotal);
  if (stash && !h->L.wblk_box.empty())
    hipLaunchKernelGGL(kWallCopy[h->storage], dim3((unsigned)h->L.wblk_box.size()), dim3(kBlock),
                       0, s, h->d_boxes, h->d_wblk_box, (const void *)stash, h->pop[1 - h->cur],
                       h->L.total, h->L.wtotal);
  return CGLBM_OK;
}

int launch_iface(cglbm_handle *h, hipStream_t s, int write_kappa) {
  hipLaunchKernelGGL((k_interface<kTX, kTY, kTZ>), dim3(h->L.ntile), dim3(kBlock), 0, s,
                     h->d_boxes, h->d_tile_box, h->aux, h->L.total, write_kappa);
  return CGLBM_OK;
}

int fork_side(cglbm_handle *h, hipStream_t s) {
  HIP_TRY(hipEventRecord(h->fork_ev, s));
  HIP_TRY(hipStreamWaitEvent(h->side, h->fork_ev, 0));
  return CGLBM_OK;
}
int join_side(cglbm_handle *h, hipStream_t s) {
  HIP_TRY(hipEventRecord(h->join_ev, h->side));
  HIP_TRY(hipStreamWaitEvent(s, h->join_ev, 0));
  return CGLBM_OK;
}

// The fused kernel over the tiles near walls (fn[1], the column entries
// after the first `nplain`), then over the others (fn[0]).  Both lists
// non-empty and bit 1 of the wall mode set: the first goes to the handle's
// side stream, which waits for everything before it on s, and s waits for it
// afterwards (also under graph capture, where the events become the graph's
// dependencies).
int launch_split(cglbm_handle *h, int32_t ncol, int32_t nplain, const FusedFn *fn, int nthreads,
                 hipStream_t s, const BoxDev *boxes, const TileEntry *cols, float *aux,
                 void *dst, int64_t plane) {
  const int32_t n[2] = {nplain, ncol - nplain};
  const bool both = (h->wmode & 2) && n[0] > 0 && n[1] > 0;
  if (both) {
    const int rc = fork_side(h, s);
    if (rc) return rc;
  }
  for (int w = 1; w >= 0; --w) {
    if (n[w] <= 0) continue;
    const TileEntry *c = cols + (w ? nplain : 0);
    void *args[] = {(void *)&boxes, (void *)&c, (void *)&aux, (void *)&dst, (void *)&plane};
    HIP_TRY(hipLaunchKernel((const void *)fn[w], dim3((unsigned)n[w]), dim3(nthreads), args, 0,
                            (both && w) ? h->side : s));
  }
  return both ? join_side(h, s) : CGLBM_OK;
}

// export == 0: interface stencils + collision of a time step; export != 0:
// the interface fields n, F, Q, kappa into aux, populations untouched.
// Compact schedule: the fused kernel writes the compact state into the
// other population buffer; k_cpull turns it into the moments of the next
// step; k_emit stores it as populations in the state buffer.
int launch_fused_compact(cglbm_handle *h, hipStream_t s) {
  const FusedVariant &F = fused_variant(h->variant);
  const BoxDev *boxes = h->d_boxes;
  const TileEntry *cols = h->d_col_tiles;
  float *aux = h->aux;
  void *dst = h->pop[1 - h->cur];
  int64_t plane = h->L.total;
  const FusedFn *fn = storage_exact(h->storage) ? F.fcx : F.fc;
  return launch_split(h, h->L.ncol, h->L.ncol_plain, fn, F.tx * F.ty, s, boxes, cols, aux, dst,
                      plane);
}
// rd: the wall stash this step's solid points emit from; the arrivals at
// solid nodes go to the other one
int launch_cpull(cglbm_handle *h, hipStream_t s, int rd = 0) {
  const CPullVariant &C = cpull_variant(h->cvariant);
  const bool x = storage_exact(h->storage);
  const int g = h->L.general ? 1 : 0;
  // the tiles away from walls, then those near them
  const CPullFn fn[2] = {x ? C.fx[0] : C.fn[g][0],
                         x ? C.fx[1] : C.fn[g][h->storage == CGLBM_FP32_PAIRS ? 2 : 1]};
  const int32_t n[2] = {h->L.nccol_plain, (int32_t)h->L.ccol_tiles.size() - h->L.nccol_plain};
  const bool both = (h->wmode & 2) && n[0] > 0 && n[1] > 0;
  if (both) {
    const int rc = fork_side(h, s);
    if (rc) return rc;
  }
  for (int w = 1; w >= 0; --w)
    if (n[w] > 0)
      hipLaunchKernelGGL(fn[w], dim3((unsigned)n[w]), dim3(C.tx * C.ty), 0,
                         (both && w) ? h->side : s, h->d_boxes, h->d_ccol_tiles + (w ? n[0] : 0),
                         (const float *)h->pop[1 - h->cur], h->aux, h->L.total,
                         (const void *)h->cstash[rd], h->cstash[1 - rd], h->L.wtotal);
  return both ? join_side(h, s) : CGLBM_OK;
}
// wi: the wall stash the last step wrote (the solid nodes' stored values)
int launch_emit(cglbm_handle *h, hipStream_t s, int wi = 0) {
  hipLaunchKernelGGL(storage_exact(h->storage)
                         ? kEmitX[h->storage]
                         : kEmit[h->storage == CGLBM_FP32_PAIRS ? 1 : 0][h->L.general ? 1 : 0],
                     dim3(h->L.nblk_pad), dim3(kBlock), 0, s, h->d_boxes, h->d_blk_box,
                     (const float *)h->pop[1 - h->cur], h->pop[h->cur], h->L.total);
  if (h->L.walls && !h->L.wblk_box.empty())
    hipLaunchKernelGGL(storage_16bit(h->storage) ? kWallEncode[h->storage]
                                                 : kWallCopy[h->storage],
                       dim3((unsigned)h->L.wblk_box.size()), dim3(kBlock),
                       0, s, h->d_boxes, h->d_wblk_box, (const void *)h->cstash[wi],
                       h->pop[h->cur], h->L.total, h->L.wtotal);
  return CGLBM_OK;
}
// The first step of a compact call: the population pull, with the solid
// nodes' reversed populations going to wall stash 0 (decoded to the
// mass-exact FP32 format for the 16-bit storages).
int launch_pull_compact(cglbm_handle *h, hipStream_t s) {
  void *stash = h->L.walls ? h->cstash[0] : nullptr;
  hipLaunchKernelGGL(stash && storage_16bit(h->storage) ? kPullDec[h->storage]
                                                        : kPull[stash ? 1 : 0][h->storage],
                     dim3(h->L.nblk_pad), dim3(kBlock), 0, s,
                     h->d_boxes, h->d_blk_box, h->pop[h->cur], h->pop[1 - h->cur], h->aux,
                     h->L.total, 1, stash, h->L.wtotal);
  return CGLBM_OK;
}
// Layouts the compact schedule serves: D3Q27, FP32 storage (either layout,
// any equilibrium family), or a mass-exact storage (FP32 or 16-bit; Model D
// with Q), two buffers, unit higher rates.  With a 16-bit storage the
// compact state (17 floats and the FP64 colour densities, 84 bytes a node)
// fits the other population buffer (at least 120 bytes a node).
bool compact_ok(const cglbm_handle *h) {
  return h->lattice == LATTICE_D3Q27 && !h->inplace && !h->L.full_rates &&
         (h->storage == CGLBM_FP32 || h->storage == CGLBM_FP32_PAIRS ||
          (storage_exact(h->storage) && !h->L.general));
}

int launch_fused(cglbm_handle *h, hipStream_t s, int export_fields) {
  const FusedVariant &F = fused_variant(h->variant);
  const BoxDev *boxes = h->d_boxes;
  const TileEntry *cols = h->d_col_tiles;
  float *aux = h->aux;
  void *dst = h->pop[1 - h->cur];
  int64_t plane = h->L.total;
  const FusedFn *fn = export_fields ? F.fx : F.fn[h->storage];
  return launch_split(h, h->L.ncol, h->L.ncol_plain, fn, F.tx * F.ty, s, boxes, cols, aux, dst,
                      plane);
}

// Select fused variant v: rebuild and upload the column tables.
void drop_graphs(cglbm_handle *h) {
  for (hipGraphExec_t &g : h->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  for (hipGraphExec_t &g : h->graphc)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Select k_cpull variant v: rebuild and upload its column table.
int select_cvariant(cglbm_handle *h, int v, hipStream_t s) {
  drop_graphs(h);
  build_ccolumns(h->L, v);
  for (const BoxDev &B : h->L.boxes)
    if (!fastdiv_ok((uint32_t)B.cncx, 1u << 20) || !fastdiv_ok((uint32_t)B.cncy, 1u << 20))
      return fail(CGLBM_EINVAL, "index division self-check failed");
  if (h->L.ccol_tiles.size() > h->ccol_cap) {
    if (h->d_ccol_tiles) HIP_TRY(hipFree(h->d_ccol_tiles));
    h->d_ccol_tiles = nullptr;
    HIP_TRY(hipMalloc(&h->d_ccol_tiles, sizeof(TileEntry) * h->L.ccol_tiles.size()));
    h->ccol_cap = h->L.ccol_tiles.size();
  }
  HIP_TRY(hipMemcpyAsync(h->d_ccol_tiles, h->L.ccol_tiles.data(),
                         sizeof(TileEntry) * h->L.ccol_tiles.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->d_boxes, h->L.boxes.data(), sizeof(BoxDev) * h->L.boxes.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  h->cvariant = v;
  return CGLBM_OK;
}

int select_variant(cglbm_handle *h, int v, hipStream_t s) {
  drop_graphs(h);
  if (h->lattice == LATTICE_D2Q9) {
    build_tiles2(h->L, v);
    for (const BoxDev &B : h->L.boxes)
      if (!fastdiv_ok((uint32_t)B.tnx, (uint32_t)(B.tnx * B.tny)))
        return fail(CGLBM_EINVAL, "index division self-check failed");
    if (h->L.col_box.size() > h->col_cap) {
      if (h->d_col_box) HIP_TRY(hipFree(h->d_col_box));
      h->d_col_box = nullptr;
      HIP_TRY(hipMalloc(&h->d_col_box, sizeof(int32_t) * h->L.col_box.size()));
      h->col_cap = h->L.col_box.size();
    }
    HIP_TRY(hipMemcpyAsync(h->d_col_box, h->L.col_box.data(),
                           sizeof(int32_t) * h->L.col_box.size(), hipMemcpyHostToDevice, s));
  } else {
    build_columns(h->L, v);
    if (h->L.col_tiles.size() > h->col_tiles_cap) {
      if (h->d_col_tiles) HIP_TRY(hipFree(h->d_col_tiles));
      h->d_col_tiles = nullptr;
      HIP_TRY(hipMalloc(&h->d_col_tiles, sizeof(TileEntry) * h->L.col_tiles.size()));
      h->col_tiles_cap = h->L.col_tiles.size();
    }
    HIP_TRY(hipMemcpyAsync(h->d_col_tiles, h->L.col_tiles.data(),
                           sizeof(TileEntry) * h->L.col_tiles.size(), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(h->d_boxes, h->L.boxes.data(), sizeof(BoxDev) * h->L.boxes.size(),
                         hipMemcpyHostToDevice, s));
  // pageable host sources: make sure the copies completed before the vectors change
  HIP_TRY(hipStreamSynchronize(s));
  h->variant = v;
  return CGLBM_OK;
}

// Fused variant v under wall mode m: rebuild the tile lists whose chunking
// changes (the k_cpull list too); graphs captured under another mode are
// dropped.
int select_mode(cglbm_handle *h, int v, int32_t m, hipStream_t s) {
  const bool zedge = (m & 1) != 0, rebuild_c = zedge != h->L.zedge;
  if (m != h->wmode) drop_graphs(h);
  h->wmode = m;
  h->L.zedge = zedge;
  int rc = select_variant(h, v, s);
  if (!rc && rebuild_c) rc = select_cvariant(h, h->cvariant, s);
  return rc;
}

int launch_collide(cglbm_handle *h, hipStream_t s) {
  hipLaunchKernelGGL(kCollide[h->storage], dim3(h->L.nblk_pad), dim3(kBlock), 0, s, h->d_boxes,
                     h->d_blk_box, h->aux, (const void *)h->pop[h->cur], h->pop[1 - h->cur],
                     h->L.total);
  return CGLBM_OK;
}

// The collision half of a compact step: the fused kernel for Model D with
// Q; for the general families the interface kernel and the collision
// writing compact states.
int launch_compact_collide(cglbm_handle *h, hipStream_t s) {
  if (!h->L.general) return launch_fused_compact(h, s);
  int rc = launch_iface(h, s, 0);
  if (rc) return rc;
  hipLaunchKernelGGL(kCollideCompact, dim3(h->L.nblk_pad), dim3(kBlock), 0, s, h->d_boxes,
                     h->d_blk_box, h->aux, (const void *)h->pop[h->cur], h->pop[1 - h->cur],
                     h->L.total);
  return CGLBM_OK;
}

template <class F>
int timed(cglbm_handle *h, hipStream_t s, int kind, F &&launch) {
  if (h->prof && h->ev_used + 2 <= h->ev.size()) {
    HIP_TRY(hipEventRecord(h->ev[h->ev_used], s));
    int rc = launch();
    HIP_TRY(hipEventRecord(h->ev[h->ev_used + 1], s));
    h->ev_kind[h->ev_used / 2] = kind;
    h->ev_used += 2;
    return rc;
  }
  return launch();
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CGLBM_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return CGLBM_OK;
}

// Local moments and interface fields of the current state into aux.
// The fused kernel implements Model D with the correction term; layouts with
// any other box run the three-kernel schedule, whose collision takes each
// box's equilibrium family and correction switch.
int effective_schedule(const cglbm_handle *h) {
  if (h->schedule == 2) return 2;  // set only where compact_ok holds
  return h->L.general ? 1 : h->schedule;
}

// D2Q9: one launch of the step kernel (export != 0: the fields of the
// stored state into aux, populations untouched).
int launch_step2(cglbm_handle *h, hipStream_t s, int export_fields) {
  const Variant2 &V = variant2(h->variant);
  const int slot = storage2_slot(h->storage);
  hipLaunchKernelGGL(export_fields ? V.fields[slot] : V.step[slot], dim3(h->L.ncol), dim3(256), 0,
                     s, h->d_boxes, h->d_col_box, (const void *)h->pop[h->cur],
                     h->pop[1 - h->cur], h->aux, h->L.total);
  return CGLBM_OK;
}

// One time step on stream s (launches only); flips the buffer parity.
int launch_step(cglbm_handle *h, hipStream_t s) {
  if (h->lattice == LATTICE_D2Q9) {
    int rc = timed(h, s, KIND_FUSED, [&] { return launch_step2(h, s, 0); });
    if (!rc) rc = check_launch();
    if (!rc) h->cur = 1 - h->cur;
    return rc;
  }
  int rc = timed(h, s, KIND_PULL, [&] { return launch_pull(h, s, 1); });
  if (effective_schedule(h) == 0) {
    if (!rc) rc = timed(h, s, KIND_FUSED, [&] { return launch_fused(h, s, 0); });
  } else {
    if (!rc) rc = timed(h, s, KIND_IFACE, [&] { return launch_iface(h, s, 0); });
    if (!rc) rc = timed(h, s, KIND_COLLIDE, [&] { return launch_collide(h, s); });
  }
  if (!rc) rc = check_launch();
  if (!rc) h->cur = 1 - h->cur;
  return rc;
}

// n steps of the compact schedule (launches only).  The state between calls
// stays in stored populations: the first step pulls them, the last converts
// the compact state back, and the state buffer parity is unchanged.
int capture_compact_pair(cglbm_handle *h) {
  if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = CGLBM_OK;
  for (int k = 0; k < 2 && !rc; ++k) {
    rc = launch_cpull(h, h->cap_stream, k);
    if (!rc) rc = launch_compact_collide(h, h->cap_stream);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(CGLBM_EHIP, "graph capture: %s", hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&h->graphc[h->cur], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    h->graphc[h->cur] = nullptr;
    return fail(CGLBM_EHIP, "graph instantiate: %s", hipGetErrorString(ei));
  }
  return CGLBM_OK;
}

// Mean milliseconds per launch(k) over `reps` replays of a graph that
// captures launch(stream, 0) and launch(stream, 1) on the capture stream.
template <class F>
int time_graph(cglbm_handle *h, hipStream_t s, int reps, hipEvent_t e0, hipEvent_t e1, F &&launch,
               double &ms_out) {
  if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = launch(h->cap_stream, 0);
  if (!rc) rc = launch(h->cap_stream, 1);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (!rc && e != hipSuccess) rc = fail(CGLBM_EHIP, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  if (!rc) {
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) rc = fail(CGLBM_EHIP, "graph instantiate: %s", hipGetErrorString(ei));
  }
  if (g) (void)hipGraphDestroy(g);
  if (rc) return rc;
  hipError_t el = hipGraphLaunch(x, s);
  if (el == hipSuccess) el = hipEventRecord(e0, s);
  for (int r = 0; r < reps && el == hipSuccess; ++r) el = hipGraphLaunch(x, s);
  if (el == hipSuccess) el = hipEventRecord(e1, s);
  if (el == hipSuccess) el = hipEventSynchronize(e1);
  float ms = 0.f;
  if (el == hipSuccess) el = hipEventElapsedTime(&ms, e0, e1);
  (void)hipGraphExecDestroy(x);
  if (el != hipSuccess) return fail(CGLBM_EHIP, "autotune: %s", hipGetErrorString(el));
  ms_out = (double)ms / (2.0 * reps);
  return CGLBM_OK;
}

// Resident compact state (cglbm_set_resident): store it as populations in the
// state buffer if the last call left it in compact form.  The next compact
// call then starts from the populations again.
int flush_compact(cglbm_handle *h, hipStream_t s) {
  if (!h->clive) return CGLBM_OK;
  h->clive = false;
  const int rc = timed(h, s, KIND_EMIT, [&] { return launch_emit(h, s, h->cwi); });
  return rc ? rc : check_launch();
}

int step_compact(cglbm_handle *h, int32_t n, hipStream_t s) {
  if (n == 0) return CGLBM_OK;
  // wall stashes (boxes with solid layers): step k's solid points emit from
  // stash wi, its arrivals at solid nodes go to 1 - wi; the first step
  // (the population pull) writes stash 0
  int wi = 0;
  int rc = CGLBM_OK;
  int32_t k = 0;
  if (h->clive) {
    // resident: continue from the compact state of the last call, with one
    // direct step first if it left the stashes at odd parity (the captured
    // pair starts from stash 0)
    wi = h->cwi;
    h->clive = false;
    if (wi == 1) {
      rc = timed(h, s, KIND_PULL, [&] { return launch_cpull(h, s, 1); });
      if (!rc) rc = timed(h, s, KIND_FUSED, [&] { return launch_compact_collide(h, s); });
      wi = 0;
      k = 1;
    }
  } else {
    rc = timed(h, s, KIND_PULL_FIRST, [&] { return launch_pull_compact(h, s); });
    if (!rc) rc = timed(h, s, KIND_FUSED, [&] { return launch_compact_collide(h, s); });
    k = 1;
  }
  if (!rc && h->use_graph && !h->prof && n - k >= 2) {
    if (!h->graphc[h->cur]) rc = capture_compact_pair(h);
    for (; !rc && k + 1 < n; k += 2) HIP_TRY(hipGraphLaunch(h->graphc[h->cur], s));
  }
  for (; k < n && !rc; ++k) {
    rc = timed(h, s, KIND_PULL, [&] { return launch_cpull(h, s, wi); });
    if (!rc) rc = timed(h, s, KIND_FUSED, [&] { return launch_compact_collide(h, s); });
    wi = 1 - wi;
  }
  if (rc) return rc;
  if (h->resident) {
    h->clive = true;
    h->cwi = wi;
    h->cstream = s;
  } else {
    rc = timed(h, s, KIND_EMIT, [&] { return launch_emit(h, s, wi); });
  }
  if (!rc) rc = check_launch();
  return rc;
}

// Capture two steps from the current parity (which they restore) on the
// handle's private stream and instantiate them as an executable graph.
int capture_pair(cglbm_handle *h) {
  if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  const int c0 = h->cur;
  HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = launch_step(h, h->cap_stream);
  if (!rc) rc = launch_step(h, h->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  h->cur = c0;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(CGLBM_EHIP, "graph capture: %s", hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&h->graph[c0], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    h->graph[c0] = nullptr;
    return fail(CGLBM_EHIP, "graph instantiate: %s", hipGetErrorString(ei));
  }
  return CGLBM_OK;
}

int compute_fields(cglbm_handle *h, hipStream_t s, int write_kappa) {
  if (h->clive) {
    const int rc = flush_compact(h, s);
    if (rc) return rc;
  }
  if (h->lattice == LATTICE_D2Q9) {
    const int rc = launch_step2(h, s, 1);
    return rc ? rc : check_launch();
  }
  int rc = launch_pull(h, s, 0);
  if (rc) return rc;
  if (effective_schedule(h) != 1)
    rc = launch_fused(h, s, 1);
  else
    rc = launch_iface(h, s, write_kappa);
  if (rc) return rc;
  return check_launch();
}

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the caller's).
int scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(CGLBM_EUNSUPPORTED, "device %d beyond the library's %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return CGLBM_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(CGLBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch[device] = (double *)ptr;
  return CGLBM_OK;
}

// The diagnostics of the current state: local moments and interface fields
// into aux, then the two chunked passes and the per-box finals (launches
// only).  centre: device array of 3 doubles per box, or NULL for the box
// centres; part: room for one partial per reduction chunk; diag: kNPart
// doubles per box; out: the packed CGLBM_NDIAG doubles per box, device.
int reduce_launch(cglbm_handle *h, hipStream_t s, const double *centre, double *part,
                  double *diag, double *out) {
  int rc = compute_fields(h, s, 0);
  if (rc) return rc;
  const double *rho64 =
      storage_exact(h->storage)
          ? (const double *)((const char *)h->aux + align256((int64_t)A_COUNT * h->L.total * 4))
          : nullptr;
  const unsigned nch = (unsigned)h->L.rch_box.size();
  hipLaunchKernelGGL(k_reduce1, dim3(nch), dim3(kBlock), 0, s, h->d_boxes, h->d_rch_box, h->aux,
                     h->L.total, rho64, centre, part);
  hipLaunchKernelGGL(k_reduce_final, dim3(h->n_boxes), dim3(kBlock), 0, s, h->d_boxes,
                     (const double *)part, 1, diag, (double *)nullptr);
  hipLaunchKernelGGL(k_reduce2, dim3(nch), dim3(kBlock), 0, s, h->d_boxes, h->d_rch_box, h->aux,
                     h->L.total, centre, (const double *)diag, part);
  hipLaunchKernelGGL(k_reduce_final, dim3(h->n_boxes), dim3(kBlock), 0, s, h->d_boxes,
                     (const double *)part, 2, diag, out);
  return check_launch();
}

// D2Q9: time every tile variant of the step kernel on the same stored state
// (the kernel reads one buffer and writes the other, so repeated launches
// are idempotent) and keep the fastest.
int autotune2(cglbm_handle *h, int32_t reps, double *ms_per_variant, hipStream_t s) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = CGLBM_OK, best = h->variant;
  double best_ms = 1e300;
  for (int v = 0; v < kNumV2 && !rc; ++v) {
    if ((rc = select_variant(h, v, s)) || (rc = launch_step2(h, s, 0))) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && !rc; ++r) rc = launch_step2(h, s, 0);
    (void)hipEventRecord(e1, s);
    if (rc || (rc = check_launch())) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(CGLBM_EHIP, "autotune: event synchronize failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double avg = (double)ms / reps;
    if (ms_per_variant) ms_per_variant[v] = avg;
    if (avg < best_ms) {
      best_ms = avg;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  return select_variant(h, best, s);
}

}  // namespace

extern "C" {

const char *cglbm_last_error(void) { return g_err.c_str(); }

const char *cglbm_version(void) { return "cglbm-gfx950 0.1"; }

}  // extern "C"

namespace {

int query_sizes(int lattice, int32_t n_boxes, const cglbm_box_params *boxes, int32_t storage,
                size_t *pop_bytes, size_t *aux_bytes, int64_t *total_nodes) {
  g_err.clear();
  int rc = lattice == LATTICE_D2Q9 ? validate_d2q9(n_boxes, boxes, storage)
                                   : validate(n_boxes, boxes, storage);
  if (rc) return rc;
  Layout L;
  build_layout(n_boxes, boxes, L, lattice);
  size_t pb, ab;
  buffer_sizes(storage, L.total, &pb, &ab, lattice);
  if (pop_bytes) *pop_bytes = pb;
  if (aux_bytes) *aux_bytes = ab;
  if (total_nodes) *total_nodes = L.total;
  return CGLBM_OK;
}

int init_handle(int lattice, cglbm_handle **out, int32_t n_boxes, const cglbm_box_params *boxes,
                int32_t storage, void *pop_a, void *pop_b, void *aux, const float *init_rho_r,
                const float *init_rho_b, const float *init_u, uint64_t noise_seed,
                double noise_amp, void *stream);

}  // namespace

extern "C" {

int cglbm_query_sizes(int32_t n_boxes, const cglbm_box_params *boxes, int32_t storage,
                      size_t *pop_bytes, size_t *aux_bytes, int64_t *total_nodes) {
  return query_sizes(LATTICE_D3Q27, n_boxes, boxes, storage, pop_bytes, aux_bytes, total_nodes);
}

int cglbm_query_sizes_d2q9(int32_t n_boxes, const cglbm_box_params *boxes, int32_t storage,
                           size_t *pop_bytes, size_t *aux_bytes, int64_t *total_nodes) {
  return query_sizes(LATTICE_D2Q9, n_boxes, boxes, storage, pop_bytes, aux_bytes, total_nodes);
}

int cglbm_init(cglbm_handle **out, int32_t n_boxes, const cglbm_box_params *boxes,
               int32_t storage, void *pop_a, void *pop_b, void *aux, const float *init_rho_r,
               const float *init_rho_b, const float *init_u, uint64_t noise_seed,
               double noise_amp, void *stream) {
  return init_handle(LATTICE_D3Q27, out, n_boxes, boxes, storage, pop_a, pop_b, aux, init_rho_r,
                     init_rho_b, init_u, noise_seed, noise_amp, stream);
}

int cglbm_init_d2q9(cglbm_handle **out, int32_t n_boxes, const cglbm_box_params *boxes,
                    int32_t storage, void *pop_a, void *pop_b, void *aux, const float *init_rho_r,
                    const float *init_rho_b, const float *init_u, uint64_t noise_seed,
                    double noise_amp, void *stream) {
  return init_handle(LATTICE_D2Q9, out, n_boxes, boxes, storage, pop_a, pop_b, aux, init_rho_r,
                     init_rho_b, init_u, noise_seed, noise_amp, stream);
}

int cglbm_lattice(const cglbm_handle *h) { return h ? h->lattice : -1; }

int64_t cglbm_box_offset(const cglbm_handle *h, int32_t box) {
  if (!h || box < 0 || box >= h->n_boxes) return -1;
  return h->L.boxes[box].base;
}

void *cglbm_state_buffer(const cglbm_handle *h) { return h ? h->pop[h->cur] : nullptr; }

int cglbm_load_state(cglbm_handle *h, const void *src, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (!src) return fail(CGLBM_EINVAL, "src must not be NULL");
  size_t pop = 0, aux = 0;
  buffer_sizes(h->storage, h->L.total, &pop, &aux, h->lattice);
  h->clive = false;  // a resident compact state is replaced by the loaded one
  if (src == h->pop[h->cur]) return CGLBM_OK;
  HIP_TRY(hipMemcpyAsync(h->pop[h->cur], src, pop, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return CGLBM_OK;
}

}  // extern "C"

namespace {

int init_handle(int lattice, cglbm_handle **out, int32_t n_boxes, const cglbm_box_params *boxes,
                int32_t storage, void *pop_a, void *pop_b, void *aux, const float *init_rho_r,
                const float *init_rho_b, const float *init_u, uint64_t noise_seed,
                double noise_amp, void *stream) {
  g_err.clear();
  if (!out) return fail(CGLBM_EINVAL, "out must not be NULL");
  *out = nullptr;
  int rc = lattice == LATTICE_D2Q9 ? validate_d2q9(n_boxes, boxes, storage)
                                   : validate(n_boxes, boxes, storage);
  if (rc) return rc;
  if (!pop_a) return fail(CGLBM_EINVAL, "pop_a must not be NULL");
  if (pop_a == pop_b) return fail(CGLBM_EINVAL, "pop_a and pop_b must differ");
  const bool inplace = pop_b == nullptr;
  if (inplace) {
    // one buffer works where populations are read by the pull alone
    if (lattice == LATTICE_D2Q9)
      return fail(CGLBM_EUNSUPPORTED, "D2Q9 steps read and write populations in one kernel: pass pop_b");
    for (int b = 0; b < n_boxes; ++b)
      for (int k = 0; k < 9; ++k)
        if (boxes[b].omega_hi[k] != 1.0)
          return fail(CGLBM_EUNSUPPORTED,
                      "box %d: non-unit higher-order rates pull the populations again: pass pop_b", b);
  }
  if (!aux || !init_rho_r || !init_rho_b || !init_u)
    return fail(CGLBM_EINVAL, "aux and the initial fields must not be NULL");
  if (!std::isfinite(noise_amp) || noise_amp < 0.0)
    return fail(CGLBM_EINVAL, "noise_amp must be finite and >= 0");
  cglbm_handle *h = new cglbm_handle();
  h->n_boxes = n_boxes;
  h->params.assign(boxes, boxes + n_boxes);
  h->storage = storage;
  h->lattice = lattice;
  build_layout(n_boxes, boxes, h->L, lattice);
  build_ccolumns(h->L, 0);
  h->ccol_cap = h->L.ccol_tiles.size();
  for (const BoxDev &B : h->L.boxes) {
    if (!fastdiv_ok((uint32_t)B.nx, (uint32_t)B.n) || !fastdiv_ok((uint32_t)B.ny, (uint32_t)B.n) ||
        !fastdiv_ok((uint32_t)B.tnx, 1u << 20) || !fastdiv_ok((uint32_t)B.tny, 1u << 20) ||
        !fastdiv_ok((uint32_t)B.cncx, 1u << 20) || !fastdiv_ok((uint32_t)B.cncy, 1u << 20)) {
      delete h;
      return fail(CGLBM_EINVAL, "index division self-check failed");
    }
  }
  h->pop[0] = pop_a;
  h->pop[1] = inplace ? pop_a : pop_b;
  h->inplace = inplace;
  h->aux = (float *)aux;
  hipStream_t s = (hipStream_t)stream;
  auto cleanup = [&](int code) {
    cglbm_destroy(h);
    return code;
  };
  hipError_t e;
  if ((e = hipGetDevice(&h->device)) != hipSuccess ||
      (e = hipMalloc(&h->d_boxes, sizeof(BoxDev) * n_boxes)) != hipSuccess ||
      (e = hipMalloc(&h->d_blk_box, sizeof(int32_t) * h->L.blk_box.size())) != hipSuccess ||
      (e = hipMalloc(&h->d_tile_box, sizeof(int32_t) * h->L.tile_box.size())) != hipSuccess ||
      (e = hipMalloc(&h->d_rch_box, sizeof(int32_t) * h->L.rch_box.size())) != hipSuccess ||
      (e = hipMalloc(&h->d_part, sizeof(double) * kNPart * h->L.rch_box.size())) != hipSuccess ||
      (e = hipMalloc(&h->d_diag, sizeof(double) * kNPart * (size_t)n_boxes)) != hipSuccess ||
      (e = hipMalloc(&h->d_centre, sizeof(double) * 3 * (size_t)n_boxes)) != hipSuccess ||
      (e = hipMalloc(&h->d_out, sizeof(double) * CGLBM_NDIAG * (size_t)n_boxes)) != hipSuccess ||
      (e = hipMemcpyAsync(h->d_rch_box, h->L.rch_box.data(),
                          sizeof(int32_t) * h->L.rch_box.size(), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMalloc(&h->d_ccol_tiles, sizeof(TileEntry) * h->L.ccol_tiles.size())) !=
          hipSuccess ||
      (e = hipMemcpyAsync(h->d_ccol_tiles, h->L.ccol_tiles.data(),
                          sizeof(TileEntry) * h->L.ccol_tiles.size(), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(h->d_boxes, h->L.boxes.data(), sizeof(BoxDev) * n_boxes,
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(h->d_blk_box, h->L.blk_box.data(),
                          sizeof(int32_t) * h->L.blk_box.size(), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(h->d_tile_box, h->L.tile_box.data(),
                          sizeof(int32_t) * h->L.tile_box.size(), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming)) != hipSuccess) {
    return cleanup(fail(CGLBM_EHIP, "init: %s", hipGetErrorString(e)));
  }
  if ((rc = scratch_lookup(h->device))) return cleanup(rc);
  if (h->L.walls) {
    // wall stashes: the in-place layout's, or the compact schedule's pair
    // (the compact schedule of the 16-bit storages keeps its stashes in the
    // mass-exact FP32 format)
    size_t sb = 0, ab = 0, csb = 0;
    buffer_sizes(storage, h->L.wtotal, &sb, &ab, lattice);
    buffer_sizes(storage_16bit(storage) ? CGLBM_FP32_EXACT : storage, h->L.wtotal, &csb, &ab,
                 lattice);
    const bool cst = lattice == LATTICE_D3Q27 && !inplace;
    if ((e = hipMalloc(&h->d_wblk_box, sizeof(int32_t) * h->L.wblk_box.size())) != hipSuccess ||
        (e = hipMemcpyAsync(h->d_wblk_box, h->L.wblk_box.data(),
                            sizeof(int32_t) * h->L.wblk_box.size(), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (inplace && (e = hipMalloc(&h->stash, sb)) != hipSuccess) ||
        (cst && ((e = hipMalloc(&h->cstash[0], csb)) != hipSuccess ||
                 (e = hipMalloc(&h->cstash[1], csb)) != hipSuccess)))
      return cleanup(fail(CGLBM_EHIP, "init: %s", hipGetErrorString(e)));
  }
  if ((rc = select_variant(h, 0, s))) return cleanup(rc);
  // the stored state lives in pop[0]
  h->cur = 0;
  if (lattice == LATTICE_D2Q9)
    hipLaunchKernelGGL(kInit2[storage2_slot(storage)], dim3(h->L.nblk), dim3(kBlock), 0, s,
                       h->d_boxes, h->d_blk_box, init_rho_r, init_rho_b, init_u, h->pop[0],
                       h->L.total, noise_seed, (float)noise_amp);
  else
    hipLaunchKernelGGL(kInit[storage], dim3(h->L.nblk), dim3(kBlock), 0, s, h->d_boxes,
                       h->d_blk_box, init_rho_r, init_rho_b, init_u, h->pop[0], h->L.total,
                       noise_seed, (float)noise_amp);
  if ((rc = check_launch())) return cleanup(rc);
  *out = h;
  return CGLBM_OK;
}

}  // namespace

extern "C" {

int cglbm_step(cglbm_handle *h, int32_t n_steps, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (n_steps < 0) return fail(CGLBM_EINVAL, "n_steps must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  if (effective_schedule(h) == 2) return step_compact(h, n_steps, s);
  if (h->clive) {
    const int rc = flush_compact(h, s);
    if (rc) return rc;
  }
  int32_t k = 0;
  if (h->use_graph && !h->prof && n_steps >= 2) {
    if (!h->graph[h->cur]) {
      const int rc = capture_pair(h);
      if (rc) return rc;
    }
    for (; k + 1 < n_steps; k += 2) HIP_TRY(hipGraphLaunch(h->graph[h->cur], s));
  }
  for (; k < n_steps; ++k) {
    const int rc = launch_step(h, s);
    if (rc) return rc;
  }
  return CGLBM_OK;
}

int cglbm_set_graph(cglbm_handle *h, int32_t enable) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (enable != 0 && enable != 1) return fail(CGLBM_EINVAL, "enable must be 0 or 1");
  h->use_graph = enable;
  return CGLBM_OK;
}

int cglbm_moments(cglbm_handle *h, int32_t box, uint32_t field_mask, float *out_dev,
                  void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (box < 0 || box >= h->n_boxes) return fail(CGLBM_EINVAL, "box %d out of range", box);
  if (field_mask == 0 || (field_mask >> 17)) return fail(CGLBM_EINVAL, "bad field mask 0x%x", field_mask);
  if (!out_dev) return fail(CGLBM_EINVAL, "out_dev must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  int rc = compute_fields(h, s, (field_mask >> 10) & 1u);
  if (rc) return rc;
  const int64_t n = h->L.boxes[box].n;
  hipLaunchKernelGGL(k_fields, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     h->d_boxes, box, h->aux, h->L.total, field_mask, out_dev);
  return check_launch();
}

int cglbm_reduce(cglbm_handle *h, const double *centre, double *out, int32_t out_is_host,
                 void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (!out) return fail(CGLBM_EINVAL, "out must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  const double *dc = nullptr;  // NULL: the kernels use each box's centre
  if (centre) {
    HIP_TRY(hipMemcpyAsync(h->d_centre, centre, sizeof(double) * 3 * (size_t)h->n_boxes,
                           hipMemcpyHostToDevice, s));
    dc = h->d_centre;
  }
  double *dout = out_is_host ? h->d_out : out;
  int rc = reduce_launch(h, s, dc, h->d_part, h->d_diag, dout);
  if (rc) return rc;
  if (!out_is_host) return CGLBM_OK;
  HIP_TRY(hipMemcpyAsync(out, h->d_out, sizeof(double) * CGLBM_NDIAG * (size_t)h->n_boxes,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int b = 0; b < h->n_boxes; ++b)
    if (out[(size_t)b * CGLBM_NDIAG + 12] != 0.0)
      return fail(CGLBM_EUNSTABLE, "non-finite values in the state");
  return CGLBM_OK;
}

int cglbm_reduce_noalloc(cglbm_handle *h, const double *centre, double *out, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (!out) return fail(CGLBM_EINVAL, "out must not be NULL");
  if (h->L.rch_box.size() > kScratchChunks || (size_t)h->n_boxes > kScratchBoxes)
    return fail(CGLBM_EINVAL,
                "%zu reduction chunks of %lld nodes and %d boxes exceed the static scratch "
                "(at most %zu chunks and %zu boxes): use cglbm_reduce",
                h->L.rch_box.size(), (long long)kRedChunk, h->n_boxes, kScratchChunks,
                kScratchBoxes);
  double *sp = h->device >= 0 && h->device < kMaxDevices ? g_scratch[h->device] : nullptr;
  if (!sp) return fail(CGLBM_ESTATE, "scratch of device %d was not looked up", h->device);
  return reduce_launch(h, (hipStream_t)stream, centre, sp, sp + kScratchChunks * kNPart, out);
}

int cglbm_set_schedule(cglbm_handle *h, int32_t schedule) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (schedule < 0 || schedule > 2) return fail(CGLBM_EINVAL, "unknown schedule %d", schedule);
  if (schedule != 0 && h->lattice == LATTICE_D2Q9)
    return fail(CGLBM_EUNSUPPORTED, "D2Q9 steps have one schedule (0)");
  if (schedule == 2 && !compact_ok(h))
    return fail(CGLBM_EUNSUPPORTED,
                "the compact schedule needs D3Q27, FP32 storage (or a mass-exact FP32 or "
                "16-bit storage with Model D and Q), two buffers and unit higher-order rates");
  if (h->clive) {
    const int rc = flush_compact(h, h->cstream);
    if (rc) return rc;
  }
  if (schedule != h->schedule) drop_graphs(h);
  h->schedule = schedule;
  // the fused geometry preferred by the schedule (the autotuner's choices);
  // work still running on any stream may read the column tables, so the
  // device is synchronized before they are replaced
  if (h->lattice == LATTICE_D3Q27) {
    const int32_t v = schedule == 2 ? h->fvar_compact : h->fvar_pop;
    const int32_t m = schedule == 2 ? h->wmode_compact : h->wmode_pop;
    if (v != h->variant || m != h->wmode) {
      HIP_TRY(hipDeviceSynchronize());
      return select_mode(h, v, m, nullptr);
    }
  }
  return CGLBM_OK;
}

int cglbm_get_schedule(const cglbm_handle *h) { return h ? effective_schedule(h) : -1; }

int cglbm_num_variants(void) { return kNumFused; }

int cglbm_variant_info(int32_t v, int32_t *info) {
  g_err.clear();
  if (v < 0 || v >= kNumFused || !info) return fail(CGLBM_EINVAL, "bad variant %d", v);
  info[0] = fused_variant(v).tx;
  info[1] = fused_variant(v).ty;
  info[2] = fused_variant(v).zc;
  info[3] = fused_variant(v).minw;
  return CGLBM_OK;
}

int cglbm_variant_info_d2q9(int32_t v, int32_t *info) {
  g_err.clear();
  if (v < 0 || v >= kNumV2 || !info) return fail(CGLBM_EINVAL, "bad D2Q9 variant %d", v);
  info[0] = variant2(v).tx;
  info[1] = variant2(v).ty;
  return CGLBM_OK;
}

int cglbm_set_variant(cglbm_handle *h, int32_t v, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  const int nv = h->lattice == LATTICE_D2Q9 ? kNumV2 : kNumFused;
  if (v < 0 || v >= nv) return fail(CGLBM_EINVAL, "variant %d out of range", v);
  if (h->clive) {
    const int rc = flush_compact(h, h->cstream);
    if (rc) return rc;
  }
  h->fvar_pop = h->fvar_compact = v;
  return select_variant(h, v, (hipStream_t)stream);
}

int cglbm_get_variant(const cglbm_handle *h) { return h ? h->variant : -1; }

int cglbm_set_wall_mode(cglbm_handle *h, int32_t mode, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (h->lattice != LATTICE_D3Q27) return fail(CGLBM_EUNSUPPORTED, "D2Q9 has no wall modes");
  if (mode < 0 || mode > 3) return fail(CGLBM_EINVAL, "wall mode %d out of range", mode);
  if (h->clive) {
    const int rc = flush_compact(h, h->cstream);
    if (rc) return rc;
  }
  h->wmode_pop = h->wmode_compact = mode;
  return select_mode(h, h->variant, mode, (hipStream_t)stream);
}

int cglbm_get_wall_mode(const cglbm_handle *h) { return h ? h->wmode : -1; }

int cglbm_set_compact_variant(cglbm_handle *h, int32_t v, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (v < 0 || v >= kNumCPull) return fail(CGLBM_EINVAL, "compact variant %d out of range", v);
  if (h->clive) {
    const int rc = flush_compact(h, h->cstream);
    if (rc) return rc;
  }
  return select_cvariant(h, v, (hipStream_t)stream);
}

int cglbm_set_resident(cglbm_handle *h, int32_t enable, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (enable != 0 && enable != 1) return fail(CGLBM_EINVAL, "enable must be 0 or 1, not %d", enable);
  h->resident = enable == 1;
  return enable ? CGLBM_OK : flush_compact(h, (hipStream_t)stream);
}

int cglbm_get_resident(const cglbm_handle *h) { return h ? (h->resident ? 1 : 0) : -1; }

int cglbm_sync_state(cglbm_handle *h, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  return flush_compact(h, (hipStream_t)stream);
}

int cglbm_compact_variant(const cglbm_handle *h, int32_t *info) {
  if (!h) return -1;
  if (info) {
    const CPullVariant &C = cpull_variant(h->cvariant);
    info[0] = C.tx;
    info[1] = C.ty;
    info[2] = C.zc;
  }
  return h->cvariant;
}

int cglbm_autotune(cglbm_handle *h, int32_t reps, double *ms_per_variant, void *stream) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (reps < 1) return fail(CGLBM_EINVAL, "reps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  if (h->lattice == LATTICE_D2Q9) return autotune2(h, reps, ms_per_variant, s);
  if (h->clive) {
    const int rc = flush_compact(h, s);
    if (rc) return rc;
  }
  // the fused kernel is idempotent for a fixed pull: time every variant on
  // the same inputs; the stored state is unchanged afterwards (in place, the
  // variants all write the next state into the one buffer: the call then
  // advances the state by exactly one step)
  int rc = launch_pull(h, s, 1);
  if (rc || (rc = check_launch())) return rc;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = h->variant;
  double best_ms = 1e300;
  for (int v = 0; v < kNumFused; ++v) {
    if ((rc = select_variant(h, v, s))) break;
    if ((rc = launch_fused(h, s, 0))) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && !rc; ++r) rc = launch_fused(h, s, 0);
    (void)hipEventRecord(e1, s);
    if (rc || (rc = check_launch())) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(CGLBM_EHIP, "autotune: event synchronize failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double avg = (double)ms / reps;
    if (ms_per_variant) ms_per_variant[v] = avg;
    if (avg < best_ms) {
      best_ms = avg;
      best = v;
    }
  }
  // the compact schedule's fused kernel on the same inputs (it writes
  // compact states into the other buffer only): its own best geometry
  int cfbest = best;
  if (!rc && compact_ok(h) && !h->L.general) {
    double cf_ms = 1e300;
    for (int v = 0; v < kNumFused && !rc; ++v) {
      if ((rc = select_variant(h, v, s)) || (rc = launch_fused_compact(h, s))) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && !rc; ++r) rc = launch_fused_compact(h, s);
      (void)hipEventRecord(e1, s);
      if (!rc) rc = check_launch();
      if (!rc && hipEventSynchronize(e1) != hipSuccess)
        rc = fail(CGLBM_EHIP, "autotune: event synchronize failed");
      if (rc) break;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if ((double)ms / reps < cf_ms) {
        cf_ms = (double)ms / reps;
        cfbest = v;
      }
    }
  }
  h->fvar_pop = best;
  h->fvar_compact = cfbest;
  // the three-kernel schedule on the same inputs (its interface and collide
  // kernels are idempotent for a fixed pull as well)
  double three_ms = 1e300;
  if (!rc) rc = select_variant(h, best, s);
  if (!rc && !(rc = launch_iface(h, s, 0)) && !(rc = launch_collide(h, s))) {
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && !rc; ++r) {
      rc = launch_iface(h, s, 0);
      if (!rc) rc = launch_collide(h, s);
    }
    (void)hipEventRecord(e1, s);
    if (!rc) rc = check_launch();
    if (!rc && hipEventSynchronize(e1) != hipSuccess)
      rc = fail(CGLBM_EHIP, "autotune: event synchronize failed");
    if (!rc) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      three_ms = (double)ms / reps;
      if (ms_per_variant) ms_per_variant[kNumFused] = three_ms;
    }
  }
  // the compact schedule's pull geometry: the compact state the fused kernel
  // writes into the other buffer from the same pull, then each k_cpull
  // variant on it (both write only that buffer and aux)
  if (!rc && compact_ok(h) && !(rc = select_variant(h, cfbest, s)) &&
      !(rc = launch_compact_collide(h, s))) {
    int cbest = h->cvariant;
    double cbest_ms = 1e300;
    for (int v = 0; v < kNumCPull && !rc; ++v) {
      if ((rc = select_cvariant(h, v, s)) || (rc = launch_cpull(h, s))) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && !rc; ++r) rc = launch_cpull(h, s);
      (void)hipEventRecord(e1, s);
      if (!rc) rc = check_launch();
      if (!rc && hipEventSynchronize(e1) != hipSuccess)
        rc = fail(CGLBM_EHIP, "autotune: event synchronize failed");
      if (rc) break;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if ((double)ms / reps < cbest_ms) {
        cbest_ms = (double)ms / reps;
        cbest = v;
      }
    }
    if (!rc) rc = select_cvariant(h, cbest, s);
  }
  // boxes with walls: the wall mode of each schedule with its chosen
  // geometries, timed as the steps run (replays of a captured graph of two
  // launches): the fused kernel alone for the population schedule (its pull
  // does not depend on the mode; layouts with the three-kernel schedule have
  // no tiled launch there), k_cpull with the compact collision for the
  // compact one (which advance only the compact state in the other buffer)
  for (int cmp = 0; cmp < 2 && !rc && h->L.walls && !h->inplace; ++cmp) {
    if (cmp ? !compact_ok(h) : h->L.general) continue;
    auto launch = [&](hipStream_t cs, int k) {
      int r = cmp ? launch_cpull(h, cs, k) : CGLBM_OK;
      if (!r) r = cmp ? launch_compact_collide(h, cs) : launch_fused(h, cs, 0);
      return r;
    };
    int32_t mbest = cmp ? h->wmode_compact : h->wmode_pop;
    double mbest_ms = 1e300;
    for (int32_t m = 0; m < 4 && !rc; ++m) {
      double ms = 0.0;
      if ((rc = select_mode(h, cmp ? cfbest : best, m, s)) ||
          (rc = time_graph(h, s, reps, e0, e1, launch, ms)))
        break;
      if (ms < mbest_ms) {
        mbest_ms = ms;
        mbest = m;
      }
    }
    (cmp ? h->wmode_compact : h->wmode_pop) = mbest;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (!rc) rc = select_mode(h, best, h->wmode_pop, s);
  if (rc) return rc;
  const int32_t sched = three_ms < best_ms ? 1 : 0;
  if (sched != h->schedule) drop_graphs(h);
  h->schedule = sched;
  if (h->inplace) h->cur = 1 - h->cur;
  return CGLBM_OK;
}

int cglbm_profile_begin(cglbm_handle *h, int32_t max_launches) {
  g_err.clear();
  if (!h) return fail(CGLBM_ESTATE, "null handle");
  if (max_launches <= 0) return fail(CGLBM_EINVAL, "max_launches must be > 0");
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.assign(2 * (size_t)max_launches, nullptr);
  h->ev_kind.assign((size_t)max_launches, -1);
  for (auto &e : h->ev) HIP_TRY(hipEventCreate(&e));
  h->ev_used = 0;
  h->prof = true;
  return CGLBM_OK;
}

int cglbm_profile_end(cglbm_handle *h, double *total_ms, int64_t *launches, int32_t n_kinds) {
  g_err.clear();
  if (!h || !h->prof) return fail(CGLBM_ESTATE, "profiling was not started");
  h->prof = false;
  std::vector<double> ms(KIND_N, 0.0);
  std::vector<int64_t> cnt(KIND_N, 0);
  for (size_t k = 0; k < h->ev_used / 2; ++k) {
    HIP_TRY(hipEventSynchronize(h->ev[2 * k + 1]));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, h->ev[2 * k], h->ev[2 * k + 1]));
    ms[h->ev_kind[k]] += t;
    cnt[h->ev_kind[k]] += 1;
  }
  for (int k = 0; k < n_kinds && k < KIND_N; ++k) {
    if (total_ms) total_ms[k] = ms[k];
    if (launches) launches[k] = cnt[k];
  }
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  h->ev_kind.clear();
  h->ev_used = 0;
  return CGLBM_OK;
}

void cglbm_destroy(cglbm_handle *h) {
  if (!h) return;
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->d_boxes) (void)hipFree(h->d_boxes);
  if (h->d_blk_box) (void)hipFree(h->d_blk_box);
  if (h->d_tile_box) (void)hipFree(h->d_tile_box);
  if (h->d_col_box) (void)hipFree(h->d_col_box);
  if (h->d_col_tiles) (void)hipFree(h->d_col_tiles);
  if (h->d_part) (void)hipFree(h->d_part);
  if (h->d_rch_box) (void)hipFree(h->d_rch_box);
  if (h->d_out) (void)hipFree(h->d_out);
  if (h->d_diag) (void)hipFree(h->d_diag);
  if (h->d_centre) (void)hipFree(h->d_centre);
  if (h->stash) (void)hipFree(h->stash);
  for (void *p : h->cstash)
    if (p) (void)hipFree(p);
  if (h->d_wblk_box) (void)hipFree(h->d_wblk_box);
  if (h->d_ccol_tiles) (void)hipFree(h->d_ccol_tiles);
  delete h;
}

}  // extern "C"
