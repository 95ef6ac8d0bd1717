// tables.hpp -- launch-geometry tables of the templated kernels.
//
// Each table is defined in a translation unit of its own (fused_tab0..2.hip,
// cpull_tab.hip, d2q9_tab.hip), so that the library's many kernel
// instantiations compile in parallel; the host code (cglbm.hip) reaches them
// through the accessors below.  The entries are host-side kernel handles:
// hipLaunchKernel resolves them to the device code of the unit that
// instantiated them.
#pragma once

#include "kernels.hpp"

namespace cglbm {

// Launch geometries of the fused kernel: column extent in x and y, z chunk,
// minimum waves per SIMD requested from the register allocator.  Every
// variant performs the same arithmetic per node (results are bitwise equal);
// cglbm_autotune picks the fastest for the boxes at hand.
using FusedFn = void (*)(const BoxDev *, const TileEntry *, float *, void *, int64_t);
struct FusedVariant {
  int tx, ty, zc, minw;
  FusedFn fn[7][2];  // time step: [storage][0: tiles away from solid layers, 1: near them]
  FusedFn fx[2];     // field export (no population store): [near solid layers]
  FusedFn fc[2];     // compact schedule: compact state out (FP32): [near solid layers]
  FusedFn fcx[2];    // compact schedule, mass-exact storage (FP64 densities): [near solid layers]
};
#define CGLBM_FV_S(TX, TY, ZC, MW, S) \
  {k_fused<TX, TY, ZC, MW, false, S, false>, k_fused<TX, TY, ZC, MW, true, S, false>}
#define CGLBM_FV(TX, TY, ZC, MW)                                                              \
  {TX, TY, ZC, MW,                                                                           \
   {CGLBM_FV_S(TX, TY, ZC, MW, StoreF32), CGLBM_FV_S(TX, TY, ZC, MW, StoreF16),               \
    CGLBM_FV_S(TX, TY, ZC, MW, StoreBF16), CGLBM_FV_S(TX, TY, ZC, MW, StoreF32X),             \
    CGLBM_FV_S(TX, TY, ZC, MW, StoreF32P), CGLBM_FV_S(TX, TY, ZC, MW, StoreF16C),             \
    CGLBM_FV_S(TX, TY, ZC, MW, StoreBF16C)},                                                 \
   {k_fused<TX, TY, ZC, MW, false, StoreF32, true>, k_fused<TX, TY, ZC, MW, true, StoreF32, true>}, \
   {k_fused<TX, TY, ZC, MW, false, StoreF32, false, true>,                                    \
    k_fused<TX, TY, ZC, MW, true, StoreF32, false, true>},                                    \
   {k_fused<TX, TY, ZC, MW, false, StoreF32X, false, true>,                                   \
    k_fused<TX, TY, ZC, MW, true, StoreF32X, false, true>}}
// the thirteen geometries, in three units
extern const FusedVariant kFusedPart0[4];
extern const FusedVariant kFusedPart1[4];
extern const FusedVariant kFusedPart2[5];
constexpr int kNumFusedVariants = 13;
inline const FusedVariant &fused_variant(int v) {
  return v < 4 ? kFusedPart0[v] : (v < 8 ? kFusedPart1[v - 4] : kFusedPart2[v - 8]);
}

// The compact schedule's pull (column tile and z chunk, chosen by the
// autotuner; equal results).
using CPullFn = void (*)(const BoxDev *, const TileEntry *, const float *, float *, int64_t,
                         const void *, void *, int64_t);
struct CPullVariant {
  int tx, ty, zc;
  // [general equilibrium family][0 tiles away from solid layers, 1 tiles near
  // them with FP32 planes, 2 tiles near them with FP32 pairs]
  CPullFn fn[2][3];
  CPullFn fx[2];  // mass-exact storage, Model D with Q: [near solid layers]
};
extern const CPullVariant kCPullTable[5];
constexpr int kNumCPullVariants = 5;
inline const CPullVariant &cpull_variant(int v) { return kCPullTable[v]; }

// Tile shapes of the two-dimensional (D2Q9) step kernel, 256 threads each;
// bitwise equal results, picked by cglbm_autotune.  Kernels per storage slot:
// FP32 pairs (for FP32 and FP32_PAIRS), FP16, BF16, FP32X.
using Step2Fn = void (*)(const BoxDev *, const int32_t *, const void *, void *, float *, int64_t);
struct Variant2 {
  int tx, ty;
  Step2Fn step[4], fields[4];
};
extern const Variant2 kVariants2Table[4];
constexpr int kNumVariants2 = 4;
inline const Variant2 &variant2(int v) { return kVariants2Table[v]; }

// Initial-state kernels (three dimensions in cglbm.hip; D2Q9 per storage slot).
using InitFn = void (*)(const BoxDev *, const int32_t *, const float *, const float *,
                        const float *, void *, int64_t, uint64_t, float);
extern const InitFn kInit2[4];

}  // namespace cglbm
