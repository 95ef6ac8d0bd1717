// d2q9_tab.hip -- tile shapes and initial-state kernels of the two-dimensional
// (D2Q9) model (tables.hpp).
#include <hip/hip_runtime.h>

#include "d2q9.hpp"
#include "tables.hpp"

namespace cglbm {
#define V2_S(S, TX, TY) d2q9::k2_step<S, TX, TY, 256, false>
#define V2_F(S, TX, TY) d2q9::k2_step<S, TX, TY, 256, true>
#define V2(TX, TY)                                                                              \
  {TX, TY,                                                                                      \
   {V2_S(StoreF32P, TX, TY), V2_S(StoreF16, TX, TY), V2_S(StoreBF16, TX, TY),                   \
    V2_S(StoreF32X, TX, TY)},                                                                   \
   {V2_F(StoreF32P, TX, TY), V2_F(StoreF16, TX, TY), V2_F(StoreBF16, TX, TY),                   \
    V2_F(StoreF32X, TX, TY)}}
const Variant2 kVariants2Table[4] = {V2(64, 16), V2(32, 32), V2(64, 8), V2(32, 16)};
#undef V2
#undef V2_S
#undef V2_F
const InitFn kInit2[4] = {d2q9::k2_init<StoreF32P>, d2q9::k2_init<StoreF16>,
                          d2q9::k2_init<StoreBF16>, d2q9::k2_init<StoreF32X>};
}  // namespace cglbm
