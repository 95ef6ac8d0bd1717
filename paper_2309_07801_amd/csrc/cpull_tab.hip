// cpull_tab.hip -- launch-geometry table of the compact schedule's pull (tables.hpp).
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace cglbm {
#define CV_M(TX, TY, ZC, G)                                                              \
  {k_cpull<TX, TY, ZC, false, StoreF32, G>, k_cpull<TX, TY, ZC, true, StoreF32, G>,      \
   k_cpull<TX, TY, ZC, true, StoreF32P, G>}
#define CV(TX, TY, ZC)                                                                   \
  {TX, TY, ZC, {CV_M(TX, TY, ZC, false), CV_M(TX, TY, ZC, true)},                        \
   {k_cpull<TX, TY, ZC, false, StoreF32X, false>, k_cpull<TX, TY, ZC, true, StoreF32X, false>}}
const CPullVariant kCPullTable[5] = {CV(64, 8, 64), CV(64, 8, 32), CV(32, 8, 32), CV(64, 4, 32),
                                     CV(32, 8, 64)};
#undef CV
#undef CV_M
}  // namespace cglbm
