// fused_tab2.hip -- part 2 of the fused kernel's launch-geometry table (tables.hpp).
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace cglbm {
const FusedVariant kFusedPart2[5] = {CGLBM_FV(32, 8, 32, 5), CGLBM_FV(64, 8, 64, 4), CGLBM_FV(64, 8, 32, 4),
                                     CGLBM_FV(64, 16, 64, 4), CGLBM_FV(64, 16, 32, 4)};
}  // namespace cglbm
