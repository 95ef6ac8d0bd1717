// fused_tab1.hip -- part 1 of the fused kernel's launch-geometry table (tables.hpp).
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace cglbm {
const FusedVariant kFusedPart1[4] = {CGLBM_FV(32, 16, 32, 4), CGLBM_FV(32, 16, 64, 4), CGLBM_FV(64, 4, 32, 4), CGLBM_FV(32, 4, 32, 4)};
}  // namespace cglbm
