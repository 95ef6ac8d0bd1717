// fused_tab0.hip -- part 0 of the fused kernel's launch-geometry table (tables.hpp).
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace cglbm {
const FusedVariant kFusedPart0[4] = {CGLBM_FV(32, 8, 32, 4), CGLBM_FV(32, 8, 64, 4), CGLBM_FV(32, 8, 16, 4), CGLBM_FV(32, 8, 32, 1)};
}  // namespace cglbm
