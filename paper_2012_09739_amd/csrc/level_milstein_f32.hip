// Level kernel instances for precision MLMC_FP32, Milstein (exact and dyadic variables).
#include "level_launch.h"

namespace mlmc {

hipError_t launch_level_milstein_f32(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s) {
    return launch_level_for<MLMC_FP32, MLMC_SCHEME_MILSTEIN, false>(v, p, grid, block, s);
}

}  // namespace mlmc
