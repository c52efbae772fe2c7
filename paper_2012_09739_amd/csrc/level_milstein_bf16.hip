// Level kernel instances for precision MLMC_BF16, Milstein (exact and dyadic variables).
#include "level_launch.h"

namespace mlmc {

hipError_t launch_level_milstein_bf16(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s) {
    return launch_level_for<MLMC_BF16, MLMC_SCHEME_MILSTEIN, false>(v, p, grid, block, s);
}

}  // namespace mlmc
