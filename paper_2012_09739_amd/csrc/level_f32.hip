// Template instantiations and launch dispatch of the level kernel for precision MLMC_FP32.
#include "level_kernel.h"

namespace mlmc {

namespace {
template <int RV, bool NESTED, bool KAHAN, bool DIAG>
hipError_t go(const LevelParams& p, int grid, int block, hipStream_t s) {
    if constexpr (NESTED || RV == MLMC_RV_EXACT) {
        if (p.n_steps < 4) {
            hipLaunchKernelGGL((level_kernel<MLMC_FP32, RV, NESTED, KAHAN, DIAG, true>), dim3(grid), dim3(block), 0, s, p);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((level_kernel<MLMC_FP32, RV, NESTED, KAHAN, DIAG>), dim3(grid), dim3(block), 0, s, p);
    return hipGetLastError();
}

template <int RV>
hipError_t by_flags(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s) {
    const int f = (v.nested ? 4 : 0) | (v.kahan ? 2 : 0) | (v.diag ? 1 : 0);
    switch (f) {
        case 0: return go<RV, false, false, false>(p, grid, block, s);
        case 1: return go<RV, false, false, true>(p, grid, block, s);
        case 2: return go<RV, false, true, false>(p, grid, block, s);
        case 3: return go<RV, false, true, true>(p, grid, block, s);
        case 4: return go<RV, true, false, false>(p, grid, block, s);
        case 5: return go<RV, true, false, true>(p, grid, block, s);
        case 6: return go<RV, true, true, false>(p, grid, block, s);
        default: return go<RV, true, true, true>(p, grid, block, s);
    }
}
}  // namespace

hipError_t launch_level_f32(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s) {
    switch (v.rv) {

        case MLMC_RV_PWL16: return by_flags<MLMC_RV_PWL16>(v, p, grid, block, s);
        case MLMC_RV_CUBIC16: return by_flags<MLMC_RV_CUBIC16>(v, p, grid, block, s);
        case MLMC_RV_MLP: return by_flags<MLMC_RV_MLP>(v, p, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mlmc
