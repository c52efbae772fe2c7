// Launch dispatch of the level kernel: the template instance for a variant, for one
// precision and one time-stepping scheme (each .hip file instantiates one pair, so the
// instances compile in parallel).
#pragma once
#include "level_kernel.h"

namespace mlmc {
namespace launch_detail {

template <int PREC, int SCHEME, int RV, bool NESTED, bool KAHAN, bool DIAG>
hipError_t go(const LevelParams& p, int grid, int block, hipStream_t s) {
    if (p.n_steps < 4) {  // levels 0 and 1: calls shared by paths
        hipLaunchKernelGGL((level_kernel<PREC, RV, NESTED, KAHAN, DIAG, true, SCHEME>), dim3(grid), dim3(block), 0, s, p);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((level_kernel<PREC, RV, NESTED, KAHAN, DIAG, false, SCHEME>), dim3(grid), dim3(block), 0, s, p);
    return hipGetLastError();
}

template <int PREC, int SCHEME, int RV>
hipError_t by_flags(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s) {
    const int f = (v.nested ? 4 : 0) | (v.kahan ? 2 : 0) | (v.diag ? 1 : 0);
    switch (f) {
        case 0: return go<PREC, SCHEME, RV, false, false, false>(p, grid, block, s);
        case 1: return go<PREC, SCHEME, RV, false, false, true>(p, grid, block, s);
        case 2: return go<PREC, SCHEME, RV, false, true, false>(p, grid, block, s);
        case 3: return go<PREC, SCHEME, RV, false, true, true>(p, grid, block, s);
        case 4: return go<PREC, SCHEME, RV, true, false, false>(p, grid, block, s);
        case 5: return go<PREC, SCHEME, RV, true, false, true>(p, grid, block, s);
        case 6: return go<PREC, SCHEME, RV, true, true, false>(p, grid, block, s);
        default: return go<PREC, SCHEME, RV, true, true, true>(p, grid, block, s);
    }
}

}  // namespace launch_detail

// The instance of variant v.  The plain exact estimator exists in binary64 only, the MLP
// variable only where kWithMlp (Euler-Maruyama in the IEEE formats); the library validates
// variants before dispatch, so the remaining cases report an invalid value.
template <int PREC, int SCHEME, bool kWithMlp>
hipError_t launch_level_for(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s) {
    using namespace launch_detail;
    switch (v.rv) {
        case MLMC_RV_EXACT:
            if constexpr (PREC == MLMC_FP64) return go<PREC, SCHEME, MLMC_RV_EXACT, false, false, false>(p, grid, block, s);
            return hipErrorInvalidValue;
        case MLMC_RV_PWL16: return by_flags<PREC, SCHEME, MLMC_RV_PWL16>(v, p, grid, block, s);
        case MLMC_RV_CUBIC16: return by_flags<PREC, SCHEME, MLMC_RV_CUBIC16>(v, p, grid, block, s);
        case MLMC_RV_PCONST4096: return by_flags<PREC, SCHEME, MLMC_RV_PCONST4096>(v, p, grid, block, s);
        case MLMC_RV_MLP:
            if constexpr (kWithMlp) return by_flags<PREC, SCHEME, MLMC_RV_MLP>(v, p, grid, block, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mlmc
