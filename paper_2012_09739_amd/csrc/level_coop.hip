// Single-level calls of a nested binary32 estimator or of the plain binary64 one with few,
// long chunks: one block of eight waves per chunk (cooperative chunks, coop.h) instead of one
// wave per chunk.  A deep level
// with a few thousand paths has too few chunks to fill the GPU, and a wave alone runs its
// chunk's 2^l dependent steps latency bound; seven producer waves drawing the variables ahead
// of the consumer cut that chain to the consumer's updates.  The consumer performs the
// single-wave code's operations in the same order and writes the same partial row, so the
// sums keep their bits.
#include <hip/hip_runtime.h>

#include "coop.h"
#include "internal.h"
#include "level_kernel.h"

namespace mlmc {

namespace {

constexpr int kCoopWaves = 8;

// One block per chunk (partial row: one chunk from level 2 for the nested estimators).
template <int RV, bool KAHAN>
__global__ __launch_bounds__(kCoopWaves * kWave) __attribute__((amdgpu_waves_per_eu(4))) void level_coop_kernel(
    const LevelParams prm) {
    constexpr bool kExactOnly = RV == MLMC_RV_EXACT;
    constexpr int DEG = RV == MLMC_RV_CUBIC16 ? 3 : 1;
    constexpr int kSteps = Coop<kCoopWaves>::kSteps;
    __shared__ float s_tab32[kExactOnly ? 1 : kTableRowsDev * (DEG + 1)];
    __shared__ __align__(16) unsigned char s_ex_raw[sizeof(ExactCols)];
    __shared__ double ring_x[2][kSteps][kWave];
    __shared__ float ring_b[kExactOnly ? 1 : 2][kSteps][kWave];
    if constexpr (!kExactOnly)
        for (int i = threadIdx.x; i < kTableRowsDev * (DEG + 1); i += blockDim.x)
            s_tab32[i] = prescaled_coeff(((const float*)prm.table)[i], i % (DEG + 1));
    stage_exact_table(s_ex_raw, prm.exact_tab, sizeof(ExactCols));
    __syncthreads();
    run_chunk_coop<RV, KAHAN, kCoopWaves>(prm, blockIdx.x, s_tab32, (const ExactLds*)s_ex_raw, ring_x, ring_b);
}

template <int RV>
hipError_t go(const LevelParams& p, uint64_t n_chunks, bool kahan, hipStream_t s) {
    if (kahan)
        hipLaunchKernelGGL((level_coop_kernel<RV, true>), dim3((uint32_t)n_chunks), dim3(kCoopWaves * kWave), 0, s, p);
    else
        hipLaunchKernelGGL((level_coop_kernel<RV, false>), dim3((uint32_t)n_chunks), dim3(kCoopWaves * kWave), 0, s, p);
    return hipGetLastError();
}

}  // namespace

bool coop_level_call(const Variant& v, int level, uint64_t n_rows, int n_cu) {
    const bool nested32 = v.precision == MLMC_FP32 && v.nested && (v.rv == MLMC_RV_PWL16 || v.rv == MLMC_RV_CUBIC16);
    const bool plain64 = v.precision == MLMC_FP64 && !v.nested && v.rv == MLMC_RV_EXACT;
    return (nested32 || plain64) && !v.diag && v.scheme == MLMC_SCHEME_EM && level >= kCoopMinLevel && n_rows > 0 &&
           n_rows <= (uint64_t)kCoopMaxRowsPerCu * (uint64_t)n_cu;
}

hipError_t launch_level_coop(const Variant& v, const LevelParams& p, uint64_t n_rows, hipStream_t s) {
    if (v.rv == MLMC_RV_EXACT) return go<MLMC_RV_EXACT>(p, n_rows, false, s);
    return v.rv == MLMC_RV_CUBIC16 ? go<MLMC_RV_CUBIC16>(p, n_rows, v.kahan, s) : go<MLMC_RV_PWL16>(p, n_rows, v.kahan, s);
}

}  // namespace mlmc
