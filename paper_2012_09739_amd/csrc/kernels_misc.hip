// Chunk-partial reduction and the parity-check kernels (uniform words, inverse CDF values).
#include <hip/hip_runtime.h>

#include "icdf.h"
#include "internal.h"
#include "mlp.h"
#include "philox.h"
#include "reduce.h"

namespace mlmc {

namespace {

// The two stages of the fixed-order reduction of n_rows rows of 8 chunk partials (the
// tree of reduce_stage1 / reduce_stage2).  The order depends only on n_rows, so results do
// not depend on the level kernel's launch shape, and the batched sweep, which runs the same
// stages per item, reproduces the single-level sums bit for bit.
__global__ __launch_bounds__(kReduceBlock) void reduce_chunks_stage1(const double* __restrict__ partials,
                                                                     uint64_t n_rows, double* __restrict__ stage) {
    __shared__ double s[kPartial][kReduceBlock];
    reduce_stage1(partials, n_rows, stage, blockIdx.x, s);
}

__global__ __launch_bounds__(kReduceBlock) void reduce_chunks_stage2(const double* __restrict__ stage,
                                                                     uint64_t n_rows, double* __restrict__ out) {
    __shared__ double s[kPartial][kReduceBlock];
    reduce_stage2(stage, n_rows, out, s);
}

__global__ void uniforms_kernel(uint32_t k0, uint32_t k1, uint32_t ctr2, uint32_t pset, uint64_t path0,
                                uint64_t n_paths, uint32_t n_steps, uint32_t* __restrict__ words) {
    const uint32_t level = ctr2 & 0xFFFFu;
    if (level < 2) {
        // one call per G = 4 >> level consecutive paths (n_steps <= 2^level, checked by the host)
        const uint32_t shift = 2 - level;
        for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_paths;
             p += (uint64_t)gridDim.x * blockDim.x) {
            const uint64_t gp = path0 + p;
            const Words4 r = philox4x32_10<0>(0u, (uint32_t)(gp >> shift), ctr2, pset, k0, k1);
            const uint32_t first = ((uint32_t)gp & ((1u << shift) - 1u)) << level;
            for (uint32_t n = 0; n < n_steps; ++n) words[p * n_steps + n] = r.w[first + n];
        }
        return;
    }
    const uint64_t n_calls = (n_steps + 3) / 4;
    const uint64_t total = n_paths * n_calls;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = g / n_calls;
        const uint32_t q = (uint32_t)(g % n_calls);
        const Words4 r = philox4x32_10<0>(q, (uint32_t)(path0 + p), ctr2, pset, k0, k1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t n = 4 * q + i;
            if (n < n_steps) words[p * n_steps + n] = r.w[i];
        }
    }
}

template <int RV, int PREC>
__global__ void icdf_kernel(const uint32_t* __restrict__ words, uint64_t n, const void* table,
                            const void* mlp, const ExactTable* __restrict__ ex, double* __restrict__ out) {
    constexpr int DEG = RV == MLMC_RV_CUBIC16 ? 3 : 1;
    // whole wavefronts step together (the learned variable uses matrix instructions): lanes
    // past the end evaluate word 0 and store nothing
    const uint64_t lane = threadIdx.x & (kWave - 1);
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < n;
         base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t g = base + lane;
        const uint32_t w = g < n ? words[g] : 0u;
        double z;
        if constexpr (RV == MLMC_RV_EXACT) {
            z = icdf_exact_f64(w, &ex->lds.top, ex->deep);
        } else if constexpr (RV == MLMC_RV_PCONST4096) {
            if constexpr (PREC == MLMC_FP64) z = icdf_pconst_f64(w, (const double*)table);
            else if constexpr (PREC == MLMC_FP16) z = (double)__half2float(icdf_pconst_f16(w, (const __half*)table));
            else z = (double)icdf_pconst_f32(w, (const float*)table);
        } else if constexpr (RV == MLMC_RV_MLP) {
            const float y = icdf_mlp_f32(w, (const float*)mlp);
            if constexpr (PREC == MLMC_FP16) z = (double)__half2float(__float2half_rn(y));
            else z = (double)y;
        } else if constexpr (PREC == MLMC_FP64) {
            z = icdf_dyadic_f64<DEG>(w, (const double*)table);
        } else if constexpr (PREC == MLMC_FP32) {
            z = (double)icdf_dyadic_f32<DEG>(w, (const float*)table);
        } else if constexpr (PREC == MLMC_BF16) {
            z = (double)icdf_dyadic_bf16<DEG>(w, (const float*)table);
        } else {
            z = (double)__half2float(icdf_dyadic_f16<DEG>(w, (const __half*)table));
        }
        if (g < n) out[g] = z;
    }
}

int grid_for(uint64_t n, int block) {
    const uint64_t g = (n + block - 1) / block;
    return (int)(g < 65536 ? (g == 0 ? 1 : g) : 65536);
}

}  // namespace

// With one stage block (at most 64 rows) that block writes the result itself: the second stage
// would add its one row to zeros and return it unchanged (a sum that starts at +0 is never -0),
// so the bits are those of the two-kernel tree with one launch fewer.
hipError_t launch_reduce(const double* partials, uint64_t n_rows, double* stage, double* d_out, hipStream_t s) {
    const uint32_t R = stage_blocks(n_rows);
    hipLaunchKernelGGL(reduce_chunks_stage1, dim3(R), dim3(kReduceBlock), 0, s, partials, n_rows, R == 1 ? d_out : stage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || R == 1) return e;
    hipLaunchKernelGGL(reduce_chunks_stage2, dim3(1), dim3(kReduceBlock), 0, s, stage, n_rows, d_out);
    return hipGetLastError();
}

hipError_t launch_uniforms(uint64_t seed, uint32_t ctr2, uint32_t pset, uint64_t path0, uint64_t n_paths,
                           uint32_t n_steps, uint32_t* d_words, hipStream_t s) {
    const uint64_t total = n_paths * ((n_steps + 3) / 4);
    hipLaunchKernelGGL(uniforms_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, (uint32_t)seed,
                       (uint32_t)(seed >> 32), ctr2, pset, path0, n_paths, n_steps, d_words);
    return hipGetLastError();
}

hipError_t launch_icdf(const uint32_t* d_words, uint64_t n, int rv, int precision, const void* table,
                       const void* mlp, const void* exact_tab, double* d_out, hipStream_t s) {
    const ExactTable* ex = (const ExactTable*)exact_tab;
    const dim3 g(grid_for(n, 256)), b(256);
#define MLMC_ICDF_CASE(R, P) \
    if (rv == R && precision == P) { \
        hipLaunchKernelGGL((icdf_kernel<R, P>), g, b, 0, s, d_words, n, table, mlp, ex, d_out); \
        return hipGetLastError(); \
    }
    if (rv == MLMC_RV_EXACT) {
        hipLaunchKernelGGL((icdf_kernel<MLMC_RV_EXACT, MLMC_FP64>), g, b, 0, s, d_words, n, table, mlp, ex, d_out);
        return hipGetLastError();
    }
    MLMC_ICDF_CASE(MLMC_RV_PWL16, MLMC_FP64)
    MLMC_ICDF_CASE(MLMC_RV_PWL16, MLMC_FP32)
    MLMC_ICDF_CASE(MLMC_RV_PWL16, MLMC_FP16)
    MLMC_ICDF_CASE(MLMC_RV_PWL16, MLMC_BF16)
    MLMC_ICDF_CASE(MLMC_RV_CUBIC16, MLMC_FP64)
    MLMC_ICDF_CASE(MLMC_RV_CUBIC16, MLMC_FP32)
    MLMC_ICDF_CASE(MLMC_RV_CUBIC16, MLMC_FP16)
    MLMC_ICDF_CASE(MLMC_RV_CUBIC16, MLMC_BF16)
    MLMC_ICDF_CASE(MLMC_RV_PCONST4096, MLMC_FP64)
    MLMC_ICDF_CASE(MLMC_RV_PCONST4096, MLMC_FP32)
    MLMC_ICDF_CASE(MLMC_RV_PCONST4096, MLMC_FP16)
    MLMC_ICDF_CASE(MLMC_RV_PCONST4096, MLMC_BF16)
    MLMC_ICDF_CASE(MLMC_RV_MLP, MLMC_FP64)
    MLMC_ICDF_CASE(MLMC_RV_MLP, MLMC_FP32)
    MLMC_ICDF_CASE(MLMC_RV_MLP, MLMC_FP16)
#undef MLMC_ICDF_CASE
    return hipErrorInvalidValue;
}

}  // namespace mlmc
