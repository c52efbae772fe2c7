// Fixed-order block reduction of chunk partial rows (shared by the single-level and the
// batched paths so that both give bit-identical sums).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace mlmc {

constexpr int kReduceBlock = 256;

// blockDim.x must be kReduceBlock.  Row c holds (sum[0..3], sumsq[0..3]) of chunk c.
__device__ __forceinline__ void reduce_rows_block(const double* __restrict__ rows, uint64_t n,
                                                  double* __restrict__ out, double (*s)[kReduceBlock]) {
    double acc[kPartial];
#pragma unroll
    for (int k = 0; k < kPartial; ++k) acc[k] = 0.0;
    // thread t adds rows t, t + B, t + 2B, ... in that order; the loads of kAhead rows are
    // issued before their additions so the loop is not bound by one memory latency per row
    constexpr int kAhead = 16;
    uint64_t c = threadIdx.x;
    for (; c + (uint64_t)(kAhead - 1) * kReduceBlock < n; c += (uint64_t)kAhead * kReduceBlock) {
        double v[kAhead][kPartial];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
#pragma unroll
            for (int k = 0; k < kPartial; ++k) v[u][k] = rows[(c + (uint64_t)u * kReduceBlock) * kPartial + k];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
#pragma unroll
            for (int k = 0; k < kPartial; ++k) acc[k] += v[u][k];
    }
    for (; c < n; c += kReduceBlock) {
#pragma unroll
        for (int k = 0; k < kPartial; ++k) acc[k] += rows[c * kPartial + k];
    }
#pragma unroll
    for (int k = 0; k < kPartial; ++k) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kReduceBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < kPartial; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < kPartial) out[threadIdx.x] = s[threadIdx.x][0];
}

// Two-stage fixed-order reduction of n chunk rows.  Stage 1 runs R = stage_blocks(n) blocks:
// block b sums rows [b per, min(n, (b + 1) per)), per = ceil(n / R), with reduce_rows_block
// into stage row b.  Stage 2 (one block) sums the R stage rows in order.  The tree depends on
// n only, never on the launch or the timing, so every caller with the same rows gets the same
// bits.  The stages are separate kernels: the kernel boundary publishes the stage rows to the
// second stage, where a device-scope fence inside one kernel would have every block write
// back its XCD's L2.
constexpr uint32_t kStageBlocks = (uint32_t)kStageRowsMax;
__host__ __device__ inline uint32_t stage_blocks(uint64_t n) {
    const uint64_t r = (n + 63) / 64;
    return r < 1 ? 1u : (r > kStageBlocks ? kStageBlocks : (uint32_t)r);
}

__device__ __forceinline__ void reduce_stage1(const double* __restrict__ rows, uint64_t n, double* __restrict__ stage,
                                              uint32_t b, double (*s)[kReduceBlock]) {
    const uint32_t R = stage_blocks(n);
    const uint64_t per = (n + R - 1) / R;
    const uint64_t lo = (uint64_t)b * per < n ? (uint64_t)b * per : n;
    const uint64_t hi = lo + per < n ? lo + per : n;
    reduce_rows_block(rows + lo * kPartial, hi - lo, stage + (uint64_t)b * kPartial, s);
}

__device__ __forceinline__ void reduce_stage2(const double* __restrict__ stage, uint64_t n, double* __restrict__ out,
                                              double (*s)[kReduceBlock]) {
    reduce_rows_block(stage, stage_blocks(n), out, s);
}

}  // namespace mlmc
