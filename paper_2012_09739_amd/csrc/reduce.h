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

}  // namespace mlmc
