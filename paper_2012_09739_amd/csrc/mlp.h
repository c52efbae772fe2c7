// The learned approximate inverse CDF: a 1-16-16-1 tanh network, device side.
//
// An approximate Gaussian variable in the sense of Section 2.1 / Assumption 2.1, mirrored
// about u = 1/2 (exactly zero mean) and bounded for 32-bit words:
//   u' = min(u, 1 - u), r = sqrt(-2 ln(2u')), x = r / 3.4 - 1,
//   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 . h2 + b3,
//   Z~ = y - r (u < 1/2), r - y (u >= 1/2);
// y learns the smooth residual Phi^{-1}(u') + r.  Inference uses the parameters rounded to
// binary16 (staged in LDS widened to binary32) with binary32 arithmetic and accumulation;
// r comes from the binary64 -log so that it stays accurate next to u' = 1/2.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "icdf.h"

namespace mlmc {

constexpr int kMlpHidden = 16;
constexpr int kMlpParams = 16 + 16 + 256 + 16 + 16 + 1;  // 321
constexpr int kMlpImage = 336;                           // padded image length
constexpr float kMlpRScale = 3.4f;
// offsets of the parameter blocks in the flat vector
constexpr int kW1 = 0, kB1 = 16, kW2 = 32, kB2 = 288, kW3 = 304, kB3 = 320;

__device__ __forceinline__ float tanh_fast(float a) {
    // tanh(a) = 1 - 2 / (exp(2a) + 1), hardware base-2 exponential and reciprocal
    const float e = __builtin_amdgcn_exp2f(a * 2.8853900817779268f);  // 2 / ln 2
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// r = sqrt(-2 ln(2u')) for the mirrored word xm, u' = (xm + 1/2) 2^-32.
__device__ __forceinline__ double mlp_radius(uint32_t xm, const LogCell* __restrict__ logtab) {
    const double two_u = ((double)xm + 0.5) * 0x1p-31;  // exact
    return __builtin_sqrt(2.0 * neg_log_f64(two_u, logtab));
}

// Network output for input x; W is the binary32 image of the binary16 parameters (LDS).
// The empty asm with a memory clobber keeps the weight reads inside the call site, so the
// 321 weights are read from LDS (uniform broadcast) instead of being hoisted into VGPRs.
__device__ __forceinline__ float mlp_eval(float x, const float* __restrict__ W) {
    asm volatile("" ::: "memory");
    float h1[kMlpHidden];
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) h1[k] = tanh_fast(__builtin_fmaf(W[kW1 + k], x, W[kB1 + k]));
    float y = W[kB3];
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) {
        asm volatile("" ::: "memory");
        float a = W[kB2 + k];
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) a = __builtin_fmaf(W[kW2 + k * kMlpHidden + j], h1[j], a);
        y = __builtin_fmaf(W[kW3 + k], tanh_fast(a), y);
    }
    return y;
}

__device__ __forceinline__ float icdf_mlp_f32(uint32_t word, const float* __restrict__ W,
                                              const LogCell* __restrict__ logtab) {
    const uint32_t xm = word ^ (uint32_t)((int32_t)word >> 31);  // ~word on the upper half
    const double r = mlp_radius(xm, logtab);
    const float x = (float)(r * (1.0 / 3.4) - 1.0);
    const float q = mlp_eval(x, W) - (float)r;
    return apply_sign(q, word & 0x80000000u);
}

}  // namespace mlmc
