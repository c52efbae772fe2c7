// The learned approximate inverse CDF: a 1-16-16-1 tanh network, device side.
//
// An approximate Gaussian variable in the sense of Section 2.1 / Assumption 2.1:
// mirrored about u = 1/2 (exactly zero mean) and bounded (|y| <= |b3| + sum |W3|).
//   u' = min(u, 1 - u), r = sqrt(-2 ln(2 u')), x = r / 3.4 - 1,
//   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 . h2 + b3,  Z~ = +-y.
// Inference uses binary16 weights with binary32 accumulation.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmc {

constexpr int kMlpHidden = 16;
constexpr int kMlpParams = 16 + 16 + 256 + 16 + 16 + 1;  // 321
constexpr float kMlpRScale = 3.4f;

// Inference image: the 321 parameters as binary16, padded to 336 entries.
struct MlpImage {
    __half p[336];
};

__device__ __forceinline__ float tanh_fast(float a) {
    // tanh(a) = 1 - 2 / (exp(2a) + 1); exp via the hardware base-2 exponential
    const float e = __builtin_amdgcn_exp2f(a * 2.8853900817779268f);  // 2 / ln 2
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ __forceinline__ float mlp_feature(uint32_t xm) {
    // u' = (xm + 1/2) 2^-32, 2u' = (xm + 1/2) 2^-31:  ln(2u') = ln(xm + 1/2) - 31 ln 2
    const float l2 = __builtin_amdgcn_logf((float)xm + 0.5f) - 31.0f;  // log2(2u')
    const float r = __builtin_sqrtf(-2.0f * 0.69314718055994531f * l2);
    return r * (1.0f / kMlpRScale) - 1.0f;
}

// y(x) for the mirrored half; W points at the binary16 image (uniform across lanes).
__device__ __forceinline__ float mlp_eval(float x, const __half* __restrict__ W) {
    const __half* W1 = W;
    const __half* b1 = W + 16;
    const __half* W2 = W + 32;
    const __half* b2 = W + 288;
    const __half* W3 = W + 304;
    const __half* b3 = W + 320;
    float h1[kMlpHidden];
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k)
        h1[k] = tanh_fast(__builtin_fmaf(__half2float(W1[k]), x, __half2float(b1[k])));
    float y = __half2float(b3[0]);
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) {
        float a = __half2float(b2[k]);
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) a = __builtin_fmaf(__half2float(W2[k * 16 + j]), h1[j], a);
        y = __builtin_fmaf(__half2float(W3[k]), tanh_fast(a), y);
    }
    return y;
}

__device__ __forceinline__ float icdf_mlp_f32(uint32_t word, const __half* __restrict__ W) {
    const bool upper = (word >> 31) != 0;
    const uint32_t xm = upper ? ~word : word;
    const float y = mlp_eval(mlp_feature(xm), W);
    return upper ? -y : y;
}

}  // namespace mlmc
