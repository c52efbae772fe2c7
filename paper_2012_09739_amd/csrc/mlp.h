// The learned approximate inverse CDF: a 1-16-16-1 tanh network, device side.
//
// An approximate Gaussian variable in the sense of Section 2.1 / Assumption 2.1, mirrored
// about u = 1/2 (exactly zero mean) and bounded for 32-bit words:
//   u' = min(u, 1 - u), r = sqrt(-2 ln(2u')), x = r / 3.4 - 1,
//   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 . h2 + b3,
//   Z~ = y - r (u < 1/2), r - y (u >= 1/2);
// y learns the smooth residual Phi^{-1}(u') + r.  Inference uses the parameters rounded to
// binary16 (staged in LDS widened to binary32) with binary32 arithmetic and accumulation, the
// 16 x 16 layer as binary32 matrix instructions; r comes from the binary64 -log so that it
// stays accurate next to u' = 1/2.
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

// Network output for every lane's own input x, the 16 x 16 layer on the matrix cores.  W is
// the binary32 image of the binary16 parameters (LDS or global memory).  All 64 lanes of
// the wavefront must call it together (a matrix instruction works on the whole wave).
//
// Lanes are split as lane = 16 g + c.  For the samples of lanes 16 b + c (b = 0..3), lane
// 16 g + c evaluates the hidden units 4 j + g of the first layer, which is the B operand of
// v_mfma_f32_16x16x4_f32 (B[k][s] in lane 16 k + s) with A[n][k] = W2[n][4 j + k] (A[n][k]
// in lane 16 k + n): four such products over j give out[n][s] for one block of 16 samples,
// returned as D[n][s] = d[n % 4] in lane 16 (n / 4) + s.  Each lane then applies the second
// tanh and the output weights to its four units n = 4 g .. 4 g + 3 of every block, the
// partial sums are added over the four lane groups, and lane 16 g + c keeps block g: its own
// sample.  The products and sums are binary32, as in the per-lane evaluation.
__device__ __forceinline__ float mlp_eval_wave(float x, const float* __restrict__ W) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t c = lane & 15u, g = lane >> 4;
    float w1[4], b1[4], w2[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t k = 4u * j + g;
        w1[j] = W[kW1 + k];
        b1[j] = W[kB1 + k];
        w2[j] = W[kW2 + c * kMlpHidden + k];
    }
    float part[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float xb = __shfl(x, 16 * b + (int)c, kWave);
        v4f d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(w2[j], tanh_fast(__builtin_fmaf(w1[j], xb, b1[j])), d, 0, 0, 0);
        float p = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t n = 4u * g + r;
            p = __builtin_fmaf(W[kW3 + n], tanh_fast(d[r] + W[kB2 + n]), p);
        }
        part[b] = p;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        part[b] += __shfl_xor(part[b], 16, kWave);
        part[b] += __shfl_xor(part[b], 32, kWave);
    }
    const float y = g == 0 ? part[0] : g == 1 ? part[1] : g == 2 ? part[2] : part[3];
    return y + W[kB3];
}

// The learned approximate variable of every lane's word (all 64 lanes together).
__device__ __forceinline__ float icdf_mlp_f32(uint32_t word, const float* __restrict__ W,
                                              const LogCell* __restrict__ logtab) {
    const uint32_t xm = word ^ (uint32_t)((int32_t)word >> 31);  // ~word on the upper half
    const double r = mlp_radius(xm, logtab);
    const float x = (float)(r * (1.0 / 3.4) - 1.0);
    const float q = mlp_eval_wave(x, W) - (float)r;
    return apply_sign(q, word & 0x80000000u);
}

}  // namespace mlmc
