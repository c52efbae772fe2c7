// The learned approximate inverse CDF: a 1-16-16-1 piecewise-linear network, device side.
//
// An approximate Gaussian variable in the sense of Section 2.1 / Assumption 2.1, mirrored
// about u = 1/2 (exactly zero mean) and bounded for 32-bit words.  Deployed form (the
// training form's hard tanh h = min(max(z, -1), 1) rewritten with c = (h + 1) / 2, so every
// activation is the clamp to [0, 1] of the instruction that forms its argument):
//   2u = R_32(2 xm + 1) 2^-32, r = sqrt(-2 ln 2u), x = R_16(r C - 1), C = R_32(1 / 3.4),
//   c1 = clamp01(A1 x + a1)            (packed binary16 fused multiply-add, clamped),
//   c2 = clamp01(A2 c1 + a2)           (binary16 matrix instruction, binary32 accumulation),
//   y  = A3 . c2 + a3                  (binary32),
//   Z~ = y - r (u < 1/2), r - y (u >= 1/2);
// y learns the smooth residual Phi^{-1}(u') + r.  The parameters are binary16 values staged
// in LDS widened to binary32; r uses the hardware base-2 logarithm and square root (no
// binary64 work, no exponential or reciprocal per unit).
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

// r = sqrt(-2 ln(2u')) in binary64 for the mirrored word xm, u' = (xm + 1/2) 2^-32 (the
// input of the training pairs).
__device__ __forceinline__ double mlp_radius(uint32_t xm, const LogCell* __restrict__ logtab) {
    const double two_u = ((double)xm + 0.5) * 0x1p-31;  // exact
    return __builtin_sqrt(2.0 * neg_log_f64(two_u, logtab));
}

typedef _Float16 mlp_h2 __attribute__((ext_vector_type(2)));
typedef _Float16 mlp_h4 __attribute__((ext_vector_type(4)));
typedef float mlp_f4 __attribute__((ext_vector_type(4)));

// Two units of the first layer: one packed binary16 fused multiply-add, clamped to [0, 1]
// (the compiler folds the clamp into the instruction's clamp modifier).  Written without
// inline assembly so that the compiler sees the operands and keeps the wait states between
// these instructions and the matrix instruction that reads them.
__device__ __forceinline__ mlp_h2 mlp_unit_pair(mlp_h2 w, mlp_h2 x, mlp_h2 b) {
    const mlp_h2 zero = {(_Float16)0.0f, (_Float16)0.0f}, one = {(_Float16)1.0f, (_Float16)1.0f};
    return __builtin_elementwise_min(__builtin_elementwise_max(__builtin_elementwise_fma(w, x, b), zero), one);
}
__device__ __forceinline__ mlp_h2 mlp_pair(float lo, float hi) {
    const mlp_h2 v = {(_Float16)lo, (_Float16)hi};  // exact: the image holds binary16 values
    return v;
}

// Network output y for every lane's own binary16 input x16 (low half of x16x2, repeated in
// the high half).  W is the binary32 image of the deployed binary16 parameters.  All 64
// lanes of the wavefront must call it together (a matrix instruction works on the whole wave).
//
// Lanes are split as lane = 16 g + c.  v_mfma_f32_16x16x16_f16 takes A[n][k] in lane
// 16 (k / 4) + n, element k % 4, B[k][s] in lane 16 (k / 4) + s, and returns D[n][s] in lane
// 16 (n / 4) + s, element n % 4.  For block b (the samples of lanes 16 b + c), lane 16 g + c
// evaluates the first-layer units 4 g .. 4 g + 3 of sample 16 b + c (two packed fused
// multiply-adds on that sample's input): the B operand.  A = A2, C = a2, so D holds the
// second layer's arguments; each lane clamps its four units, weighs them with A3, and the
// partial sums are added over the four lane groups (two lane-permutation swaps, no LDS), lane
// 16 g + c keeping block g: its own sample.
__device__ __forceinline__ float mlp_eval_wave(uint32_t x16x2, const float* __restrict__ W) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t c = lane & 15u, g = lane >> 4;
    const uint32_t k0 = 4u * g;
    const mlp_h2 w1a = mlp_pair(W[kW1 + k0], W[kW1 + k0 + 1]), w1b = mlp_pair(W[kW1 + k0 + 2], W[kW1 + k0 + 3]);
    const mlp_h2 b1a = mlp_pair(W[kB1 + k0], W[kB1 + k0 + 1]), b1b = mlp_pair(W[kB1 + k0 + 2], W[kB1 + k0 + 3]);
    const mlp_h4 w2 = {(_Float16)W[kW2 + c * kMlpHidden + k0], (_Float16)W[kW2 + c * kMlpHidden + k0 + 1],
                       (_Float16)W[kW2 + c * kMlpHidden + k0 + 2], (_Float16)W[kW2 + c * kMlpHidden + k0 + 3]};
    const mlp_f4 b2 = {W[kB2 + k0], W[kB2 + k0 + 1], W[kB2 + k0 + 2], W[kB2 + k0 + 3]};
    float part[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const mlp_h2 xb = __builtin_bit_cast(mlp_h2, (uint32_t)__shfl((int)x16x2, 16 * b + (int)c, kWave));
        const mlp_h2 h01 = mlp_unit_pair(w1a, xb, b1a), h23 = mlp_unit_pair(w1b, xb, b1b);
        const mlp_h4 bop = {h01[0], h01[1], h23[0], h23[1]};
        const mlp_f4 d = __builtin_amdgcn_mfma_f32_16x16x16f16(w2, bop, b2, 0, 0, 0);
        float p = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            p = __builtin_fmaf(W[kW3 + k0 + r], __builtin_amdgcn_fmed3f(d[r], 0.0f, 1.0f), p);
        part[b] = p;
    }
    // sum over the four lane groups, each lane keeping its own block: swapping the lane halves
    // pairs block 0 with 2 and 1 with 3 (lanes 0..31 keep blocks 0, 1), swapping odd and even
    // rows of 16 lanes leaves row g with block g
    const auto s02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(part[0]), __float_as_uint(part[2]), false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(part[1]), __float_as_uint(part[3]), false, false);
    const float q0 = __uint_as_float(s02[0]) + __uint_as_float(s02[1]);
    const float q1 = __uint_as_float(s13[0]) + __uint_as_float(s13[1]);
    const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(q0), __float_as_uint(q1), false, false);
    return (__uint_as_float(t[0]) + __uint_as_float(t[1])) + W[kB3];
}

// The learned approximate variable of every lane's word (all 64 lanes together).
__device__ __forceinline__ float icdf_mlp_f32(uint32_t word, const float* __restrict__ W) {
    const uint32_t xm = word ^ (uint32_t)((int32_t)word >> 31);  // ~word on the upper half
    const float two_u = (float)(2u * xm + 1u) * 0x1p-32f;         // R_32(2 xm + 1), scaled exactly
    const float r = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(two_u) * -1.38629436111989061f);  // -2 ln 2
    const float x = __builtin_fmaf(r, (float)(1.0 / 3.4), -1.0f);
    const uint32_t x16 = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
    const float q = mlp_eval_wave(x16 | (x16 << 16), W) - r;
    return apply_sign(q, word & 0x80000000u);
}

}  // namespace mlmc
