// The learned approximate inverse CDF: a 1-16-16-1 piecewise-linear network, device side.
//
// An approximate Gaussian variable in the sense of Section 2.1 / Assumption 2.1, mirrored
// about u = 1/2 (exactly zero mean) and bounded for 32-bit words.  Deployed form (the
// training form's hard tanh h = min(max(z, -1), 1) rewritten with c = (h + 1) / 2, so every
// activation is the clamp to [0, 1] of the instruction that forms its argument):
//   2u = R_32(2 xm + 1) 2^-32, r = sqrt(-2 ln 2u), x = R_16(R_32(r C - 1)), C = R_32(1 / 3.4),
//   c1 = clamp01(A1 x + a1)            (packed binary16 fused multiply-add, clamped),
//   c2 = clamp01(R_16(A2 c1 + a2))     (binary16 matrix instruction, binary32 accumulation,
//                                       rounded to binary16 and clamped in one conversion),
//   y  = A3 . c2 + a3                  (binary16 matrix instruction, binary32 accumulation),
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
constexpr float kMlpRScale = 3.4f;
// offsets of the parameter blocks in the flat vector
constexpr int kW1 = 0, kB1 = 16, kW2 = 32, kB2 = 288, kW3 = 304, kB3 = 320;
// The inference image (binary32 words): the deployed parameters widened to binary32 at the
// offsets above (padded to 336), then the matrix-instruction operands of mlp_eval_wave already
// packed as binary16 pairs, so that a wavefront loads them without conversions:
//   kPkL1   16 words: row g: (A1[4g], A1[4g+1]), (A1[4g+2], A1[4g+3]), (a1[4g], a1[4g+1]),
//                     (a1[4g+2], a1[4g+3])
//   kPkA2  128 words: lane 16 g + c: (A2[c][4g], A2[c][4g+1]), (A2[c][4g+2], A2[c][4g+3])
//   kPkA3  128 words: block b, r = c / 4, row g: A3[4g .. 4g+3] as two pairs when r = b, else 0
//   kPkB3    4 words: a3 four times (binary32)
constexpr int kPkL1 = 336, kPkA2 = 352, kPkA3 = 480, kPkB3 = 608;
constexpr int kMlpImage = 612;

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
// second layer's arguments in exactly the B layout of the next product: one conversion to
// binary16 with the clamp modifier per pair of units gives c2 as a B operand.  The output
// layer is a second product whose A operand is A3 in the rows n of block b (n / 4 = b) and
// zero elsewhere, accumulated over the four blocks from C = a3: row n of the result then holds
// y of sample 16 (n / 4) + s, so lane 16 g + c finds its own sample's y in every element.
__device__ __forceinline__ float mlp_eval_wave(uint32_t x16x2, const float* __restrict__ W) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t c = lane & 15u, g = lane >> 4;
    const float4 l1 = *(const float4*)(W + kPkL1 + 4 * g);
    const mlp_h2 w1a = __builtin_bit_cast(mlp_h2, l1.x), w1b = __builtin_bit_cast(mlp_h2, l1.y);
    const mlp_h2 b1a = __builtin_bit_cast(mlp_h2, l1.z), b1b = __builtin_bit_cast(mlp_h2, l1.w);
    const mlp_h4 w2 = __builtin_bit_cast(mlp_h4, *(const float2*)(W + kPkA2 + 2 * lane));
    const mlp_f4 b2 = __builtin_bit_cast(mlp_f4, *(const float4*)(W + kB2 + 4 * g));
    const float* a3 = W + kPkA3 + 2 * (4 * (c >> 2) + g);
    mlp_f4 y = __builtin_bit_cast(mlp_f4, *(const float4*)(W + kPkB3));
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const mlp_h2 xb = __builtin_bit_cast(mlp_h2, (uint32_t)__shfl((int)x16x2, 16 * b + (int)c, kWave));
        const mlp_h2 h01 = mlp_unit_pair(w1a, xb, b1a), h23 = mlp_unit_pair(w1b, xb, b1b);
        const mlp_h4 bop = {h01[0], h01[1], h23[0], h23[1]};
        const mlp_f4 d = __builtin_amdgcn_mfma_f32_16x16x16f16(w2, bop, b2, 0, 0, 0);
        // round to binary16, then clamp (the same as clamping first: 0 and 1 are binary16
        // values and rounding is monotone); one conversion with the clamp modifier per pair
        const mlp_h2 zero = {(_Float16)0.0f, (_Float16)0.0f}, one = {(_Float16)1.0f, (_Float16)1.0f};
        mlp_h2 c01 = {(_Float16)d[0], (_Float16)d[1]}, c23 = {(_Float16)d[2], (_Float16)d[3]};
        c01 = __builtin_elementwise_min(__builtin_elementwise_max(c01, zero), one);
        c23 = __builtin_elementwise_min(__builtin_elementwise_max(c23, zero), one);
        const mlp_h4 c2 = {c01[0], c01[1], c23[0], c23[1]};
        const mlp_h4 w3 = __builtin_bit_cast(mlp_h4, *(const float2*)(a3 + 32 * b));
        y = __builtin_amdgcn_mfma_f32_16x16x16f16(w3, c2, y, 0, 0, 0);
    }
    return y[0];
}

// y for K inputs per lane at once (the K variables of one Philox call): the same operations as
// K mlp_eval_wave calls, ordered block by block so that the K independent chains of matrix
// instructions interleave and hide each other's latency.
template <int K>
__device__ __forceinline__ void mlp_eval_wave_k(const uint32_t (&x16x2)[K], const float* __restrict__ W,
                                                float (&out)[K]) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t c = lane & 15u, g = lane >> 4;
    const float4 l1 = *(const float4*)(W + kPkL1 + 4 * g);
    const mlp_h2 w1a = __builtin_bit_cast(mlp_h2, l1.x), w1b = __builtin_bit_cast(mlp_h2, l1.y);
    const mlp_h2 b1a = __builtin_bit_cast(mlp_h2, l1.z), b1b = __builtin_bit_cast(mlp_h2, l1.w);
    const mlp_h4 w2 = __builtin_bit_cast(mlp_h4, *(const float2*)(W + kPkA2 + 2 * lane));
    const mlp_f4 b2 = __builtin_bit_cast(mlp_f4, *(const float4*)(W + kB2 + 4 * g));
    const float* a3 = W + kPkA3 + 2 * (4 * (c >> 2) + g);
    const mlp_f4 y0 = __builtin_bit_cast(mlp_f4, *(const float4*)(W + kPkB3));
    const mlp_h2 zero = {(_Float16)0.0f, (_Float16)0.0f}, one = {(_Float16)1.0f, (_Float16)1.0f};
    mlp_f4 y[K];
#pragma unroll
    for (int v = 0; v < K; ++v) y[v] = y0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const mlp_h4 w3 = __builtin_bit_cast(mlp_h4, *(const float2*)(a3 + 32 * b));
        mlp_f4 d[K];
#pragma unroll
        for (int v = 0; v < K; ++v) {
            const mlp_h2 xb = __builtin_bit_cast(mlp_h2, (uint32_t)__shfl((int)x16x2[v], 16 * b + (int)c, kWave));
            const mlp_h2 h01 = mlp_unit_pair(w1a, xb, b1a), h23 = mlp_unit_pair(w1b, xb, b1b);
            const mlp_h4 bop = {h01[0], h01[1], h23[0], h23[1]};
            d[v] = __builtin_amdgcn_mfma_f32_16x16x16f16(w2, bop, b2, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < K; ++v) {
            mlp_h2 c01 = {(_Float16)d[v][0], (_Float16)d[v][1]}, c23 = {(_Float16)d[v][2], (_Float16)d[v][3]};
            c01 = __builtin_elementwise_min(__builtin_elementwise_max(c01, zero), one);
            c23 = __builtin_elementwise_min(__builtin_elementwise_max(c23, zero), one);
            const mlp_h4 c2 = {c01[0], c01[1], c23[0], c23[1]};
            y[v] = __builtin_amdgcn_mfma_f32_16x16x16f16(w3, c2, y[v], 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < K; ++v) out[v] = y[v][0];
}

// The learned variables of K words per lane (all 64 lanes together), as icdf_mlp_f32 each.
template <int K>
__device__ __forceinline__ void icdf_mlp_f32_k(const uint32_t* word, const float* __restrict__ W, float (&z)[K]) {
    uint32_t x16x2[K];
    float r[K], y[K];
#pragma unroll
    for (int v = 0; v < K; ++v) {
        const uint32_t xm = word[v] ^ (uint32_t)((int32_t)word[v] >> 31);
        const float two_u = (float)(2u * xm + 1u) * 0x1p-32f;
        r[v] = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(two_u) * -1.38629436111989061f);
        const float x = __builtin_fmaf(r[v], (float)(1.0 / 3.4), -1.0f);
        asm("v_cvt_pk_f16_f32 %0, %1, %1" : "=v"(x16x2[v]) : "v"(x));
    }
    mlp_eval_wave_k<K>(x16x2, W, y);
#pragma unroll
    for (int v = 0; v < K; ++v) z[v] = apply_sign(y[v] - r[v], word[v] & 0x80000000u);
}

// The learned approximate variable of every lane's word (all 64 lanes together).
__device__ __forceinline__ float icdf_mlp_f32(uint32_t word, const float* __restrict__ W) {
    const uint32_t xm = word ^ (uint32_t)((int32_t)word >> 31);  // ~word on the upper half
    const float two_u = (float)(2u * xm + 1u) * 0x1p-32f;         // R_32(2 xm + 1), scaled exactly
    const float r = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(two_u) * -1.38629436111989061f);  // -2 ln 2
    const float x = __builtin_fmaf(r, (float)(1.0 / 3.4), -1.0f);
    // R_16(x) in both halves with one conversion (written as the instruction: the compiler
    // would fuse the fma and the narrowing into a mixed-precision fma, then duplicate the half)
    uint32_t x16x2;
    asm("v_cvt_pk_f16_f32 %0, %1, %1" : "=v"(x16x2) : "v"(x));
    const float q = mlp_eval_wave(x16x2, W) - r;
    return apply_sign(q, word & 0x80000000u);
}

}  // namespace mlmc
