// Exact and approximate Gaussian variables from one 32-bit uniform word, device side.
//
// Section 3 couples the exact variable Z = Phi^{-1}(U) and the approximate variable
// Z~ = Phi~^{-1}(U) through the same uniform U; here U = (x + 1/2) 2^-32 for a word x.
//
// Exact (binary64): Phi^{-1}(u) = x g(w) with x = 2u - 1 and w = -log((1 - x)(1 + x)),
// g an entire function of w evaluated by one polynomial in w on w <= 6.25 (more than
// 99.9% of words, so a wavefront almost never diverges) and by one in sqrt(w) beyond;
// -log is table driven (128 cells, the table in LDS or global memory).
// x, 1 - x and 1 + x are exact; the result is exactly odd under x -> 2^32 - 1 - x.
//
// Approximate (Section 2.1, Lemmas 2.2 and 2.3): a polynomial of degree 1 or 3 in the
// local coordinate t of one of 16 dyadic intervals of (0, 1/2] -- I_j = [2^-(j+1), 2^-j)
// for j = 1..15, I_16 = (0, 2^-16) -- mirrored to (1/2, 1).  Horner's rule is unfused
// (one rounding per product and per sum), in the working precision.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "icdf_exact_coeffs.h"

namespace mlmc {

// Cell of the table-driven log: f = R(1/c) for the cell centre c, l = -log(f) rounded.
struct LogCell {
    double f;
    double l;
};
constexpr int kLogCells = 128;

// -log(y) for normal 0 < y <= 1 (Tang's table method).  y = 2^(e-1023) m with m in [1, 2)
// read off the bit pattern; the top 7 mantissa bits pick a cell (centre c, f = R(1/c));
// r = R(m f - 1) with |r| <= 2^-8, and log y = (e - 1023) ln2 - log f + log1p(r).  Storing
// -log f (not log c) makes the rounding of f harmless.  Absolute error about 1e-16 plus
// the rounding of the result.
__device__ __forceinline__ double neg_log_f64(double y, const LogCell* __restrict__ tab) {
    constexpr double kP[] = MLMC_LOG1P_COEFFS;
    const uint32_t hi = (uint32_t)__double2hiint(y);
    const uint32_t lo = (uint32_t)__double2loint(y);
    const int k = (int)((hi >> 20) & 0x7FFu) - 1023;
    const double m = __hiloint2double((int)((hi & 0x000FFFFFu) | 0x3FF00000u), (int)lo);
    const LogCell c = tab[(hi >> 13) & (kLogCells - 1)];
    const double r = __builtin_fma(m, c.f, -1.0);
    double p = kP[MLMC_LOG1P_DEG];
#pragma unroll
    for (int i = MLMC_LOG1P_DEG - 1; i >= 0; --i) p = __builtin_fma(p, r, kP[i]);
    const double log_m = c.l + __builtin_fma(r * r, p, r);
    const double kd = (double)k;
    // ln 2 split so that k * kLn2Hi is exact for |k| < 2^11
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
    constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
    return -__builtin_fma(kd, kLn2Hi, __builtin_fma(kd, kLn2Lo, log_m));
}

// g(w) on the tail w > 6.25 (fewer than one word in a thousand): out of line so that its
// coefficients are materialised only when a lane needs them.
__device__ __noinline__ double icdf_tail_g(double w) {
    constexpr double kTail[] = MLMC_ICDF_TAIL_COEFFS;
    double acc = kTail[MLMC_ICDF_TAIL_DEG];
    const double d = __builtin_sqrt(w) - MLMC_ICDF_MID2;
#pragma unroll
    for (int i = MLMC_ICDF_TAIL_DEG - 1; i >= 0; --i) acc = __builtin_fma(acc, d, kTail[i]);
    return acc;
}

__device__ __forceinline__ double icdf_exact_f64(uint32_t word, const LogCell* __restrict__ tab) {
    // x = 2u - 1 = (v + 1/2) 2^-31 with v = word - 2^31 (exact in binary64)
    const int32_t v = (int32_t)(word ^ 0x80000000u);
    const double x = __builtin_fma((double)v, 0x1p-31, 0x1p-32);
    const double y = (1.0 - x) * (1.0 + x);
    const double w = neg_log_f64(y, tab);
    constexpr double kCentral[] = MLMC_ICDF_CENTRAL_COEFFS;
    double g;
    if (w <= MLMC_ICDF_W1) {
        double acc = kCentral[MLMC_ICDF_CENTRAL_DEG];
        const double d = w - MLMC_ICDF_MID1;
#pragma unroll
        for (int i = MLMC_ICDF_CENTRAL_DEG - 1; i >= 0; --i) acc = __builtin_fma(acc, d, kCentral[i]);
        g = acc;
    } else {
        g = icdf_tail_g(w);
    }
    return x * g;
}

// Places a binary64 constant in an SGPR pair at its point of use.  The polynomial
// coefficients are then scalar operands of v_fma_f64 (one instruction per Horner step)
// instead of loop-invariant VGPR copies that cost a v_mov per step and occupancy.
__device__ __forceinline__ double sgpr_const(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// Exact variables of four words at once: the four Horner chains share every
// coefficient (one scalar materialisation per coefficient for four FMAs) and give the
// scheduler four independent dependency chains.
__device__ __forceinline__ void icdf_exact_f64x4(const uint32_t (&word)[4], double (&z)[4],
                                                 const LogCell* __restrict__ tab) {
    constexpr double kCentral[] = MLMC_ICDF_CENTRAL_COEFFS;
    double x[4], w[4], d[4], acc[4];
    bool tail = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t v = (int32_t)(word[k] ^ 0x80000000u);
        x[k] = __builtin_fma((double)v, 0x1p-31, 0x1p-32);
        w[k] = neg_log_f64((1.0 - x[k]) * (1.0 + x[k]), tab);
        tail |= w[k] > MLMC_ICDF_W1;
        d[k] = w[k] - MLMC_ICDF_MID1;
        acc[k] = kCentral[MLMC_ICDF_CENTRAL_DEG];
    }
#pragma unroll
    for (int i = MLMC_ICDF_CENTRAL_DEG - 1; i >= 0; --i) {
        const double c = sgpr_const(kCentral[i]);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = __builtin_fma(acc[k], d[k], c);
    }
    if (tail) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (w[k] > MLMC_ICDF_W1) acc[k] = icdf_tail_g(w[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) z[k] = x[k] * acc[k];
}

// Interval j-1 (0-based row of the table), mirror flag and the local coordinate scaled to
// an integer: t = T 2^-31 exactly, T < 2^31 + 2^14.
struct DyadicPos {
    uint32_t row;
    uint32_t T;
    bool upper;
};

__device__ __forceinline__ DyadicPos dyadic_locate(uint32_t word) {
    DyadicPos p;
    p.upper = (word >> 31) != 0;
    const uint32_t xm = p.upper ? ~word : word;  // 2^32 - 1 - word on the upper half
    const uint32_t k = (uint32_t)__clz((int)xm);  // 1..32 since xm < 2^31
    if (k <= 15u) {
        // u' = 2^-(k+1) (1 + t):  t = ((xm << k) - 2^31 + 2^(k-1)) 2^-31
        p.T = ((xm << k) & 0x7FFFFFFFu) + (1u << (k - 1u));
        p.row = k - 1u;
    } else {
        // u' = 2^-16 t:  t = (xm + 1/2) 2^-16 = ((xm << 15) + 2^14) 2^-31
        p.T = (xm << 15) + (1u << 14);
        p.row = 15u;
    }
    return p;
}

// Z~ in binary32; tab holds 16 rows of (DEG + 1) binary32 coefficients c_0..c_d.
template <int DEG>
__device__ __forceinline__ float icdf_dyadic_f32(uint32_t word, const float* __restrict__ tab) {
    const DyadicPos p = dyadic_locate(word);
    const float t = (float)p.T * 0x1p-31f;  // one correctly rounded conversion: R_32(t)
    const float* c = tab + p.row * (DEG + 1);
    float q = c[DEG];
#pragma unroll
    for (int i = DEG - 1; i >= 0; --i) {
        q = __fmul_rn(q, t);
        q = __fadd_rn(q, c[i]);
    }
    return p.upper ? -q : q;
}

// Z~ in binary64 (the high-precision approximate variable of the diagnostic paths).
template <int DEG>
__device__ __forceinline__ double icdf_dyadic_f64(uint32_t word, const double* __restrict__ tab) {
    const DyadicPos p = dyadic_locate(word);
    const double t = (double)p.T * 0x1p-31;  // exact
    const double* c = tab + p.row * (DEG + 1);
    double q = c[DEG];
#pragma unroll
    for (int i = DEG - 1; i >= 0; --i) {
        q = __dmul_rn(q, t);
        q = __dadd_rn(q, c[i]);
    }
    return p.upper ? -q : q;
}

// Z~ in binary16 for one word; the coordinate is formed in binary32 and narrowed,
// t = R_16(R_32(t)).
template <int DEG>
__device__ __forceinline__ __half icdf_dyadic_f16(uint32_t word, const __half* __restrict__ tab) {
    const DyadicPos p = dyadic_locate(word);
    const __half t = __float2half_rn((float)p.T * 0x1p-31f);
    const __half* c = tab + p.row * (DEG + 1);
    __half q = c[DEG];
#pragma unroll
    for (int i = DEG - 1; i >= 0; --i) {
        q = __hmul(q, t);
        q = __hadd(q, c[i]);
    }
    return p.upper ? __hneg(q) : q;
}

}  // namespace mlmc
