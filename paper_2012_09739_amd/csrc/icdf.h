// Exact and approximate Gaussian variables from one 32-bit uniform word, device side.
//
// Section 3 couples the exact variable Z = Phi^{-1}(U) and the approximate variable
// Z~ = Phi~^{-1}(U) through the same uniform U; here U = (x + 1/2) 2^-32 for a word x.
//
// Exact (binary64): Phi^{-1}(u) = x g(w) with x = 2u - 1 and w = -log((1 - x)(1 + x)),
// g an entire function of w.  -log is table driven (256 cells) and g is piecewise: on each
// of 344 intervals of width 1/16 covering every w of a 32-bit word, one polynomial of
// degree 5 in the local coordinate, its coefficients read per lane from the same table (in
// LDS or global memory), so every lane runs the same instructions whatever its interval.
// x is exact and y = 1 - x^2 = (1 - x)(1 + x) is rounded once (one fma); the result is
// exactly odd under word -> 2^32 - 1 - word.
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
#include "internal.h"

namespace mlmc {

// Cell of the table-driven log: f = R(1/c) for the cell centre c in [1/2, 1), l = -log(f)
// rounded.
struct LogCell {
    double f;
    double l;
};
constexpr int kLogCells = 256;

// -log(y) for normal 0 < y < 1 (Tang's table method).  y = m 2^e with m in [1/2, 1) from
// the hardware frexp; the top 8 mantissa bits pick a cell (centre c, f = R(1/c)),
// r = R(m f - 1) with |r| <= 2^-9, and log y = e ln2 - log f + log1p(r).  Storing -log f
// (not log c) makes the rounding of f harmless; for y in [1/2, 1) the exponent is 0 and no
// cancellation against e ln2 occurs.  Absolute error about 1e-16 plus the rounding of the
// result.
__device__ __forceinline__ double neg_log_f64(double y, const LogCell* __restrict__ tab,
                                              double p_top = 0.0, bool p_top_given = false) {
    constexpr double kP[] = MLMC_LOG1P_COEFFS;
    const uint32_t hi = (uint32_t)__double2hiint(y);
    const double m = __builtin_amdgcn_frexp_mant(y);
    const double kd = (double)__builtin_amdgcn_frexp_exp(y);
    const LogCell c = tab[(hi >> 12) & (kLogCells - 1)];
    const double r = __builtin_fma(m, c.f, -1.0);
    double p = p_top_given ? p_top : kP[MLMC_LOG1P_DEG];
#pragma unroll
    for (int i = MLMC_LOG1P_DEG - 1; i >= 0; --i) p = __builtin_fma(p, r, kP[i]);
    const double log_m = c.l + __builtin_fma(r * r, p, r);
    // e ln 2 with ln 2 rounded once: the error |e| 2.3e-17 vanishes for y in [1/2, 1), where
    // w = -log y is small, and stays below 1e-15 absolute (relative 3e-17 of w) at y = 2^-32
    constexpr double kLn2 = 0x1.62e42fefa39efp-1;
    return -__builtin_fma(kd, kLn2, log_m);
}

// Places a binary64 constant in an SGPR pair at its point of use, as the scalar operand of
// a v_fma_f64, instead of a loop-invariant VGPR copy that costs a v_mov and occupancy.
__device__ __forceinline__ double sgpr_const(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// Table of the exact variable: the log cells and, interval-major, the piecewise
// coefficients of g (piece[k][j] is coefficient j of interval k: one 48-byte row per
// interval, read with three 16-byte loads from one address).
constexpr int kPieces = MLMC_ICDF_PIECES;
constexpr int kPieceDeg = MLMC_ICDF_PIECE_DEG;
static_assert((kPieceDeg + 1) % 2 == 0, "rows of whole 16-byte pairs of coefficients");
struct ExactTable {
    LogCell log[kLogCells];
    double piece[kPieces][kPieceDeg + 1];
};
static_assert(sizeof(ExactTable) % 16 == 0, "staged in 16-byte pieces");

// x = 2u - 1 = word 2^-31 + (2^-32 - 1), exact in binary64 (a multiple of 2^-32 below 1 in
// magnitude), and y = (1 - x)(1 + x) = 1 - x^2 rounded once.
__device__ __forceinline__ double icdf_x(uint32_t word) {
    return __builtin_fma((double)word, 0x1p-31, 0x1p-32 - 1.0);
}
__device__ __forceinline__ double icdf_y(double x) {
    return __builtin_fma(-x, x, 1.0);
}

// g(w): interval k = floor(16 |w|) and local coordinate f = 16 |w| - k, both exact.  w is
// below 0 only by a rounding when y rounds to 1 (|x| < 2^-26.5), where g(|w|) = g(0) to
// far below binary64 resolution; the absolute value is a free source modifier.
__device__ __forceinline__ double icdf_g(double w, const double (*__restrict__ piece)[kPieceDeg + 1]) {
    const double t = __builtin_fabs(w) * (double)MLMC_ICDF_PIECE_SCALE;
    const uint32_t k0 = (uint32_t)(int)t;
    const uint32_t k = k0 < (uint32_t)(kPieces - 1) ? k0 : (uint32_t)(kPieces - 1);
    const double f = __builtin_amdgcn_fract(t);
    const double* c = piece[k];
    double acc = c[kPieceDeg];
#pragma unroll
    for (int j = kPieceDeg - 1; j >= 0; --j) acc = __builtin_fma(acc, f, c[j]);
    return acc;
}

__device__ __forceinline__ double icdf_exact_f64(uint32_t word, const ExactTable* __restrict__ tab) {
    const double x = icdf_x(word);
    return x * icdf_g(neg_log_f64(icdf_y(x), tab->log), tab->piece);
}

// Binary64 constants held in VGPRs for a whole chunk.  Each is an operand of an fma whose
// other constant operand is already scalar; an instruction reads at most one scalar
// register here, so without this each use would cost a move.
struct ExactConsts {
    double x0;     // 2^-32 - 1, the addend of x = word 2^-31 + x0
    double p_top;  // leading log1p coefficient
};

__device__ __forceinline__ ExactConsts exact_consts() {
    constexpr double kP[] = MLMC_LOG1P_COEFFS;
    ExactConsts k{0x1p-32 - 1.0, kP[MLMC_LOG1P_DEG]};
    asm volatile("" : "+v"(k.x0), "+v"(k.p_top));
    return k;
}

// Exact variables of four words at once (four independent chains for the scheduler).
__device__ __forceinline__ void icdf_exact_f64x4(const uint32_t (&word)[4], double (&z)[4],
                                                 const ExactTable* __restrict__ tab, const ExactConsts& kc) {
    double x[4], w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = __builtin_fma((double)word[k], sgpr_const(0x1p-31), kc.x0);
        w[k] = neg_log_f64(icdf_y(x[k]), tab->log, kc.p_top, true);
    }
    // one word's coefficient row at a time: each result is pinned before the next row is
    // read (the asm takes the result as an operand and clobbers memory), so at most one
    // row of 8 coefficients (16 VGPRs) is live instead of all of them
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        z[k] = x[k] * icdf_g(w[k], tab->piece);
        asm volatile("" : "+v"(z[k])::"memory");
    }
}

// Interval j-1 (0-based row of the table), mirror flag and the local coordinate scaled to
// an integer: t = T 2^-31 exactly, T < 2^31 + 2^14.
struct DyadicPos {
    uint32_t row;
    uint32_t T;
    uint32_t sign;  // 0x80000000 on the upper half, else 0 (xor into the result's sign bit)
};

// Branch-free: with xm the mirrored word (u' = (xm + 1/2) 2^-32 in I_k, k = clz(xm)) and
// a = 2 xm + 1, clz(a) = k - 1 and, for s = min(k - 1, 14),
//   k <= 15:  (a << s) mod 2^31 = (xm << k) - 2^31 + 2^(k-1)    (u' = 2^-(k+1) (1 + t))
//   k >= 16:  (a << s)          = (xm << 15) + 2^14             (u' = 2^-16 t)
__device__ __forceinline__ DyadicPos dyadic_locate(uint32_t word) {
    DyadicPos p;
    p.sign = word & 0x80000000u;
    const uint32_t xm = word ^ (uint32_t)((int32_t)word >> 31);  // 2^32 - 1 - word on the upper half
    const uint32_t a = (xm << 1) | 1u;
    const uint32_t km1 = (uint32_t)__builtin_clz(a);  // a != 0
    p.T = (a << (km1 < 14u ? km1 : 14u)) & 0x7FFFFFFFu;
    p.row = km1 < 15u ? km1 : 15u;
    return p;
}

__device__ __forceinline__ float apply_sign(float q, uint32_t sign) {
    return __uint_as_float(__float_as_uint(q) ^ sign);
}
__device__ __forceinline__ double apply_sign(double q, uint32_t sign) {
    return __hiloint2double((int)((uint32_t)__double2hiint(q) ^ sign), __double2loint(q));
}

// Z~ in binary32; tab holds 16 rows of (DEG + 1) binary32 coefficients c_0..c_d, or, with
// kPrescaled, c_i 2^(-31 i) (see prescaled_coeff): then T itself serves as the coordinate and
// every Horner value is the unscaled one times an exact power of two (all stay normal), so
// the result is bit-for-bit the same with one multiplication less.
template <int DEG, bool kPrescaled = false>
__device__ __forceinline__ float icdf_dyadic_f32(uint32_t word, const float* __restrict__ tab) {
    const DyadicPos p = dyadic_locate(word);
    // one correctly rounded conversion: R_32(t) = R_32(T) 2^-31
    const float t = kPrescaled ? (float)p.T : (float)p.T * 0x1p-31f;
    const float* c = tab + p.row * (DEG + 1);
    float q = c[DEG];
#pragma unroll
    for (int i = DEG - 1; i >= 0; --i) {
        q = __fmul_rn(q, t);
        q = __fadd_rn(q, c[i]);
    }
    return apply_sign(q, p.sign);
}

// Coefficient i of a row, scaled for icdf_dyadic_f32<DEG, true> (exact: a power of two).
__device__ __forceinline__ float prescaled_coeff(float c, int i) {
    return __builtin_ldexpf(c, -31 * i);
}

// R_bf16(x): x rounded to 8 significant bits, to nearest with ties to even, from the bit
// pattern (finite x); the result is a binary32 value.  Rounding the correctly rounded
// binary32 result of + - x on 8-bit operands gives the correctly rounded bfloat16 result
// (24 >= 2 * 8 + 2).
__device__ __forceinline__ float round_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t r = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    return __uint_as_float(r);
}

// Z~ in emulated bfloat16; tab holds 16 rows of (DEG + 1) coefficients rounded to bfloat16
// (as binary32 values).  The coordinate is formed in binary32 and narrowed, R_bf16(R_32(t)).
template <int DEG>
__device__ __forceinline__ float icdf_dyadic_bf16(uint32_t word, const float* __restrict__ tab) {
    const DyadicPos p = dyadic_locate(word);
    const float t = round_bf16((float)p.T * 0x1p-31f);
    const float* c = tab + p.row * (DEG + 1);
    float q = c[DEG];
#pragma unroll
    for (int i = DEG - 1; i >= 0; --i) q = round_bf16(round_bf16(q * t) + c[i]);
    return apply_sign(q, p.sign);
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
    return apply_sign(q, p.sign);
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
    return p.sign ? __hneg(q) : q;
}

// ---- piecewise-constant variable (table lookup) ------------------------------------------
// 2^kPcBits equal cells of (0, 1); row i of the table holds the mean of Phi^-1 over
// [i 2^-b, (i + 1) 2^-b) for the lower half.  With xm the mirrored word, u' = (xm + 1/2) 2^-32
// lies in cell xm >> (32 - b) (the cells align with the word grid), and the upper half takes
// the negated value.  No arithmetic: a shift, a load and a sign.
__device__ __forceinline__ uint32_t pconst_row(uint32_t word) {
    const uint32_t xm = word ^ (uint32_t)((int32_t)word >> 31);
    return xm >> (32 - kPcBits);
}
__device__ __forceinline__ float icdf_pconst_f32(uint32_t word, const float* __restrict__ tab) {
    return apply_sign(tab[pconst_row(word)], word & 0x80000000u);
}
__device__ __forceinline__ double icdf_pconst_f64(uint32_t word, const double* __restrict__ tab) {
    return apply_sign(tab[pconst_row(word)], word & 0x80000000u);
}
__device__ __forceinline__ __half icdf_pconst_f16(uint32_t word, const __half* __restrict__ tab) {
    const __half q = tab[pconst_row(word)];
    return (word >> 31) ? __hneg(q) : q;
}

}  // namespace mlmc
