// Exact and approximate Gaussian variables from one 32-bit uniform word, device side.
//
// Section 3 couples the exact variable Z = Phi^{-1}(U) and the approximate variable
// Z~ = Phi~^{-1}(U) through the same uniform U; here U = (x + 1/2) 2^-32 for a word x.
//
// Exact (binary64): Phi^{-1}(u) = x g(w) with x = 2u - 1 and w = -log((1 - x)(1 + x)),
// g an entire function of w.  w itself is never formed: G(y) = g(-log y) is piecewise
// polynomial in y = (1 - x)(1 + x) on cells of y -- 32 per binade, chosen by the exponent
// and the five leading mantissa bits -- of degree 6 in the offset from the cell centre, its
// coefficients read per lane from a table (in LDS or global memory), so every lane runs
// the same instructions whatever its cell.  x is exact and y is rounded once (one fma); the
// result is exactly odd under word -> 2^32 - 1 - word.
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

// Cell of the table-driven log (the learned variable's input): f = R(1/c) for the cell
// centre c in [1/2, 1), l = -log(f) rounded.
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
__device__ __forceinline__ double neg_log_f64(double y, const LogCell* __restrict__ tab) {
    constexpr double kP[] = MLMC_LOG1P_COEFFS;
    const uint32_t hi = (uint32_t)__double2hiint(y);
    const double m = __builtin_amdgcn_frexp_mant(y);
    const double kd = (double)__builtin_amdgcn_frexp_exp(y);
    const LogCell c = tab[(hi >> 12) & (kLogCells - 1)];
    const double r = __builtin_fma(m, c.f, -1.0);
    double p = kP[MLMC_LOG1P_DEG];
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

// Table of the exact variable: the 7 coefficients of G on each cell of y.  Cell k has the
// key kKeyMin + k, the key of y being its biased exponent and five leading mantissa bits
// (the upper word shifted right by 15).  The cells of y >= 2^-10 (the top cells) sit in LDS
// as four arrays of 16-byte entries -- (c0, c1), (c2, c3), (c4, c5) and (c6, unused) -- so a
// lane reads its cell with loads from one address plus fixed offsets and no conversion (c5
// and c6 are binary32 values, stored widened).  The deep cells below 2^-10 stay in global
// memory as 64-byte rows of binary64 coefficients and are read only by lanes whose y falls
// there (probability 2^-11 per word).
constexpr int kCellBits = MLMC_EXACT_CELL_BITS;
constexpr int kExactDeg = MLMC_EXACT_DEG;
static_assert(kExactDeg == 6, "four 16-byte entries per top cell");
constexpr int kRowLen = 8;
constexpr uint32_t kKeyMin = (uint32_t)MLMC_EXACT_E_MIN << kCellBits;
constexpr int kExactRows = MLMC_EXACT_ROWS;
constexpr uint32_t kKeyMax = 1023u << kCellBits;  // y = 1: the constant row G(1) = g(0)
static_assert(kKeyMin + kExactRows - 1 == kKeyMax, "one row per cell, then y = 1");
constexpr uint32_t kKeyTop = (uint32_t)MLMC_EXACT_E_TOP << kCellBits;  // y >= 2^-10
constexpr int kTopCells = (int)(kKeyMax + 1 - kKeyTop);
constexpr int kDeepRows = kExactRows - kTopCells;

struct ExactCols {
    double2 c01[kTopCells];
    double2 c23[kTopCells];
    double2 c45[kTopCells];
    double2 c6[kTopCells];  // (c6, 0)
};
// what kernels stage into LDS: the top cells, then the log cells (only for the learned variable)
struct ExactLds {
    ExactCols top;
    LogCell log[kLogCells];
};
// the device image: the LDS part, then the deep rows
struct ExactTable {
    ExactLds lds;
    double deep[kDeepRows][kRowLen];
};
static_assert(sizeof(ExactCols) % 16 == 0 && sizeof(ExactLds) % 16 == 0, "staged in 16-byte pieces");

// x = 2u - 1 = word 2^-31 + (2^-32 - 1), exact in binary64 (a multiple of 2^-32 below 1 in
// magnitude), and y = (1 - x)(1 + x) = 1 - x^2 rounded once.
__device__ __forceinline__ double icdf_x(uint32_t word) {
    return __builtin_fma((double)word, 0x1p-31, 0x1p-32 - 1.0);
}
__device__ __forceinline__ double icdf_y(double x) {
    return __builtin_fma(-x, x, 1.0);
}

// Horner's rule for the 7 coefficients of a cell at t.
__device__ __forceinline__ double cell_poly(const double (&co)[kExactDeg + 1], double t) {
    double acc = co[kExactDeg];
#pragma unroll
    for (int j = kExactDeg - 1; j >= 0; --j) acc = __builtin_fma(acc, t, co[j]);
    return acc;
}

// G(y) = g(-log y) for 2^-32 < y <= 1.  c is the centre of y's cell (its key with one half
// of the bits below), so t = y - c is exact (same binade; y = 1 reads a constant row).
// Every lane evaluates a top cell (the deep lanes the lowest one, a finite value they
// discard); the deep lanes then evaluate their own row from global memory.
__device__ __forceinline__ double icdf_G(double y, const ExactCols* __restrict__ top,
                                         const double (*__restrict__ deep)[kRowLen]) {
    constexpr uint32_t kHalf = 1u << (19 - kCellBits);
    uint32_t key = (uint32_t)__double2hiint(y) >> (20 - kCellBits);
    asm volatile("" : "+v"(key));  // the deep test stays a 32-bit compare of the key
    const double c = __hiloint2double((int)((key << (20 - kCellBits)) | kHalf), 0);
    const double t = y - c;
    const uint32_t k = (key > kKeyTop ? key : kKeyTop) - kKeyTop;
    const double2 p01 = top->c01[k], p23 = top->c23[k], p45 = top->c45[k];
    const double p6 = top->c6[k].x;
    double g = cell_poly({p01.x, p01.y, p23.x, p23.y, p45.x, p45.y, p6}, t);
    // g is final here for the top lanes: the deep branch below then neither merges its loads
    // with the LDS ones (a flat load) nor shares this Horner chain through copies
    asm volatile("" : "+v"(g));
    if (key < kKeyTop) {
        const double2* d = (const double2*)deep[key - kKeyMin];
        const double2 q0 = d[0], q1 = d[1], q2 = d[2], q3 = d[3];
        g = cell_poly({q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x}, t);
    }
    return g;
}

__device__ __forceinline__ double icdf_exact_f64(uint32_t word, const ExactCols* __restrict__ top,
                                                 const double (*__restrict__ deep)[kRowLen]) {
    const double x = icdf_x(word);
    return x * icdf_G(icdf_y(x), top, deep);
}

// The binary64 addend 2^-32 - 1 of x = word 2^-31 + x0 held in a VGPR pair for a whole
// chunk: the fma's other constant operand is already scalar, and an instruction reads at
// most one scalar register here, so without this each use would cost a move.
struct ExactConsts {
    double x0;
};

__device__ __forceinline__ ExactConsts exact_consts() {
    ExactConsts k{0x1p-32 - 1.0};
    asm volatile("" : "+v"(k.x0));
    return k;
}

// Exact variables of four words at once (four independent chains for the scheduler).
__device__ __forceinline__ void icdf_exact_f64x4(const uint32_t (&word)[4], double (&z)[4],
                                                 const ExactCols* __restrict__ top,
                                                 const double (*__restrict__ deep)[kRowLen], const ExactConsts& kc) {
    double x[4], y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = __builtin_fma((double)word[k], sgpr_const(0x1p-31), kc.x0);
        y[k] = icdf_y(x[k]);
    }
    // one word's cell at a time: each result is pinned before the next cell is read (the
    // asm takes the result as an operand and clobbers memory), so at most one cell's
    // coefficients (14 VGPRs) are live instead of all four
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        z[k] = x[k] * icdf_G(y[k], top, deep);
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
// The row is k - 1 itself: the device tables repeat the last interval's row in rows 15..31.
__device__ __forceinline__ DyadicPos dyadic_locate(uint32_t word) {
    DyadicPos p;
    p.sign = word & 0x80000000u;
    const uint32_t xm = word ^ (uint32_t)((int32_t)word >> 31);  // 2^32 - 1 - word on the upper half
    const uint32_t a = (xm << 1) | 1u;
    const uint32_t km1 = (uint32_t)__builtin_clz(a);  // a != 0
    p.T = (a << (km1 < 14u ? km1 : 14u)) & 0x7FFFFFFFu;
    p.row = km1;
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
    return __ushort_as_half((unsigned short)(__half_as_ushort(q) ^ (p.sign >> 16)));
}

// The binary16 variables of two words as one pair (the two packed paths of a lane): the same
// values as two icdf_dyadic_f16 calls, with both coordinates narrowed by one conversion of the
// pair and both signs applied by one 32-bit xor.
template <int DEG>
__device__ __forceinline__ __half2 icdf_dyadic_f16x2(uint32_t w0, uint32_t w1, const __half* __restrict__ tab) {
    const DyadicPos p0 = dyadic_locate(w0), p1 = dyadic_locate(w1);
    // R_16(R_32(T) 2^-31) for both in one conversion (the scaling by 2^-31 is exact, T >= 1;
    // v_cvt_pk_f16_f32 rounds to nearest like the scalar conversion).  Written as the
    // instruction itself: the compiler would otherwise fuse each product and its narrowing
    // into a mixed-precision multiply-add, at twice the issue cost of the pair.
    const float a0 = (float)p0.T * 0x1p-31f, a1 = (float)p1.T * 0x1p-31f;
    uint32_t tp;
    asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(tp) : "v"(a0), "v"(a1));
    const _Float16 t0 = __builtin_bit_cast(_Float16, (uint16_t)tp);
    const _Float16 t1 = __builtin_bit_cast(_Float16, (uint16_t)(tp >> 16));
    const _Float16* c0 = (const _Float16*)(tab + p0.row * (DEG + 1));
    const _Float16* c1 = (const _Float16*)(tab + p1.row * (DEG + 1));
    _Float16 q0 = c0[DEG], q1 = c1[DEG];
#pragma unroll
    for (int i = DEG - 1; i >= 0; --i) {
        q0 = q0 * t0;  // separately rounded (the build does not contract)
        q0 = q0 + c0[i];
        q1 = q1 * t1;
        q1 = q1 + c1[i];
    }
    // bit 31 of w0 to bit 15 and bit 31 of w1 to bit 31 (bytes 3 of each, then the sign bits)
    const uint32_t sgn = __builtin_amdgcn_perm(w1, w0, 0x070C030Cu) & 0x80008000u;
    const uint32_t q = (uint32_t)__builtin_bit_cast(uint16_t, q0) | ((uint32_t)__builtin_bit_cast(uint16_t, q1) << 16);
    const uint32_t bits = q ^ sgn;
    __half2 z;
    __builtin_memcpy(&z, &bits, sizeof z);
    return z;
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
