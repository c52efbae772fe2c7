/*
 * libvalurates -- issue rates of single vector-ALU opcodes on gfx950 (not part of the
 * method: the measured weights behind the level kernels' issue roofline).
 *
 * valu_rate(op, waves_per_simd, iters, &rate, &kernel_ms) launches the probe kernel of opcode
 * `op` twice on every CU of the current device (waves_per_simd 1..8 resident wavefronts per
 * SIMD, iters 1..2^20 loop trips of 32 instructions of the opcode per lane; the first launch
 * warms the clocks) and returns in *rate the lane-instructions of the second launch per CU
 * per nanosecond of its HIP-event time, and in *kernel_ms (host, may be NULL) that time.
 * Divided by the shader clock of the launch (GHz) the rate is lane-instructions per CU per
 * clock (64 = one wavefront instruction per clock per CU).  Synchronous on the null stream;
 * allocates and frees its own small device buffer.  Returns 0, or -1 (invalid argument),
 * -2 (allocation), -3 (no device), -4 (launch or execution error).
 */
#ifndef VALU_RATES_H
#define VALU_RATES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VALU_FMA_F64 = 0,
    VALU_MUL_F64,
    VALU_ADD_F64,
    VALU_FMA_F32,
    VALU_MUL_F32,
    VALU_PK_FMA_F16,   /* packed binary16 FMA: two lanes' worth of FMAs per lane */
    VALU_PK_MUL_F16,
    VALU_FMA_F16,      /* scalar binary16 FMA */
    VALU_XOR3_B32,     /* three-input xor (v_bitop3_b32 with the table 0x96) */
    VALU_ADD_U32,
    VALU_MUL_LO_U32,
    VALU_MUL_HI_U32,
    VALU_FFBH_U32,     /* count leading zeros */
    VALU_EXP_F32,      /* transcendental unit */
    VALU_RCP_F32,      /* transcendental unit */
    VALU_MED3_F32,
    VALU_MAD_U64_U32,  /* 32 x 32 -> 64 integer product with 64-bit addend */
    VALU_CVT_F64_F32,  /* v_cvt_f32_f64 + v_cvt_f64_f32 (rate per instruction) */
    VALU_CVT_F16_F32,  /* v_cvt_f16_f32 + v_cvt_f32_f16 (rate per instruction) */
    VALU_MIN_U32,
    VALU_LSHL_OR_B32,
    VALU_CNDMASK_B32,  /* v_cmp_gt_u32 + v_cndmask_b32 (rate per instruction) */
    VALU_PERM_B32,
    VALU_AND_B32,
    VALU_ASHR_I32,
    VALU_ADD_F16,      /* scalar binary16 */
    VALU_MUL_F16,      /* scalar binary16 */
    VALU_PK_ADD_F16,
    VALU_CVT_PK_F16_F32,
    VALU_CVT_F32_U32,
    VALU_CVT_F64_U32,
    VALU_LSHL_B64,
    VALU_LSHL_ADD_U64,
    VALU_MOV_B64,
    VALU_MAX_F32_CLAMP, /* v_max_f32 with the clamp modifier (a clamp to [0, 1]) */
    VALU_SUB_U32_CLAMP, /* saturating 32-bit subtract */
    VALU_LSHR_B32,
    VALU_FMA_MIX_F16,   /* v_fma_mixlo_f16: binary32 operands, binary16 result */
    VALU_BITOP3_B16,
    VALU_LOG_F32,       /* transcendental unit */
    VALU_SQRT_F32,      /* transcendental unit */
    VALU_CMP_U32,       /* v_cmp_gt_u32 into a scalar register pair (no select) */
    VALU_N_OPS
};

int valu_rate(int op, int waves_per_simd, uint32_t iters, double* lane_instr_per_cu_ns, double* kernel_ms);

#ifdef __cplusplus
}
#endif

#endif /* VALU_RATES_H */
