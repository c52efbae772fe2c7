// VALU issue rates of single opcodes on gfx950: the weights of the issue roofline.
//
// The level kernels are bound by vector-ALU issue, and a wavefront instruction's issue cost
// depends on its opcode (a binary64 FMA, a 32-bit operation, a packed binary16 FMA and the
// 32x32->64 integer product do not issue at the same rate).  Each probe kernel runs one
// opcode, written as inline assembly so the instruction is exactly that one, on eight
// independent register chains per lane, for a fixed number of iterations, on a grid of
// exactly the requested resident wavefronts per SIMD on every CU.  The rate is the lane-
// instructions of the timed launch per CU per nanosecond of its HIP-event time; divided by the
// shader clock of that launch (GRBM_GUI_ACTIVE cycles over its duration, from a counter run)
// it gives lane-instructions per CU per clock: 64 is one wavefront instruction per clock per
// CU, the binary64 FMA rate of the published 78.6 TFLOP/s vector peak at 2.4 GHz.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/valu_rates.h"

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 4;  // iterations of the eight chains per loop trip

// one instruction of the opcode on chain register r (inputs a, b loop-invariant)
#define VR_F64(op) asm volatile(op " %0, %1, %2, %0" : "+v"(r) : "v"(a), "v"(b))
#define VR_F64_2(op) asm volatile(op " %0, %0, %1" : "+v"(r) : "v"(a))
#define VR_32_3(op) asm volatile(op " %0, %1, %2, %0" : "+v"(r) : "v"(a), "v"(b))
#define VR_32_2(op) asm volatile(op " %0, %0, %1" : "+v"(r) : "v"(a))
#define VR_32_1(op) asm volatile(op " %0, %0" : "+v"(r))

template <int OP>
struct Chain;

// 64-bit register chains
template <>
struct Chain<VALU_FMA_F64> {
    double r;
    __device__ void step(double a, double b) { VR_F64("v_fma_f64"); }
};
template <>
struct Chain<VALU_MUL_F64> {
    double r;
    __device__ void step(double a, double) { VR_F64_2("v_mul_f64"); }
};
template <>
struct Chain<VALU_ADD_F64> {
    double r;
    __device__ void step(double a, double) { VR_F64_2("v_add_f64"); }
};

// 32-bit register chains
template <>
struct Chain<VALU_FMA_F32> {
    float r;
    __device__ void step(float a, float b) { VR_32_3("v_fma_f32"); }
};
template <>
struct Chain<VALU_MUL_F32> {
    float r;
    __device__ void step(float a, float) { VR_32_2("v_mul_f32"); }
};
template <>
struct Chain<VALU_PK_FMA_F16> {
    uint32_t r;
    __device__ void step(uint32_t a, uint32_t b) { VR_32_3("v_pk_fma_f16"); }
};
template <>
struct Chain<VALU_PK_MUL_F16> {
    uint32_t r;
    __device__ void step(uint32_t a, uint32_t) { VR_32_2("v_pk_mul_f16"); }
};
template <>
struct Chain<VALU_FMA_F16> {
    uint32_t r;
    __device__ void step(uint32_t a, uint32_t b) { VR_32_3("v_fma_f16"); }
};
template <>
struct Chain<VALU_XOR3_B32> {
    uint32_t r;
    // gfx950's three-input bitwise operation with the truth table of a ^ b ^ c
    __device__ void step(uint32_t a, uint32_t b) {
        asm volatile("v_bitop3_b32 %0, %1, %2, %0 bitop3:0x96" : "+v"(r) : "v"(a), "v"(b));
    }
};
template <>
struct Chain<VALU_ADD_U32> {
    uint32_t r;
    __device__ void step(uint32_t a, uint32_t) { VR_32_2("v_add_u32"); }
};
template <>
struct Chain<VALU_MUL_LO_U32> {
    uint32_t r;
    __device__ void step(uint32_t a, uint32_t) { VR_32_2("v_mul_lo_u32"); }
};
template <>
struct Chain<VALU_MUL_HI_U32> {
    uint32_t r;
    __device__ void step(uint32_t a, uint32_t) { VR_32_2("v_mul_hi_u32"); }
};
template <>
struct Chain<VALU_FFBH_U32> {
    uint32_t r;
    __device__ void step(uint32_t, uint32_t) { VR_32_1("v_ffbh_u32"); }
};
template <>
struct Chain<VALU_EXP_F32> {
    float r;
    __device__ void step(float, float) { VR_32_1("v_exp_f32"); }
};
template <>
struct Chain<VALU_RCP_F32> {
    float r;
    __device__ void step(float, float) { VR_32_1("v_rcp_f32"); }
};
template <>
struct Chain<VALU_MED3_F32> {
    float r;
    __device__ void step(float a, float b) { VR_32_3("v_med3_f32"); }
};

// further opcodes of the level kernels' loops (32-bit unless named otherwise)
#define VR_CHAIN32(ID, T, BODY)                                  \
    template <>                                                  \
    struct Chain<ID> {                                           \
        T r;                                                     \
        __device__ void step(uint32_t a, uint32_t b) { BODY; }   \
    };
VR_CHAIN32(VALU_MIN_U32, uint32_t, VR_32_2("v_min_u32"))
VR_CHAIN32(VALU_LSHL_OR_B32, uint32_t, VR_32_3("v_lshl_or_b32"))
VR_CHAIN32(VALU_CNDMASK_B32, uint32_t,
           asm volatile("v_cmp_gt_u32 vcc, %1, %2\n\tv_cndmask_b32 %0, %0, %1, vcc" : "+v"(r) : "v"(a), "v"(b) : "vcc"))
VR_CHAIN32(VALU_PERM_B32, uint32_t, VR_32_3("v_perm_b32"))
VR_CHAIN32(VALU_AND_B32, uint32_t, VR_32_2("v_and_b32"))
VR_CHAIN32(VALU_ASHR_I32, uint32_t, VR_32_2("v_ashrrev_i32"))
VR_CHAIN32(VALU_ADD_F16, uint32_t, VR_32_2("v_add_f16"))
VR_CHAIN32(VALU_MUL_F16, uint32_t, VR_32_2("v_mul_f16"))
VR_CHAIN32(VALU_PK_ADD_F16, uint32_t, VR_32_2("v_pk_add_f16"))
VR_CHAIN32(VALU_CVT_PK_F16_F32, uint32_t, asm volatile("v_cvt_pk_f16_f32 %0, %1, %2" : "+v"(r) : "v"(a), "v"(b)))
VR_CHAIN32(VALU_CVT_F32_U32, uint32_t, asm volatile("v_cvt_f32_u32 %0, %1" : "+v"(r) : "v"(a)))
VR_CHAIN32(VALU_MAX_F32_CLAMP, float, asm volatile("v_max_f32_e64 %0, %0, %1 clamp" : "+v"(r) : "v"(a)))
VR_CHAIN32(VALU_SUB_U32_CLAMP, uint32_t, asm volatile("v_sub_u32_e64 %0, %0, %1 clamp" : "+v"(r) : "v"(a)))
VR_CHAIN32(VALU_LSHR_B32, uint32_t, VR_32_2("v_lshrrev_b32"))
VR_CHAIN32(VALU_FMA_MIX_F16, float, VR_32_3("v_fma_mixlo_f16"))
VR_CHAIN32(VALU_BITOP3_B16, uint32_t,
           asm volatile("v_bitop3_b16 %0, %1, %2, %0 bitop3:0x96" : "+v"(r) : "v"(a), "v"(b)))
#undef VR_CHAIN32
template <>
struct Chain<VALU_CMP_U32> {
    uint32_t r;
    uint64_t m;  // each chain's own scalar register pair
    __device__ void step(uint32_t a, uint32_t) { asm volatile("v_cmp_gt_u32_e64 %0, %1, %2" : "=s"(m) : "v"(a), "v"(r)); }
};
template <>
struct Chain<VALU_LOG_F32> {
    float r;
    // from the loop-invariant operand: a chain of logarithms would leave the finite range
    __device__ void step(float a, float) { asm volatile("v_log_f32 %0, %1" : "+v"(r) : "v"(a)); }
};
template <>
struct Chain<VALU_SQRT_F32> {
    float r;
    __device__ void step(float, float) { VR_32_1("v_sqrt_f32"); }
};
template <>
struct Chain<VALU_CVT_F64_U32> {
    double r;
    __device__ void step(uint32_t a, uint32_t) { asm volatile("v_cvt_f64_u32 %0, %1" : "+v"(r) : "v"(a)); }
};
template <>
struct Chain<VALU_LSHL_B64> {
    uint64_t r;
    __device__ void step(uint32_t a, uint32_t) { asm volatile("v_lshlrev_b64 %0, %1, %0" : "+v"(r) : "v"(a)); }
};
template <>
struct Chain<VALU_LSHL_ADD_U64> {
    uint64_t r;
    __device__ void step(uint32_t a, uint32_t) {
        const uint64_t c = 0x100000001ull;
        asm volatile("v_lshl_add_u64 %0, %0, 1, %1" : "+v"(r) : "v"(c));
    }
};
template <>
struct Chain<VALU_MOV_B64> {
    uint64_t r;
    __device__ void step(uint32_t a, uint32_t) {
        const uint64_t c = 0x100000001ull + a;
        asm volatile("v_mov_b64 %0, %1" : "+v"(r) : "v"(c));
    }
};

// the 32x32->64 integer product in the form Philox uses it: a lane value times a uniform
// (SGPR) multiplier, zero addend
template <>
struct Chain<VALU_MAD_U64_U32> {
    uint64_t r;
    uint64_t carry;
    __device__ void step(uint32_t a, uint32_t b) {
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, 0" : "+v"(r), "+s"(carry) : "v"(a), "s"(b));
    }
};

// conversions between the formats (the exact variable widens binary32 coefficients; the
// binary16 paths narrow their variable): one narrowing and one widening per step, each
// from a loop-invariant source into the chain's own register
template <>
struct Chain<VALU_CVT_F64_F32> {
    double r;
    float f;
    __device__ void step(double a, double) {
        const float fa = 1.5f;
        asm volatile("v_cvt_f32_f64 %0, %1" : "+v"(f) : "v"(a));
        asm volatile("v_cvt_f64_f32 %0, %1" : "+v"(r) : "v"(fa));
    }
};
template <>
struct Chain<VALU_CVT_F16_F32> {
    float r;
    uint32_t h;
    __device__ void step(float a, float) {
        const uint32_t ha = 0x3C00u;
        asm volatile("v_cvt_f16_f32 %0, %1" : "+v"(h) : "v"(a));
        asm volatile("v_cvt_f32_f16 %0, %1" : "+v"(r) : "v"(ha));
    }
};

template <int OP>
__device__ void seed(Chain<OP>& c, uint32_t lane, int k) {
    using T = decltype(c.r);
    if constexpr (OP == VALU_MAD_U64_U32) {
        c.r = (uint64_t)lane * 2654435761u + k;
        c.carry = 0;
    } else if constexpr (OP == VALU_CMP_U32) {
        c.r = lane * 747796405u + (uint32_t)k;
        c.m = 0;
    }
    else if constexpr (OP == VALU_CVT_F64_F32) {
        c.r = 1.0;
        c.f = 1.0f + k;
    } else if constexpr (OP == VALU_CVT_F16_F32) {
        c.r = 1.0f;
        c.h = (uint32_t)k;
    } else if constexpr (sizeof(T) == 8) c.r = 1.0 + 1e-3 * (double)(lane + k);
    else if constexpr (OP == VALU_PK_FMA_F16 || OP == VALU_PK_MUL_F16 || OP == VALU_FMA_F16 || OP == VALU_ADD_F16 ||
                       OP == VALU_MUL_F16 || OP == VALU_PK_ADD_F16)
        c.r = 0x3C003C00u + k;
    else if constexpr (std::is_same<T, float>::value) c.r = 1.0f + 1e-3f * (float)(lane + k);
    else c.r = lane * 747796405u + (uint32_t)k;
}

template <int OP>
__global__ __launch_bounds__(256) void probe_kernel(uint32_t iters, uint64_t* sink) {
    const uint32_t lane = threadIdx.x;
    Chain<OP> c[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) seed<OP>(c[k], lane, k);
    // operands near one keep the floating-point chains finite and normal
    using T = decltype(c[0].r);
    const uint32_t a = lane | 1u;
    const double af64 = 0.999999, bf64 = 1e-7;
    const float af32 = 0.999999f, bf32 = 1e-7f;
    const uint32_t ah = 0x3BFF3BFFu, bh = 0x00010001u;  // half2 (0.9995, 0.9995), (tiny, tiny)
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                if constexpr (sizeof(T) == 8 && OP != VALU_MAD_U64_U32) c[k].step(af64, bf64);
                else if constexpr (OP == VALU_MAD_U64_U32) c[k].step(a, 0xD2511F53u);
                else if constexpr (OP == VALU_PK_FMA_F16 || OP == VALU_PK_MUL_F16 || OP == VALU_FMA_F16 ||
                                   OP == VALU_ADD_F16 || OP == VALU_MUL_F16 || OP == VALU_PK_ADD_F16)
                    c[k].step(ah, bh);
                else if constexpr (OP == VALU_CVT_PK_F16_F32)
                    c[k].step(__float_as_uint(af32), __float_as_uint(bf32));
                else if constexpr (std::is_same<T, float>::value) c[k].step(af32, bf32);
                else c[k].step(a, a ^ 0x9E3779B9u);
            }
    }
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        uint64_t bits = 0;
        __builtin_memcpy(&bits, &c[k].r, sizeof(c[k].r));
        acc ^= bits;
    }
    sink[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int OP>
hipError_t launch(uint32_t grid, uint32_t iters, uint64_t* sink, hipStream_t s) {
    hipLaunchKernelGGL(probe_kernel<OP>, dim3(grid), dim3(256), 0, s, iters, sink);
    return hipGetLastError();
}

// instructions of the opcode per loop trip and chain (the conversion probes run two)
int instrs_per_step(int op) {
    return (op == VALU_CVT_F64_F32 || op == VALU_CVT_F16_F32 || op == VALU_CNDMASK_B32) ? 2 : 1;
}

}  // namespace

extern "C" int valu_rate(int op, int waves_per_simd, uint32_t iters, double* lane_instr_per_cu_ns, double* kernel_ms) {
    if (op < 0 || op >= VALU_N_OPS || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || iters > (1u << 20) ||
        !lane_instr_per_cu_ns)
        return -1;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return -3;
    const int n_cu = prop.multiProcessorCount;
    // 4 SIMDs per CU, four-wave blocks: waves_per_simd blocks per CU, all resident at once
    const uint32_t grid = (uint32_t)(n_cu * waves_per_simd);
    uint64_t* sink = nullptr;
    if (hipMalloc(&sink, (size_t)grid * 256 * sizeof(uint64_t)) != hipSuccess) return -2;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) {
        (void)hipFree(sink);
        return -4;
    }
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipFree(sink);
        return -4;
    }
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first launch warms the clocks up
        if (rep == 1) e = hipEventRecord(e0, nullptr);
        if (e != hipSuccess) break;
        switch (op) {
#define VR_CASE(x) case x: e = launch<x>(grid, iters, sink, nullptr); break;
            VR_CASE(VALU_FMA_F64) VR_CASE(VALU_MUL_F64) VR_CASE(VALU_ADD_F64) VR_CASE(VALU_FMA_F32)
            VR_CASE(VALU_MUL_F32) VR_CASE(VALU_PK_FMA_F16) VR_CASE(VALU_PK_MUL_F16) VR_CASE(VALU_FMA_F16)
            VR_CASE(VALU_XOR3_B32) VR_CASE(VALU_ADD_U32) VR_CASE(VALU_MUL_LO_U32) VR_CASE(VALU_MUL_HI_U32)
            VR_CASE(VALU_FFBH_U32) VR_CASE(VALU_EXP_F32) VR_CASE(VALU_RCP_F32) VR_CASE(VALU_MED3_F32)
            VR_CASE(VALU_MAD_U64_U32) VR_CASE(VALU_CVT_F64_F32) VR_CASE(VALU_CVT_F16_F32) VR_CASE(VALU_MIN_U32)
            VR_CASE(VALU_LSHL_OR_B32) VR_CASE(VALU_CNDMASK_B32) VR_CASE(VALU_PERM_B32) VR_CASE(VALU_AND_B32)
            VR_CASE(VALU_ASHR_I32) VR_CASE(VALU_ADD_F16) VR_CASE(VALU_MUL_F16) VR_CASE(VALU_PK_ADD_F16)
            VR_CASE(VALU_CVT_PK_F16_F32) VR_CASE(VALU_CVT_F32_U32) VR_CASE(VALU_CVT_F64_U32) VR_CASE(VALU_LSHL_B64)
            VR_CASE(VALU_LSHL_ADD_U64) VR_CASE(VALU_MOV_B64) VR_CASE(VALU_MAX_F32_CLAMP)
            VR_CASE(VALU_SUB_U32_CLAMP) VR_CASE(VALU_LSHR_B32) VR_CASE(VALU_FMA_MIX_F16) VR_CASE(VALU_BITOP3_B16)
            VR_CASE(VALU_LOG_F32) VR_CASE(VALU_SQRT_F32) VR_CASE(VALU_CMP_U32)
#undef VR_CASE
            default: e = hipErrorInvalidValue;
        }
        if (rep == 1 && e == hipSuccess) e = hipEventRecord(e1, nullptr);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    int rc = 0;
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess || ms <= 0.0f) {
        rc = -4;
    } else {
        const double lane_instr = 64.0 * 4.0 * grid * (double)iters * kUnroll * kChains * instrs_per_step(op);
        *lane_instr_per_cu_ns = lane_instr / n_cu / (1e6 * (double)ms);
        if (kernel_ms) *kernel_ms = (double)ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return rc;
}
