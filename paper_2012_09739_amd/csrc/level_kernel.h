// The MLMC level kernel: coupled fine/coarse Euler-Maruyama paths, register resident.
//
// One wavefront owns one chunk of 64 paths (128 in binary16, two paths per lane packed in
// half2) and walks all 2^l fine steps of them: per group of four fine steps one Philox
// call, then per step the exact and/or approximate variable, the fine update, and after
// every second step the coarse update from the pairwise-summed variables (Section 3).
// At the end each lane forms the payoffs and differences and adds them to its (sum, sum of
// squares) of every term; after the chunks of one partial row (several at the coarse levels)
// the wave reduces them into the row, and a second kernel reduces the rows in a fixed order.
//
// Arithmetic (Section 2.2): X <- X (+) (A (+) B), A = ca (x) X, B = (cb (x) X) (x) Z with
// one rounding per operation (the build uses -ffp-contract=off), and the optional
// Kahan-compensated update of Algorithm 1 / Code 1 on every low-precision path.
// The Milstein instances (the higher-order scheme of Sections 2 and 4) add, for GBM, the
// rounded correction M = (cm (x) X) (x) (Z (x) Z (-) k), cm = R_p(sigma^2 delta_f / 2),
// as dX = (A (+) B) (+) M, with k = 1 on the fine path and k = 2 on the coarse path (whose
// variable is the sum of two fine ones).
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "icdf.h"
#include "internal.h"
#include "mlp.h"
#include "philox.h"

namespace mlmc {

// ---- one Euler-Maruyama update in precision T --------------------------------------
// R is the rounding applied to the result of every operation: none for the IEEE formats
// (the hardware rounds), R_bf16 for emulated bfloat16.
struct NoRound {
    template <typename T>
    __device__ __forceinline__ T operator()(T x) const { return x; }
};
struct RoundBF16 {
    __device__ __forceinline__ float operator()(float x) const { return round_bf16(x); }
};

// The increment dX of one step in a low-precision path: A (+) B, and for Milstein
// (A (+) B) (+) M, every operation rounded as the method states.
template <int SCHEME, typename T, typename R>
__device__ __forceinline__ T increment(T X, T z, T ca, T cb, T cm, T k, R r) {
    const T A = r(ca * X);
    const T B = r(r(cb * X) * z);
    const T dX = r(A + B);
    if constexpr (SCHEME == MLMC_SCHEME_MILSTEIN) {
        const T M = r(r(cm * X) * r(r(z * z) - k));
        return r(dX + M);
    } else {
        return dX;
    }
}

// One state update.  The binary64 paths (the exact pair, the binary64 approximate pair and
// the diagnostic's reference) stand for exact arithmetic; for GBM the drift and diffusion
// are linear in X, so there X + ca X + cb X Z = X (1 + d) with d = ca + cb Z (Milstein:
// + cm (Z^2 - k)) is evaluated as fma(X, d, X), d by fmas that do not depend on X: two
// roundings per step instead of four, a one-instruction dependent chain, and an error far
// below every tolerance these paths are compared with.  The low-precision paths keep the
// separately rounded X (+) dX.
template <int SCHEME, typename T, typename R = NoRound>
__device__ __forceinline__ void em_step(T& X, T z, T ca, T cb, T cm, T k, R r = R{}) {
    if constexpr (sizeof(T) == 8) {
        double d = __builtin_fma(cb, z, ca);
        if constexpr (SCHEME == MLMC_SCHEME_MILSTEIN) d = __builtin_fma(cm, __builtin_fma(z, z, -k), d);
        X = __builtin_fma(X, d, X);
    } else {
        X = r(X + increment<SCHEME>(X, z, ca, cb, cm, k, r));
    }
}

template <int SCHEME, typename T, typename R = NoRound>
__device__ __forceinline__ void em_step_kahan(T& X, T& c, T z, T ca, T cb, T cm, T k, R r = R{}) {
    const T dX = increment<SCHEME>(X, z, ca, cb, cm, k, r);
    const T y = r(dX - c);
    const T s = r(X + y);
    c = r(r(s - X) - y);
    X = s;
}

template <int SCHEME>
__device__ __forceinline__ __half2 increment_h2(__half2 X, __half2 z, __half2 ca, __half2 cb, __half2 cm, __half2 k) {
    const __half2 A = __hmul2(ca, X);
    const __half2 B = __hmul2(__hmul2(cb, X), z);
    const __half2 dX = __hadd2(A, B);
    if constexpr (SCHEME == MLMC_SCHEME_MILSTEIN) {
        const __half2 M = __hmul2(__hmul2(cm, X), __hsub2(__hmul2(z, z), k));
        return __hadd2(dX, M);
    } else {
        return dX;
    }
}

template <int SCHEME>
__device__ __forceinline__ void em_step_h2(__half2& X, __half2 z, __half2 ca, __half2 cb, __half2 cm, __half2 k) {
    X = __hadd2(X, increment_h2<SCHEME>(X, z, ca, cb, cm, k));
}

template <int SCHEME>
__device__ __forceinline__ void em_step_kahan_h2(__half2& X, __half2& c, __half2 z, __half2 ca, __half2 cb, __half2 cm,
                                                 __half2 k) {
    const __half2 dX = increment_h2<SCHEME>(X, z, ca, cb, cm, k);
    const __half2 y = __hsub2(dX, c);
    const __half2 s = __hadd2(X, y);
    c = __hsub2(__hsub2(s, X), y);
    X = s;
}

template <typename T, typename R = NoRound>
__device__ __forceinline__ T payoff(T X, T K, int kind, R r = R{}) {
    if (kind == MLMC_PAYOFF_X) return X;
    const T d = r(X - K);
    return d > T(0) ? d : T(0);
}

__device__ __forceinline__ __half payoff_h(__half X, __half K, int kind) {
    if (kind == MLMC_PAYOFF_X) return X;
    const __half d = __hsub(X, K);
    return __hgt(d, __float2half(0.0f)) ? d : __float2half(0.0f);
}

// ---- fixed-order wave reduction of the 8 partial values ------------------------------
// Lane i and lane i ^ 32 swap half of their eight values and each adds the half it keeps
// (lanes with bit 5 clear keep values 0..3, the others 4..7); then i ^ 16 halves again and
// i ^ 8 leaves one value per lane; three exchanges inside each group of eight lanes (its
// mirror image, then i ^ 2, then i ^ 1) complete the sums.  Lane 8k ends with the total of
// value k.  The order of every addition depends on the lane numbers only, so the result is
// reproducible.  The exchanges stay in the VALU: the half-wave and row swaps of gfx950
// (v_permlane32_swap, v_permlane16_swap) for the first two, row-local DPP moves for the rest,
// each on the two 32-bit halves of a double.
__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__builtin_bit_cast(uint64_t, x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32); }
__device__ __forceinline__ double join64(uint32_t lo, uint32_t hi) {
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// a's lanes 32..63 trade places with b's lanes 0..31: a lane of the lower half then holds its
// own a and the upper partner's a, a lane of the upper half the lower partner's b and its own b
__device__ __forceinline__ void swap_half_waves(double& a, double& b) {
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    a = join64(l[0], h[0]);
    b = join64(l[1], h[1]);
}
// the same between the odd rows (16 lanes) of a and the even rows of b
__device__ __forceinline__ void swap_rows(double& a, double& b) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    a = join64(l[0], h[0]);
    b = join64(l[1], h[1]);
}
// the value of the lane that DPP control CTRL names (inside the lane's row)
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
    return join64((uint32_t)__builtin_amdgcn_mov_dpp((int)lo32(x), CTRL, 0xf, 0xf, false),
                  (uint32_t)__builtin_amdgcn_mov_dpp((int)hi32(x), CTRL, 0xf, 0xf, false));
}
constexpr int kDppRowRor8 = 0x128;       // lane i of a row reads lane (i + 8) mod 16 = i ^ 8
constexpr int kDppHalfMirror = 0x141;    // lane i of a group of eight reads lane 7 - i
constexpr int kDppQuadXor2 = 0x4e;       // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadXor1 = 0xb1;       // quad_perm [1, 0, 3, 2]

// Every lane of the wave takes part (called with the full execution mask).
__device__ __forceinline__ void store_row(const double (&acc)[kPartial], uint32_t lane, double* out) {
    static_assert(kPartial == 8, "three halving exchanges");
    double v4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double a = acc[j], b = acc[4 + j];
        swap_half_waves(a, b);
        v4[j] = a + b;  // value j in the lower half-wave, 4 + j in the upper
    }
    double v2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        double a = v4[j], b = v4[2 + j];
        swap_rows(a, b);
        v2[j] = a + b;  // even rows keep the first two of their four values, odd rows the last two
    }
    const bool h3 = (lane & 8) != 0;
    double v = (h3 ? v2[1] : v2[0]) + dpp64<kDppRowRor8>(h3 ? v2[0] : v2[1]);
    v += dpp64<kDppHalfMirror>(v);
    v += dpp64<kDppQuadXor2>(v);
    v += dpp64<kDppQuadXor1>(v);
    if ((lane & 7) == 0) out[lane >> 3] = v;
}

// Copies the first `bytes` of the exact-variable table (the top cells, then the log cells)
// into LDS.
__device__ __forceinline__ void stage_exact_table(unsigned char* dst, const void* src, size_t bytes) {
    const uint4* s = (const uint4*)src;
    uint4* d = (uint4*)dst;
    for (int i = threadIdx.x; i < (int)(bytes / 16); i += blockDim.x) d[i] = s[i];
}

// The exact variable's deep rows (global memory) of a level.
__device__ __forceinline__ const double (*deep_rows(const LevelParams& prm))[kRowLen] {
    return ((const ExactTable*)prm.exact_tab)->deep;
}

// ---- the kernel ------------------------------------------------------------------------
// Approximate variable of one word in the working precision (binary64 or binary32).
template <int RV, int DEG, typename T, int PREC = MLMC_FP32>
__device__ __forceinline__ T approx_rv(uint32_t w, const T* tab, const float* mlpw) {
    if constexpr (RV == MLMC_RV_MLP) {
        return (T)icdf_mlp_f32(w, mlpw);
    } else if constexpr (RV == MLMC_RV_PCONST4096) {
        if constexpr (sizeof(T) == 8) return icdf_pconst_f64(w, (const double*)tab);
        else return icdf_pconst_f32(w, (const float*)tab);  // binary32, or bfloat16 values held in binary32
    } else if constexpr (PREC == MLMC_BF16) {
        return icdf_dyadic_bf16<DEG>(w, (const float*)tab);
    } else if constexpr (sizeof(T) == 8) {
        return icdf_dyadic_f64<DEG>(w, (const double*)tab);
    } else {
        return icdf_dyadic_f32<DEG, true>(w, (const float*)tab);  // table staged prescaled
    }
}

// One wave simulates one chunk of 64 paths (128 for binary16: two paths per lane) of one
// level and adds each lane's (sum, sum of squares) of every term to acc.  s_tab is the
// coefficient table in the working precision (binary32: prescaled, see prescaled_coeff) and
// s_tab64 the binary64 one (diagnostic), both in LDS.  SHORT (levels 0 and 1): the caller
// draws the words, whose calls several paths share, and names each lane's paths in
// sh_words / sh_local (chunk is then unused); NS is then the level's fine step count (1 or 2),
// known at compile time so that the step loop and the payoffs unroll without tests.
template <int PREC, int RV, bool NESTED, bool KAHAN, bool DIAG, bool SHORT = false, int SCHEME = MLMC_SCHEME_EM,
          int NS = 0>
__device__ __forceinline__ void chunk_terms(const LevelParams& prm, uint64_t chunk, uint32_t lane, const void* s_tab_v,
                                            const double* s_tab64, const ExactLds* s_ex, double (&acc)[kPartial],
                                            const Words4* sh_words = nullptr, const uint64_t* sh_local = nullptr) {
    constexpr int DEG = (RV == MLMC_RV_CUBIC16) ? 3 : 1;
    constexpr bool kExactOnly = (RV == MLMC_RV_EXACT);
    constexpr bool kNeedExact = kExactOnly || NESTED;
    constexpr bool kNeedApprox = !kExactOnly;
    constexpr bool kKahan = KAHAN && PREC != MLMC_FP64;
    constexpr int L = (PREC == MLMC_FP16) ? 2 : 1;  // paths per lane
    using AT = typename std::conditional<PREC == MLMC_FP64, double, float>::type;
    using Rnd = typename std::conditional<PREC == MLMC_BF16, RoundBF16, NoRound>::type;
    const Rnd rnd{};
    const AT* s_tab = (const AT*)s_tab_v;
    const __half* s_tab16 = (const __half*)s_tab_v;
    const float* mlpw = (const float*)s_tab_v;  // the MLP image when RV is MLMC_RV_MLP
    constexpr uint32_t kChunk = kWave * L;
    static_assert(SHORT == (NS == 1 || NS == 2) && (SHORT || NS == 0), "SHORT instances know their step count");
    const uint32_t n_calls = SHORT ? 1u : (prm.n_steps + 3) / 4;

    uint64_t local[L];
    bool valid[L];
    uint32_t path[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        local[l] = SHORT ? sh_local[l] : chunk * kChunk + (uint64_t)l * kWave + lane;
        valid[l] = local[l] < prm.n_paths;
        path[l] = (uint32_t)(prm.path_offset + (valid[l] ? local[l] : 0));
    }

    // exact pair (binary64)
    double Xfh[L], Xch[L], zh_prev[L];
    // binary64 fine path with approximate variables (diagnostic)
    double Xft[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        Xfh[l] = prm.x0_f64; Xch[l] = prm.x0_f64; zh_prev[l] = 0.0; Xft[l] = prm.x0_f64;
    }
    // approximate pair
    AT Xfb = (AT)(PREC == MLMC_FP64 ? prm.x0_f64 : prm.x0_f32), Xcb = Xfb, cfb = 0, ccb = 0, zb_prev = 0;
    const AT ca_b = (AT)(PREC == MLMC_FP64 ? prm.ca_f64 : prm.ca_f32);
    const AT cac_b = (AT)(PREC == MLMC_FP64 ? prm.cac_f64 : prm.cac_f32);
    const AT cb_b = (AT)(PREC == MLMC_FP64 ? prm.cb_f64 : prm.cb_f32);
    const AT cm_b = (AT)(PREC == MLMC_FP64 ? prm.cm_f64 : prm.cm_f32);
    const AT one_b = (AT)1, two_b = (AT)2;  // the Milstein offsets k, exact in every format
    __half2 Xf2 = __half2half2(prm.x0_f16), Xc2 = Xf2, cf2 = __float2half2_rn(0.0f), cc2 = cf2,
            z2_prev = cf2;
    const __half2 ca2 = __half2half2(prm.ca_f16), cac2 = __half2half2(prm.cac_f16),
                  cb2 = __half2half2(prm.cb_f16), cm2 = __half2half2(prm.cm_f16);
    const __half2 one2 = __float2half2_rn(1.0f), two2 = __float2half2_rn(2.0f);

    ExactConsts kc{};
    if constexpr (kNeedExact) kc = exact_consts();
    // the binary64 addends ca, cac of d = fma(cb, Z, ca) held in VGPRs for the chunk: an fma
    // reads at most one scalar operand, and cb is the other constant
    double ca64 = prm.ca_f64, cac64 = prm.cac_f64;
    asm volatile("" : "+v"(ca64), "+v"(cac64));
    for (uint32_t q = 0; q < n_calls; ++q) {
        Words4 r[L];
#pragma unroll
        for (int l = 0; l < L; ++l)
            r[l] = SHORT ? sh_words[l] : philox4x32_10(q, path[l], prm.ctr2, prm.pset, prm.key0, prm.key1);
        double zx[L][4];
        if constexpr (kNeedExact) {
            if constexpr (!SHORT) {
                // the exact pair of one path at a time: its four variables, then its four fine
                // and two coarse steps in step order (the binary16 lanes' second path reuses
                // the registers of the first)
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    double z4[4];
                    icdf_exact_f64x4(r[l].w, z4, &s_ex->top, deep_rows(prm), kc);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        em_step<SCHEME, double>(Xfh[l], z4[i], ca64, prm.cb_f64, prm.cm_f64, 1.0);
                        if (i & 1) em_step<SCHEME, double>(Xch[l], zh_prev[l] + z4[i], cac64, prm.cb_f64, prm.cm_f64, 2.0);
                        else zh_prev[l] = z4[i];
                    }
                }
            } else {
                // levels 0 and 1 use only the first one or two words of the call
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    zx[l][0] = icdf_exact_f64(r[l].w[0], &s_ex->top, deep_rows(prm));
                    if constexpr (NS > 1) zx[l][1] = icdf_exact_f64(r[l].w[1], &s_ex->top, deep_rows(prm));
                }
            }
        }
        // the learned variable of the call's four words together (binary64/binary32 paths,
        // levels >= 2): their matrix-instruction chains interleave
        float zmlp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (RV == MLMC_RV_MLP && PREC != MLMC_FP16 && !SHORT) {
            float za[2], zb[2];
            icdf_mlp_f32_k<2>(r[0].w, mlpw, za);
            icdf_mlp_f32_k<2>(r[0].w + 2, mlpw, zb);
            zmlp[0] = za[0]; zmlp[1] = za[1]; zmlp[2] = zb[0]; zmlp[3] = zb[1];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // only levels 0 and 1 stop inside a call, and they run as SHORT instances
            if constexpr (SHORT)
                if (i >= NS) break;
            const bool coarse = (i & 1) != 0;
            if constexpr (kNeedExact && SHORT) {
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    const double z = zx[l][i];
                    em_step<SCHEME, double>(Xfh[l], z, ca64, prm.cb_f64, prm.cm_f64, 1.0);
                    if (coarse)
                        em_step<SCHEME, double>(Xch[l], zh_prev[l] + z, cac64, prm.cb_f64, prm.cm_f64, 2.0);
                    else zh_prev[l] = z;
                }
            }
            if constexpr (kNeedApprox && PREC != MLMC_FP16) {
                AT z;
                if constexpr (RV == MLMC_RV_MLP && !SHORT) z = (AT)zmlp[i];
                else z = approx_rv<RV, DEG, AT, PREC>(r[0].w[i], s_tab, mlpw);
                if constexpr (kKahan) {
                    em_step_kahan<SCHEME, AT>(Xfb, cfb, z, ca_b, cb_b, cm_b, one_b, rnd);
                    if (coarse) em_step_kahan<SCHEME, AT>(Xcb, ccb, rnd(zb_prev + z), cac_b, cb_b, cm_b, two_b, rnd);
                } else {
                    em_step<SCHEME, AT>(Xfb, z, ca_b, cb_b, cm_b, one_b, rnd);
                    if (coarse) em_step<SCHEME, AT>(Xcb, rnd(zb_prev + z), cac_b, cb_b, cm_b, two_b, rnd);
                }
                if (!coarse) zb_prev = z;
            }
            if constexpr (kNeedApprox && PREC == MLMC_FP16) {
                __half2 z;
                if constexpr (RV == MLMC_RV_MLP) {
                    z = __halves2half2(__float2half_rn(icdf_mlp_f32(r[0].w[i], mlpw)),
                                       __float2half_rn(icdf_mlp_f32(r[1].w[i], mlpw)));
                } else if constexpr (RV == MLMC_RV_PCONST4096) {
                    z = __halves2half2(icdf_pconst_f16(r[0].w[i], s_tab16), icdf_pconst_f16(r[1].w[i], s_tab16));
                } else {
                    z = icdf_dyadic_f16x2<DEG>(r[0].w[i], r[1].w[i], s_tab16);
                }
                if constexpr (kKahan) {
                    em_step_kahan_h2<SCHEME>(Xf2, cf2, z, ca2, cb2, cm2, one2);
                    if (coarse) em_step_kahan_h2<SCHEME>(Xc2, cc2, __hadd2(z2_prev, z), cac2, cb2, cm2, two2);
                } else {
                    em_step_h2<SCHEME>(Xf2, z, ca2, cb2, cm2, one2);
                    if (coarse) em_step_h2<SCHEME>(Xc2, __hadd2(z2_prev, z), cac2, cb2, cm2, two2);
                }
                if (!coarse) z2_prev = z;
            }
            if constexpr (DIAG) {
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    double zt;
                    if constexpr (RV == MLMC_RV_MLP) zt = (double)icdf_mlp_f32(r[l].w[i], mlpw);
                    else if constexpr (RV == MLMC_RV_PCONST4096) zt = icdf_pconst_f64(r[l].w[i], s_tab64);
                    else zt = icdf_dyadic_f64<DEG>(r[l].w[i], s_tab64);
                    em_step<SCHEME, double>(Xft[l], zt, ca64, prm.cb_f64, prm.cm_f64, 1.0);
                }
            }
        }
    }

    // payoffs and differences (binary64), then the lane's contribution to the sums
    const bool has_coarse = SHORT ? NS > 1 : prm.level >= 1;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        double t[kTerms] = {0.0, 0.0, 0.0, 0.0};
        double pfh = 0.0, pch = 0.0, pfb = 0.0, pcb = 0.0, xfb = 0.0;
        if constexpr (kNeedExact) {
            pfh = payoff<double>(Xfh[l], prm.k_f64, prm.payoff);
            pch = has_coarse ? payoff<double>(Xch[l], prm.k_f64, prm.payoff) : 0.0;
        }
        if constexpr (kNeedApprox) {
            if constexpr (PREC == MLMC_FP16) {
                const __half xf = l == 0 ? __low2half(Xf2) : __high2half(Xf2);
                const __half xc = l == 0 ? __low2half(Xc2) : __high2half(Xc2);
                pfb = (double)__half2float(payoff_h(xf, prm.k_f16, prm.payoff));
                pcb = has_coarse ? (double)__half2float(payoff_h(xc, prm.k_f16, prm.payoff)) : 0.0;
                xfb = (double)__half2float(xf);
            } else {
                const AT kk = (AT)(PREC == MLMC_FP64 ? prm.k_f64 : prm.k_f32);
                pfb = (double)payoff<AT>(Xfb, kk, prm.payoff, rnd);
                pcb = has_coarse ? (double)payoff<AT>(Xcb, kk, prm.payoff, rnd) : 0.0;
                xfb = (double)Xfb;
            }
        }
        if constexpr (kExactOnly) {
            t[MLMC_TERM_TWO_WAY] = pfh - pch;
        } else {
            t[MLMC_TERM_TWO_WAY] = pfb - pcb;
            if constexpr (NESTED) {
                t[MLMC_TERM_TWO_WAY_EXACT] = pfh - pch;
                t[MLMC_TERM_FOUR_WAY] = t[MLMC_TERM_TWO_WAY_EXACT] - t[MLMC_TERM_TWO_WAY];
            }
            if constexpr (DIAG) t[MLMC_TERM_ROUNDING] = xfb - Xft[l];
        }
        if (valid[l]) {
#pragma unroll
            for (int k = 0; k < kTerms; ++k) {
                acc[k] += t[k];
                acc[kTerms + k] += t[k] * t[k];
            }
            const uint64_t o = local[l];
            if constexpr (kNeedExact) {
                if (prm.out_pf_hat) prm.out_pf_hat[o] = pfh;
                if (prm.out_pc_hat) prm.out_pc_hat[o] = pch;
            }
            if constexpr (kNeedApprox) {
                if (prm.out_pf_bar) prm.out_pf_bar[o] = pfb;
                if (prm.out_pc_bar) prm.out_pc_bar[o] = pcb;
            }
            if constexpr (DIAG) {
                if (prm.out_xf_tilde) prm.out_xf_tilde[o] = Xft[l];
            }
        }
    }
}

// One wave runs partial row `row`: chunks row * g .. row * g + g - 1 (g = row_chunks(level),
// those below the chunk count) one after another, each lane adding its terms in that order,
// then one wave reduction into prm.partials[row].  The instances that serve only levels >= 2
// (every one with the exact variable but the SHORT ones) have one-chunk rows, so their sums
// need no registers during the steps.
// Levels 0 and 1 (S = 2^LEVEL fine steps): one Philox call serves the G = 4 / S
// consecutive paths whose words it holds, so the lanes take a row's paths in groups of G:
// lane i takes groups k 64 + i of the row (k = 0, 1, ...), draws one call per group (two when
// the first path index is not a multiple of G), and runs the group's paths L at a time (two
// packed binary16 paths, else one), each lane adding them in that order.
template <int LEVEL, int PREC, int RV, bool NESTED, bool KAHAN, bool DIAG, int SCHEME>
__device__ __forceinline__ void short_row_terms(const LevelParams& prm, uint64_t row, uint32_t lane, const void* s_tab_v,
                                                const double* s_tab64, const ExactLds* s_ex, double (&acc)[kPartial]) {
    constexpr uint32_t S = 1u << LEVEL, G = 4u >> LEVEL;
    constexpr uint32_t L = (PREC == MLMC_FP16) ? 2 : 1;
    constexpr uint32_t kRowPaths = row_chunks(LEVEL, false) * kWave * L;
    static_assert(kRowPaths % (kWave * G) == 0 && G % L == 0, "whole groups per lane");
    const uint64_t first = row * kRowPaths;
    const uint32_t shift = (uint32_t)(prm.path_offset % G);  // wave-uniform
    for (uint32_t k = 0; k < kRowPaths / (kWave * G); ++k) {
        const uint64_t base = first + (uint64_t)G * (k * kWave + lane);  // the group's first path (local)
        const uint64_t gp = prm.path_offset + base;
        const Words4 c0 = philox4x32_10(0u, (uint32_t)(gp / G), prm.ctr2, prm.pset, prm.key0, prm.key1);
        Words4 c1 = c0;
        if (shift != 0) c1 = philox4x32_10(0u, (uint32_t)(gp / G + 1), prm.ctr2, prm.pset, prm.key0, prm.key1);
#pragma unroll
        for (uint32_t j = 0; j < G; j += L) {
            Words4 w[L] = {};
            uint64_t loc[L];
#pragma unroll
            for (uint32_t l = 0; l < L; ++l) {
                loc[l] = base + j + l;
#pragma unroll
                for (uint32_t n = 0; n < S; ++n) {
                    // word (shift + j + l) S + n of the two calls, in order
                    if (shift == 0) {
                        w[l].w[n] = c0.w[(j + l) * S + n];
                    } else {
                        const uint32_t e = (shift + j + l) * S + n;  // uniform, < 8
                        uint32_t x = c0.w[0];
#pragma unroll
                        for (uint32_t t = 1; t < 8; ++t)
                            if (e == t) x = t < 4 ? c0.w[t] : c1.w[t - 4];
                        w[l].w[n] = x;
                    }
                }
            }
            chunk_terms<PREC, RV, NESTED, KAHAN, DIAG, true, SCHEME, S>(prm, 0, lane, s_tab_v, s_tab64, s_ex, acc, w,
                                                                       loc);
        }
    }
}

template <int PREC, int RV, bool NESTED, bool KAHAN, bool DIAG, bool SHORT = false, int SCHEME = MLMC_SCHEME_EM>
__device__ __forceinline__ void run_row(const LevelParams& prm, uint64_t row, uint32_t lane, const void* s_tab_v,
                                        const double* s_tab64, const ExactLds* s_ex) {
    constexpr bool kOneChunkRows = !SHORT && (NESTED || RV == MLMC_RV_EXACT);
    double acc[kPartial];
#pragma unroll
    for (int k = 0; k < kPartial; ++k) acc[k] = 0.0;
    if constexpr (SHORT) {
        if (prm.level == 0) short_row_terms<0, PREC, RV, NESTED, KAHAN, DIAG, SCHEME>(prm, row, lane, s_tab_v, s_tab64, s_ex, acc);
        else short_row_terms<1, PREC, RV, NESTED, KAHAN, DIAG, SCHEME>(prm, row, lane, s_tab_v, s_tab64, s_ex, acc);
    } else if constexpr (kOneChunkRows) {
        chunk_terms<PREC, RV, NESTED, KAHAN, DIAG, SHORT, SCHEME>(prm, row, lane, s_tab_v, s_tab64, s_ex, acc);
    } else {
        constexpr uint32_t kChunk = kWave * ((PREC == MLMC_FP16) ? 2 : 1);
        const uint64_t n_chunks = (prm.n_paths + kChunk - 1) / kChunk;
        const uint64_t g = row_chunks(prm.level, true);  // approximate-only instances
        const uint64_t c0 = row * g;
        const uint64_t c1 = c0 + g < n_chunks ? c0 + g : n_chunks;
        for (uint64_t c = c0; c < c1; ++c)
            chunk_terms<PREC, RV, NESTED, KAHAN, DIAG, SHORT, SCHEME>(prm, c, lane, s_tab_v, s_tab64, s_ex, acc);
    }
    store_row(acc, lane, prm.partials + row * kPartial);
}

// SHORT: the instance for levels with fewer than 4 fine steps (exact variables one word at a time).
// SCHEME: MLMC_SCHEME_EM or MLMC_SCHEME_MILSTEIN.
template <int PREC, int RV, bool NESTED, bool KAHAN, bool DIAG, bool SHORT = false, int SCHEME = MLMC_SCHEME_EM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SHORT ? 1 : RV == MLMC_RV_MLP ? 6 : (PREC == MLMC_FP32 || PREC == MLMC_FP64) ? 7 : PREC == MLMC_FP16 ? 6 : 1))) void level_kernel(const LevelParams prm) {
    constexpr int DEG = (RV == MLMC_RV_CUBIC16) ? 3 : 1;
    constexpr bool kDyadic = (RV == MLMC_RV_PWL16 || RV == MLMC_RV_CUBIC16);
    constexpr bool kPconst = (RV == MLMC_RV_PCONST4096);
    constexpr int L = (PREC == MLMC_FP16) ? 2 : 1;
    using AT = typename std::conditional<PREC == MLMC_FP64, double, float>::type;

    // coefficient tables or cell means in LDS (working precision, and binary64 for the
    // diagnostic), each sized for the variant that reads it
    constexpr int kTabN = kPconst ? kPcEntries : kTableRowsDev * (DEG + 1);
    constexpr bool kTab16 = PREC == MLMC_FP16 && (kDyadic || kPconst);
    __shared__ AT s_tab[(kDyadic || kPconst) && !kTab16 ? kTabN : 1];
    __shared__ __half s_tab16[kTab16 ? kTabN : 1];
    __shared__ double s_tab64[(kDyadic || kPconst) && DIAG ? kTabN : 1];
    __shared__ __align__(16) float s_mlp[RV == MLMC_RV_MLP ? kMlpImage : 1];  // 16-byte operand loads
    // the exact variable's top cells
    constexpr size_t kExBytes = (RV == MLMC_RV_EXACT || NESTED) ? sizeof(ExactCols) : 0;
    __shared__ __align__(16) unsigned char s_ex_raw[kExBytes ? kExBytes : 16];
    const ExactLds* s_ex = (const ExactLds*)s_ex_raw;
    if constexpr (kExBytes > 0) {
        stage_exact_table(s_ex_raw, prm.exact_tab, kExBytes);
        __syncthreads();
    }
    if constexpr (kDyadic) {
        for (int i = threadIdx.x; i < kTabN; i += blockDim.x) {
            if constexpr (PREC == MLMC_FP16) s_tab16[i] = ((const __half*)prm.table)[i];
            else if constexpr (PREC == MLMC_FP32) s_tab[i] = prescaled_coeff(((const float*)prm.table)[i], i % (DEG + 1));
            else if constexpr (PREC == MLMC_BF16) s_tab[i] = ((const float*)prm.table)[i];  // bfloat16 values, unscaled
            else s_tab[i] = ((const AT*)prm.table)[i];
            if constexpr (DIAG) s_tab64[i] = prm.table64[i];
        }
        __syncthreads();
    }
    if constexpr (kPconst) {
        for (int i = threadIdx.x; i < kTabN; i += blockDim.x) {
            if constexpr (PREC == MLMC_FP16) s_tab16[i] = ((const __half*)prm.table)[i];
            else s_tab[i] = ((const AT*)prm.table)[i];
            if constexpr (DIAG) s_tab64[i] = prm.table64[i];
        }
        __syncthreads();
    }
    if constexpr (RV == MLMC_RV_MLP) {
        for (int i = threadIdx.x; i < kMlpImage; i += blockDim.x) s_mlp[i] = ((const float*)prm.mlp)[i];
        __syncthreads();
    }
    const void* tab = RV == MLMC_RV_MLP ? (const void*)s_mlp
                                        : (PREC == MLMC_FP16 ? (const void*)s_tab16 : (const void*)s_tab);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    constexpr uint32_t kChunk = kWave * L;
    const uint64_t n_rows = rows_of((prm.n_paths + kChunk - 1) / kChunk, prm.level, !NESTED && RV != MLMC_RV_EXACT);
    for (uint64_t row = wave; row < n_rows; row += n_waves)
        run_row<PREC, RV, NESTED, KAHAN, DIAG, SHORT, SCHEME>(prm, row, lane, tab, s_tab64, s_ex);
}

}  // namespace mlmc
