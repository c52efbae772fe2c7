// Cooperative chunks: one 64-path chunk of a nested binary32 level run by a whole block, its
// producer waves drawing the uniforms and both inverse CDFs ahead of the consumer wave that
// advances the coupled paths.  Shared by the batched sweep and by the single-level calls whose
// few long chunks would otherwise run one wave each, latency bound.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "level_kernel.h"

namespace mlmc {

// Blocks of WAVES = 8 or 4 wavefronts; a cooperative chunk's producers are waves
// 1 .. WAVES - 1, each drawing one Philox call (four fine steps) per phase.
template <int WAVES>
struct Coop {
    static constexpr int kProducers = WAVES - 1;
    static constexpr int kSteps = 4 * kProducers;  // fine steps per phase
};

// One cooperative chunk of a nested binary32 item, or (RV = MLMC_RV_EXACT) of the plain
// binary64 estimator, (n_steps >= 4, a multiple of 4) run by the whole block of WAVES waves,
// P = WAVES - 1 of them producers.  Phase f covers fine steps [4 P f, 4 P f + 4 P): producer
// wave p draws Philox call P f + p - 1 and writes its four exact (binary64) and approximate
// (binary32) variables into ring slot f & 1; the consumer, wave 0, reads slot f & 1 while the
// producers fill slot (f + 1) & 1, and a barrier closes every phase (the same number of
// barriers in every wave).  The consumer's updates and payoff terms are those of the
// single-wave code for this variant, in the same order.  The plain estimator has no
// approximate pair: ring_b and s_tab are then not used (may be null).
template <int RV, bool KAHAN, int WAVES>
__device__ inline void run_chunk_coop(const LevelParams& prm, uint64_t chunk, const float* s_tab, const ExactLds* s_ex,
                                      double (*ring_x)[Coop<WAVES>::kSteps][kWave],
                                      float (*ring_b)[Coop<WAVES>::kSteps][kWave]) {
    constexpr int kCoopProducers = Coop<WAVES>::kProducers;
    constexpr int kCoopSteps = Coop<WAVES>::kSteps;
    constexpr int DEG = RV == MLMC_RV_CUBIC16 ? 3 : 1;
    constexpr bool kExactOnly = RV == MLMC_RV_EXACT;
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t local = chunk * kWave + lane;
    const bool valid = local < prm.n_paths;
    const uint32_t path = (uint32_t)(prm.path_offset + (valid ? local : 0));
    const uint32_t n_calls = prm.n_steps / 4;
    const uint32_t n_phases = (n_calls + kCoopProducers - 1) / kCoopProducers;

    if (wave != 0) {
        const ExactConsts kc = exact_consts();
        const uint32_t base = 4 * (wave - 1);
        for (uint32_t f = 0; f <= n_phases; ++f) {
            const uint32_t q = f * kCoopProducers + (wave - 1);
            if (f < n_phases && q < n_calls) {
                const Words4 r = philox4x32_10(q, path, prm.ctr2, prm.pset, prm.key0, prm.key1);
                double zx[4];
                icdf_exact_f64x4(r.w, zx, &s_ex->top, deep_rows(prm), kc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ring_x[f & 1][base + i][lane] = zx[i];
                    if constexpr (!kExactOnly)
                        ring_b[f & 1][base + i][lane] = approx_rv<RV, DEG, float, MLMC_FP32>(r.w[i], s_tab, nullptr);
                }
            }
            __syncthreads();  // phase f written; the consumer is done with slot (f + 1) & 1
        }
        return;
    }

    double Xfh = prm.x0_f64, Xch = prm.x0_f64, zh_prev = 0.0;
    float Xfb = prm.x0_f32, Xcb = Xfb, cfb = 0.0f, ccb = 0.0f, zb_prev = 0.0f;
    const NoRound rnd{};
    // step i of a phase (phases start at an even step, so odd steps close a coarse step)
    auto step = [&](int i, double z, float zb) {
        const bool coarse = (i & 1) != 0;
        em_step<MLMC_SCHEME_EM, double>(Xfh, z, prm.ca_f64, prm.cb_f64, prm.cm_f64, 1.0);
        if (coarse) em_step<MLMC_SCHEME_EM, double>(Xch, zh_prev + z, prm.cac_f64, prm.cb_f64, prm.cm_f64, 2.0);
        else zh_prev = z;
        if constexpr (kExactOnly) return;
        if constexpr (KAHAN) {
            em_step_kahan<MLMC_SCHEME_EM, float>(Xfb, cfb, zb, prm.ca_f32, prm.cb_f32, prm.cm_f32, 1.0f, rnd);
            if (coarse)
                em_step_kahan<MLMC_SCHEME_EM, float>(Xcb, ccb, rnd(zb_prev + zb), prm.cac_f32, prm.cb_f32, prm.cm_f32,
                                                     2.0f, rnd);
        } else {
            em_step<MLMC_SCHEME_EM, float>(Xfb, zb, prm.ca_f32, prm.cb_f32, prm.cm_f32, 1.0f, rnd);
            if (coarse) em_step<MLMC_SCHEME_EM, float>(Xcb, rnd(zb_prev + zb), prm.cac_f32, prm.cb_f32, prm.cm_f32, 2.0f, rnd);
        }
        if (!coarse) zb_prev = zb;
    };
    __syncthreads();  // phase 0 written
    for (uint32_t f = 0; f < n_phases; ++f) {
        const uint32_t left = prm.n_steps - f * kCoopSteps;
        if (left >= (uint32_t)kCoopSteps) {
            // a full phase, unrolled with no exits: the ring reads of all its steps can be
            // issued ahead of the dependent updates instead of one LDS round trip per step
            double z[kCoopSteps];
            float zb[kCoopSteps];
#pragma unroll
            for (int i = 0; i < kCoopSteps; ++i) {
                z[i] = ring_x[f & 1][i][lane];
                zb[i] = kExactOnly ? 0.0f : ring_b[f & 1][i][lane];
            }
#pragma unroll
            for (int i = 0; i < kCoopSteps; ++i) step(i, z[i], zb[i]);
        } else {
            for (int i = 0; i < (int)left; ++i) step(i, ring_x[f & 1][i][lane], kExactOnly ? 0.0f : ring_b[f & 1][i][lane]);
        }
        __syncthreads();  // phase f + 1 written; slot f & 1 free again
    }

    // payoffs and differences (binary64), as the single-wave code for the chunk
    double acc[kPartial];
#pragma unroll
    for (int k = 0; k < kPartial; ++k) acc[k] = 0.0;
    const bool has_coarse = prm.level >= 1;
    double t[kTerms] = {0.0, 0.0, 0.0, 0.0};
    const double pfh = payoff<double>(Xfh, prm.k_f64, prm.payoff);
    const double pch = has_coarse ? payoff<double>(Xch, prm.k_f64, prm.payoff) : 0.0;
    if constexpr (kExactOnly) {
        t[MLMC_TERM_TWO_WAY] = pfh - pch;
    } else {
        const float kk = prm.k_f32;
        const double pfb = (double)payoff<float>(Xfb, kk, prm.payoff, rnd);
        const double pcb = has_coarse ? (double)payoff<float>(Xcb, kk, prm.payoff, rnd) : 0.0;
        t[MLMC_TERM_TWO_WAY] = pfb - pcb;
        t[MLMC_TERM_TWO_WAY_EXACT] = pfh - pch;
        t[MLMC_TERM_FOUR_WAY] = t[MLMC_TERM_TWO_WAY_EXACT] - t[MLMC_TERM_TWO_WAY];
    }
    if (valid) {
#pragma unroll
        for (int k = 0; k < kTerms; ++k) {
            acc[k] += t[k];
            acc[kTerms + k] += t[k] * t[k];
        }
    }
    // cooperative items are at least level 2, where a partial row is one chunk
    store_row(acc, lane, prm.partials + chunk * kPartial);
}

}  // namespace mlmc
