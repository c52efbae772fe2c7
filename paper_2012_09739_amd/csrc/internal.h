// Internal definitions shared by the host library and its kernels (not part of the C-ABI).
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mlmc.h"

namespace mlmc {

constexpr int kTerms = 4;           // two-way, four-way, two-way exact part, rounding diagnostic
constexpr int kPartial = 2 * kTerms;  // (sum, sum of squares) per term
constexpr int kWave = 64;
constexpr int kMaxLevel = 24;
constexpr int kTableRows = 16;
// Device layout of a dyadic table: row r serves clz(2 xm + 1) = r, so rows 15..31 all hold
// the coefficients of the last interval (0, 2^-16) and the row needs no clamp.
constexpr int kTableRowsDev = 32;
// piecewise-constant variable: 2^kPcBits equal cells of (0, 1), the lower half stored
constexpr int kPcBits = 12;
constexpr int kPcEntries = 1 << (kPcBits - 1);

// Per-launch parameters of one MLMC level (one parameter set).  Constants are rounded
// on the host from binary64, once, to the working precision p (R_p(mu delta) etc.).
struct LevelParams {
    // exact pair (binary64); cm is the Milstein constant sigma^2 delta_f / 2
    double ca_f64, cac_f64, cb_f64, x0_f64, k_f64, cm_f64;
    // approximate pair in binary32, or in emulated bfloat16 (then rounded to 8 bits)
    float ca_f32, cac_f32, cb_f32, x0_f32, k_f32, cm_f32;
    // approximate pair in binary16
    __half ca_f16, cac_f16, cb_f16, x0_f16, k_f16, cm_f16;
    int payoff;
    int level;
    uint32_t n_steps;
    uint64_t n_paths;      // paths in this launch
    uint64_t path_offset;  // first global path index (Philox counter word 1)
    uint32_t key0, key1;   // seed
    uint32_t ctr2;         // (stream << 16) | level
    uint32_t pset;
    const void* table;     // 16 x (DEG + 1) coefficients (dyadic) or kPcEntries cell means, working precision
    const double* table64; // the same in binary64 (diagnostic)
    const void* mlp;       // MLP inference image (rv = MLP)
    const void* exact_tab; // ExactTable: rows of the exact inverse CDF, log cells
    double* partials;      // [n_rows][kPartial] partial sums of the rows (row_chunks chunks each)
    // optional per-path outputs (device, n_paths entries each, may be null)
    double* out_pf_hat;
    double* out_pc_hat;
    double* out_pf_bar;
    double* out_pc_bar;
    double* out_xf_tilde;
};

// Template variant selector.
struct Variant {
    int precision;  // MLMC_FP64 / MLMC_FP32 / MLMC_FP16 / MLMC_BF16
    int rv;         // MLMC_RV_EXACT / PWL16 / CUBIC16 / MLP
    bool nested;
    bool kahan;
    bool diag;
    int scheme;     // MLMC_SCHEME_EM / MLMC_SCHEME_MILSTEIN
};

// Launch helpers implemented in the .hip translation units.
hipError_t launch_level(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
// Single-level calls of the nested binary32 estimators and of the plain binary64 one (EM, no
// diagnostic) at level >= kCoopMinLevel with at most kCoopMaxRowsPerCu partial rows per CU run
// one eight-wave block per chunk (cooperative chunks): same partial rows, same bits, a shorter
// dependent chain.
constexpr int kCoopMinLevel = 6;
constexpr int kCoopMaxRowsPerCu = 4;
bool coop_level_call(const Variant& v, int level, uint64_t n_rows, int n_cu);
hipError_t launch_level_coop(const Variant& v, const LevelParams& p, uint64_t n_rows, hipStream_t s);
hipError_t launch_reduce(const double* partials, uint64_t n_rows, double* stage, double* d_out, hipStream_t s);

// Chunks per partial row.  A row is the unit of the fixed-order reduction: a wave simulates
// the row's chunks one after another, each lane adding its paths' terms in that order, then
// reduces the row once.  At the coarse levels a chunk is only a few steps long, so the wave
// reduction and the per-wave set-up would otherwise cost more than the paths.  Levels 0 and 1
// take 8 and 4 chunks per row; from level 2 the instances with the exact variable take one
// (their sums then hold no registers during the steps), the approximate-only ones 8, 4 and 2
// at levels 2, 3 and 4 (at least 32 steps per lane between two reductions) and one above.
// Grouping depends on the level and the estimator's kind alone, so every call and batch item
// of a level and kind reduces its paths alike.
__host__ __device__ constexpr inline uint32_t row_chunks(int level, bool approx_only) {
    return level < 2 ? (8u >> level) : (approx_only && level < 5) ? (32u >> level) : 1u;
}
__host__ __device__ inline uint64_t rows_of(uint64_t n_chunks, int level, bool approx_only) {
    const uint64_t g = row_chunks(level, approx_only);
    return (n_chunks + g - 1) / g;
}

// Workspace of one level call: the partial rows and the stage rows of the two-stage
// reduction (at most 128 rows of kPartial doubles), plus 64 bytes of slack.
constexpr uint64_t kStageRowsMax = 128;
inline size_t level_workspace_bytes(uint64_t n_rows) {
    return (size_t)((n_rows == 0 ? 1 : n_rows) + kStageRowsMax) * kPartial * sizeof(double) + 64;
}
hipError_t launch_uniforms(uint64_t seed, uint32_t ctr2, uint32_t pset, uint64_t path0,
                           uint64_t n_paths, uint32_t n_steps, uint32_t* d_words, hipStream_t s);
hipError_t launch_icdf(const uint32_t* d_words, uint64_t n, int rv, int precision, const void* table,
                       const void* mlp, const void* exact_tab, double* d_out, hipStream_t s);

// Device resources the library keeps for the current device (lazily initialised).
struct DeviceInfo {
    int n_cu;
    const void* tables[2][4];  // [pwl, cubic][precision]
    const double* tables64[2];
    const void* pconst[4];     // cell means of the piecewise-constant variable, [precision]
    const void* mlp;
    bool mlp_loaded;
    const void* exact_tab;
};
int device_info(DeviceInfo* out);
int set_error(int code, const char* fmt, ...);
int validate_sde_public(const mlmc_gbm_t* s);
void fill_level_params(LevelParams* p, const mlmc_gbm_t& s, int level, int precision, uint64_t n_paths,
                       uint64_t path_offset, uint64_t seed, uint32_t stream, uint32_t pset);

// Paths covered by one wave-chunk (the unit of the fixed-order reduction).
inline uint32_t chunk_paths(int precision) { return precision == MLMC_FP16 ? 2 * kWave : kWave; }

}  // namespace mlmc
