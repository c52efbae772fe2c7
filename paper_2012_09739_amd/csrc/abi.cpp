// The C-ABI of libmlmc: argument validation, per-device state, constants, dispatch.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp.h"

namespace mlmc {

bool build_l2_table(int degree, double out[16][4]);
bool build_pconst_table(int bits, double* out);
hipError_t launch_mlp_deploy(const float* d_params, float* image, hipStream_t s);
hipError_t launch_level_f64(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
hipError_t launch_level_f32(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
hipError_t launch_level_f16(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
hipError_t launch_level_bf16(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
hipError_t launch_level_milstein_f64(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
hipError_t launch_level_milstein_f32(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
hipError_t launch_level_milstein_f16(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);
hipError_t launch_level_milstein_bf16(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s);

hipError_t launch_level(const Variant& v, const LevelParams& p, int grid, int block, hipStream_t s) {
    if (v.scheme == MLMC_SCHEME_MILSTEIN) {
        switch (v.precision) {
            case MLMC_FP64: return launch_level_milstein_f64(v, p, grid, block, s);
            case MLMC_FP32: return launch_level_milstein_f32(v, p, grid, block, s);
            case MLMC_BF16: return launch_level_milstein_bf16(v, p, grid, block, s);
            default: return launch_level_milstein_f16(v, p, grid, block, s);
        }
    }
    switch (v.precision) {
        case MLMC_FP64: return launch_level_f64(v, p, grid, block, s);
        case MLMC_FP32: return launch_level_f32(v, p, grid, block, s);
        case MLMC_BF16: return launch_level_bf16(v, p, grid, block, s);
        default: return launch_level_f16(v, p, grid, block, s);
    }
}

// R_bf16(x): a finite binary64 value rounded once to 8 significant bits, to nearest with
// ties to even (the constants and tables of the emulated bfloat16 paths).
double bf16_of(double x) {
    uint64_t u;
    std::memcpy(&u, &x, sizeof u);
    const uint64_t d = 45;  // 53 - 8 dropped bits
    u = (u + ((1ull << (d - 1)) - 1) + ((u >> d) & 1ull)) & ~((1ull << d) - 1);
    std::memcpy(&x, &u, sizeof x);
    return x;
}

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(MLMC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- host tables (binary64 masters of the two dyadic approximations) ------------------
struct HostTables {
    double pwl[16][4];
    double cubic[16][4];
    double pconst[kPcEntries];  // lower-half cell means of the piecewise-constant variable
    bool ok = false;
    HostTables() { ok = build_l2_table(1, pwl) && build_l2_table(3, cubic) && build_pconst_table(kPcBits, pconst); }
};

// value of a binary64 master rounded once to precision p, widened back to binary64
double rounded_to(int precision, double c);

const HostTables& host_tables() {
    static const HostTables t;
    return t;
}

int degree_of(int rv) { return rv == MLMC_RV_CUBIC16 ? 3 : 1; }

// binary64 -> binary16 with one correctly rounded conversion (round to nearest even)
__half half_of(double d) {
    const _Float16 f = (_Float16)d;
    __half h;
    std::memcpy(&h, &f, sizeof h);
    return h;
}

double rounded_to(int precision, double c) {
    if (precision == MLMC_FP32) return (double)(float)c;
    if (precision == MLMC_FP16) return (double)__half2float(half_of(c));
    if (precision == MLMC_BF16) return bf16_of(c);
    return c;
}

// ---- device scratch of mlmc_level_noalloc --------------------------------------------------
// The chunk partials and stage rows of one level call, for callers that cannot allocate: a
// file-scope device array (each device holds its own copy from the time the code object is
// loaded until the process ends).  Host code never passes `scratch` itself to a kernel (on the
// host the name is a stand-in, not a device address); device_state() looks up each device's
// address once with hipGetSymbolAddress and keeps it in DevState::noalloc_scratch.
constexpr uint64_t kNoAllocMaxChunks = 65536;  // 2^22 paths in binary32/64, 2^23 in binary16
constexpr size_t kNoAllocBytes = (size_t)(kNoAllocMaxChunks + kStageRowsMax) * kPartial * sizeof(double) + 64;
static_assert(kNoAllocBytes % 8 == 0, "scratch holds doubles");
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

// ---- per-device state -------------------------------------------------------------------
constexpr int kSetStreams = 4;     // streams of a level set (the hardware queues of a process)
constexpr int kMaxSetCalls = 4096;  // calls per level set

struct DevState {
    bool ready = false;
    int n_cu = 256;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    void* tables[2][4] = {{nullptr}};  // [pwl, cubic][precision], 16 x (d+1) coefficients
    double* tables64[2] = {nullptr, nullptr};
    void* pconst[4] = {nullptr};       // [precision], kPcEntries cell means
    double* scratch = nullptr;
    size_t scratch_bytes = 0;
    double* noalloc_scratch = nullptr;  // this device's address of `scratch`
    double* out8 = nullptr;             // result slot of the synchronous entry point
    float* mlp = nullptr;               // MLP inference image (binary16 values as binary32)
    void* exact_tab = nullptr;          // ExactTable: cells of the exact variable, log cells
    bool mlp_loaded = false;
    // level sets: their own streams, events (two per call and two per set) and device memory
    // (result slots, then one workspace per call), created on first use
    hipStream_t set_stream[kSetStreams] = {nullptr};
    std::vector<hipEvent_t> set_events;
    void* set_mem = nullptr;
    size_t set_mem_bytes = 0;
};

std::mutex g_mutex;
std::map<int, DevState> g_devs;

int current_device(int* dev) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(MLMC_ENODEV, "no HIP device available");
    }
    e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return MLMC_OK;
}

int upload_tables(DevState& st) {
    const HostTables& ht = host_tables();
    if (!ht.ok) return fail(MLMC_EHIP, "dyadic table construction failed");
    for (int r = 0; r < 2; ++r) {
        const double(*src)[4] = r == 0 ? ht.pwl : ht.cubic;
        const int d = r == 0 ? 1 : 3;
        const int n = kTableRowsDev * (d + 1);  // device layout: rows 15..31 repeat interval 16
        double h64[kTableRowsDev * 4];
        float h32[kTableRowsDev * 4];
        __half h16[kTableRowsDev * 4];
        float hbf[kTableRowsDev * 4];
        for (int j = 0; j < kTableRowsDev; ++j)
            for (int i = 0; i <= d; ++i) {
                const double c = src[j < kTableRows ? j : kTableRows - 1][i];
                h64[j * (d + 1) + i] = c;
                h32[j * (d + 1) + i] = (float)c;
                h16[j * (d + 1) + i] = half_of(c);  // one rounding from binary64
                hbf[j * (d + 1) + i] = (float)bf16_of(c);  // one rounding from binary64, exact in binary32
            }
        hipError_t e;
        if ((e = hipMalloc(&st.tables[r][MLMC_FP64], n * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipMalloc(&st.tables[r][MLMC_FP32], n * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipMalloc(&st.tables[r][MLMC_FP16], n * sizeof(__half))) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipMalloc(&st.tables[r][MLMC_BF16], n * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipMemcpy(st.tables[r][MLMC_FP64], h64, n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(st.tables[r][MLMC_FP32], h32, n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(st.tables[r][MLMC_FP16], h16, n * sizeof(__half), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(st.tables[r][MLMC_BF16], hbf, n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "hipMemcpy");
        st.tables64[r] = (double*)st.tables[r][MLMC_FP64];
    }
    {
        static double h64[kPcEntries];
        static float h32[kPcEntries], hbf[kPcEntries];
        static __half h16[kPcEntries];
        for (int i = 0; i < kPcEntries; ++i) {
            const double c = ht.pconst[i];
            h64[i] = c;
            h32[i] = (float)c;
            h16[i] = half_of(c);
            hbf[i] = (float)bf16_of(c);
        }
        const void* src[4] = {h64, h32, h16, hbf};
        const size_t bytes[4] = {sizeof h64, sizeof h32, sizeof h16, sizeof hbf};
        for (int q = 0; q < 4; ++q) {
            hipError_t e;
            if ((e = hipMalloc(&st.pconst[q], bytes[q])) != hipSuccess) return hip_fail(e, "hipMalloc");
            if ((e = hipMemcpy(st.pconst[q], src[q], bytes[q], hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(e, "hipMemcpy");
        }
    }
    return MLMC_OK;
}

// Returns the initialised state of the current device (lazily created).
int device_state(DevState** out) {
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mutex);
    DevState& st = g_devs[dev];
    if (!st.ready) {
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(MLMC_ENODEV, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
        st.n_cu = prop.multiProcessorCount;
        if ((e = hipGetSymbolAddress((void**)&st.noalloc_scratch, HIP_SYMBOL(scratch))) != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if ((e = hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
        if ((e = hipEventCreate(&st.ev0)) != hipSuccess || (e = hipEventCreate(&st.ev1)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");
        if ((e = hipMalloc(&st.out8, kPartial * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipMalloc(&st.mlp, kMlpImage * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc");
        {
            // log cells (the learned variable's input): cell i covers the frexp mantissa m in
            // [(1 + i/256)/2, (1 + (i+1)/256)/2): f = R(1/c), l = R(-log f), c the centre; then
            // the generated rows of G, row k for the key kKeyMin + k: the deep ones as rows, the
            // top ones in three arrays
            static ExactTable h;
            for (int i = 0; i < kLogCells; ++i) {
                const double c = 0.5 + (i + 0.5) / (2.0 * kLogCells);
                const double f = 1.0 / c;
                h.lds.log[i].f = f;
                h.lds.log[i].l = (double)(-std::log((long double)f));
            }
            static const double kRows[] = MLMC_EXACT_COEFFS;
            static_assert(sizeof kRows == sizeof(double) * kExactRows * (kExactDeg + 1), "exact table size");
            for (int k = 0; k < kExactRows; ++k) {
                const double* v = kRows + k * (kExactDeg + 1);
                if (k < kDeepRows) {
                    for (int j = 0; j < kRowLen; ++j) h.deep[k][j] = j <= kExactDeg ? v[j] : 0.0;
                } else {  // (coefficients 5 and 6 of a top cell are binary32 values)
                    const int i = k - kDeepRows;
                    h.lds.top.c01[i] = make_double2(v[0], v[1]);
                    h.lds.top.c23[i] = make_double2(v[2], v[3]);
                    h.lds.top.c45[i] = make_double2(v[4], v[5]);
                    h.lds.top.c6[i] = make_double2(v[6], 0.0);
                }
            }
            if ((e = hipMalloc(&st.exact_tab, sizeof h)) != hipSuccess) return hip_fail(e, "hipMalloc");
            if ((e = hipMemcpy(st.exact_tab, &h, sizeof h, hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(e, "hipMemcpy");
        }
        rc = upload_tables(st);
        if (rc) return rc;
        st.ready = true;
    }
    *out = &st;
    return MLMC_OK;
}

int ensure_scratch(DevState& st, size_t bytes) {
    if (bytes <= st.scratch_bytes) return MLMC_OK;
    if (st.scratch) {
        hipError_t e = hipStreamSynchronize(st.stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(st.scratch);
        st.scratch = nullptr;
        st.scratch_bytes = 0;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    hipError_t e = hipMalloc(&st.scratch, want);
    if (e != hipSuccess) return fail(MLMC_ENOMEM, "hipMalloc of %zu scratch bytes failed", want);
    st.scratch_bytes = want;
    return MLMC_OK;
}

// ---- argument validation (no HIP calls) ---------------------------------------------------
bool finite(double v) { return std::isfinite(v); }

int validate_sde(const mlmc_gbm_t* s) {
    if (!s) return fail(MLMC_EINVAL, "sde is NULL");
    if (!finite(s->mu) || !finite(s->sigma) || !finite(s->x0) || !finite(s->T) || !finite(s->strike))
        return fail(MLMC_EINVAL, "sde has a non-finite field");
    if (!(s->T > 0)) return fail(MLMC_EINVAL, "sde.T must be positive");
    if (s->sigma < 0) return fail(MLMC_EINVAL, "sde.sigma must be non-negative");
    if (s->payoff != MLMC_PAYOFF_X && s->payoff != MLMC_PAYOFF_CALL)
        return fail(MLMC_EINVAL, "sde.payoff %d is not MLMC_PAYOFF_X or MLMC_PAYOFF_CALL", s->payoff);
    return MLMC_OK;
}

int rv_of_mode(int rv_mode, int* rv, bool* nested) {
    switch (rv_mode) {
        case MLMC_EXACT: *rv = MLMC_RV_EXACT; *nested = false; return MLMC_OK;
        case MLMC_APPROX_PWL16: *rv = MLMC_RV_PWL16; *nested = false; return MLMC_OK;
        case MLMC_APPROX_CUBIC16: *rv = MLMC_RV_CUBIC16; *nested = false; return MLMC_OK;
        case MLMC_APPROX_MLP: *rv = MLMC_RV_MLP; *nested = false; return MLMC_OK;
        case MLMC_NESTED_PWL16: *rv = MLMC_RV_PWL16; *nested = true; return MLMC_OK;
        case MLMC_NESTED_CUBIC16: *rv = MLMC_RV_CUBIC16; *nested = true; return MLMC_OK;
        case MLMC_NESTED_MLP: *rv = MLMC_RV_MLP; *nested = true; return MLMC_OK;
        case MLMC_APPROX_PCONST4096: *rv = MLMC_RV_PCONST4096; *nested = false; return MLMC_OK;
        case MLMC_NESTED_PCONST4096: *rv = MLMC_RV_PCONST4096; *nested = true; return MLMC_OK;
        default: return fail(MLMC_EINVAL, "rv_mode %d is not a valid MLMC_EXACT/APPROX/NESTED mode", rv_mode);
    }
}

int validate_args(const mlmc_level_args_t* a, Variant* v) {
    if (!a) return fail(MLMC_EINVAL, "args is NULL");
    int rc = validate_sde(&a->sde);
    if (rc) return rc;
    if (a->level < 0 || a->level > kMaxLevel) return fail(MLMC_EINVAL, "level %d outside 0..%d", a->level, kMaxLevel);
    if (a->precision < MLMC_FP64 || a->precision > MLMC_BF16)
        return fail(MLMC_EINVAL, "precision %d is not MLMC_FP64/FP32/FP16/BF16", a->precision);
    if (a->kahan != 0 && a->kahan != 1) return fail(MLMC_EINVAL, "kahan must be 0 or 1");
    if (a->diag != 0 && a->diag != 1) return fail(MLMC_EINVAL, "diag must be 0 or 1");
    if (a->stream > 0xFFFFu) return fail(MLMC_EINVAL, "stream %u exceeds 65535", a->stream);
    const uint64_t lim = 1ull << 32;
    if (a->n_paths > lim || a->path_offset > lim || a->path_offset + a->n_paths > lim)
        return fail(MLMC_EINVAL, "path_offset + n_paths exceeds 2^32");
    int rv;
    bool nested;
    rc = rv_of_mode(a->rv_mode, &rv, &nested);
    if (rc) return rc;
    if (rv == MLMC_RV_EXACT && a->precision != MLMC_FP64)
        return fail(MLMC_EINVAL, "MLMC_EXACT (the plain estimator) runs in MLMC_FP64");
    if (rv == MLMC_RV_EXACT && a->diag) return fail(MLMC_EINVAL, "diag needs an approximate rv_mode");
    if (a->precision == MLMC_BF16 && rv == MLMC_RV_MLP)
        return fail(MLMC_EINVAL, "MLMC_BF16 runs the table approximations (PWL16, CUBIC16, PCONST4096) only");
    if (a->scheme != MLMC_SCHEME_EM && a->scheme != MLMC_SCHEME_MILSTEIN)
        return fail(MLMC_EINVAL, "scheme %u is not MLMC_SCHEME_EM/MILSTEIN", a->scheme);
    if (a->scheme == MLMC_SCHEME_MILSTEIN && rv == MLMC_RV_MLP)
        return fail(MLMC_EINVAL, "MLMC_SCHEME_MILSTEIN runs with exact and dyadic variables only");
    v->scheme = (int)a->scheme;
    v->precision = a->precision;
    v->rv = rv;
    v->nested = nested;
    v->kahan = a->kahan && a->precision != MLMC_FP64;
    v->diag = a->diag != 0;
    return MLMC_OK;
}

uint64_t n_chunks_of(const mlmc_level_args_t* a) {
    const uint64_t cp = chunk_paths(a->precision);
    return (a->n_paths + cp - 1) / cp;
}

// approximate-only estimators (no exact variable): their rows group more chunks from level 2
bool approx_only_mode(int rv_mode) { return rv_mode != MLMC_EXACT && rv_mode < MLMC_NESTED_PWL16; }
uint64_t n_rows_of(const mlmc_level_args_t* a) {
    return rows_of(n_chunks_of(a), a->level, approx_only_mode(a->rv_mode));
}

LevelParams make_params(const mlmc_level_args_t* a, const Variant& v, const DevState& st, double* partials) {
    LevelParams p;
    fill_level_params(&p, a->sde, a->level, a->precision, a->n_paths, a->path_offset, a->seed, a->stream, a->pset);
    if (v.rv == MLMC_RV_PWL16 || v.rv == MLMC_RV_CUBIC16) {
        const int r = v.rv == MLMC_RV_PWL16 ? 0 : 1;
        p.table = st.tables[r][v.precision];
        p.table64 = st.tables64[r];
    }
    if (v.rv == MLMC_RV_PCONST4096) {
        p.table = st.pconst[v.precision];
        p.table64 = (const double*)st.pconst[MLMC_FP64];
    }
    p.mlp = st.mlp;
    p.exact_tab = st.exact_tab;
    p.partials = partials;
    return p;
}

// Four-wave blocks, one partial row per wave up to 32 blocks per CU (several times what is
// resident at once), past that an equal number of rows per wave.  With more blocks than fit,
// the dispatcher hands the last rows to whichever CU frees first, so the tail of the launch
// stays busy; a grid of only the resident waves, two rows each, left it to a few CUs.
void launch_shape(const DevState& st, uint64_t n_rows, int* grid, int* block) {
    const int waves_per_block = 4;
    *block = waves_per_block * kWave;
    const uint64_t max_blocks = (uint64_t)st.n_cu * 32;
    uint64_t blocks = (n_rows + waves_per_block - 1) / waves_per_block;
    if (blocks > max_blocks) {  // ceil(blocks / rounds) <= max_blocks
        const uint64_t rounds = (blocks + max_blocks - 1) / max_blocks;
        blocks = (blocks + rounds - 1) / rounds;
    }
    if (blocks == 0) blocks = 1;
    *grid = (int)blocks;
}

// Enqueue level + reduction on `s`; result (8 doubles) to d_out.
int enqueue_level(DevState& st, const mlmc_level_args_t* a, const Variant& v, double* d_out, double* partials,
                  double* out_pf_hat, double* out_pc_hat, double* out_pf_bar, double* out_pc_bar,
                  double* out_xf_tilde, hipStream_t s) {
    if (v.rv == MLMC_RV_MLP && !st.mlp_loaded)
        return fail(MLMC_EUNSUPPORTED, "MLMC_RV_MLP needs weights: call mlmc_mlp_load first");
    const uint64_t n_rows = n_rows_of(a);
    LevelParams p = make_params(a, v, st, partials);
    p.out_pf_hat = out_pf_hat;
    p.out_pc_hat = out_pc_hat;
    p.out_pf_bar = out_pf_bar;
    p.out_pc_bar = out_pc_bar;
    p.out_xf_tilde = out_xf_tilde;
    hipError_t e;
    // layout of the workspace: partial rows, then the stage rows
    double* stage = partials + (n_rows == 0 ? 1 : n_rows) * kPartial;
    int grid, block;
    launch_shape(st, n_rows, &grid, &block);
    const bool per_path = out_pf_hat || out_pc_hat || out_pf_bar || out_pc_bar || out_xf_tilde;
    if (n_rows > 0 && !per_path && coop_level_call(v, a->level, n_rows, st.n_cu)) {
        e = launch_level_coop(v, p, n_rows, s);
        if (e != hipSuccess) return hip_fail(e, "cooperative level kernel launch");
    } else if (n_rows > 0) {
        e = launch_level(v, p, grid, block, s);
        if (e != hipSuccess) return hip_fail(e, "level kernel launch");
    }
    if (d_out) {  // with no rows the first stage reads no row and the sums are zero
        e = launch_reduce(partials, n_rows, stage, d_out, s);
        if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
    }
    return MLMC_OK;
}

void term_mask(const Variant& v, bool m[4]) {
    m[MLMC_TERM_TWO_WAY] = true;
    m[MLMC_TERM_FOUR_WAY] = v.nested;
    m[MLMC_TERM_TWO_WAY_EXACT] = v.nested;
    m[MLMC_TERM_ROUNDING] = v.diag;
}

}  // namespace

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int validate_sde_public(const mlmc_gbm_t* s) { return validate_sde(s); }

// binary64 constants of one level, then one rounding to each working precision
void fill_level_params(LevelParams* p, const mlmc_gbm_t& s, int level, int precision, uint64_t n_paths,
                       uint64_t path_offset, uint64_t seed, uint32_t stream, uint32_t pset) {
    std::memset(p, 0, sizeof *p);
    const double dt = s.T * std::ldexp(1.0, -level);
    const double ca = s.mu * dt;
    const double cac = s.mu * (2.0 * dt);
    const double cb = s.sigma * std::sqrt(dt);
    const double cm = 0.5 * s.sigma * s.sigma * dt;
    p->ca_f64 = ca; p->cac_f64 = cac; p->cb_f64 = cb; p->x0_f64 = s.x0; p->k_f64 = s.strike; p->cm_f64 = cm;
    p->ca_f32 = (float)ca; p->cac_f32 = (float)cac; p->cb_f32 = (float)cb; p->x0_f32 = (float)s.x0;
    p->k_f32 = (float)s.strike; p->cm_f32 = (float)cm;
    if (precision == MLMC_BF16) {  // one rounding from binary64 to 8 bits, exact in binary32
        p->ca_f32 = (float)bf16_of(ca); p->cac_f32 = (float)bf16_of(cac); p->cb_f32 = (float)bf16_of(cb);
        p->x0_f32 = (float)bf16_of(s.x0); p->k_f32 = (float)bf16_of(s.strike); p->cm_f32 = (float)bf16_of(cm);
    }
    p->ca_f16 = half_of(ca); p->cac_f16 = half_of(cac); p->cb_f16 = half_of(cb);
    p->x0_f16 = half_of(s.x0); p->k_f16 = half_of(s.strike); p->cm_f16 = half_of(cm);
    p->payoff = s.payoff;
    p->level = level;
    p->n_steps = 1u << level;
    p->n_paths = n_paths;
    p->path_offset = path_offset;
    p->key0 = (uint32_t)seed;
    p->key1 = (uint32_t)(seed >> 32);
    p->ctr2 = (stream << 16) | (uint32_t)level;
    p->pset = pset;
}

int device_info(DeviceInfo* out) {
    DevState* st;
    int rc = device_state(&st);
    if (rc) return rc;
    out->n_cu = st->n_cu;
    for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < 4; ++q) out->tables[r][q] = st->tables[r][q];
        out->tables64[r] = st->tables64[r];
    }
    for (int q = 0; q < 4; ++q) out->pconst[q] = st->pconst[q];
    out->mlp = st->mlp;
    out->mlp_loaded = st->mlp_loaded;
    out->exact_tab = st->exact_tab;
    return MLMC_OK;
}

}  // namespace mlmc

using namespace mlmc;

extern "C" {

int mlmc_init(int device) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(MLMC_ENODEV, "no HIP device available");
    }
    if (device < 0 || device >= n) return fail(MLMC_EINVAL, "device %d outside 0..%d", device, n - 1);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    DevState* st;
    return device_state(&st);
}

int mlmc_shutdown(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_devs) {
        DevState& st = kv.second;
        if (hipSetDevice(kv.first) != hipSuccess) continue;
        (void)hipDeviceSynchronize();
        for (auto& row : st.tables)
            for (void*& t : row)
                if (t) (void)hipFree(t);
        for (void*& t : st.pconst)
            if (t) (void)hipFree(t);
        if (st.scratch) (void)hipFree(st.scratch);
        if (st.out8) (void)hipFree(st.out8);
        if (st.mlp) (void)hipFree(st.mlp);
        if (st.exact_tab) (void)hipFree(st.exact_tab);
        if (st.ev0) (void)hipEventDestroy(st.ev0);
        if (st.ev1) (void)hipEventDestroy(st.ev1);
        if (st.stream) (void)hipStreamDestroy(st.stream);
        for (hipStream_t& q : st.set_stream)
            if (q) (void)hipStreamDestroy(q);
        for (hipEvent_t ev : st.set_events) (void)hipEventDestroy(ev);
        if (st.set_mem) (void)hipFree(st.set_mem);
    }
    g_devs.clear();
    (void)hipSetDevice(cur);
    return MLMC_OK;
}

const char* mlmc_last_error(void) { return g_error.c_str(); }

size_t mlmc_level_workspace_bytes(const mlmc_level_args_t* args) {
    Variant v;
    if (validate_args(args, &v)) return 0;
    return level_workspace_bytes(n_rows_of(args));
}

int mlmc_level_ex(const mlmc_level_args_t* args, double* d_out, void* d_workspace, size_t workspace_bytes,
                  void* hip_stream) {
    Variant v;
    int rc = validate_args(args, &v);
    if (rc) return rc;
    if (!d_out) return fail(MLMC_EINVAL, "d_out is NULL");
    const size_t need = level_workspace_bytes(n_rows_of(args));
    if (d_workspace && workspace_bytes < need)
        return fail(MLMC_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
    DevState* st;
    if ((rc = device_state(&st))) return rc;
    double* partials = (double*)d_workspace;
    if (!partials) {
        if ((rc = ensure_scratch(*st, need))) return rc;
        partials = st->scratch;
    }
    return enqueue_level(*st, args, v, d_out, partials, nullptr, nullptr, nullptr, nullptr, nullptr,
                         (hipStream_t)hip_stream);
}

int mlmc_level_noalloc(const mlmc_level_args_t* args, double* d_out, void* hip_stream) {
    Variant v;
    int rc = validate_args(args, &v);
    if (rc) return rc;
    if (!d_out) return fail(MLMC_EINVAL, "d_out is NULL");
    const uint64_t n_chunks = n_chunks_of(args);
    if (n_chunks > kNoAllocMaxChunks)
        return fail(MLMC_EINVAL,
                    "n_paths %llu needs %llu chunks; mlmc_level_noalloc holds at most %llu (2^22 paths, 2^23 in "
                    "binary16)",
                    (unsigned long long)args->n_paths, (unsigned long long)n_chunks,
                    (unsigned long long)kNoAllocMaxChunks);
    int dev = 0;
    if ((rc = current_device(&dev))) return rc;
    DevState* st = nullptr;
    {
        // look the device up without creating it: set-up allocates, this entry point does not
        std::lock_guard<std::mutex> lock(g_mutex);
        auto it = g_devs.find(dev);
        if (it != g_devs.end() && it->second.ready) st = &it->second;
    }
    if (!st) return fail(MLMC_EUNSUPPORTED, "mlmc_level_noalloc allocates nothing: call mlmc_init(%d) first", dev);
    return enqueue_level(*st, args, v, d_out, st->noalloc_scratch, nullptr, nullptr, nullptr, nullptr, nullptr,
                         (hipStream_t)hip_stream);
}

int mlmc_level_run(const mlmc_level_args_t* args, mlmc_result_t* out) {
    if (!out) return fail(MLMC_EINVAL, "out is NULL");
    Variant v;
    int rc = validate_args(args, &v);
    if (rc) return rc;
    DevState* st;
    if ((rc = device_state(&st))) return rc;
    const size_t need = level_workspace_bytes(n_rows_of(args));
    if ((rc = ensure_scratch(*st, need))) return rc;
    hipError_t e = hipEventRecord(st->ev0, st->stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    rc = enqueue_level(*st, args, v, st->out8, st->scratch, nullptr, nullptr, nullptr, nullptr, nullptr, st->stream);
    if (rc) return rc;
    if ((e = hipEventRecord(st->ev1, st->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    double h[kPartial];
    if ((e = hipMemcpyAsync(h, st->out8, sizeof h, hipMemcpyDeviceToHost, st->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(st->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, st->ev0, st->ev1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    bool m[4];
    term_mask(v, m);
    for (int k = 0; k < kTerms; ++k) {
        out->sum[k] = m[k] ? h[k] : NAN;
        out->sumsq[k] = m[k] ? h[kTerms + k] : NAN;
    }
    out->n_paths = args->n_paths;
    out->path_steps = args->n_paths << args->level;
    out->cost_seconds = 1e-3 * (double)ms;
    return MLMC_OK;
}

int mlmc_level_set_run(const mlmc_level_args_t* args, int n_calls, mlmc_result_t* out, double* span_seconds) {
    if (!args) return fail(MLMC_EINVAL, "args is NULL");
    if (!out) return fail(MLMC_EINVAL, "out is NULL");
    if (n_calls < 1 || n_calls > kMaxSetCalls) return fail(MLMC_EINVAL, "n_calls must be 1..%d", kMaxSetCalls);
    std::vector<Variant> v(n_calls);
    for (int i = 0; i < n_calls; ++i) {
        const int rc = validate_args(&args[i], &v[i]);
        if (rc) return fail(rc, "call %d: %s", i, g_error.c_str());
    }
    DevState* st;
    int rc = device_state(&st);
    if (rc) return rc;
    for (int i = 0; i < n_calls; ++i)
        if (v[i].rv == MLMC_RV_MLP && !st->mlp_loaded)
            return fail(MLMC_EUNSUPPORTED, "call %d: MLMC_RV_MLP needs weights: call mlmc_mlp_load first", i);
    // device memory: n_calls result slots of 8 doubles, then each call's workspace (256-byte aligned)
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    std::vector<size_t> ws_off(n_calls);
    size_t total = up((size_t)n_calls * kPartial * sizeof(double));
    for (int i = 0; i < n_calls; ++i) {
        ws_off[i] = total;
        total += up(level_workspace_bytes(n_rows_of(&args[i])));
    }
    hipError_t e;
    for (hipStream_t& q : st->set_stream)
        if (!q && (e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreate");
    while (st->set_events.size() < (size_t)(2 * n_calls + kSetStreams + 1)) {
        hipEvent_t ev;
        if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        st->set_events.push_back(ev);
    }
    if (total > st->set_mem_bytes) {
        if (st->set_mem) {
            (void)hipFree(st->set_mem);  // the previous set has completed (every set is synchronous)
            st->set_mem = nullptr;
            st->set_mem_bytes = 0;
        }
        if ((e = hipMalloc(&st->set_mem, total)) != hipSuccess)
            return fail(MLMC_ENOMEM, "hipMalloc of %zu level-set bytes failed", total);
        st->set_mem_bytes = total;
    }
    unsigned char* mem = (unsigned char*)st->set_mem;
    double* results = (double*)mem;
    hipEvent_t* ev = st->set_events.data();  // [2i, 2i+1]: call i; then the set's begin, joins, end
    hipEvent_t ev_begin = ev[2 * n_calls], ev_end = ev[2 * n_calls + kSetStreams];
    // the longest serial chains first (level, then samples), dealt round-robin over the
    // streams, so that the deep levels' few long paths overlap the shallow levels' many short ones
    std::vector<int> order(n_calls);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (args[a].level != args[b].level) return args[a].level > args[b].level;
        return args[a].n_paths > args[b].n_paths;
    });
    hipStream_t s0 = st->set_stream[0];
    if ((e = hipEventRecord(ev_begin, s0)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int q = 1; q < kSetStreams; ++q)
        if ((e = hipStreamWaitEvent(st->set_stream[q], ev_begin, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    for (int k = 0; k < n_calls && rc == MLMC_OK; ++k) {
        const int i = order[k];
        hipStream_t q = st->set_stream[k % kSetStreams];
        if ((e = hipEventRecord(ev[2 * i], q)) != hipSuccess) {
            rc = hip_fail(e, "hipEventRecord");
            break;
        }
        rc = enqueue_level(*st, &args[i], v[i], results + (size_t)i * kPartial, (double*)(mem + ws_off[i]), nullptr,
                           nullptr, nullptr, nullptr, nullptr, q);
        if (rc == MLMC_OK && (e = hipEventRecord(ev[2 * i + 1], q)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
    }
    // join the streams into the first one (also after a failed launch, so nothing is left running)
    for (int q = 1; q < kSetStreams; ++q) {
        if ((e = hipEventRecord(ev[2 * n_calls + q], st->set_stream[q])) != hipSuccess ||
            (e = hipStreamWaitEvent(s0, ev[2 * n_calls + q], 0)) != hipSuccess) {
            for (hipStream_t r : st->set_stream) (void)hipStreamSynchronize(r);
            return rc ? rc : hip_fail(e, "stream join");
        }
    }
    if ((e = hipEventRecord(ev_end, s0)) != hipSuccess && rc == MLMC_OK) rc = hip_fail(e, "hipEventRecord");
    if ((e = hipStreamSynchronize(s0)) != hipSuccess && rc == MLMC_OK) rc = hip_fail(e, "hipStreamSynchronize");
    if (rc) return rc;
    std::vector<double> h((size_t)n_calls * kPartial);
    if ((e = hipMemcpy(h.data(), results, h.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy");
    for (int i = 0; i < n_calls; ++i) {
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1])) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        bool m[4];
        term_mask(v[i], m);
        for (int t = 0; t < kTerms; ++t) {
            out[i].sum[t] = m[t] ? h[(size_t)i * kPartial + t] : NAN;
            out[i].sumsq[t] = m[t] ? h[(size_t)i * kPartial + kTerms + t] : NAN;
        }
        out[i].n_paths = args[i].n_paths;
        out[i].path_steps = args[i].n_paths << args[i].level;
        out[i].cost_seconds = 1e-3 * (double)ms;
    }
    if (span_seconds) {
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, ev_begin, ev_end)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        *span_seconds = 1e-3 * (double)ms;
    }
    return MLMC_OK;
}

int mlmc_level(const mlmc_gbm_t* sde, int level, uint64_t n_paths, int precision, int rv_mode, int kahan,
               uint64_t seed, mlmc_result_t* out) {
    if (!sde) return fail(MLMC_EINVAL, "sde is NULL");
    if (!out) return fail(MLMC_EINVAL, "out is NULL");
    mlmc_level_args_t a;
    std::memset(&a, 0, sizeof a);
    a.sde = *sde;
    a.level = level;
    a.precision = precision;
    a.rv_mode = rv_mode;
    a.kahan = kahan;
    a.stream = rv_mode >= MLMC_NESTED_PWL16 ? 1u : 0u;
    a.seed = seed;
    a.n_paths = n_paths;
    a.scheme = MLMC_SCHEME_EM;
    return mlmc_level_run(&a, out);
}

int mlmc_paths(const mlmc_level_args_t* args, double* d_pf_hat, double* d_pc_hat, double* d_pf_bar,
               double* d_pc_bar, double* d_xf_tilde, void* hip_stream) {
    Variant v;
    int rc = validate_args(args, &v);
    if (rc) return rc;
    DevState* st;
    if ((rc = device_state(&st))) return rc;
    const size_t need = level_workspace_bytes(n_rows_of(args));
    if ((rc = ensure_scratch(*st, need))) return rc;
    return enqueue_level(*st, args, v, nullptr, st->scratch, d_pf_hat, d_pc_hat, d_pf_bar, d_pc_bar, d_xf_tilde,
                         (hipStream_t)hip_stream);
}

int mlmc_uniforms(uint64_t seed, uint32_t stream, int level, uint32_t pset, uint64_t path0, uint64_t n_paths,
                  uint32_t n_steps, uint32_t* d_words, void* hip_stream) {
    if (!d_words && n_paths > 0 && n_steps > 0) return fail(MLMC_EINVAL, "d_words is NULL");
    if (stream > 0xFFFFu) return fail(MLMC_EINVAL, "stream %u exceeds 65535", stream);
    if (level < 0 || level > 0xFFFF) return fail(MLMC_EINVAL, "level %d outside 0..65535", level);
    if (n_steps > (1u << kMaxLevel)) return fail(MLMC_EINVAL, "n_steps exceeds 2^%d", kMaxLevel);
    if (level < 2 && n_steps > (1u << level))
        return fail(MLMC_EINVAL, "level %d has at most %u steps (its calls are shared by paths)", level, 1u << level);
    if (path0 + n_paths > (1ull << 32)) return fail(MLMC_EINVAL, "path0 + n_paths exceeds 2^32");
    DevState* st;
    int rc = device_state(&st);
    if (rc) return rc;
    if (n_paths == 0 || n_steps == 0) return MLMC_OK;
    hipError_t e = launch_uniforms(seed, (stream << 16) | (uint32_t)level, pset, path0, n_paths, n_steps, d_words,
                                   (hipStream_t)hip_stream);
    return e == hipSuccess ? MLMC_OK : hip_fail(e, "uniforms kernel launch");
}

int mlmc_icdf(const uint32_t* d_words, uint64_t n, int rv, int precision, double* d_out, void* hip_stream) {
    if ((!d_words || !d_out) && n > 0) return fail(MLMC_EINVAL, "NULL buffer");
    if (rv < MLMC_RV_EXACT || rv > MLMC_RV_PCONST4096) return fail(MLMC_EINVAL, "rv %d is not an MLMC_RV_* kind", rv);
    if (precision < MLMC_FP64 || precision > MLMC_BF16) return fail(MLMC_EINVAL, "precision %d invalid", precision);
    if (precision == MLMC_BF16 && (rv == MLMC_RV_EXACT || rv == MLMC_RV_MLP))
        return fail(MLMC_EINVAL, "MLMC_BF16 is available for the table approximations only");
    DevState* st;
    int rc = device_state(&st);
    if (rc) return rc;
    if (rv == MLMC_RV_MLP && !st->mlp_loaded)
        return fail(MLMC_EUNSUPPORTED, "MLMC_RV_MLP needs weights: call mlmc_mlp_load first");
    if (n == 0) return MLMC_OK;
    const void* table = nullptr;
    if (rv == MLMC_RV_PWL16 || rv == MLMC_RV_CUBIC16) table = st->tables[rv == MLMC_RV_PWL16 ? 0 : 1][precision];
    if (rv == MLMC_RV_PCONST4096) table = st->pconst[precision];
    hipError_t e = launch_icdf(d_words, n, rv, precision, table, st->mlp, st->exact_tab, d_out,
                               (hipStream_t)hip_stream);
    return e == hipSuccess ? MLMC_OK : hip_fail(e, "icdf kernel launch");
}

int mlmc_mlp_load(const float* d_params, void* hip_stream) {
    if (!d_params) return fail(MLMC_EINVAL, "d_params is NULL");
    DevState* st;
    int rc = device_state(&st);
    if (rc) return rc;
    hipError_t e = launch_mlp_deploy(d_params, st->mlp, (hipStream_t)hip_stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "MLP deploy");
    st->mlp_loaded = true;
    return MLMC_OK;
}

int mlmc_table(int rv, int precision, double* h_out) {
    if (!h_out) return fail(MLMC_EINVAL, "h_out is NULL");
    if (rv != MLMC_RV_PWL16 && rv != MLMC_RV_CUBIC16) return fail(MLMC_EINVAL, "rv must be PWL16 or CUBIC16");
    if (precision < MLMC_FP64 || precision > MLMC_BF16) return fail(MLMC_EINVAL, "precision %d invalid", precision);
    const HostTables& ht = host_tables();
    if (!ht.ok) return fail(MLMC_EHIP, "dyadic table construction failed");
    const double(*src)[4] = rv == MLMC_RV_PWL16 ? ht.pwl : ht.cubic;
    const int d = degree_of(rv);
    for (int j = 0; j < 16; ++j)
        for (int i = 0; i < 4; ++i) h_out[j * 4 + i] = rounded_to(precision, i <= d ? src[j][i] : 0.0);
    return MLMC_OK;
}

int mlmc_pconst_table(int precision, double* h_out) {
    if (!h_out) return fail(MLMC_EINVAL, "h_out is NULL");
    if (precision < MLMC_FP64 || precision > MLMC_BF16) return fail(MLMC_EINVAL, "precision %d invalid", precision);
    const HostTables& ht = host_tables();
    if (!ht.ok) return fail(MLMC_EHIP, "table construction failed");
    for (int i = 0; i < kPcEntries; ++i) h_out[i] = rounded_to(precision, ht.pconst[i]);
    return MLMC_OK;
}

}  // extern "C"
