// Batched MLMC sweep: every (parameter set, level) item of a sweep in one persistent
// launch, captured in a hipGraph, with a host autotuner for the launch shape.
//
// Items are split into tasks (a range of 64-path chunks of one item).  Tasks are ordered
// by decreasing work -- the few long fine-level chunks (up to 2^24 sequential steps each)
// start first, the many short coarse-level chunks fill in behind them -- and each
// wavefront pops tasks from a device counter until the queue is empty, so every wave
// reaches the exit.  Tasks at or above a chosen level run at raised wave priority, which
// keeps the long dependent chains issuing while short tasks share the SIMD.  A chunk
// writes its 8 partial sums to a per-item row; the rows of every item are then reduced in
// the same fixed order as the single-level path.
//
// Cooperative chunks: the chunks of the deepest binary32 items (level >= coop_level) are
// serial chains of up to 2^24 steps, and one wavefront alone runs them latency bound.  Each
// block (eight or four waves) first pops such chunks from a block queue and runs one chunk
// with all its waves (coop.h): seven or three producer waves draw the uniforms and both
// inverse CDFs for the next phase of 28 or 12 steps into an LDS ring while the consumer wave
// advances the four coupled paths through the current phase, one barrier per phase.  The
// consumer performs exactly the operations of the single-wave code in the same order, so
// every sum keeps its bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "coop.h"
#include "internal.h"
#include "level_kernel.h"
#include "reduce.h"

struct mlmc_batch {
    int device = 0;
    int rv = MLMC_RV_PWL16;
    std::vector<mlmc_item_t> items;
    mlmc_batch_cfg_t cfg{};
    int n_cu = 256;
    double* d_out = nullptr;
    // device data
    mlmc::LevelParams* d_params = nullptr;
    int* d_variant = nullptr;
    uint64_t* d_row_off = nullptr;
    uint64_t* d_rows = nullptr;
    double* d_partials = nullptr;
    uint4* d_tasks = nullptr;
    uint2* d_coop = nullptr;                 // cooperative chunks (item, chunk), longest first
    uint64_t n_coop = 0;
    uint64_t coop_capacity = 0;
    uint32_t* d_counter = nullptr;           // [0] wave queue, [1] cooperative block queue
    unsigned long long* d_ticks = nullptr;  // per item: wall-clock ticks summed over its tasks
    double* d_stage = nullptr;               // per item: stage rows of the two-stage reduction
    uint2* d_reduce_blocks = nullptr;        // (item, stage block) of every reduction block
    uint32_t n_reduce_blocks = 0;
    uint64_t n_tasks = 0;
    uint64_t task_capacity = 0;
    const void* tab32 = nullptr;
    const void* tab16 = nullptr;
    const void* exact_tab = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace mlmc {

namespace {

// variant of an item: binary16 or binary32 approximate pair, with or without Kahan
__host__ __device__ inline int variant_of(int precision, int kahan) {
    return (precision == MLMC_FP16 ? 0 : 2) + (kahan ? 1 : 0);
}

// Clears the queue counter and the per-item tick sums (a kernel, not a memset, so that the
// captured graph holds no memset node).
__global__ void batch_reset(uint32_t* counter, unsigned long long* ticks, uint32_t n_items) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        counter[0] = 0u;
        counter[1] = 0u;
    }
    for (uint32_t k = i; k < n_items; k += gridDim.x * blockDim.x) ticks[k] = 0ull;
}

constexpr int kDefaultBlockWaves = 8;

template <int RV, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(4))) void batch_kernel(const LevelParams* __restrict__ params, const int* __restrict__ variant,
                                                    const uint4* __restrict__ tasks, uint32_t n_tasks,
                                                    const uint2* __restrict__ coop, uint32_t n_coop,
                                                    uint32_t* __restrict__ counter, const float* __restrict__ tab32,
                                                    const __half* __restrict__ tab16, const void* __restrict__ exact_tab,
                                                    unsigned long long* __restrict__ ticks) {
    constexpr int DEG = RV == MLMC_RV_CUBIC16 ? 3 : 1;
    __shared__ float s_tab32[kTableRowsDev * 4];
    __shared__ __half s_tab16[kTableRowsDev * 4];
    __shared__ __align__(16) unsigned char s_ex_raw[sizeof(ExactCols)];
    __shared__ double ring_x[2][Coop<WAVES>::kSteps][kWave];
    __shared__ float ring_b[2][Coop<WAVES>::kSteps][kWave];
    __shared__ uint32_t s_pop;
    const ExactLds* s_ex = (const ExactLds*)s_ex_raw;  // the top rows only (no learned variable here)
    for (int i = threadIdx.x; i < kTableRowsDev * (DEG + 1); i += blockDim.x) {
        s_tab32[i] = prescaled_coeff(tab32[i], i % (DEG + 1));
        s_tab16[i] = tab16[i];
    }
    stage_exact_table(s_ex_raw, exact_tab, sizeof(ExactCols));
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    // cooperative chunks first: the block pops one, all its waves run it (block-uniform loop)
    for (;;) {
        if (threadIdx.x == 0) s_pop = atomicAdd(&counter[1], 1u);
        __syncthreads();
        const uint32_t c = s_pop;
        __syncthreads();  // every thread has read s_pop before it is written again
        if (c >= n_coop) break;
        const uint2 ct = coop[c];
        const LevelParams& prm = params[ct.x];
        __builtin_amdgcn_s_setprio(3);
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        if (variant[ct.x] & 1) run_chunk_coop<RV, true, WAVES>(prm, ct.y, s_tab32, s_ex, ring_x, ring_b);
        else run_chunk_coop<RV, false, WAVES>(prm, ct.y, s_tab32, s_ex, ring_x, ring_b);
        const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
        if (lane == 0) atomicAdd(&ticks[ct.x], (unsigned long long)(t1 - t0));
        __builtin_amdgcn_s_setprio(0);
    }
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(counter, 1u);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, kWave));
        if (t >= n_tasks) break;
        const uint4 task = tasks[t];  // (item, first row, row count, raised priority)
        const LevelParams& prm = params[task.x];
        const int var = variant[task.x];
        if (task.w) __builtin_amdgcn_s_setprio(3);
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        // levels 0 and 1 (fewer than 4 steps) take the per-word exact variable
        const int v = var + (prm.n_steps < 4 ? 4 : 0);
        for (uint32_t c = task.y; c < task.y + task.z; ++c) {
            switch (v) {
                case 0: run_row<MLMC_FP16, RV, true, false, false>(prm, c, lane, s_tab16, nullptr, s_ex); break;
                case 1: run_row<MLMC_FP16, RV, true, true, false>(prm, c, lane, s_tab16, nullptr, s_ex); break;
                case 2: run_row<MLMC_FP32, RV, true, false, false>(prm, c, lane, s_tab32, nullptr, s_ex); break;
                case 3: run_row<MLMC_FP32, RV, true, true, false>(prm, c, lane, s_tab32, nullptr, s_ex); break;
                case 4: run_row<MLMC_FP16, RV, true, false, false, true>(prm, c, lane, s_tab16, nullptr, s_ex); break;
                case 5: run_row<MLMC_FP16, RV, true, true, false, true>(prm, c, lane, s_tab16, nullptr, s_ex); break;
                case 6: run_row<MLMC_FP32, RV, true, false, false, true>(prm, c, lane, s_tab32, nullptr, s_ex); break;
                default: run_row<MLMC_FP32, RV, true, true, false, true>(prm, c, lane, s_tab32, nullptr, s_ex); break;
            }
        }
        const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
        if (lane == 0) atomicAdd(&ticks[task.x], (unsigned long long)(t1 - t0));
        if (task.w) __builtin_amdgcn_s_setprio(0);
    }
}

// Per item the same two-stage fixed-order reduction as a single-level call.  First stage:
// block k is stage block blocks[k].y of item blocks[k].x; an item's stage rows sit at the
// start of its own range of partial-row slots in `stage` (it has at most as many stage rows
// as rows).  Second stage: block i sums the stage rows of item i.
__global__ __launch_bounds__(kReduceBlock) void batch_reduce_stage1(const double* __restrict__ partials,
                                                                    const uint64_t* __restrict__ row_off,
                                                                    const uint64_t* __restrict__ rows,
                                                                    const uint2* __restrict__ blocks,
                                                                    double* __restrict__ stage) {
    __shared__ double s[kPartial][kReduceBlock];
    const uint2 bl = blocks[blockIdx.x];
    const uint32_t item = bl.x;
    reduce_stage1(partials + row_off[item] * kPartial, rows[item], stage + row_off[item] * kPartial, bl.y, s);
}

__global__ __launch_bounds__(kReduceBlock) void batch_reduce_stage2(const uint64_t* __restrict__ row_off,
                                                                    const uint64_t* __restrict__ rows,
                                                                    const double* __restrict__ stage,
                                                                    double* __restrict__ out) {
    __shared__ double s[kPartial][kReduceBlock];
    const uint32_t item = blockIdx.x;
    reduce_stage2(stage + row_off[item] * kPartial, rows[item], out + (uint64_t)item * kPartial, s);
}

constexpr mlmc_batch_cfg_t kDefaultCfg = {16, 1024, 12, 12, kDefaultBlockWaves};

int validate_cfg(const mlmc_batch_cfg_t& c) {
    if (c.waves_per_cu < 4 || c.waves_per_cu > 32) return set_error(MLMC_EINVAL, "waves_per_cu must be 4..32");
    if (c.task_steps < 1 || c.task_steps > (1 << 20)) return set_error(MLMC_EINVAL, "task_steps must be 1..2^20");
    if (c.priority_level < 0 || c.priority_level > 25) return set_error(MLMC_EINVAL, "priority_level must be 0..25");
    if (c.coop_level < 2 || c.coop_level > 25) return set_error(MLMC_EINVAL, "coop_level must be 2..25");
    if (c.block_waves != 4 && c.block_waves != 8) return set_error(MLMC_EINVAL, "block_waves must be 4 or 8");
    if (c.waves_per_cu < c.block_waves) return set_error(MLMC_EINVAL, "waves_per_cu is below one block");
    return MLMC_OK;
}

mlmc_batch_cfg_t merged(const mlmc_batch_cfg_t* c) {
    mlmc_batch_cfg_t r = kDefaultCfg;
    if (c) {
        if (c->waves_per_cu) r.waves_per_cu = c->waves_per_cu;
        if (c->task_steps) r.task_steps = c->task_steps;
        if (c->priority_level) r.priority_level = c->priority_level;
        if (c->coop_level) r.coop_level = c->coop_level;
        if (c->block_waves) r.block_waves = c->block_waves;
    }
    return r;
}

// whether an item's chunks run cooperatively (binary32, at least coop_level; n_steps >= 4,
// where a partial row is one chunk)
bool is_coop(const mlmc_item_t& it, const mlmc_batch_cfg_t& c) {
    return it.precision == MLMC_FP32 && it.level >= c.coop_level && it.level >= 2;
}

std::string signature(const mlmc_batch& b) {
    // item list + device shape; FNV-1a over the item records
    uint64_t h = 1469598103934665603ull;
    for (const mlmc_item_t& it : b.items) {
        const unsigned char* p = (const unsigned char*)&it;
        for (size_t i = 0; i < sizeof it; ++i) h = (h ^ p[i]) * 1099511628211ull;
    }
    char buf[96];
    std::snprintf(buf, sizeof buf, "gfx950-cu%d-rv%d-n%zu-%016llx", b.n_cu, b.rv, b.items.size(),
                  (unsigned long long)h);
    return buf;
}

bool cache_lookup(const std::string& key, mlmc_batch_cfg_t* c) {
    const char* path = std::getenv("MLMC_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k;
        int a, s, p, q, w;
        if ((in >> k >> a >> s >> p >> q >> w) && k == key) {
            *c = mlmc_batch_cfg_t{a, s, p, q, w};
            return validate_cfg(*c) == MLMC_OK;
        }
    }
    return false;
}

void cache_store(const std::string& key, const mlmc_batch_cfg_t& c) {
    const char* path = std::getenv("MLMC_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line))
            if (line.compare(0, key.size() + 1, key + " ") != 0 && !line.empty()) keep.push_back(line);
    }
    std::ofstream f(path, std::ios::trunc);
    for (const std::string& l : keep) f << l << "\n";
    f << key << " " << c.waves_per_cu << " " << c.task_steps << " " << c.priority_level << " " << c.coop_level << " "
      << c.block_waves << "\n";
}

int hipck(hipError_t e, const char* what) {
    return e == hipSuccess ? MLMC_OK : set_error(MLMC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Task list for the current configuration: ordered by decreasing work.  Chunks of
// cooperative items go to `coop` instead (one entry per chunk, deepest first).
std::vector<uint4> build_tasks(const mlmc_batch& b, const std::vector<uint64_t>& rows, std::vector<uint2>* coop) {
    struct T {
        uint64_t work;
        uint4 t;
    };
    std::vector<T> ts;
    std::vector<std::pair<int, uint2>> cs;
    for (size_t i = 0; i < b.items.size(); ++i) {
        const int l = b.items[i].level;
        if (is_coop(b.items[i], b.cfg)) {
            for (uint64_t c = 0; c < rows[i]; ++c) cs.push_back({l, make_uint2((uint32_t)i, (uint32_t)c)});
            continue;
        }
        // rows of row_chunks(l) chunks: about task_steps steps per path and task
        const uint64_t g = row_chunks(l, false);  // nested items
        const uint64_t per = std::max<uint64_t>(1, ((uint64_t)b.cfg.task_steps >> l) / g);
        const uint32_t prio = l >= b.cfg.priority_level ? 1u : 0u;
        for (uint64_t c = 0; c < rows[i]; c += per) {
            const uint64_t n = std::min<uint64_t>(per, rows[i] - c);
            ts.push_back({(n * g) << l, make_uint4((uint32_t)i, (uint32_t)c, (uint32_t)n, prio)});
        }
    }
    std::stable_sort(ts.begin(), ts.end(), [](const T& a, const T& c) { return a.work > c.work; });
    std::stable_sort(cs.begin(), cs.end(), [](const std::pair<int, uint2>& a, const std::pair<int, uint2>& c) {
        return a.first > c.first;
    });
    coop->resize(cs.size());
    for (size_t i = 0; i < cs.size(); ++i) (*coop)[i] = cs[i].second;
    std::vector<uint4> out(ts.size());
    for (size_t i = 0; i < ts.size(); ++i) out[i] = ts[i].t;
    return out;
}

template <int RV, int WAVES>
void launch_batch(const mlmc_batch* b, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((batch_kernel<RV, WAVES>), dim3(blocks), dim3(WAVES * kWave), 0, s, b->d_params, b->d_variant,
                       b->d_tasks, (uint32_t)b->n_tasks, b->d_coop, (uint32_t)b->n_coop, b->d_counter,
                       (const float*)b->tab32, (const __half*)b->tab16, b->exact_tab, b->d_ticks);
}

int enqueue(mlmc_batch* b, hipStream_t s) {
    const int bw = b->cfg.block_waves;
    const int blocks = std::max(1, b->n_cu * b->cfg.waves_per_cu / bw);
    const uint32_t n_items = (uint32_t)b->items.size();
    hipLaunchKernelGGL(batch_reset, dim3(std::min<uint32_t>(64, (n_items + 255) / 256)), dim3(256), 0, s, b->d_counter,
                       b->d_ticks, n_items);
    int rc = hipck(hipGetLastError(), "queue reset launch");
    if (rc) return rc;
    if (b->rv == MLMC_RV_CUBIC16) {
        if (bw == 4) launch_batch<MLMC_RV_CUBIC16, 4>(b, blocks, s);
        else launch_batch<MLMC_RV_CUBIC16, 8>(b, blocks, s);
    } else {
        if (bw == 4) launch_batch<MLMC_RV_PWL16, 4>(b, blocks, s);
        else launch_batch<MLMC_RV_PWL16, 8>(b, blocks, s);
    }
    rc = hipck(hipGetLastError(), "batch kernel launch");
    if (rc) return rc;
    hipLaunchKernelGGL(batch_reduce_stage1, dim3(b->n_reduce_blocks), dim3(kReduceBlock), 0, s, b->d_partials,
                       b->d_row_off, b->d_rows, b->d_reduce_blocks, b->d_stage);
    rc = hipck(hipGetLastError(), "batch reduction launch");
    if (rc) return rc;
    hipLaunchKernelGGL(batch_reduce_stage2, dim3(n_items), dim3(kReduceBlock), 0, s, b->d_row_off, b->d_rows,
                       b->d_stage, b->d_out);
    return hipck(hipGetLastError(), "batch reduction launch");
}

void drop_graph(mlmc_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// (Re)build the task list for b->cfg, upload it and capture the launch sequence.
int prepare(mlmc_batch* b) {
    std::vector<uint64_t> rows(b->items.size());
    for (size_t i = 0; i < b->items.size(); ++i) {
        const uint64_t cp = chunk_paths(b->items[i].precision);
        rows[i] = rows_of((b->items[i].n_paths + cp - 1) / cp, b->items[i].level, false);
    }
    std::vector<uint2> coop;
    const std::vector<uint4> tasks = build_tasks(*b, rows, &coop);
    // the 32-bit queue counters end at (tasks + waves) and (cooperative chunks + blocks): every
    // wave (block) takes one index past the end before it leaves
    const uint64_t waves = (uint64_t)b->n_cu * (uint64_t)b->cfg.waves_per_cu;
    if ((uint64_t)tasks.size() + waves >= (1ull << 32) || (uint64_t)coop.size() + waves >= (1ull << 32))
        return set_error(MLMC_EINVAL, "the plan needs %zu wave tasks and %zu cooperative chunks; at most 2^32 - %llu "
                         "each fit the queue counters (fewer paths, or a larger task_steps)",
                         tasks.size(), coop.size(), (unsigned long long)waves);
    int rc;
    if (tasks.size() > b->task_capacity || (b->d_tasks == nullptr && !tasks.empty())) {
        if (b->d_tasks) (void)hipFree(b->d_tasks);
        b->d_tasks = nullptr;
        if ((rc = hipck(hipMalloc(&b->d_tasks, std::max<size_t>(1, tasks.size()) * sizeof(uint4)), "hipMalloc tasks")))
            return rc;
        b->task_capacity = tasks.size();
    }
    if (!tasks.empty() &&
        (rc = hipck(hipMemcpy(b->d_tasks, tasks.data(), tasks.size() * sizeof(uint4), hipMemcpyHostToDevice),
                    "hipMemcpy tasks")))
        return rc;
    b->n_tasks = tasks.size();
    if (coop.size() > b->coop_capacity || (b->d_coop == nullptr && !coop.empty())) {
        if (b->d_coop) (void)hipFree(b->d_coop);
        b->d_coop = nullptr;
        if ((rc = hipck(hipMalloc(&b->d_coop, std::max<size_t>(1, coop.size()) * sizeof(uint2)), "hipMalloc coop")))
            return rc;
        b->coop_capacity = coop.size();
    }
    if (!coop.empty() &&
        (rc = hipck(hipMemcpy(b->d_coop, coop.data(), coop.size() * sizeof(uint2), hipMemcpyHostToDevice),
                    "hipMemcpy coop")))
        return rc;
    b->n_coop = coop.size();
    drop_graph(b);
    if ((rc = hipck(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")))
        return rc;
    rc = enqueue(b, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if ((rc = hipck(e, "hipStreamEndCapture"))) return rc;
    b->graph = g;
    return hipck(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

void free_plan(mlmc_batch* b) {
    drop_graph(b);
    for (void* p : {(void*)b->d_params, (void*)b->d_variant, (void*)b->d_row_off, (void*)b->d_rows,
                    (void*)b->d_partials, (void*)b->d_tasks, (void*)b->d_coop, (void*)b->d_counter,
                    (void*)b->d_ticks, (void*)b->d_stage, (void*)b->d_reduce_blocks})
        if (p) (void)hipFree(p);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

}  // namespace
}  // namespace mlmc

using namespace mlmc;

extern "C" {

int mlmc_batch_create(const mlmc_item_t* items, int n_items, int rv, const mlmc_batch_cfg_t* cfg, double* d_out,
                      mlmc_batch_t** out_plan) {
    if (!out_plan) return set_error(MLMC_EINVAL, "out_plan is NULL");
    *out_plan = nullptr;
    if (!items || n_items <= 0) return set_error(MLMC_EINVAL, "need at least one item");
    if (n_items > (1 << 20)) return set_error(MLMC_EINVAL, "at most 2^20 items");
    if (!d_out) return set_error(MLMC_EINVAL, "d_out is NULL");
    if (rv != MLMC_RV_PWL16 && rv != MLMC_RV_CUBIC16) return set_error(MLMC_EINVAL, "rv must be PWL16 or CUBIC16");
    uint64_t total_rows = 0;
    for (int i = 0; i < n_items; ++i) {
        const mlmc_item_t& it = items[i];
        int rc = validate_sde_public(&it.sde);
        if (rc) return rc;
        if (it.level < 0 || it.level > kMaxLevel) return set_error(MLMC_EINVAL, "item %d: level outside 0..24", i);
        if (it.precision != MLMC_FP16 && it.precision != MLMC_FP32)
            return set_error(MLMC_EINVAL, "item %d: precision must be MLMC_FP16 or MLMC_FP32", i);
        if (it.kahan != 0 && it.kahan != 1) return set_error(MLMC_EINVAL, "item %d: kahan must be 0 or 1", i);
        if (it.stream > 0xFFFFu) return set_error(MLMC_EINVAL, "item %d: stream exceeds 65535", i);
        if (it.n_paths == 0 || it.n_paths > (1ull << 32))
            return set_error(MLMC_EINVAL, "item %d: n_paths must be 1..2^32", i);
        total_rows += rows_of((it.n_paths + chunk_paths(it.precision) - 1) / chunk_paths(it.precision), it.level, false);
    }
    const mlmc_batch_cfg_t c0 = merged(cfg);
    int rc = validate_cfg(c0);
    if (rc) return rc;
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;

    mlmc_batch* b = new mlmc_batch();
    (void)hipGetDevice(&b->device);
    b->rv = rv;
    b->items.assign(items, items + n_items);
    b->n_cu = di.n_cu;
    b->cfg = c0;
    if (!cfg) {
        mlmc_batch_cfg_t cached;
        if (cache_lookup(signature(*b), &cached)) b->cfg = cached;
    }
    b->d_out = d_out;
    const int r = rv == MLMC_RV_PWL16 ? 0 : 1;
    b->tab32 = di.tables[r][MLMC_FP32];
    b->tab16 = di.tables[r][MLMC_FP16];
    b->exact_tab = di.exact_tab;

    std::vector<LevelParams> prm(n_items);
    std::vector<int> var(n_items);
    std::vector<uint64_t> off(n_items), rows(n_items);
    uint64_t acc = 0;
    for (int i = 0; i < n_items; ++i) {
        const mlmc_item_t& it = items[i];
        rows[i] = rows_of((it.n_paths + chunk_paths(it.precision) - 1) / chunk_paths(it.precision), it.level, false);
        off[i] = acc;
        acc += rows[i];
        var[i] = variant_of(it.precision, it.kahan);
    }
    rc = MLMC_OK;
    auto alloc = [&](void** p, size_t bytes, const char* what) {
        if (!rc) rc = hipck(hipMalloc(p, bytes), what);
    };
    alloc((void**)&b->d_params, sizeof(LevelParams) * n_items, "hipMalloc params");
    alloc((void**)&b->d_variant, sizeof(int) * n_items, "hipMalloc variants");
    alloc((void**)&b->d_row_off, sizeof(uint64_t) * n_items, "hipMalloc offsets");
    alloc((void**)&b->d_rows, sizeof(uint64_t) * n_items, "hipMalloc rows");
    alloc((void**)&b->d_partials, sizeof(double) * kPartial * total_rows, "hipMalloc partials");
    alloc((void**)&b->d_counter, sizeof(uint32_t) * 64, "hipMalloc counter");
    alloc((void**)&b->d_ticks, sizeof(unsigned long long) * n_items, "hipMalloc item ticks");
    alloc((void**)&b->d_stage, sizeof(double) * kPartial * total_rows, "hipMalloc stage rows");
    if (!rc) rc = hipck(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    if (rc) {
        free_plan(b);
        return rc == MLMC_EHIP ? MLMC_ENOMEM : rc;
    }
    for (int i = 0; i < n_items; ++i) {
        const mlmc_item_t& it = items[i];
        fill_level_params(&prm[i], it.sde, it.level, it.precision, it.n_paths, 0, it.seed, it.stream, it.pset);
        prm[i].partials = b->d_partials + off[i] * kPartial;
        prm[i].mlp = di.mlp;
        prm[i].exact_tab = di.exact_tab;
    }
    if (!rc) rc = hipck(hipMemcpy(b->d_params, prm.data(), sizeof(LevelParams) * n_items, hipMemcpyHostToDevice), "copy");
    if (!rc) rc = hipck(hipMemcpy(b->d_variant, var.data(), sizeof(int) * n_items, hipMemcpyHostToDevice), "copy");
    if (!rc) rc = hipck(hipMemcpy(b->d_row_off, off.data(), sizeof(uint64_t) * n_items, hipMemcpyHostToDevice), "copy");
    if (!rc) rc = hipck(hipMemcpy(b->d_rows, rows.data(), sizeof(uint64_t) * n_items, hipMemcpyHostToDevice), "copy");
    if (!rc) {
        std::vector<uint2> blocks;
        for (int i = 0; i < n_items; ++i)
            for (uint32_t k = 0; k < stage_blocks(rows[i]); ++k) blocks.push_back(make_uint2((uint32_t)i, k));
        b->n_reduce_blocks = (uint32_t)blocks.size();
        alloc((void**)&b->d_reduce_blocks, sizeof(uint2) * blocks.size(), "hipMalloc reduction blocks");
        if (!rc)
            rc = hipck(hipMemcpy(b->d_reduce_blocks, blocks.data(), sizeof(uint2) * blocks.size(),
                                 hipMemcpyHostToDevice), "copy");
    }
    if (!rc) rc = prepare(b);
    if (rc) {
        free_plan(b);
        return rc;
    }
    *out_plan = b;
    return MLMC_OK;
}

int mlmc_batch_run(mlmc_batch_t* plan, void* hip_stream) {
    if (!plan || !plan->exec) return set_error(MLMC_EINVAL, "plan is NULL or not prepared");
    return hipck(hipGraphLaunch(plan->exec, (hipStream_t)hip_stream), "hipGraphLaunch");
}

int mlmc_batch_run_eager(mlmc_batch_t* plan, void* hip_stream) {
    if (!plan) return set_error(MLMC_EINVAL, "plan is NULL");
    return enqueue(plan, (hipStream_t)hip_stream);
}

int mlmc_batch_item_times(mlmc_batch_t* plan, double* h_wave_seconds, void* hip_stream) {
    if (!plan) return set_error(MLMC_EINVAL, "plan is NULL");
    if (!h_wave_seconds) return set_error(MLMC_EINVAL, "h_wave_seconds is NULL");
    int rc = hipck(hipStreamSynchronize((hipStream_t)hip_stream), "hipStreamSynchronize");
    if (rc) return rc;
    int khz = 0;
    if ((rc = hipck(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, plan->device), "wall clock rate")))
        return rc;
    if (khz <= 0) return set_error(MLMC_EHIP, "device reports no wall clock rate");
    std::vector<unsigned long long> t(plan->items.size());
    if ((rc = hipck(hipMemcpy(t.data(), plan->d_ticks, t.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost),
                    "hipMemcpy item ticks")))
        return rc;
    for (size_t i = 0; i < t.size(); ++i) h_wave_seconds[i] = (double)t[i] / (1e3 * khz);
    return MLMC_OK;
}

int mlmc_batch_info(const mlmc_batch_t* plan, mlmc_batch_cfg_t* cfg, uint64_t* n_tasks) {
    if (!plan) return set_error(MLMC_EINVAL, "plan is NULL");
    if (cfg) *cfg = plan->cfg;
    if (n_tasks) *n_tasks = plan->n_tasks;
    return MLMC_OK;
}

int mlmc_batch_autotune(mlmc_batch_t* plan, int repeats, mlmc_batch_cfg_t* best) {
    if (!plan) return set_error(MLMC_EINVAL, "plan is NULL");
    if (repeats < 1 || repeats > 100) return set_error(MLMC_EINVAL, "repeats must be 1..100");
    hipEvent_t e0, e1;
    int rc = hipck(hipEventCreate(&e0), "hipEventCreate");
    if (rc) return rc;
    if ((rc = hipck(hipEventCreate(&e1), "hipEventCreate"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    // block shapes (8 or 4 waves) and, for each, wavefronts per CU in whole blocks up to what
    // the kernel's registers and LDS let reside at once (a persistent wave that cannot start
    // before the queue drains is idle)
    std::vector<std::pair<int, int>> shapes;  // (block waves, waves per CU)
    for (int bw : {8, 4}) {
        int blocks_per_cu = 0;
        const void* fn = plan->rv == MLMC_RV_CUBIC16
                             ? (bw == 8 ? (const void*)batch_kernel<MLMC_RV_CUBIC16, 8>
                                        : (const void*)batch_kernel<MLMC_RV_CUBIC16, 4>)
                             : (bw == 8 ? (const void*)batch_kernel<MLMC_RV_PWL16, 8>
                                        : (const void*)batch_kernel<MLMC_RV_PWL16, 4>);
        if ((rc = hipck(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, fn, bw * kWave, 0),
                        "occupancy query"))) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
        bool any = false;
        for (int w = bw; w <= 32; w += bw)
            if (w <= bw * blocks_per_cu) {
                shapes.push_back({bw, w});
                any = true;
            }
        if (!any) shapes.push_back({bw, bw});
    }
    const int steps[] = {64, 256, 1024};
    const int prios[] = {12, 25};
    const int coops[] = {11, 12, 13, 14, 25};
    mlmc_batch_cfg_t winner = plan->cfg;
    float best_ms = 1e30f;
    for (const auto& shape : shapes)
        for (int st : steps)
            for (int pr : prios)
                for (int co : coops) {
                plan->cfg = mlmc_batch_cfg_t{shape.second, st, pr, co, shape.first};
                if ((rc = prepare(plan))) goto done;
                if ((rc = hipck(hipGraphLaunch(plan->exec, plan->cap_stream), "warm-up replay"))) goto done;
                if ((rc = hipck(hipEventRecord(e0, plan->cap_stream), "hipEventRecord"))) goto done;
                for (int k = 0; k < repeats; ++k)
                    if ((rc = hipck(hipGraphLaunch(plan->exec, plan->cap_stream), "replay"))) goto done;
                if ((rc = hipck(hipEventRecord(e1, plan->cap_stream), "hipEventRecord"))) goto done;
                if ((rc = hipck(hipEventSynchronize(e1), "hipEventSynchronize"))) goto done;
                float ms = 0.f;
                if ((rc = hipck(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime"))) goto done;
                if (ms < best_ms) {
                    best_ms = ms;
                    winner = plan->cfg;
                }
            }
    plan->cfg = winner;
    rc = prepare(plan);
    if (!rc) cache_store(signature(*plan), winner);
    if (!rc && best) *best = winner;
done:
    (void)hipStreamSynchronize(plan->cap_stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int mlmc_batch_destroy(mlmc_batch_t* plan) {
    if (!plan) return MLMC_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    (void)hipSetDevice(cur);
    return MLMC_OK;
}

}  // extern "C"
