// Training of the learned inverse CDF on the GPU: pair generation, fused forward and
// backward pass with fixed-order gradient sums, and Adam, one epoch captured in a hipGraph.
//
// Pairs (Philox stream 2): pair i draws words w0, w1 of counter (0, i, 2 << 16, 0); even
// pairs are uniform (w0 mirrored to the lower half), odd pairs tail-weighted
// (xm = (w0 >> 1) >> (w1 mod 31)).  Input x = r / 3.4 - 1 and target Phi^{-1}(u') + r with
// the binary64 exact inverse.  The trained network uses the hard tanh min(max(z, -1), 1)
// (slope 1 inside, 0 outside); deployment rewrites it with clamps to [0, 1] (mlp.h).  Loss:
// mean squared error over a mini-batch.  Every sum (per-block gradient, across blocks) is
// taken in a fixed order, so training is bit-reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "icdf.h"
#include "internal.h"
#include "mlp.h"
#include "philox.h"

namespace mlmc {

namespace {

constexpr int kTB = 128;          // samples per training block
constexpr int kGradStride = 324;  // 321 gradients + loss, padded
constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;

__device__ __forceinline__ float hard_tanh(float z) { return fminf(fmaxf(z, -1.0f), 1.0f); }
// slope of the hard tanh at its argument z, from its value h = hard_tanh(z): 1 inside (-1, 1)
__device__ __forceinline__ float hard_tanh_slope(float h) { return (h > -1.0f && h < 1.0f) ? 1.0f : 0.0f; }

__device__ __forceinline__ uint32_t pair_word(uint32_t i, uint32_t k0, uint32_t k1) {
    const Words4 r = philox4x32_10(0u, i, 2u << 16, 0u, k0, k1);
    if ((i & 1u) == 0u) return (r.w[0] >> 31) ? ~r.w[0] : r.w[0];
    return (r.w[0] >> 1) >> (r.w[1] % 31u);
}

__global__ void pairs_kernel(uint32_t k0, uint32_t k1, uint32_t first, uint32_t n, uint32_t* __restrict__ words,
                             float* __restrict__ xs, float* __restrict__ ts, const ExactTable* __restrict__ ex) {
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
        const uint32_t xm = pair_word(first + g, k0, k1);
        const double r = mlp_radius(xm, ex->lds.log);
        if (words) words[g] = xm;
        xs[g] = (float)(r * (1.0 / 3.4) - 1.0);
        ts[g] = (float)(icdf_exact_f64(xm, &ex->lds.top, ex->deep) + r);
    }
}

// One block: kTB samples of pairs [first + blockIdx.x * kTB, ...) clipped to `last`.
// Writes the block's gradient of  scale * sum (y - t)^2  (scale = 1 / batch) and the
// block's sum of squared residuals.
__global__ __launch_bounds__(kTB) void grad_kernel(const float* __restrict__ params, const float* __restrict__ xs,
                                                   const float* __restrict__ ts, uint32_t first, uint32_t last,
                                                   float scale, float* __restrict__ block_grad) {
    __shared__ float sW[kMlpParams];
    __shared__ float s_h1[kMlpHidden][kTB], s_da1[kMlpHidden][kTB], s_da2[kMlpHidden][kTB], s_h2[kMlpHidden][kTB];
    __shared__ float s_x[kTB], s_dy[kTB], s_l[kTB];
    for (int i = threadIdx.x; i < kMlpParams; i += kTB) sW[i] = params[i];
    __syncthreads();
    const uint32_t t = threadIdx.x;
    const uint32_t i = first + blockIdx.x * kTB + t;
    const bool valid = i < last;
    const float x = valid ? xs[i] : 0.0f;
    const float target = valid ? ts[i] : 0.0f;
    float h1[kMlpHidden], h2[kMlpHidden];
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) h1[k] = hard_tanh(__builtin_fmaf(sW[kW1 + k], x, sW[kB1 + k]));
    float y = sW[kB3];
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) {
        asm volatile("" ::: "memory");  // read each weight row from LDS when it is used
        float a = sW[kB2 + k];
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) a = __builtin_fmaf(sW[kW2 + k * kMlpHidden + j], h1[j], a);
        h2[k] = hard_tanh(a);
        y = __builtin_fmaf(sW[kW3 + k], h2[k], y);
    }
    const float res = valid ? y - target : 0.0f;
    const float dy = 2.0f * scale * res;
    float dh1[kMlpHidden];
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j) dh1[j] = 0.0f;
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) {
        asm volatile("" ::: "memory");
        const float da2 = dy * sW[kW3 + k] * hard_tanh_slope(h2[k]);
        s_da2[k][t] = da2;
        s_h2[k][t] = h2[k];
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) dh1[j] = __builtin_fmaf(da2, sW[kW2 + k * kMlpHidden + j], dh1[j]);
    }
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j) {
        s_h1[j][t] = h1[j];
        s_da1[j][t] = dh1[j] * hard_tanh_slope(h1[j]);
    }
    s_x[t] = x;
    s_dy[t] = dy;
    s_l[t] = res * res;
    __syncthreads();
    float* out = block_grad + (uint64_t)blockIdx.x * kGradStride;
    // dW2[k][j] = sum_b da2[k][b] h1[j][b]: thread t handles entries t and t + 128
    for (int e = t; e < 256; e += kTB) {
        const int k = e / kMlpHidden, j = e % kMlpHidden;
        float acc = 0.0f;
        for (int b = 0; b < kTB; ++b) acc = __builtin_fmaf(s_da2[k][b], s_h1[j][b], acc);
        out[kW2 + e] = acc;
    }
    // W1, b1, b2, W3, b3 and the loss: 66 sums
    if (t < 66) {
        float acc = 0.0f;
        for (int b = 0; b < kTB; ++b) {
            float v;
            if (t < 16) v = s_da1[t][b] * s_x[b];
            else if (t < 32) v = s_da1[t - 16][b];
            else if (t < 48) v = s_da2[t - 32][b];
            else if (t < 64) v = s_dy[b] * s_h2[t - 48][b];
            else if (t == 64) v = s_dy[b];
            else v = s_l[b];
            acc += v;
        }
        const int dst = t < 16 ? kW1 + t : t < 32 ? kB1 + (t - 16) : t < 48 ? kB2 + (t - 32) : t < 64 ? kW3 + (t - 48)
                      : t == 64 ? kB3 : kMlpParams;  // slot 321 holds the loss
        out[dst] = acc;
    }
}

// Sums the block gradients in block order: grad[i] = sum_b block_grad[b][i] (i < 322).
__device__ __forceinline__ float sum_blocks(const float* __restrict__ block_grad, uint32_t n_blocks, int i) {
    float acc = 0.0f;
    for (uint32_t b = 0; b < n_blocks; ++b) acc += block_grad[(uint64_t)b * kGradStride + i];
    return acc;
}

__global__ void reduce_grad_kernel(const float* __restrict__ block_grad, uint32_t n_blocks, float* __restrict__ grad,
                                   float* __restrict__ loss, float loss_scale) {
    const int i = threadIdx.x;
    if (i < kMlpParams) grad[i] = sum_blocks(block_grad, n_blocks, i);
    if (i == kMlpParams && loss) loss[0] = sum_blocks(block_grad, n_blocks, kMlpParams) * loss_scale;
}

// Adam on the summed gradient.  state: [m(321) | v(321)], counter[0] = steps taken.  The
// learning rate decays geometrically per epoch from lr0 to lr1 over `epochs` epochs.
__global__ void adam_kernel(float* __restrict__ params, float* __restrict__ state, uint32_t* __restrict__ counter,
                            const float* __restrict__ block_grad, uint32_t n_blocks, uint32_t steps_per_epoch,
                            uint32_t epochs, float lr0, float lr1, float* __restrict__ loss_hist, float loss_scale) {
    const int i = threadIdx.x;
    const uint32_t step = counter[0] + 1u;  // read by every thread before thread 0 advances it
    const uint32_t epoch = (step - 1u) / steps_per_epoch;
    const float frac = epochs > 1 ? (float)epoch / (float)(epochs - 1) : 0.0f;
    const float lr = lr0 * powf(lr1 / lr0, frac);
    if (i < kMlpParams) {
        const float g = sum_blocks(block_grad, n_blocks, i);
        float* m = state;
        float* v = state + kMlpParams;
        m[i] = kBeta1 * m[i] + (1.0f - kBeta1) * g;
        v[i] = kBeta2 * v[i] + (1.0f - kBeta2) * g * g;
        const float mhat = m[i] / (1.0f - powf(kBeta1, (float)step));
        const float vhat = v[i] / (1.0f - powf(kBeta2, (float)step));
        params[i] -= lr * mhat / (sqrtf(vhat) + kEps);
    }
    if (i == kMlpParams && loss_hist && step % steps_per_epoch == 0u)
        loss_hist[epoch] = sum_blocks(block_grad, n_blocks, kMlpParams) * loss_scale;
    __syncthreads();
    if (i == 0) counter[0] = step;
}

__global__ void fill_kernel(float* __restrict__ p, uint32_t n, float v, uint32_t* __restrict__ counter) {
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) p[g] = v;
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) counter[0] = 0u;
}

// Inference image: the deployed form of the parameters (c = (h + 1) / 2 for every hard-tanh
// unit h), A1 = W1 / 2, a1 = (b1 + 1) / 2, A2 = W2, a2 = (b2 - W2 1 + 1) / 2, A3 = 2 W3,
// a3 = b3 - W3 . 1, each formed in binary32 (sums in index order), rounded once to binary16
// and stored widened to binary32, followed by the same binary16 values packed as the matrix
// operands of the inference (layout in mlp.h).
__device__ __forceinline__ float pack_halves(_Float16 lo, _Float16 hi) {
    return __uint_as_float((uint32_t)__builtin_bit_cast(uint16_t, lo) |
                           ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16));
}

__global__ void deploy_kernel(const float* __restrict__ params, float* __restrict__ image) {
    __shared__ _Float16 h[kMlpParams];
    const int i = threadIdx.x;
    if (i < kMlpParams) {
        float v = 0.0f;
        if (i < kB1) {
            v = params[i] * 0.5f;
        } else if (i < kW2) {
            v = (params[i] + 1.0f) * 0.5f;
        } else if (i < kB2) {
            v = params[i];
        } else if (i < kW3) {
            const int n = i - kB2;
            float s = 0.0f;
            for (int k = 0; k < kMlpHidden; ++k) s = __fadd_rn(s, params[kW2 + n * kMlpHidden + k]);
            v = __fmul_rn(__fadd_rn(__fadd_rn(params[i], -s), 1.0f), 0.5f);
        } else if (i < kB3) {
            v = params[i] * 2.0f;
        } else {
            float s = 0.0f;
            for (int k = 0; k < kMlpHidden; ++k) s = __fadd_rn(s, params[kW3 + k]);
            v = __fadd_rn(params[i], -s);
        }
        h[i] = (_Float16)__float2half_rn(v);
        image[i] = (float)h[i];
    } else if (i < kPkL1) {
        image[i] = 0.0f;
    }
    __syncthreads();
    if (i < kPkA2 - kPkL1) {                       // first layer, per row g
        const int g = i / 4, q = i % 4;
        const int base = (q < 2 ? kW1 : kB1) + 4 * g + 2 * (q & 1);
        image[kPkL1 + i] = pack_halves(h[base], h[base + 1]);
    } else if (i < kPkA3 - kPkL1) {                // 16 x 16 layer, per lane
        const int j = i - (kPkA2 - kPkL1), lane = j / 2, c = lane % 16, g = lane / 16;
        const int base = kW2 + c * kMlpHidden + 4 * g + 2 * (j & 1);
        image[kPkL1 + i] = pack_halves(h[base], h[base + 1]);
    } else if (i < kPkB3 - kPkL1) {                // output layer, masked per block
        const int j = i - (kPkA3 - kPkL1), e = j / 2, b = e / 16, r = (e / 4) % 4, g = e % 4;
        const int base = kW3 + 4 * g + 2 * (j & 1);
        image[kPkL1 + i] = r == b ? pack_halves(h[base], h[base + 1]) : 0.0f;
    } else if (i < kMlpImage - kPkL1) {
        image[kPkL1 + i] = (float)h[kB3];
    }
}

int ck(hipError_t e, const char* what) {
    return e == hipSuccess ? MLMC_OK : set_error(MLMC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

hipError_t launch_mlp_deploy(const float* d_params, float* image, hipStream_t s) {
    static_assert(kMlpImage - kPkL1 <= 384 && kMlpParams <= 384 && kPkL1 <= 384, "one thread per entry");
    hipLaunchKernelGGL(deploy_kernel, dim3(1), dim3(384), 0, s, d_params, image);
    return hipGetLastError();
}

}  // namespace mlmc

using namespace mlmc;

extern "C" {

int mlmc_mlp_pairs(uint64_t seed, uint32_t first, uint32_t n, uint32_t* d_words, float* d_x, float* d_target,
                   void* hip_stream) {
    if (n > 0 && (!d_x || !d_target)) return set_error(MLMC_EINVAL, "NULL buffer");
    if ((uint64_t)first + n > (1ull << 32)) return set_error(MLMC_EINVAL, "first + n exceeds 2^32");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc || n == 0) return rc;
    const uint32_t grid = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    hipLaunchKernelGGL(pairs_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream, (uint32_t)seed,
                       (uint32_t)(seed >> 32), first, n, d_words, d_x, d_target, (const ExactTable*)di.exact_tab);
    return ck(hipGetLastError(), "pairs kernel launch");
}

int mlmc_mlp_grad(const float* d_params, uint64_t seed, uint32_t first, uint32_t n, float* d_grad, float* d_loss,
                  void* hip_stream) {
    if (!d_params || !d_grad) return set_error(MLMC_EINVAL, "NULL buffer");
    if (n == 0 || n > (1u << 24)) return set_error(MLMC_EINVAL, "n must be 1..2^24");
    if ((uint64_t)first + n > (1ull << 32)) return set_error(MLMC_EINVAL, "first + n exceeds 2^32");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    const hipStream_t s = (hipStream_t)hip_stream;
    const uint32_t blocks = (n + kTB - 1) / kTB;
    DevBuf xs, ts, bg;
    if ((rc = ck(hipMalloc(&xs.p, n * sizeof(float)), "hipMalloc")) || (rc = ck(hipMalloc(&ts.p, n * sizeof(float)), "hipMalloc")) ||
        (rc = ck(hipMalloc(&bg.p, (size_t)blocks * kGradStride * sizeof(float)), "hipMalloc")))
        return MLMC_ENOMEM;
    const uint32_t grid = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    hipLaunchKernelGGL(pairs_kernel, dim3(grid), dim3(256), 0, s, (uint32_t)seed, (uint32_t)(seed >> 32), first, n,
                       nullptr, (float*)xs.p, (float*)ts.p, (const ExactTable*)di.exact_tab);
    hipLaunchKernelGGL(grad_kernel, dim3(blocks), dim3(kTB), 0, s, d_params, (const float*)xs.p, (const float*)ts.p,
                       0u, n, 1.0f / (float)n, (float*)bg.p);
    hipLaunchKernelGGL(reduce_grad_kernel, dim3(1), dim3(384), 0, s, (const float*)bg.p, blocks, d_grad, d_loss,
                       1.0f / (float)n);
    if ((rc = ck(hipGetLastError(), "gradient kernels launch"))) return rc;
    return ck(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int mlmc_mlp_train(const mlmc_mlp_cfg_t* cfg, float* d_params, float* h_loss, void* hip_stream) {
    if (!cfg || !d_params) return set_error(MLMC_EINVAL, "NULL argument");
    if (cfg->n_pairs < cfg->batch || cfg->batch < kTB || cfg->batch % kTB != 0 || cfg->n_pairs % cfg->batch != 0)
        return set_error(MLMC_EINVAL, "batch must be a multiple of %d dividing n_pairs", kTB);
    if (cfg->n_pairs > (1u << 26)) return set_error(MLMC_EINVAL, "n_pairs must be at most 2^26");
    if (cfg->epochs < 1 || cfg->epochs > 100000) return set_error(MLMC_EINVAL, "epochs must be 1..100000");
    if (!(cfg->lr > 0) || !(cfg->lr_final > 0)) return set_error(MLMC_EINVAL, "learning rates must be positive");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    const hipStream_t s = (hipStream_t)hip_stream;
    const uint32_t n = cfg->n_pairs, B = cfg->batch, spe = n / B, blocks = B / kTB;
    DevBuf xs, ts, bg, st, cnt, lh;
    if ((rc = ck(hipMalloc(&xs.p, n * sizeof(float)), "hipMalloc")) || (rc = ck(hipMalloc(&ts.p, n * sizeof(float)), "hipMalloc")) ||
        (rc = ck(hipMalloc(&bg.p, (size_t)blocks * kGradStride * sizeof(float)), "hipMalloc")) ||
        (rc = ck(hipMalloc(&st.p, 2 * kMlpParams * sizeof(float)), "hipMalloc")) ||
        (rc = ck(hipMalloc(&cnt.p, 64 * sizeof(uint32_t)), "hipMalloc")) ||
        (rc = ck(hipMalloc(&lh.p, (size_t)cfg->epochs * sizeof(float)), "hipMalloc")))
        return MLMC_ENOMEM;
    const uint32_t grid = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    hipLaunchKernelGGL(pairs_kernel, dim3(grid), dim3(256), 0, s, (uint32_t)cfg->seed, (uint32_t)(cfg->seed >> 32),
                       0u, n, nullptr, (float*)xs.p, (float*)ts.p, (const ExactTable*)di.exact_tab);
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, s, (float*)st.p, (uint32_t)(2 * kMlpParams), 0.0f,
                       (uint32_t*)cnt.p);
    if ((rc = ck(hipGetLastError(), "training set-up launch"))) return rc;
    if ((rc = ck(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;

    // capture one epoch: spe x (gradient, Adam)
    hipStream_t cs;
    if ((rc = ck(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate"))) return rc;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    rc = ck(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (!rc) {
        for (uint32_t k = 0; k < spe; ++k) {
            hipLaunchKernelGGL(grad_kernel, dim3(blocks), dim3(kTB), 0, cs, (const float*)d_params,
                               (const float*)xs.p, (const float*)ts.p, k * B, (k + 1) * B, 1.0f / (float)B,
                               (float*)bg.p);
            hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(384), 0, cs, d_params, (float*)st.p, (uint32_t*)cnt.p,
                               (const float*)bg.p, blocks, spe, cfg->epochs, cfg->lr, cfg->lr_final, (float*)lh.p,
                               1.0f / (float)B);
        }
        rc = ck(hipGetLastError(), "training kernels launch");
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (!rc) rc = ck(e, "hipStreamEndCapture");
    }
    if (!rc) rc = ck(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    for (uint32_t ep = 0; !rc && ep < cfg->epochs; ++ep) rc = ck(hipGraphLaunch(exec, cs), "hipGraphLaunch");
    if (!rc) rc = ck(hipStreamSynchronize(cs), "hipStreamSynchronize");
    if (!rc && h_loss)
        rc = ck(hipMemcpy(h_loss, lh.p, (size_t)cfg->epochs * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    return rc;
}

}  // extern "C"
