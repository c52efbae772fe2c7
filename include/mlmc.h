/*
 * libmlmc -- the multilevel Monte Carlo level-correction estimator for Euler-Maruyama SDE
 * paths with exact or low-precision approximate Gaussian variables, on AMD Instinct
 * MI355X (gfx950).  C-ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The method (Giles and Sheridan-Methven, "Rounding error using low precision
 * approximate random variables"):
 *   - Euler-Maruyama for dX = a(X) dt + b(X) dW in finite precision,
 *     X_{n+1} = X_n (+) (A_n (+) B_n), A_n = a (x) delta, B_n = (b (x) sqrt(delta)) (x) Z_n
 *     (Section 2.2), here for geometric Brownian motion a = mu X, b = sigma X;
 *   - optional Kahan-compensated state update (Section 2.3, Algorithm 1);
 *   - MLMC level l: fine step delta_f = T 2^-l, coarse step 2 delta_f, coarse Wiener
 *     increments the pairwise sums of fine ones, exact and approximate variables from the
 *     same uniform (Section 3);
 *   - the plain two-way difference P_l - P_{l-1} and the nested four-way difference
 *     (P^_l - P^_{l-1}) - (P-_l - P-_{l-1}) with their sums and sums of squares, from
 *     which the caller forms the estimators theta^ and theta- and the variances v_l, V_l
 *     (Section 3), and the device time of each call, the cost c_l.
 *
 * Conventions for every entry point:
 *   - return MLMC_OK (0) on success or a negative MLMC_E* code; mlmc_last_error() then
 *     holds a message for the calling thread.  Nothing aborts or throws across the ABI.
 *   - arguments are validated before any HIP call, so invalid arguments are reported
 *     as MLMC_EINVAL even on a machine without a GPU; a valid call on a machine without a
 *     usable gfx950 device returns MLMC_ENODEV.
 *   - "device" pointers are HIP device memory of the current device; "host" pointers are
 *     ordinary host memory.  The caller owns every buffer it passes; the library owns only
 *     its per-device scratch (chunk partial sums, coefficient tables, MLP image), created
 *     on first use and released by mlmc_shutdown().
 *   - hip_stream arguments are hipStream_t values (NULL = the null stream).
 *   - results are bit-reproducible for identical arguments: uniforms depend only on
 *     (seed, stream, level, pset, path, step) and sums are reduced in a fixed order over
 *     fixed 64-path chunks (128 for binary16), independent of the launch shape.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
#define MLMC_OK 0
#define MLMC_EINVAL (-1)       /* an argument is out of range or a pointer is NULL      */
#define MLMC_ENOMEM (-2)       /* device or host allocation failed                      */
#define MLMC_ENODEV (-3)       /* no usable HIP device                                   */
#define MLMC_EHIP (-4)         /* a HIP runtime call failed                              */
#define MLMC_EUNSUPPORTED (-5) /* valid but unsupported combination (e.g. no MLP loaded) */

/* ---- enumerations ---------------------------------------------------------------- */
/* arithmetic of the approximate (or only) path pair; the exact pair is always binary64 */
#define MLMC_FP64 0
#define MLMC_FP32 1
#define MLMC_FP16 2 /* packed half2: two paths per lane */
/* bfloat16 (8 significant bits, the binary32 exponent range), emulated: binary32 registers,
 * every operation rounded to 8 bits, to nearest even; approximate and nested modes with
 * the table approximations only (the precision-width experiments around Figure 3) */
#define MLMC_BF16 3

/* inverse-CDF kind (Section 2.1; 16 dyadic intervals of (0,1/2], mirrored) */
#define MLMC_RV_EXACT 0   /* Z = Phi^-1(U), binary64                                   */
#define MLMC_RV_PWL16 1   /* piecewise linear, L2-optimal per interval (Lemma 2.2)     */
#define MLMC_RV_CUBIC16 2 /* piecewise cubic, L2-optimal per interval (Lemma 2.3)      */
#define MLMC_RV_MLP 3     /* 1-16-16-1 tanh network (binary16 weights), mirrored        */
#define MLMC_RV_PCONST4096 4 /* piecewise constant by table lookup (Section 2.1 names   */
                             /* table lookups among the substitutes for Z): the mean of */
                             /* Phi^-1 on each of 4096 equal cells of (0,1), mirrored;  */
                             /* cell = top 12 bits of the mirrored word                */

/* rv_mode of mlmc_level: which differences one call samples (Section 3) */
#define MLMC_EXACT 0          /* term 0 = P^_l - P^_{l-1}, binary64, exact variables      */
#define MLMC_APPROX_PWL16 1   /* term 0 = P-_l - P-_{l-1}, precision p, approx variables  */
#define MLMC_APPROX_CUBIC16 2
#define MLMC_APPROX_MLP 3
#define MLMC_NESTED_PWL16 5   /* nested: terms 0, 1 (four-way) and 2 on the same samples  */
#define MLMC_NESTED_CUBIC16 6
#define MLMC_NESTED_MLP 7
#define MLMC_APPROX_PCONST4096 4
#define MLMC_NESTED_PCONST4096 8

/* terms of a result */
#define MLMC_TERM_TWO_WAY 0       /* two-way difference of the call's own pair            */
#define MLMC_TERM_FOUR_WAY 1      /* (P^_l - P^_{l-1}) - (P-_l - P-_{l-1})  (nested only)   */
#define MLMC_TERM_TWO_WAY_EXACT 2 /* P^_l - P^_{l-1} of the nested samples (nested only)    */
#define MLMC_TERM_ROUNDING 3      /* X-_N - X~_N: fine terminal state in precision p minus  */
                                  /* binary64 with the same approximate variables (Lemma  */
                                  /* 2.6), only when diag is set                          */

/* time-stepping scheme of mlmc_level_args_t.scheme */
#define MLMC_SCHEME_EM 0       /* Euler-Maruyama, X <- X (+) (A (+) B) (Section 2.2)       */
#define MLMC_SCHEME_MILSTEIN 1 /* Milstein (named in Sections 2 and 4, not analysed there): */
                               /* for GBM dX = (A (+) B) (+) M, M = (cm (x) X) (x)         */
                               /* (Z (x) Z (-) k), cm = R_p(sigma^2 delta_f / 2), k = 1    */
                               /* fine, 2 coarse (the coarse variable is the sum of two    */
                               /* fine ones).  Exact and dyadic variables (not the MLP).   */

#define MLMC_PAYOFF_X 0    /* P(X) = X_T (Section 3 takes P(X) = X)                    */
#define MLMC_PAYOFF_CALL 1 /* P(X) = max(X_T - K, 0)                                   */

/* ---- data -------------------------------------------------------------------------- */
/* geometric Brownian motion dX = mu X dt + sigma X dW on [0, T], X_0 = x0 (Section 2.2) */
typedef struct {
    double mu;
    double sigma;
    double x0;
    double T;
    int32_t payoff; /* MLMC_PAYOFF_* */
    int32_t reserved;
    double strike;  /* K of the call payoff */
} mlmc_gbm_t;

/* result of one level call: per term, the sum and sum of squares over n_paths samples
 * (NaN for a term the call does not sample); mean = sum/m and unbiased variance
 * (sumsq - sum^2/m)/(m-1) are for the caller to form. */
typedef struct {
    double sum[4];
    double sumsq[4];
    uint64_t n_paths;
    uint64_t path_steps;  /* n_paths * 2^level fine steps (coupled path-steps)        */
    double cost_seconds;  /* device time of the call, from HIP events                 */
} mlmc_result_t;

/* full argument set of one level (extended entry points) */
typedef struct {
    mlmc_gbm_t sde;
    int32_t level;       /* 0..24: 2^level fine steps                                 */
    int32_t precision;   /* MLMC_FP64 / FP32 / FP16 / BF16                            */
    int32_t rv_mode;     /* MLMC_EXACT, MLMC_APPROX_*, MLMC_NESTED_*                  */
    int32_t kahan;       /* 0/1: Kahan-compensated low-precision updates              */
    int32_t diag;        /* 0/1: also sample MLMC_TERM_ROUNDING                        */
    uint32_t stream;     /* Philox stream id 0..65535 (independent sample sets)       */
    uint32_t pset;       /* parameter-set id (Philox counter word 3)                  */
    uint32_t scheme;     /* MLMC_SCHEME_EM or MLMC_SCHEME_MILSTEIN                     */
    uint64_t seed;       /* Philox key                                                */
    uint64_t n_paths;    /* samples; path_offset + n_paths <= 2^32                    */
    uint64_t path_offset;/* first path index (shards / resumes a sample set)          */
} mlmc_level_args_t;

/* ---- entry points ------------------------------------------------------------------ */

/* Initialise the library on HIP device `device` (optional: every call initialises the
 * current device lazily).  Builds the binary64 master tables of the dyadic
 * approximations (L2-optimal fit per interval, Section 2.1) on the host and uploads
 * them in each working precision.  Errors: MLMC_ENODEV, MLMC_EHIP, MLMC_ENOMEM. */
int mlmc_init(int device);

/* Release every per-device resource the library holds.  Always MLMC_OK. */
int mlmc_shutdown(void);

/* One MLMC level, synchronously (Section 3; the estimator sums of theta^ / theta-).
 * sde: host, GBM and payoff.  level: 0..24.  n_paths: 0..2^32 (0 gives zero sums).
 * precision: MLMC_FP64/FP32/FP16 (MLMC_EXACT requires MLMC_FP64).  rv_mode: MLMC_EXACT,
 * MLMC_APPROX_*, MLMC_NESTED_*.  kahan: 0/1 (ignored for binary64).  seed: Philox key.
 * Philox stream 0 for MLMC_EXACT / MLMC_APPROX_*, 1 for MLMC_NESTED_* (so the two sums
 * of theta- are independent), pset 0, path_offset 0.  out: host, filled on success,
 * including the device time of the call.  Runs on a library-owned stream.  The sums do not
 * depend on how the call is launched: a level >= 6 with few 64-path chunks (at most
 * four per CU) of the nested binary32 or the plain binary64 estimator runs one block of eight
 * waves per chunk instead of one wave, with the same partial sums and the same bits. */
int mlmc_level(const mlmc_gbm_t* sde, int level, uint64_t n_paths, int precision,
               int rv_mode, int kahan, uint64_t seed, mlmc_result_t* out);

/* mlmc_level with the full argument set (any scheme, stream, pset, path_offset, diag):
 * args, out: host.  Synchronous on the library's stream; out receives the sums and the
 * device time of the call.  Errors as mlmc_level. */
int mlmc_level_run(const mlmc_level_args_t* args, mlmc_result_t* out);

/* Several level calls at once, synchronously: the final sampling of an MLMC estimate
 * (Section 3) draws every term of every level, and a deep level with few samples is a few
 * long serial paths that leave most of the GPU idle.  The calls are issued longest chain
 * first (level, then n_paths), dealt round-robin over four library streams, so that such
 * calls overlap the shallow levels' many short paths.  args: host, n_calls (1..4096) argument
 * sets, each validated as for mlmc_level_run before anything is launched (the message names
 * the failing call).  out: host, n_calls results, each equal to what mlmc_level_run returns
 * for the same arguments except cost_seconds, the device time from the call's start to its
 * end while it shared the GPU.  span_seconds: host, may be NULL: device time from the first
 * call's start to the last call's end.  Uses its own streams and device memory (one
 * workspace per call, kept for the next set); sets that overlap on one device race. */
int mlmc_level_set_run(const mlmc_level_args_t* args, int n_calls, mlmc_result_t* out,
                       double* span_seconds);

/* Asynchronous level call on hip_stream.  args: host.  d_out: device, 8 doubles
 * (sum[0..3], sumsq[0..3]) written when the stream reaches the call.  d_workspace:
 * device scratch of at least mlmc_level_workspace_bytes(args) bytes (8-byte aligned; it
 * holds the partial sums of the call's rows of 64-path chunks and the stage rows of the
 * fixed-order two-stage reduction,
 * all written by the call before they are read), or NULL to use the library's per-device
 * scratch (calls that overlap on one device then race). */
int mlmc_level_ex(const mlmc_level_args_t* args, double* d_out, void* d_workspace,
                  size_t workspace_bytes, void* hip_stream);

/* mlmc_level_ex for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same fixed-order reduction (so the same bits), with the chunk partials and stage rows in a
 * library-owned device array of 4 MiB (room for 65536 chunks: n_paths <= 2^22, or 2^23 in
 * MLMC_FP16) that each device holds from library load until the process ends.  The call
 * allocates and frees nothing: the current device must have been set up by mlmc_init first
 * (else MLMC_EUNSUPPORTED).  args: host; d_out: device, 8 doubles (sum[0..3], sumsq[0..3]),
 * written when hip_stream reaches the call.  Larger n_paths: MLMC_EINVAL (checked before any
 * HIP call).  Every call on one device shares that device's array and writes every entry it
 * reads, so nothing carries over between calls; calls that overlap on one device race. */
int mlmc_level_noalloc(const mlmc_level_args_t* args, double* d_out, void* hip_stream);

/* Bytes of device scratch one mlmc_level_ex call needs (0 on invalid arguments). */
size_t mlmc_level_workspace_bytes(const mlmc_level_args_t* args);

/* Per-path payoffs of a level call, same kernel and launch as mlmc_level_ex (parity
 * checks).  Each device pointer receives n_paths doubles or may be NULL:
 * d_pf_hat / d_pc_hat  exact pair P^_l, P^_{l-1} (MLMC_EXACT or nested)
 * d_pf_bar / d_pc_bar  approximate pair P-_l, P-_{l-1} (approx or nested)
 * d_xf_tilde           binary64 fine state with approximate variables (diag)
 * Coarse entries are 0 at level 0 (P_{-1} = 0). */
int mlmc_paths(const mlmc_level_args_t* args, double* d_pf_hat, double* d_pc_hat,
               double* d_pf_bar, double* d_pc_bar, double* d_xf_tilde, void* hip_stream);

/* The uniform words the level kernels consume (parity checks): d_words (device,
 * n_paths * n_steps uint32, row-major [path][step]) for paths path0.. of the given
 * seed, Philox stream, level and pset.  n_steps <= 2^24, and at most 2^level at levels 0
 * and 1, where one Philox call serves 4 / 2^level consecutive paths (counter (0, path div
 * G, (stream << 16) | level, pset), word (path mod G) 2^level + n); from level 2 on the
 * counter is (n >> 2, path, (stream << 16) | level, pset) and step n takes word n & 3. */
int mlmc_uniforms(uint64_t seed, uint32_t stream, int level, uint32_t pset, uint64_t path0,
                  uint64_t n_paths, uint32_t n_steps, uint32_t* d_words, void* hip_stream);

/* Z = Phi^-1(U) or Z~ for n device words (Section 3: same U for both), widened to
 * binary64 into d_out (device, n doubles).  rv: MLMC_RV_*; precision: arithmetic of the
 * approximation (ignored for MLMC_RV_EXACT, which is binary64). */
int mlmc_icdf(const uint32_t* d_words, uint64_t n, int rv, int precision, double* d_out,
              void* hip_stream);

/* The library's coefficient table of a dyadic approximation (Section 2.1): 16 rows of
 * (degree + 1) coefficients c_0..c_d in the local coordinate, rounded to `precision`
 * and widened to binary64, written to h_out (host, 16 * 4 doubles; unused columns 0).
 * rv: MLMC_RV_PWL16 or MLMC_RV_CUBIC16.  Host-only: needs no GPU. */
int mlmc_table(int rv, int precision, double* h_out);

/* Lower-half cell means of MLMC_RV_PCONST4096 (cell i = [i/4096, (i+1)/4096), i < 2048;
 * the upper half is the mirror) rounded to `precision` and widened to binary64, written to
 * h_out (host, 2048 doubles).  Built on the host as 4096 (phi(Phi^-1(a)) - phi(Phi^-1(b)))
 * in long double.  Host-only: needs no GPU. */
int mlmc_pconst_table(int precision, double* h_out);

/* ---- batched sweep: many (parameter set, level) items in one persistent launch -------
 * Not in the paper: a full MLMC sweep (Section 3: every level l = 0..L, here also many
 * GBM parameter sets) as one launch.  Each item is a nested sample set (terms 0, 1, 2 as
 * in mlmc_level) of one level of one GBM.  Work is split into tasks (chunk ranges of one
 * item), ordered longest first and popped by each wavefront from a device work queue;
 * per-item sums are reduced in the same fixed order as mlmc_level, so every item's result
 * equals the corresponding single-level call bit for bit. */
typedef struct {
    mlmc_gbm_t sde;
    int32_t level;      /* 0..24                                                        */
    int32_t precision;  /* MLMC_FP16 or MLMC_FP32 (the approximate pair)                 */
    int32_t kahan;      /* 0/1                                                          */
    uint32_t pset;      /* parameter-set id (Philox counter word 3)                     */
    uint32_t stream;    /* Philox stream id 0..65535                                    */
    uint32_t reserved;
    uint64_t n_paths;   /* 1..2^32                                                      */
    uint64_t seed;      /* Philox key                                                   */
} mlmc_item_t;

/* launch shape of a batch (0 in a field selects the default or the autotuned value) */
typedef struct {
    int32_t waves_per_cu;    /* wavefronts per CU of the persistent grid (rounded down to */
                             /* whole blocks): 4..32, at least one block                  */
    int32_t task_steps;      /* fine steps per task at level 0 (tasks of level l hold      */
                             /* max(1, task_steps >> l) chunks): 1..2^20                 */
    int32_t priority_level;  /* tasks of level >= this run at raised wave priority; 25=off */
    int32_t coop_level;      /* binary32 items of level >= this (2..25; 25 = off) run each   */
                             /* chunk on a whole block: its other waves draw the variables */
                             /* of the next 4 (block_waves - 1) steps into LDS while one   */
                             /* wave advances the paths (same operations, same bits)       */
    int32_t block_waves;     /* wavefronts per block: 8 or 4                               */
} mlmc_batch_cfg_t;

typedef struct mlmc_batch mlmc_batch_t; /* opaque plan (device task list + captured graph) */

/* Build a plan for n_items items (host array, copied) that all use approximation rv
 * (MLMC_RV_PWL16 or MLMC_RV_CUBIC16).  d_out: device, n_items x 8 doubles (sum[0..3],
 * sumsq[0..3] per item; term 3 is 0), owned by the caller and written by every run.  cfg:
 * host, may be NULL (defaults, or the cached autotuned shape for this item list).  The
 * launch sequence (queue reset, persistent kernel, per-item reduction) is captured into a
 * hipGraph.  *out_plan receives the plan; free it with mlmc_batch_destroy. */
int mlmc_batch_create(const mlmc_item_t* items, int n_items, int rv, const mlmc_batch_cfg_t* cfg,
                      double* d_out, mlmc_batch_t** out_plan);

/* Replay the plan's graph on hip_stream (asynchronous). */
int mlmc_batch_run(mlmc_batch_t* plan, void* hip_stream);

/* Launch the same kernels directly, without the graph (asynchronous). */
int mlmc_batch_run_eager(mlmc_batch_t* plan, void* hip_stream);

/* Time candidate launch shapes (each replayed `repeats` times, 1..100), keep the fastest in
 * the plan (re-captured) and in the autotune cache file named by MLMC_AUTOTUNE_CACHE (no
 * cache when unset).  best: host, may be NULL.  Synchronous; d_out is overwritten. */
int mlmc_batch_autotune(mlmc_batch_t* plan, int repeats, mlmc_batch_cfg_t* best);

/* Cost of each item in the plan's last run (Section 3's c_l, per item): h_wave_seconds
 * (host, n_items doubles) receives the wall-clock time that wavefronts spent on the item's
 * tasks, summed over wavefronts (the device's constant-rate counter, read at the start and
 * end of every task).  Dividing by the sum over items and multiplying by the sweep time
 * attributes the device time to items.  Synchronous: waits for hip_stream first. */
int mlmc_batch_item_times(mlmc_batch_t* plan, double* h_wave_seconds, void* hip_stream);

/* The plan's current launch shape and task count (host outputs, either may be NULL). */
int mlmc_batch_info(const mlmc_batch_t* plan, mlmc_batch_cfg_t* cfg, uint64_t* n_tasks);

/* Release a plan (NULL is allowed). */
int mlmc_batch_destroy(mlmc_batch_t* plan);

/* ---- learned inverse CDF (MLMC_RV_MLP) -------------------------------------------------
 * Not in the paper: a 1-16-16-1 tanh network used as an approximate Gaussian variable in
 * the sense of Section 2.1 / Assumption 2.1 (mirrored, so exactly zero mean; bounded).
 * u' = min(u, 1-u), r = sqrt(-2 ln 2u'), input x = r/3.4 - 1, output y, Z~ = +-(y - r).
 * Parameters: 321 binary32 values W1(16) b1(16) W2(16x16 row-major [out][in]) b2(16)
 * W3(16) b3(1).  Training pairs (Philox stream 2): pair i uses words w0, w1 of counter
 * (0, i, 2<<16, 0); even pairs take w0 mirrored to (0, 1/2), odd pairs the tail-weighted
 * word (w0 >> 1) >> (w1 mod 31); target Phi^-1(u') + r from the binary64 exact inverse. */
typedef struct {
    uint64_t seed;     /* Philox key of the training pairs                               */
    uint32_t n_pairs;  /* training set size (multiple of batch), <= 2^26                 */
    uint32_t batch;    /* mini-batch size, a multiple of 128                              */
    uint32_t epochs;   /* passes over the training set, 1..100000                         */
    float lr;          /* Adam learning rate of the first epoch                           */
    float lr_final;    /* learning rate of the last epoch (geometric decay per epoch)     */
    uint32_t reserved;
} mlmc_mlp_cfg_t;

/* Training pairs first..first+n-1 (parity checks): d_words (device, n uint32, may be NULL)
 * the mirrored words, d_x (device, n floats) the network inputs, d_target (device, n
 * floats) Phi^-1(u') + r. */
int mlmc_mlp_pairs(uint64_t seed, uint32_t first, uint32_t n, uint32_t* d_words, float* d_x,
                   float* d_target, void* hip_stream);

/* Gradient of the mean squared error over pairs first..first+n-1 (1 <= n <= 2^24) at the
 * parameters d_params (device, 321 floats): d_grad (device, 321 floats), d_loss (device,
 * 1 float, may be NULL).  Synchronous on hip_stream. */
int mlmc_mlp_grad(const float* d_params, uint64_t seed, uint32_t first, uint32_t n, float* d_grad,
                  float* d_loss, void* hip_stream);

/* Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on cfg->n_pairs pairs; d_params
 * (device, 321 floats) holds the initial parameters on entry and the trained ones on
 * return.  h_loss (host, cfg->epochs floats, may be NULL) receives the mini-batch loss
 * at the end of each epoch.  Synchronous: waits for hip_stream, then runs one captured
 * hipGraph per epoch on a library stream. */
int mlmc_mlp_train(const mlmc_mlp_cfg_t* cfg, float* d_params, float* h_loss, void* hip_stream);

/* Deploy parameters (device, 321 floats) as the MLMC_RV_MLP inference model of the
 * current device: each is rounded once to binary16.  Synchronous on hip_stream. */
int mlmc_mlp_load(const float* d_params, void* hip_stream);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* mlmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_H */
