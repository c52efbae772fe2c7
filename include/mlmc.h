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

/* inverse-CDF kind (Section 2.1; 16 dyadic intervals of (0,1/2], mirrored) */
#define MLMC_RV_EXACT 0   /* Z = Phi^-1(U), binary64                                   */
#define MLMC_RV_PWL16 1   /* piecewise linear, L2-optimal per interval (Lemma 2.2)     */
#define MLMC_RV_CUBIC16 2 /* piecewise cubic, L2-optimal per interval (Lemma 2.3)      */
#define MLMC_RV_MLP 3     /* 1-16-16-1 tanh network (binary16 weights), mirrored        */

/* rv_mode of mlmc_level: which differences one call samples (Section 3) */
#define MLMC_EXACT 0          /* term 0 = P^_l - P^_{l-1}, binary64, exact variables      */
#define MLMC_APPROX_PWL16 1   /* term 0 = P-_l - P-_{l-1}, precision p, approx variables  */
#define MLMC_APPROX_CUBIC16 2
#define MLMC_APPROX_MLP 3
#define MLMC_NESTED_PWL16 5   /* nested: terms 0, 1 (four-way) and 2 on the same samples  */
#define MLMC_NESTED_CUBIC16 6
#define MLMC_NESTED_MLP 7

/* terms of a result */
#define MLMC_TERM_TWO_WAY 0       /* two-way difference of the call's own pair            */
#define MLMC_TERM_FOUR_WAY 1      /* (P^_l - P^_{l-1}) - (P-_l - P-_{l-1})  (nested only)   */
#define MLMC_TERM_TWO_WAY_EXACT 2 /* P^_l - P^_{l-1} of the nested samples (nested only)    */
#define MLMC_TERM_ROUNDING 3      /* X-_N - X~_N: fine terminal state in precision p minus  */
                                  /* binary64 with the same approximate variables (Lemma  */
                                  /* 2.6), only when diag is set                          */

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
    int32_t precision;   /* MLMC_FP64 / FP32 / FP16                                   */
    int32_t rv_mode;     /* MLMC_EXACT, MLMC_APPROX_*, MLMC_NESTED_*                  */
    int32_t kahan;       /* 0/1: Kahan-compensated low-precision updates              */
    int32_t diag;        /* 0/1: also sample MLMC_TERM_ROUNDING                        */
    uint32_t stream;     /* Philox stream id 0..65535 (independent sample sets)       */
    uint32_t pset;       /* parameter-set id (Philox counter word 3)                  */
    uint32_t reserved;
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
 * including the device time of the call.  Runs on a library-owned stream. */
int mlmc_level(const mlmc_gbm_t* sde, int level, uint64_t n_paths, int precision,
               int rv_mode, int kahan, uint64_t seed, mlmc_result_t* out);

/* Asynchronous level call on hip_stream.  args: host.  d_out: device, 8 doubles
 * (sum[0..3], sumsq[0..3]) written when the stream reaches the call.  d_workspace:
 * device scratch of at least mlmc_level_workspace_bytes(args) bytes, or NULL to use the
 * library's per-device scratch (calls that overlap on one device then race). */
int mlmc_level_ex(const mlmc_level_args_t* args, double* d_out, void* d_workspace,
                  size_t workspace_bytes, void* hip_stream);

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
 * seed, Philox stream, level and pset.  n_steps <= 2^24. */
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

/* Thread-local message of the last failure on this thread ("" if none). */
const char* mlmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_H */
