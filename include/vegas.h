/*
 * vegas.h -- C ABI of the MI355X (gfx950) VEGAS+ iteration library.
 *
 * One VEGAS+ iteration (Tolotti et al., arXiv:2408.09229, Sec. 2.1 and
 * Alg. 1-2) runs entirely in HIP kernels on the caller's stream:
 * stratified sampling over hypercubes (Sec. 2.1.2), the separable adaptive
 * importance map and its Jacobian (Sec. 2.1.1, Eq. 2-4), the integrand,
 * per-hypercube mean/variance (Eq. 5-6), per-axis refinement histograms,
 * then the map refinement (damping alpha) and the sample reallocation
 * n_h ~ sigma_h^beta (Eq. 7).  Iteration estimates combine by Eq. 8-9.
 *
 * Conventions
 *  - Every function is extern "C", takes plain pointers and sizes, and never
 *    throws.  Failures return a negative vegas_status; vegas_last_error()
 *    gives a thread-local message.
 *  - "device pointer" means memory on the current HIP device; "host pointer"
 *    means ordinary host memory.  Each argument below says which.
 *  - A context borrows the caller's device workspace and HIP stream; both
 *    must outlive it.  The library allocates no device memory of its own.
 *  - A context is not thread-safe.  Distinct contexts are independent.
 *  - All work is asynchronous on the stream, except functions documented as
 *    synchronous (they synchronise that stream before returning).
 */
#ifndef VEGAS_MI355X_H
#define VEGAS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VEGAS_OK = 0,
    VEGAS_EINVAL = -1,        /* invalid argument or configuration */
    VEGAS_ENOMEM = -2,        /* workspace too small / sizes overflow */
    VEGAS_EDEVICE = -3,       /* a HIP call failed (message has the HIP error) */
    VEGAS_ESTATE = -4,        /* call not valid in the context's state */
    VEGAS_ENONFINITE = -5,    /* the integrand returned NaN/Inf (counted; those samples weigh 0),
                                 or an iteration's estimate or variance is not finite */
    VEGAS_EUNSUPPORTED = -6   /* valid request this build does not implement */
} vegas_status;

/* Arithmetic of the per-sample path (map, Jacobian, integrand, weight). */
enum { VEGAS_PREC_FP64 = 0, VEGAS_PREC_FP32 = 1 };

/* Accumulation of per-cube sums and iteration totals.
 *  FP64    : shifted FP64 sums per cube, FP64 totals (default).
 *  KAHAN   : FP32 sample path with per-cube sums and totals in compensated
 *            FP32 (Kahan) form.  Squares of weights must fit FP32 (|w| below
 *            about 1e19); past that an iteration's variance overflows and
 *            vegas_result reports VEGAS_ENONFINITE.
 *  ORDERED : every sum taken in increasing sample order, as a sequential
 *            program would; bit-reproducible, for small problems only
 *            (n_eval * n_intervals <= 2^26). */
enum { VEGAS_ACC_FP64 = 0, VEGAS_ACC_KAHAN = 1, VEGAS_ACC_ORDERED = 2 };

/* Built-in integrand families (params layout in vegas_integrand). */
enum {
    VEGAS_GAUSS_DIAG = 1,   /* A sum_j exp(-sum_d (x_d-c_j)^2/(2 s^2)) : [A, s, M, c_0..c_{M-1}] */
    VEGAS_GENZ_PPEAK = 2,   /* A prod_d 1/(a_d^-2 + (x_d-u_d)^2)        : [A, a_0..a_{D-1}, u_0..u_{D-1}] */
    VEGAS_GENZ_GAUSS = 3,   /* A exp(-sum_d a_d^2 (x_d-u_d)^2)           : [A, a_0..a_{D-1}, u_0..u_{D-1}] */
    VEGAS_GAUSS_CORR = 4,   /* N(x; mu 1, s^2((1-rho)I + rho 1 1^T))      : [mu, s, rho] */
    VEGAS_LINEAR = 5,       /* A sum_d x_d                               : [A]  (Tab. 3 #2) */
    VEGAS_ROOS = 6,         /* A prod_d |4 x_d - 2|                      : [A]  (Tab. 3 #5) */
    VEGAS_CONST = 7,        /* A                                         : [A] */
    VEGAS_COSINE = 8,       /* A prod_d cos x_d                          : [A]  (Tab. 3 #3) */
    VEGAS_SIN_EXP = 9,      /* A (sin x_0 + exp x_1), dim >= 2           : [A]  (Tab. 3 #1) */
    VEGAS_EXP_SQ = 10,      /* A exp(sum_d x_d^2)                        : [A]  (Tab. 3 #4) */
    VEGAS_MOROKOFF = 11,    /* A (1 + 1/D)^D prod_d x_d^(1/D), box x >= 0: [A]  (Tab. 3 #6) */
    VEGAS_USER = 12         /* compiled at run time (vegas_user_compile): any params, 0..4096 */
};

/* Problem parameters (Tab. 2: n_intervals, alpha, beta).  Copied at create. */
typedef struct {
    int32_t  dim;            /* D, 1..16 */
    int32_t  n_intervals;    /* N_g >= 1 intervals per axis (paper default 1024) */
    int64_t  n_eval;         /* N_ev evaluations per iteration, < 2^32 */
    int32_t  n_strat;        /* strata per axis; 0 = largest m with 4 m^D <= N_ev */
    int32_t  n_min;          /* samples reserved per hypercube, >= 2 */
    double   alpha;          /* map damping >= 0 (0 freezes the map) */
    double   beta;           /* allocation damping >= 0 (0 = uniform) */
    uint64_t seed;           /* Philox key */
    uint32_t instance;       /* Philox counter word 3 high bits (< 2^24) */
    int32_t  precision;      /* VEGAS_PREC_* */
    int32_t  accum;          /* VEGAS_ACC_* */
    int32_t  adapt_map;      /* 1: refine the map after each iteration */
    int32_t  adapt_strat;    /* 1: reallocate samples after each iteration */
    int32_t  max_iter;       /* capacity of the per-iteration result log; 0 = 4096 */
} vegas_config;

/* Integrand: family id, parameters and the box [lo_d, hi_d].  Host
 * pointers, copied at create.  lo/hi may be NULL (unit box). */
typedef struct {
    int32_t       family;
    int32_t       n_params;
    const double* params;
    const double* lo;
    const double* hi;
} vegas_integrand;

/* Combined estimate (Eq. 8-9) over the iterations run by vegas_integrate. */
typedef struct {
    double  integral;
    double  sigma2;
    double  chi2_dof;         /* sum (I_t - I)^2/sigma_t^2 / (n-1); 0 when n < 2 */
    int32_t n_iter_combined;
    int32_t n_iter_total;     /* adapt + integrate iterations run so far */
    int64_t n_eval_total;
    int64_t n_nonfinite;      /* samples whose weight was NaN/Inf (counted as 0) */
} vegas_estimate;

/* Derived sizes of a context (for tests and tools). */
typedef struct {
    int64_t n_strat;          /* N_st per axis */
    int64_t n_cubes;          /* N_c = N_st^D */
    int64_t n_rest;           /* R = N_ev - n_min N_c, split by sigma^beta */
    int32_t tile;             /* samples per fill tile */
    int32_t n_tiles;
    int32_t n_workgroups;     /* persistent fill workgroups */
    int32_t lds_hist;         /* 1: histograms privatised in LDS */
    size_t  workspace_bytes;
} vegas_info;

typedef struct vegas_ctx vegas_ctx;

/* Bytes of device workspace a context needs.  Host pointers; no HIP call. */
vegas_status vegas_workspace_size(const vegas_config* cfg, const vegas_integrand* f,
                                  size_t* bytes);

/* Validate, carve the caller's device workspace (d_workspace, >= bytes,
 * 256-byte aligned) and initialise the uniform map and uniform allocation
 * (asynchronous, on hip_stream; NULL = the null stream).  *out receives a
 * host-owned handle released by vegas_destroy. */
vegas_status vegas_create(const vegas_config* cfg, const vegas_integrand* f,
                          void* d_workspace, size_t bytes, void* hip_stream,
                          vegas_ctx** out);

/* Run n_iter iterations whose estimates are discarded (the paper's `skip`,
 * Alg. 1); map and allocation still adapt.  Asynchronous. */
vegas_status vegas_adapt(vegas_ctx* ctx, int32_t n_iter);

/* Run n_iter iterations whose estimates enter the Eq. 8-9 combination.
 * Asynchronous. */
vegas_status vegas_integrate(vegas_ctx* ctx, int32_t n_iter);

/* Synchronous: wait for the stream, combine the integrate iterations by
 * Eq. 8-9 (host FP64) and fill *out (host pointer).  Returns
 * VEGAS_ENONFINITE (after filling *out) if any sample weight was NaN/Inf. */
vegas_status vegas_result(vegas_ctx* ctx, vegas_estimate* out);

/* Synchronous: release the handle (the workspace stays the caller's). */
void vegas_destroy(vegas_ctx* ctx);

/* ---- integrands compiled at run time (hipRTC) -------------------------
 * The counterpart of the paper's user-supplied integrand compiled for the
 * GPU at run time (Sec. 3.6).  source (host string) defines the device
 * function vegas_user_f, taking (const vegas_real* x, int dim,
 * const double* params) and returning vegas_real,
 * where vegas_real is double for precision VEGAS_PREC_FP64 and float for
 * VEGAS_PREC_FP32, x holds the point in the box (dim values) and params the
 * context's n_params parameters (device memory, FP64).  It may define other
 * device functions and constants, and use the HIP device math functions.
 * The fill kernel (the built-ins' tile body, specialised to dim) is compiled
 * for the current device with hipRTC, with the library's own flags.
 * Errors: VEGAS_EINVAL for bad arguments or source that does not compile
 * (the compiler's log is in vegas_last_error()); VEGAS_EDEVICE when loading
 * fails.  *out is a host handle, valid on that device, released by
 * vegas_user_destroy (after every context that uses it). */
typedef struct vegas_user_fn vegas_user_fn;
vegas_status vegas_user_compile(const char* source, int32_t dim, int32_t precision,
                                vegas_user_fn** out);
/* Compile only, for gfx950, and discard the code: checks a source without a
 * device (no HIP call).  Errors as vegas_user_compile. */
vegas_status vegas_user_check(const char* source, int32_t dim, int32_t precision);
void vegas_user_destroy(vegas_user_fn* fn);
/* As vegas_create, for f->family == VEGAS_USER (0..4096 parameters; params
 * may be NULL when there are none): the fill runs fn, whose dim and
 * precision must equal cfg's.  Accumulation FP64 or KAHAN (not ORDERED);
 * the sample probe and the learned warp do not take user integrands
 * (VEGAS_EUNSUPPORTED).  fn must outlive the context. */
vegas_status vegas_create_user(const vegas_config* cfg, const vegas_integrand* f, const vegas_user_fn* fn,
                               void* d_workspace, size_t bytes, void* hip_stream, vegas_ctx** out);

/* ---- for callers that cannot allocate device memory ---------------------
 * Code under HIP graph capture, tight serving loops, or harnesses that
 * forbid hipMalloc: the same context as vegas_create, but its workspace is a
 * device array the library holds (VEGAS_STATIC_SCRATCH_BYTES, 256-byte
 * aligned), one per device, kept until the process ends.  Allocates no
 * device memory (no hipMalloc/hipFree, no allocating library routine); the
 * handle itself is host memory, released by vegas_destroy.
 *  - The problem's workspace (vegas_workspace_size) must fit the array,
 *    else VEGAS_ENOMEM and no context.
 *  - Every context made by this call on one device uses the same array:
 *    creating one overwrites the state of any earlier one on that device,
 *    whose handle may then only be destroyed.  Calls on such contexts that
 *    overlap (any thread, any stream) race.
 *  - The array keeps the last context's contents; create writes everything
 *    an iteration reads before writing it, so no clearing is needed.
 *  - Set-up as vegas_create (asynchronous on hip_stream, NULL = null
 *    stream); errors as vegas_create, plus VEGAS_EDEVICE when the array's
 *    device address cannot be obtained. */
#define VEGAS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
vegas_status vegas_create_static(const vegas_config* cfg, const vegas_integrand* f,
                                 void* hip_stream, vegas_ctx** out);

/* Host pointer out. */
vegas_status vegas_get_info(const vegas_ctx* ctx, vegas_info* out);

/* ---- inspection / injection hooks (all synchronous, host pointers) ----- */
/* Switch the map refinement and the sample reallocation on or off (1 / 0)
 * for the iterations that follow, as cfg.adapt_map and cfg.adapt_strat do
 * at create (the usual last phase of a VEGAS run keeps the grid fixed).
 * No HIP call. */
vegas_status vegas_set_adapt(vegas_ctx* ctx, int32_t adapt_map, int32_t adapt_strat);

/* Map grid, FP64, layout [D][N_g+1] row-major. */
vegas_status vegas_get_map(vegas_ctx* ctx, double* grid);
vegas_status vegas_set_map(vegas_ctx* ctx, const double* grid);
/* Replace the integrand's parameters (same family and count, validated as
 * at create) for the iterations that follow; map, allocation and iteration
 * log stay.  Meant for continuation: adapting first on a wider version of a
 * sharply peaked integrand whose values would otherwise underflow
 * everywhere the uniform start samples.  Estimates of iterations run under
 * other parameters belong to that other integrand (run them as adapt). */
vegas_status vegas_set_params(vegas_ctx* ctx, const double* params);
/* Samples per hypercube n_h of the next iteration, uint32 [N_c]
 * (set: must sum to N_ev with every n_h >= n_min). */
vegas_status vegas_get_nh(vegas_ctx* ctx, uint32_t* nh);
vegas_status vegas_set_nh(vegas_ctx* ctx, const uint32_t* nh);
/* Accumulators of the last iteration: per-axis histograms H = sum w^2 and
 * counts C, FP64 [D][N_g] each; per-cube unbiased variance v_h FP64 [N_c].
 * Any pointer may be NULL. */
vegas_status vegas_get_accumulators(vegas_ctx* ctx, double* H, double* C, double* v);
/* Replace the accumulators (same layouts) so that vegas_update refines the
 * map and the allocation from injected values. */
vegas_status vegas_set_accumulators(vegas_ctx* ctx, const double* H, const double* C,
                                    const double* v);
/* Run only the update half of an iteration (allocation, then map) from the
 * current accumulators.  Asynchronous. */
vegas_status vegas_update(vegas_ctx* ctx);
/* Per-iteration (I_t, sigma_t^2) of every iteration run so far, host
 * arrays of capacity cap; *n receives the count. */
vegas_status vegas_get_iterations(vegas_ctx* ctx, double* I, double* sigma2, int32_t cap,
                                  int32_t* n);

/* Checkpoint: opaque byte image of the adaptive state (map, allocation,
 * iteration log, counters).  Call with buf = NULL to query *bytes. */
vegas_status vegas_get_state(vegas_ctx* ctx, void* buf, size_t* bytes);
vegas_status vegas_set_state(vegas_ctx* ctx, const void* buf, size_t bytes);

/* Test hook: the per-sample path of Alg. 2 (getCube, getPoint, getJac,
 * integrand) for samples k0 .. k0+n-1 of iteration t under the current map
 * and allocation, written to DEVICE arrays (any may be NULL):
 * cube uint32 [n], bins uint32 [n][D], delta / x FP64 [n][D], jac / f FP64
 * [n].  delta, x, jac, f are computed in the context's precision and
 * widened.  Asynchronous. */
vegas_status vegas_sample_probe(vegas_ctx* ctx, uint32_t t, uint64_t k0, int64_t n,
                                uint32_t* d_cube, uint32_t* d_bins, double* d_delta,
                                double* d_x, double* d_jac, double* d_f);

/* Phase timing with HIP events on the context's stream.  on = 1 starts
 * (and clears) the record; vegas_get_timing synchronises and returns the
 * summed milliseconds of each phase over the recorded iterations:
 * ms[0] fill (Alg. 2), ms[1] cube fix-up + iteration estimate,
 * ms[2] allocation update, ms[3] map refinement; *n_iter the count.
 * ms is a host array of 4 doubles. */
vegas_status vegas_set_timing(vegas_ctx* ctx, int32_t on);
vegas_status vegas_get_timing(vegas_ctx* ctx, double* ms, int32_t* n_iter);

/* ---- learned warp: a coupling flow stacked on the VEGAS map ------------- */
/* Not in the paper; an extension of the method.  With the warp enabled,
 * every iteration draws the stratified points y as before, maps them by a
 * normalising flow F to w = F(y), and w goes through the VEGAS map to x.
 * A sample weighs f(x) J_map(w) J_F(y).  J_F is the exact Jacobian
 * determinant, so every estimate stays unbiased.  The map and allocation
 * adapt to the warped samples exactly as before.
 * F: four affine coupling layers in Gaussian coordinates.  z_0 = Phi^-1(y)
 *   (Phi the standard normal distribution function), z_4 after the layers,
 *   w = Phi(z_4).  Layer l keeps the axes A_l ({0..7}, {8..15}, the even
 *   axes, the odd axes) and moves the other 8: z_B -> z_B e^s + t with
 *   s = 3 tanh(a/3).  (a, t) come from an MLP of x = z_A / 2:
 *   8 -> 64 -> 64 -> 16 with ReLU (outputs a_0..a_7, t_0..t_7).  The matrix
 *   products run on BF16 MFMA with FP32 accumulation.
 *   log J_F(y) = sum s + sum_d (z_0d^2 - z_4d^2)/2, exact.
 * Parameters: vegas_flow_n_params() floats, layer by layer
 *   W1[64][8], b1[64], W2[64][64], b2[64], W3[16][64], b3[16] (row-major
 *   [out][in]).  A zero W3 and b3 make F the identity.
 * Restrictions: dim 16, FP32 precision, accum FP64 or KAHAN, families
 *   GAUSS_DIAG, GENZ_PPEAK, GENZ_GAUSS, GAUSS_CORR. */
typedef struct {
    float    lr;              /* Adam step of the warp's training */
    int32_t  train;           /* 1: train after every kept warped iteration */
    int32_t  loss;            /* 0: variance, c_k ~ omega_k^2; 1: KL, c_k ~ |omega_k| */
    int32_t  judge;           /* 0: none; 1: guard; 2: guard and cost (see vegas_flow_enable) */
    int32_t  steps_per_iter;  /* Adam steps after each kept warped iteration, 0..64 (0 = 1) */
    int32_t  control_period;  /* judge > 0: every control_period-th iteration of the warp's
                                 phase samples plain VEGAS+; 0 (= 16) or 2..32 */
    int32_t  train_stride;    /* a training step uses every train_stride-th sample of the
                                 iteration (offset turning with the steps); 0 (= 1) .. 1024 */
    uint64_t init_seed;       /* seed of the library's starting weights (params NULL at attach) */
} vegas_flow_config;

int32_t vegas_flow_n_params(void);
/* Bytes of the warp's own device workspace for this context. */
vegas_status vegas_flow_workspace_size(const vegas_ctx* ctx, size_t* bytes);
/* Attach a warp.  params: host pointer to n_params floats, or NULL for the
 * library's own starting weights: W1 and W2 uniform in +-1/sqrt(fan_in)
 * (fan_in 8 and 64) from Philox4x32-10 keyed by cfg->init_seed, every other
 * parameter 0, so that F starts as the identity (s = t = 0,
 * log J_F = 0).  d_workspace: device memory of at least the size
 * above, 256-byte aligned; it must outlive the context.  Synchronous.  The
 * warp starts disabled. */
vegas_status vegas_flow_attach(vegas_ctx* ctx, const vegas_flow_config* cfg, const float* params,
                               void* d_workspace, size_t bytes);
/* Replace the warp's configuration (lr, training, loss, judge, steps,
 * control period) for the iterations that follow; parameters and Adam
 * state stay.  A new judge mode starts its cost records afresh.  Host
 * pointer; no HIP call. */
vegas_status vegas_flow_set_config(vegas_ctx* ctx, const vegas_flow_config* cfg);
/* on = 1: the following iterations sample through the warp; the parameters
 * in place become the kept ones.
 * The judge (cfg.judge > 0):
 *  - control: every control_period-th iteration of the warp's phase samples
 *    plain VEGAS+ (the same map and allocation, no warp), so 1/period of
 *    the evaluations measure plain VEGAS+.  Control iterations are not
 *    combined by Eq. 8-9: a separable importance density can miss most of a
 *    correlated integrand's mass, and its variance estimate is then far
 *    too small to be weighted by.
 *  - guard, every warped iteration: rejected when its estimate or variance
 *    is not finite or its relative variance sigma_t^2/I_t^2 exceeds 10x the
 *    median of the last (up to) 4 kept warped iterations (of the last plain
 *    iterations before any was kept).  A rejected iteration restores the
 *    last kept parameters and restarts Adam; three rejections in a row
 *    switch the warp off.
 *  - cost (judge = 2), after each control iteration: the warp's efficiency,
 *    the median of sigma_t^2/I_t^2 x GPU time over its last (up to) 8
 *    warped iterations (training included), against the same over the last
 *    (up to) 3 controls; a control whose estimate lies more than 5 sigma
 *    from the kept warped iterations' combined estimate has missed the
 *    integrand and counts as infinitely costly.  The warp losing two
 *    checks in a row switches it off; plain VEGAS+ continues.
 * Warped iterations combine by Eq. 8-9 with the plain ones run outside the
 * warp's phase.  The judge reads each warped iteration's estimate, so it
 * synchronises the stream once per warped iteration. */
vegas_status vegas_flow_enable(vegas_ctx* ctx, int32_t on);
/* Timing of the warp with HIP events on the context's stream: on = 1
 * starts (and clears) the record; vegas_flow_get_timing synchronises and
 * returns, summed over the recorded warped iterations, ms[0] the sampling
 * pass (y -> w = F(y)) and ms[1] the training (gradient passes, Adam,
 * repack), and *n_iter their count.  ms: host array of 2 doubles. */
vegas_status vegas_flow_set_timing(vegas_ctx* ctx, int32_t on);
vegas_status vegas_flow_get_timing(vegas_ctx* ctx, double* ms, int32_t* n_iter);
/* With the same timing on: the gradient kernel alone (the training's
 * dominant kernel: inverse pass and every layer's backward pass), events
 * just before and after each of its launches.  Synchronises; *ms receives
 * the summed duration in ms and *n_launch the launch count.  ms: host
 * pointer to one double. */
vegas_status vegas_flow_get_grad_timing(vegas_ctx* ctx, double* ms, int32_t* n_launch);
/* Kind of every iteration run so far: 0 plain, 1 through the warp, 2 plain
 * control of the judge.  kinds: host array of capacity cap; *n receives
 * the iteration count.  No HIP call. */
vegas_status vegas_flow_get_kinds(vegas_ctx* ctx, int32_t* kinds, int32_t cap, int32_t* n);
/* The warp's state: enabled now, warped iterations kept and rejected by the
 * judge (host pointers, any may be NULL). */
vegas_status vegas_flow_status(const vegas_ctx* ctx, int32_t* on, int32_t* accepted, int32_t* rejected);
/* Synchronous copies of the FP32 parameters (host pointers). */
vegas_status vegas_flow_get_params(vegas_ctx* ctx, float* params);
vegas_status vegas_flow_set_params(vegas_ctx* ctx, const float* params);
/* Test hook, synchronous.  The last warped iteration's samples: w [N][16],
 * log J_F [N], weight omega [N] and the final Gaussian coordinates z_4
 * [N][16] (FP32, host pointers; any may be NULL). */
vegas_status vegas_flow_get_samples(vegas_ctx* ctx, float* w, float* lj, float* omega, float* z);
/* Test hook, synchronous.  Gradient of the warp's training loss on the last
 * warped iteration's samples (no parameter update), host pointer
 * grad[n_params].  Loss: sum_k c_k log J_F(F^-1(w_k)) with c_k as set by
 * vegas_flow_config.loss, normalised to sum 1.  With the variance loss its
 * gradient is a positive multiple of the gradient of the estimator's
 * variance. */
vegas_status vegas_flow_grad(vegas_ctx* ctx, float* grad);
/* Test hook, synchronous.  One Adam step of the warp's training (the step
 * counter advances) on a given gradient instead of the computed one: host
 * pointer grad[n_params], all finite.  Adam: beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected, step cfg.lr, in FP32. */
vegas_status vegas_flow_adam_step(vegas_ctx* ctx, const float* grad);
/* Test hook, synchronous, on the current device.  One BF16 matrix product
 * D = A B.  Device pointers: A [32][16], B [16][32], D [32][32], all FP32
 * row-major.  A and B are rounded to BF16 first.  It checks the lane layout
 * the warp's kernels assume. */
vegas_status vegas_mfma_probe(const float* d_A, const float* d_B, float* d_D);

/* ---- batches: many independent problems advanced together ------------- */
/* A batch holds n problems, each with its own configuration (dimension,
 * intervals, budget, alpha, beta, seed, instance) and integrand, advanced
 * one iteration at a time together.  Every problem computes exactly what a
 * single context with the same config computes (Alg. 1-2, Eq. 5-9).
 * Two launch schedules:
 *  - VEGAS_BATCH_STREAMS: each problem runs the single-problem kernels in a
 *    context of its own; the problems are spread over a few streams of the
 *    library (longest first onto the least loaded stream), which start after
 *    the caller's stream and which the caller's stream waits for at the end
 *    of every iteration.  The stream count (1, 2, 4 or 8) comes from the
 *    autotuner, which times the fill of every problem under each count.
 *    Results do not depend on the stream count.
 *  - VEGAS_BATCH_PERSISTENT: one persistent fill launch whose workgroups pop
 *    work items (runs of consecutive sample tiles of one problem) from a
 *    queue ordered longest first, then one launch per update phase for all
 *    problems.  Switched off: its first device run ended in a memory fault
 *    whose cause is not yet found, so vegas_batch_create returns
 *    VEGAS_EUNSUPPORTED for it (vegas_batch_workspace_size still sizes it).
 * Restrictions: families GENZ_PPEAK, GENZ_GAUSS and GAUSS_DIAG; dim <= 12;
 * every config has the same precision and accumulation, FP64 or KAHAN (or
 * ORDERED under the streams schedule, which then follows the single
 * contexts bit for bit); n in 1..2^20.  The iteration log holds
 * max(max_iter) iterations (256 if every max_iter is 0).  With FP64 or
 * KAHAN accumulation the histogram bins are LDS atomic sums whose last bits
 * follow the order of the adds, as in a single context. */
typedef struct vegas_batch vegas_batch;

typedef enum { VEGAS_BATCH_STREAMS = 0, VEGAS_BATCH_PERSISTENT = 1 } vegas_batch_schedule;

typedef struct {
    int32_t n;                /* problems */
    int32_t per_lane;         /* persistent layout: samples per lane (0 for streams) */
    int64_t item_samples;     /* persistent layout: target samples per work item (0 for streams) */
    int64_t n_items;          /* persistent: work items per fill; streams: n */
    int64_t n_tiles;          /* sample tiles of all problems */
    int32_t n_workgroups;     /* persistent fill workgroups; streams: sum over problems */
    int32_t tuned;            /* 0 default, 1 timed at create, 2 read from the cache */
    double  tune_ms;          /* fill time of the chosen schedule when tuned */
    size_t  lds_bytes;        /* largest LDS of a fill launch */
    size_t  workspace_bytes;  /* bytes of the workspace in use */
    int64_t n_eval_total;     /* sum of n_eval over the problems (one iteration) */
    int64_t n_cubes_total;
    int32_t schedule;         /* vegas_batch_schedule */
    int32_t n_streams;        /* streams schedule: streams in use */
} vegas_batch_info;

/* Bytes of device workspace for n problems (cfgs[n], fs[n], host arrays)
 * under a schedule (for the persistent one: enough for every layout the
 * autotuner may pick).  No HIP call. */
vegas_status vegas_batch_workspace_size(int32_t n, const vegas_config* cfgs,
                                        const vegas_integrand* fs, int32_t schedule, size_t* bytes);

/* Validate and set up n problems in the caller's workspace (device,
 * 256-byte aligned, >= the size above for the same schedule) after the work
 * already queued on hip_stream.  tune_cache: path of a text file of tuned
 * schedules, or NULL for the default (4 streams; the first persistent
 * layout).  When the file has no entry for this batch shape on this device,
 * the fill is timed over the candidates, the fastest is used, and a line is
 * appended to the file (a file that cannot be written is ignored).
 * Synchronous.  *out is released by vegas_batch_destroy. */
vegas_status vegas_batch_create(int32_t n, const vegas_config* cfgs, const vegas_integrand* fs,
                                void* d_workspace, size_t bytes, void* hip_stream, int32_t schedule,
                                const char* tune_cache, vegas_batch** out);
/* Synchronous: release the handle (and the streams the batch made). */
void vegas_batch_destroy(vegas_batch* b);
/* Persistent schedule: choose one of the candidate layouts by hand
 * (per_lane 8/4/2 with item_samples 2^16, 2^18 or 2^20, as listed by the
 * tuner); only before the first iteration.  Synchronous; VEGAS_EINVAL for
 * other values, VEGAS_EUNSUPPORTED under the streams schedule. */
vegas_status vegas_batch_set_layout(vegas_batch* b, int32_t per_lane, int64_t item_samples);
/* Streams schedule: choose the stream count (1..8) by hand; only before the
 * first iteration.  Synchronous; VEGAS_EUNSUPPORTED under the persistent
 * schedule. */
vegas_status vegas_batch_set_streams(vegas_batch* b, int32_t n_streams);
/* Iterations for every problem: discarded (adapt) or combined by Eq. 8-9
 * (integrate).  Asynchronous with respect to the host; ordered on the
 * caller's stream. */
vegas_status vegas_batch_adapt(vegas_batch* b, int32_t n_iter);
vegas_status vegas_batch_integrate(vegas_batch* b, int32_t n_iter);
/* Synchronous: out[n] (host) receives each problem's combined estimate.
 * VEGAS_ENONFINITE (after filling out) if any weight was NaN/Inf. */
vegas_status vegas_batch_results(vegas_batch* b, vegas_estimate* out);
/* Synchronous inspection of problem i (host pointers): its per-iteration
 * estimates, its map [D][N_g+1] and its next allocation n_h [N_c]. */
vegas_status vegas_batch_get_iterations(vegas_batch* b, int32_t i, double* I, double* sigma2,
                                        int32_t cap, int32_t* n);
vegas_status vegas_batch_get_map(vegas_batch* b, int32_t i, double* grid);
vegas_status vegas_batch_get_nh(vegas_batch* b, int32_t i, uint32_t* nh);
vegas_status vegas_batch_get_info(const vegas_batch* b, vegas_batch_info* out);
/* Timing of the iterations that follow.  Persistent schedule: per phase,
 * summed over all problems (ms[0] fill, ms[1] fix-up + estimates, ms[2]
 * allocation, ms[3] map refinement).  Streams schedule: ms[0] is the whole
 * iteration of all problems on the caller's stream, ms[1..3] are 0. */
vegas_status vegas_batch_set_timing(vegas_batch* b, int32_t on);
vegas_status vegas_batch_get_timing(vegas_batch* b, double* ms, int32_t* n_iter);

const char* vegas_status_string(vegas_status s);
const char* vegas_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VEGAS_MI355X_H */
