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
    VEGAS_ENONFINITE = -5,    /* the integrand returned NaN/Inf (counted; those samples weigh 0) */
    VEGAS_EUNSUPPORTED = -6   /* valid request this build does not implement */
} vegas_status;

/* Arithmetic of the per-sample path (map, Jacobian, integrand, weight). */
enum { VEGAS_PREC_FP64 = 0, VEGAS_PREC_FP32 = 1 };

/* Accumulation of per-cube sums and iteration totals.
 *  FP64    : shifted FP64 sums per cube, FP64 totals (default).
 *  KAHAN   : FP32 sample path with per-cube sums and totals in compensated
 *            FP32 (Kahan) form.
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
    VEGAS_COSINE = 8        /* A prod_d cos x_d                          : [A]  (Tab. 3 #3) */
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

/* Host pointer out. */
vegas_status vegas_get_info(const vegas_ctx* ctx, vegas_info* out);

/* ---- inspection / injection hooks (all synchronous, host pointers) ----- */
/* Map grid, FP64, layout [D][N_g+1] row-major. */
vegas_status vegas_get_map(vegas_ctx* ctx, double* grid);
vegas_status vegas_set_map(vegas_ctx* ctx, const double* grid);
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

const char* vegas_status_string(vegas_status s);
const char* vegas_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VEGAS_MI355X_H */
