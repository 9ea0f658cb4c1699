// Host helpers shared by the single-problem and the batched C ABI:
// error reporting, configuration validation into a problem geometry, and
// the Eq. 8-9 combination of iteration estimates.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/vegas.h"

namespace vgh {

// record a thread-local message and return s
vegas_status fail(vegas_status s, const char* fmt, ...);

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return vgh::fail(VEGAS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kMaxNg = 4096;

// Problem geometry derived from a validated config (no HIP call).
struct Geometry {
    int D, ng, n_min, family, n_params;
    uint32_t n_eval;
    uint32_t nst;
    uint32_t n_cubes;
    uint64_t R;
    uint32_t magic;
    int shift;
    int per_lane, tile, n_tiles;
    int lds_hist_ok;
    int n_aux;
};

// validate (cfg, f) and derive the strata, cube count, magic divisor and
// the single-problem tile layout
vegas_status geometry(const vegas_config* c, const vegas_integrand* f, Geometry* g);

// Eq. 8-9: inverse-variance weighted mean, its variance and chi^2/dof of the
// iteration estimates (iterations with sigma^2 = 0 are exact and decide)
void combine(const std::vector<double>& I, const std::vector<double>& s2, double* Ib, double* s2b, double* chi);

// Hooks for the batch driver, which runs one single-problem context per
// problem: move a context to another stream (between iterations only), and
// enqueue the fill of the next iteration alone, leaving the iteration count,
// the allocation and the map as they are (its accumulators are overwritten
// by the iteration itself; used to time launch schedules).
void ctx_set_stream(vegas_ctx* c, hipStream_t s);
vegas_status ctx_fill_pass(vegas_ctx* c);

// integrands compiled at run time (rtc.hip)
int user_fn_dim(const vegas_user_fn* fn);
int user_fn_precision(const vegas_user_fn* fn);

}  // namespace vgh

namespace vg {
struct FillArgs;
}

namespace vgh {
hipError_t launch_user_fill(const vegas_user_fn* fn, const vg::FillArgs& a, int n_wg, size_t lds, hipStream_t st);

}  // namespace vgh
