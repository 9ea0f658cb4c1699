// VegasFill (Alg. 2) for gfx950: the data-parallel half of one VEGAS+
// iteration.
//
// Layout of the work.  Samples k = 0 .. N_ev-1 of an iteration are ordered by
// hypercube: cube h owns the contiguous range [start_h, start_{h+1}) (its
// n_h samples, Sec. 2.1.2).  The fill is a persistent kernel, one 1024-lane
// workgroup per CU, that walks tiles of `tile` consecutive samples; lane l of
// a tile owns `per_lane` consecutive samples.  Every sample costs the same
// whatever the allocation (the balance requirement of Sec. 3.1), and a lane
// meets the cubes of its range in order, so most cubes are summed inside one
// lane with no atomics.
//
// Per sample (Alg. 2): its cube (getCube) from the tile's cube starts in
// LDS; its stratum digits; Philox4x32-10 words keyed by (k, t, instance);
// the fixed-point point and bin index (getPoint, Eq. 3); x and the Jacobian
// J = prod N_g dx from the map held in LDS (getJac, Eq. 2-4); f(x); w = J f.
// Then w^2 and a count go to the per-axis histograms (privatised in LDS,
// written once per workgroup) and w to the running shifted sums of its cube.
//
// Per cube (Eq. 5-6): runs of a cube that cross lanes merge with Chan's
// pairwise formula in a segmented scan over wavefront shuffles, with one
// carry per wave through LDS; runs that cross tiles go to a side record and
// a fix-up kernel merges them in tile order.  Each finished cube yields its
// mean m_h and unbiased variance v_h; the iteration estimate is
// I = sum m_h / N_c and sigma^2 = sum v_h / (N_c^2 n_h), reduced in a fixed
// order so that a run is reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "layout.hpp"
#include "launch.hpp"
#include "sample.hpp"
#include "fill_dev.hpp"

namespace vg {

template <typename R, int FAM, int MAXD, bool KAHAN, bool EXACT>
__global__ __launch_bounds__(kFillThreads) void k_fill(FillArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    fill_body<R, FAM, MAXD, KAHAN, EXACT>(a, smem);
}

// ---------------------------------------------------------------------------
// cubes that cross tiles: merge their runs in tile order
// ---------------------------------------------------------------------------
__global__ void k_fixup(FixupArgs a)
{
    // one maximum per wavefront: the lanes' atomics on one address would
    // queue one behind another
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long vb = j < a.n_tiles ? fixup_chain_v(a.side, a.n_tiles, j, a.v_out, a.fix_part + 2 * j) : 0ull;
    wave_atomic_max(vb, a.vmax);
}

// ---------------------------------------------------------------------------
// iteration estimate: fixed-order sum of workgroup and fix-up partials
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_final(FinalArgs a)
{
    __shared__ double rI[1024], rV[1024];
    final_reduce(a, rI, rV);
}

// ---------------------------------------------------------------------------
// probe: the per-sample path for a range of samples, outputs widened to FP64
// ---------------------------------------------------------------------------
template <typename R, int FAM, int MAXD>
__global__ void k_probe(ProbeArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t k = (uint32_t)(a.k0 + (uint64_t)i);
    // cube of k: largest h with start[h] <= k
    uint32_t lo = 0, hi = a.sc.n_cubes;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.start[mid] <= k) lo = mid; else hi = mid;
    }
    const R* aux = std::is_same<R, double>::value ? reinterpret_cast<const R*>(a.sc.aux_d)
                                                  : reinterpret_cast<const R*>(a.sc.aux_f);
    SamplePath<R, FAM, MAXD> sp(a.sc, aux);
    uint32_t s[MAXD], bins[MAXD];
    R delta[MAXD], x[MAXD], J, f;
    sp.digits(lo, s);
    sp.template eval<true>(k, a.t, s, reinterpret_cast<const R*>(a.grid), bins, delta, x, J, f);
    const int D = a.sc.D;
    if (a.cube) a.cube[i] = lo;
#pragma unroll
    for (int d = 0; d < MAXD; ++d) {
        if (d < D) {
            if (a.bins) a.bins[i * D + d] = bins[d];
            if (a.delta) a.delta[i * D + d] = (double)delta[d];
            if (a.x) a.x[i * D + d] = (double)x[d];
        }
    }
    if (a.jac) a.jac[i] = (double)J;
    if (a.f) a.f[i] = (double)f;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
// the kernel for dimension bound MAXD; its guard-free form when D == MAXD
template <typename R, int FAM, int MAXD, bool KAHAN>
static void launch_fill_d(const FillArgs& a, int n_wg, size_t lds, hipStream_t st)
{
    if (a.sc.D == MAXD) {
        hipFuncSetAttribute((const void*)k_fill<R, FAM, MAXD, KAHAN, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_fill<R, FAM, MAXD, KAHAN, true>), dim3(n_wg), dim3(kFillThreads), lds, st, a);
    } else {
        hipFuncSetAttribute((const void*)k_fill<R, FAM, MAXD, KAHAN, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_fill<R, FAM, MAXD, KAHAN, false>), dim3(n_wg), dim3(kFillThreads), lds, st, a);
    }
}

template <typename R, int FAM, bool KAHAN>
static hipError_t launch_fill_k(const FillArgs& a, int n_wg, size_t lds, hipStream_t st)
{
    const int D = a.sc.D;
    if (D <= 4) launch_fill_d<R, FAM, 4, KAHAN>(a, n_wg, lds, st);
    else if (D <= 8) launch_fill_d<R, FAM, 8, KAHAN>(a, n_wg, lds, st);
    else if (D <= 12) launch_fill_d<R, FAM, 12, KAHAN>(a, n_wg, lds, st);
    else launch_fill_d<R, FAM, 16, KAHAN>(a, n_wg, lds, st);
    return hipGetLastError();
}

template <typename R, int FAM>
static hipError_t launch_fill_fam(const FillArgs& a, int n_wg, size_t lds, hipStream_t st)
{
    // compensated FP32 accumulators only exist for the FP32 sample path
    if constexpr (std::is_same<R, float>::value) {
        if (a.accum == 1) return launch_fill_k<R, FAM, true>(a, n_wg, lds, st);
    }
    return launch_fill_k<R, FAM, false>(a, n_wg, lds, st);
}

template <typename R, int FAM>
static hipError_t launch_probe_fam(const ProbeArgs& a, hipStream_t st)
{
    const int D = a.sc.D;
    const int bs = 256;
    const unsigned nb = (unsigned)((a.n + bs - 1) / bs);
    if (D <= 4) hipLaunchKernelGGL((k_probe<R, FAM, 4>), dim3(nb), dim3(bs), 0, st, a);
    else if (D <= 8) hipLaunchKernelGGL((k_probe<R, FAM, 8>), dim3(nb), dim3(bs), 0, st, a);
    else if (D <= 12) hipLaunchKernelGGL((k_probe<R, FAM, 12>), dim3(nb), dim3(bs), 0, st, a);
    else hipLaunchKernelGGL((k_probe<R, FAM, 16>), dim3(nb), dim3(bs), 0, st, a);
    return hipGetLastError();
}

#define VG_FAMILY_SWITCH(R, CALL, ...)                                          \
    switch (fam) {                                                             \
    case F_GAUSS_DIAG: return CALL<R, F_GAUSS_DIAG>(__VA_ARGS__);              \
    case F_GENZ_PPEAK: return CALL<R, F_GENZ_PPEAK>(__VA_ARGS__);              \
    case F_GENZ_GAUSS: return CALL<R, F_GENZ_GAUSS>(__VA_ARGS__);              \
    case F_GAUSS_CORR: return CALL<R, F_GAUSS_CORR>(__VA_ARGS__);              \
    case F_LINEAR: return CALL<R, F_LINEAR>(__VA_ARGS__);                      \
    case F_ROOS: return CALL<R, F_ROOS>(__VA_ARGS__);                          \
    case F_CONST: return CALL<R, F_CONST>(__VA_ARGS__);                        \
    case F_COSINE: return CALL<R, F_COSINE>(__VA_ARGS__);                      \
    case F_SIN_EXP: return CALL<R, F_SIN_EXP>(__VA_ARGS__);                    \
    case F_EXP_SQ: return CALL<R, F_EXP_SQ>(__VA_ARGS__);                      \
    case F_MOROKOFF: return CALL<R, F_MOROKOFF>(__VA_ARGS__);                  \
    default: return hipErrorInvalidValue;                                      \
    }

hipError_t launch_fill(const FillArgs& a, bool fp64, int n_wg, size_t lds, hipStream_t st)
{
    const int fam = a.sc.family;
    if (fp64) {
        VG_FAMILY_SWITCH(double, launch_fill_fam, a, n_wg, lds, st)
    } else {
        VG_FAMILY_SWITCH(float, launch_fill_fam, a, n_wg, lds, st)
    }
}

hipError_t launch_probe(const ProbeArgs& a, bool fp64, hipStream_t st)
{
    const int fam = a.sc.family;
    if (fp64) {
        VG_FAMILY_SWITCH(double, launch_probe_fam, a, st)
    } else {
        VG_FAMILY_SWITCH(float, launch_probe_fam, a, st)
    }
}

hipError_t launch_fixup(const FixupArgs& a, hipStream_t st)
{
    const int bs = 256;
    hipLaunchKernelGGL(k_fixup, dim3((a.n_tiles + bs - 1) / bs), dim3(bs), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_final(const FinalArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

size_t fill_lds_bytes(int D, int ng, bool fp64, int lds_hist, int tile, int n_aux, int map_lds)
{
    return lds_plan(D, ng, fp64 ? 8 : 4, lds_hist, tile, n_aux, map_lds).total;
}

}  // namespace vg
