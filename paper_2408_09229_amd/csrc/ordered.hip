// ORDERED accumulation: one VEGAS+ iteration whose every sum runs in the
// order a sequential program takes (samples k = 0 .. N_ev-1, cubes in index
// order), so that a whole trajectory -- estimates, map, allocation -- is
// reproducible bit for bit.  FP64 only; meant for small problems (the
// histogram pass reads every sample once per interval).
//
//   k_ord_eval   per sample: cube, point, map, f, w = J f (Alg. 2), stored
//   k_ord_cube   per cube: mean, then the sum of squared deviations (Eq. 5-6)
//   k_ord_hist   per (axis, interval): sum of w^2 and count over samples in
//                increasing k
//   k_ord_total  I = sum m_h / N_c, sigma^2 = sum v_h / (N_c^2 n_h) in cube
//                order, and max v_h for the allocation
//
// For the rational and polynomial families (GENZ_PPEAK, LINEAR, ROOS, CONST)
// f is evaluated exactly as the formula reads, factor by factor, so that w
// itself is reproducible across machines; other families use the fill's
// evaluation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "launch.hpp"
#include "sample.hpp"

namespace vg {

// f as the formula reads, one correctly rounded operation at a time
__device__ __forceinline__ bool f_in_formula_order(int fam, int D, const double* p, const double* x, double& f)
{
    switch (fam) {
    case F_GENZ_PPEAK: {
        double v = p[0];
        for (int d = 0; d < D; ++d) {
            const double a = p[1 + d];
            const double u = x[d] - p[1 + D + d];
            v *= 1.0 / (1.0 / (a * a) + u * u);
        }
        f = v;
        return true;
    }
    case F_LINEAR: {
        double s = 0.0;
        for (int d = 0; d < D; ++d) s += x[d];
        f = p[0] * s;
        return true;
    }
    case F_ROOS: {
        double v = p[0];
        for (int d = 0; d < D; ++d) v *= fabs(4.0 * x[d] - 2.0);
        f = v;
        return true;
    }
    case F_CONST:
        f = p[0];
        return true;
    default:
        return false;
    }
}

template <int FAM, int MAXD>
__global__ void k_ord_eval(OrderedArgs a)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.sc.n_eval) return;
    uint32_t lo = 0, hi = a.sc.n_cubes;      // largest h with start[h] <= k
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.start[mid] <= k) lo = mid; else hi = mid;
    }
    SamplePath<double, FAM, MAXD> sp(a.sc, a.sc.aux_d);
    uint32_t s[MAXD], bins[MAXD];
    double delta[MAXD], x[MAXD], J, f;
    sp.digits(lo, s);
    sp.template eval<true>(k, a.t, s, a.grid, bins, delta, x, J, f);
    const int D = a.sc.D;
    double fs;
    if (f_in_formula_order(a.sc.family, D, a.sc.prm, x, fs)) f = fs;
    double w = J * f;
    if (!__builtin_isfinite(w)) {
        w = 0.0;
        atomicAdd(a.nonfinite, 1ull);
    }
    a.w[k] = w;
#pragma unroll
    for (int d = 0; d < MAXD; ++d)
        if (d < D) a.bins[(size_t)k * D + d] = bins[d];
}

__global__ void k_ord_cube(OrderedArgs a)
{
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= a.sc.n_cubes) return;
    const uint32_t k0 = a.start[h], k1 = a.start[h + 1];
    const double n = (double)(k1 - k0);
    double sum = 0.0;
    for (uint32_t k = k0; k < k1; ++k) sum += a.w[k];
    const double m = sum / n;
    double ss = 0.0;
    for (uint32_t k = k0; k < k1; ++k) {
        const double u = a.w[k] - m;
        ss += u * u;
    }
    a.m[h] = m;
    a.v[h] = ss / (n - 1.0);
}

__global__ void k_ord_hist(OrderedArgs a)
{
    const int D = a.sc.D;
    const int ng = (int)a.sc.ng;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D * ng) return;
    const int d = i / ng;
    const uint32_t bin = (uint32_t)(i - d * ng);
    double H = 0.0;
    uint32_t C = 0;
    for (uint32_t k = 0; k < a.sc.n_eval; ++k) {
        if (a.bins[(size_t)k * D + d] == bin) {
            const double w = a.w[k];
            H += w * w;
            ++C;
        }
    }
    a.hist_H[i] = H;
    a.hist_C[i] = C;
}

__global__ void k_ord_total(OrderedArgs a)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double Nc = (double)a.sc.n_cubes;
    const double Nc2 = Nc * Nc;
    double I = 0.0, S2 = 0.0, vmax = 0.0;
    for (uint32_t h = 0; h < a.sc.n_cubes; ++h) {
        const double n = (double)(a.start[h + 1] - a.start[h]);
        I += a.m[h] / Nc;
        S2 += a.v[h] / (Nc2 * n);
        vmax = a.v[h] > vmax ? a.v[h] : vmax;
    }
    a.iter_out[0] = I;
    a.iter_out[1] = S2;
    *a.vmax = (unsigned long long)__double_as_longlong(vmax);
}

template <int FAM>
static hipError_t launch_ord_eval_fam(const OrderedArgs& a, hipStream_t st)
{
    const unsigned nb = (a.sc.n_eval + 255) / 256;
    const int D = a.sc.D;
    if (D <= 4) hipLaunchKernelGGL((k_ord_eval<FAM, 4>), dim3(nb), dim3(256), 0, st, a);
    else if (D <= 8) hipLaunchKernelGGL((k_ord_eval<FAM, 8>), dim3(nb), dim3(256), 0, st, a);
    else if (D <= 12) hipLaunchKernelGGL((k_ord_eval<FAM, 12>), dim3(nb), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_ord_eval<FAM, 16>), dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_ordered(const OrderedArgs& a, hipStream_t st)
{
    hipError_t e;
    switch (a.sc.family) {
    case F_GAUSS_DIAG: e = launch_ord_eval_fam<F_GAUSS_DIAG>(a, st); break;
    case F_GENZ_PPEAK: e = launch_ord_eval_fam<F_GENZ_PPEAK>(a, st); break;
    case F_GENZ_GAUSS: e = launch_ord_eval_fam<F_GENZ_GAUSS>(a, st); break;
    case F_GAUSS_CORR: e = launch_ord_eval_fam<F_GAUSS_CORR>(a, st); break;
    case F_LINEAR: e = launch_ord_eval_fam<F_LINEAR>(a, st); break;
    case F_ROOS: e = launch_ord_eval_fam<F_ROOS>(a, st); break;
    case F_CONST: e = launch_ord_eval_fam<F_CONST>(a, st); break;
    case F_COSINE: e = launch_ord_eval_fam<F_COSINE>(a, st); break;
    case F_SIN_EXP: e = launch_ord_eval_fam<F_SIN_EXP>(a, st); break;
    case F_EXP_SQ: e = launch_ord_eval_fam<F_EXP_SQ>(a, st); break;
    case F_MOROKOFF: e = launch_ord_eval_fam<F_MOROKOFF>(a, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ord_cube, dim3((a.sc.n_cubes + 255) / 256), dim3(256), 0, st, a);
    const int nb = a.sc.D * (int)a.sc.ng;
    hipLaunchKernelGGL(k_ord_hist, dim3((nb + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_ord_total, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace vg
