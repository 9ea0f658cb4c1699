// The update half of a VEGAS+ iteration (Alg. 1 updateEvalsPerCube,
// adjustWeights, updateMap) and set-up kernels.
//
// Allocation (Sec. 2.1.2, Eq. 7): n_h ~ sigma_h^beta with sum n_h = N_ev.
// n_min samples are reserved per cube and the rest R is split in proportion
// to q_h = v_h^(beta/2) by integer systematic rounding:
//   Q_h = floor(q_h / q_max * 2^32), C_h = Q_0 + .. + Q_h, T = C_{N_c-1},
//   n_h = n_min + floor(R C_h / T) - floor(R C_{h-1} / T).
// Integer sums are associative, so a parallel scan gives exactly the
// sequential result; the first sample of cube h is h n_min + floor(R C_{h-1}/T).
//
// Map refinement (Sec. 2.1.1): per axis, mean weight per interval
// d_i = H_i / C_i; smoothing with (7,1)/8 at the ends and (1,6,1)/8 inside;
// normalisation by the sum taken in interval order; damping
// g_i = ((1 - e_i)/ln(1/e_i))^alpha; then every new interval receives G/N_g of
// the damped weight, linearly inside the old intervals.  The two sums are
// sequential (one lane) so the result is the same bit for bit as any
// in-order evaluation; the element-wise steps and the rebin search run in
// parallel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "fill_dev.hpp"
#include "launch.hpp"
#include "update_dev.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// set-up: derived integrand constants and the uniform initial grid
// ---------------------------------------------------------------------------
__global__ void k_prep(PrepArgs a)
{
    prep_problem(a, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void k_reset(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_grid32(const double* g64, float* g32, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g32[i] = (float)g64[i];
}

__global__ __launch_bounds__(kAllocThreads) void k_alloc_qmax(AllocArgs a, unsigned long long* qmax_bits)
{
    __shared__ double red[kAllocThreads];
    alloc_qmax_block(a, blockIdx.x, qmax_bits, red);
}

__global__ __launch_bounds__(kAllocThreads) void k_alloc_sum(AllocArgs a, const unsigned long long* qmax_bits)
{
    __shared__ uint64_t sh[kAllocThreads / 64 + 1];
    alloc_sum_block(a, qmax_bits, blockIdx.x, a.bsum + blockIdx.x, sh);
}

__global__ __launch_bounds__(kAllocThreads) void k_alloc_scan(AllocArgs a, int nb)
{
    __shared__ uint64_t sh[kAllocThreads / 64 + 1];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += kAllocThreads) {
        const int i = base + threadIdx.x;
        const uint64_t v = i < nb ? a.bsum[i] : 0ull;
        uint64_t total;
        const uint64_t ex = block_exscan(v, sh, total);
        if (i < nb) a.boff[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.boff[nb] = carry;
}

__global__ __launch_bounds__(kAllocThreads) void k_alloc_write(AllocArgs a, const unsigned long long* qmax_bits, int nb)
{
    __shared__ uint64_t sh[kAllocThreads / 64 + 1];
    alloc_write_block(a, qmax_bits, blockIdx.x, a.boff[blockIdx.x], a.boff[nb], sh);
}

hipError_t launch_alloc(const AllocArgs& a, unsigned long long* qmax_bits, hipStream_t st)
{
    const int nb = (int)((a.n_cubes + kAllocPerBlock - 1) / kAllocPerBlock);
    if (!a.uniform && !beta_monotone(a.beta))
        hipLaunchKernelGGL(k_alloc_qmax, dim3(nb), dim3(kAllocThreads), 0, st, a, qmax_bits);
    hipLaunchKernelGGL(k_alloc_sum, dim3(nb), dim3(kAllocThreads), 0, st, a, qmax_bits);
    hipLaunchKernelGGL(k_alloc_scan, dim3(1), dim3(kAllocThreads), 0, st, a, nb);
    hipLaunchKernelGGL(k_alloc_write, dim3(nb), dim3(kAllocThreads), 0, st, a, qmax_bits, nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// histogram slots -> a few partials: thread (bin, part) adds its part's
// slots in slot order; the map kernel then adds the parts in part order, so
// the sum is the same on every run
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hist_reduce(HistReduceArgs a)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.nbins * a.parts) return;
    const int part = idx / a.nbins;
    const int bin = idx - part * a.nbins;
    const int per = (a.n_slots + a.parts - 1) / a.parts;
    const int w0 = part * per;
    const int w1 = min(w0 + per, a.n_slots);
    double h = 0.0;
    uint32_t c = 0;
    int w = w0;
    for (; w + 4 <= w1; w += 4) {
        const double h0 = a.hist_H[(size_t)w * a.nbins + bin];
        const double h1 = a.hist_H[(size_t)(w + 1) * a.nbins + bin];
        const double h2 = a.hist_H[(size_t)(w + 2) * a.nbins + bin];
        const double h3 = a.hist_H[(size_t)(w + 3) * a.nbins + bin];
        c += a.hist_C[(size_t)w * a.nbins + bin] + a.hist_C[(size_t)(w + 1) * a.nbins + bin] +
             a.hist_C[(size_t)(w + 2) * a.nbins + bin] + a.hist_C[(size_t)(w + 3) * a.nbins + bin];
        h = (((h + h0) + h1) + h2) + h3;
    }
    for (; w < w1; ++w) {
        h += a.hist_H[(size_t)w * a.nbins + bin];
        c += a.hist_C[(size_t)w * a.nbins + bin];
    }
    a.part_H[(size_t)part * a.nbins + bin] = h;
    a.part_C[(size_t)part * a.nbins + bin] = c;
}

hipError_t launch_hist_reduce(const HistReduceArgs& a, hipStream_t st)
{
    const int n = a.nbins * a.parts;
    hipLaunchKernelGGL(k_hist_reduce, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_map_update(MapArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double S_sh;
    map_update_axis(a, blockIdx.x, smem, S_sh);
}

hipError_t launch_map_update(const MapArgs& a, hipStream_t st)
{
    const size_t lds = (size_t)3 * (a.ng + 1) * sizeof(double);
    hipFuncSetAttribute((const void*)k_map_update, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_map_update, dim3(a.D), dim3(1024), lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the cube fix-up, the iteration estimate and the map refinement of a small
// problem in one launch: workgroup d < D refines axis d; workgroup D runs the
// fix-up and then the estimate (the same device code and order of operations
// as the separate kernels).  The allocation follows in its own kernels,
// whose blocks then run on as many CUs.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_update_small(UpdateArgs u)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double S_sh;
    if ((int)blockIdx.x < u.map.D) {
        map_update_axis(u.map, (int)blockIdx.x, smem, S_sh);
        return;
    }
    const int tid = threadIdx.x;
    unsigned long long vb = 0ull;
    for (int j = tid; j < u.fx.n_tiles; j += 1024) {
        const unsigned long long b = fixup_chain_v(u.fx.side, u.fx.n_tiles, j, u.fx.v_out, u.fx.fix_part + 2 * j);
        vb = b > vb ? b : vb;
    }
    wave_atomic_max(vb, u.fx.vmax);
    // the fix-up's partials are read below by other lanes of this workgroup:
    // the barrier's workgroup-scope release and acquire order them (a
    // device-scope fence here would write back the whole L2)
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);      // 2 x 1024 doubles
    final_reduce(u.fin, red, red + 1024);
}

size_t update_small_lds(int ng, int parts)
{
    const size_t map = (size_t)3 * (ng + 1) * sizeof(double) + (size_t)parts * ng * (sizeof(double) + sizeof(uint32_t));
    const size_t red = (size_t)2 * 1024 * sizeof(double);
    return map > red ? map : red;
}

hipError_t launch_update_small(const UpdateArgs& u, hipStream_t st)
{
    const size_t lds = update_small_lds(u.map.ng, u.map.parts);
    hipFuncSetAttribute((const void*)k_update_small, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_update_small, dim3(u.map.D + 1), dim3(1024), lds, st, u);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_prep, dim3(64), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reset(unsigned long long* p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_grid32(const double* g64, float* g32, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_grid32, dim3((n + 255) / 256), dim3(256), 0, st, g64, g32, n);
    return hipGetLastError();
}

}  // namespace vg
