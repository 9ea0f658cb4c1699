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
#include "launch.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// set-up: derived integrand constants and the uniform initial grid
// ---------------------------------------------------------------------------
__global__ void k_prep(PrepArgs a)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    const int D = a.D;
    if (a.family == F_GAUSS_DIAG) {
        const double s = a.prm[1];
        const int M = (int)a.prm[2];
        const double K = sqrt((double)D / (2.0 * s * s * kLn2));
        for (int j = tid; j < M; j += nth) {
            a.aux_d[j] = a.prm[3 + j];
            a.aux_f[j] = (float)(K * a.prm[3 + j]);
        }
    } else if (a.family == F_GENZ_PPEAK || a.family == F_GENZ_GAUSS) {
        for (int d = tid; d < D; d += nth) {
            const double c = a.prm[1 + d];
            const double u = a.prm[1 + D + d];
            if (a.family == F_GENZ_PPEAK) {
                a.aux_d[d] = 1.0 / (c * c);
                a.aux_f[d] = (float)(1.0 / (c * c));
            } else {
                a.aux_d[d] = c * c;
                a.aux_f[d] = (float)(c * c / kLn2);
            }
            a.aux_d[D + d] = u;
            a.aux_f[D + d] = (float)u;
        }
    }
    if (a.grid64) {
        const int row = a.ng + 1;
        for (int i = tid; i < D * row; i += nth) {
            const int d = i / row, j = i % row;
            const double x = a.lo[d] + ((a.hi[d] - a.lo[d]) * (double)j) / (double)a.ng;
            a.grid64[i] = x;
            a.grid32[i] = (float)x;
        }
    }
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

// ---------------------------------------------------------------------------
// allocation
// ---------------------------------------------------------------------------
// floor(R C / T) exactly, R < 2^32, C <= T < 2^63: a double estimate is
// within one of the answer; 128-bit products settle it.
__device__ __forceinline__ uint64_t floor_mul_div(uint64_t R, uint64_t C, uint64_t T)
{
    const double est = ((double)R * (double)C) / (double)T;
    uint64_t m = (uint64_t)est;
    const unsigned __int128 rc = (unsigned __int128)R * C;
    unsigned __int128 mt = (unsigned __int128)m * T;
    while (mt > rc) {
        --m;
        mt -= T;
    }
    while (mt + T <= rc) {
        ++m;
        mt += T;
    }
    return m;
}

struct QPlan {
    int uniform;
    double qmax;
};

__device__ __forceinline__ QPlan q_plan(const AllocArgs& a, const unsigned long long* qmax_bits)
{
    QPlan p;
    p.uniform = a.uniform;
    p.qmax = 0.0;
    if (!p.uniform) {
        if (beta_monotone(a.beta)) p.qmax = pow_half_beta(__longlong_as_double((long long)*a.vmax), a.beta);
        else p.qmax = __longlong_as_double((long long)*qmax_bits);
        if (!(p.qmax > 0.0)) p.uniform = 1;
    }
    return p;
}

__device__ __forceinline__ uint64_t quant(const AllocArgs& a, const QPlan& p, uint32_t h)
{
    if (p.uniform) return 1ull;
    const double q = pow_half_beta(a.v[h], a.beta);
    return (uint64_t)floor((q / p.qmax) * 4294967296.0);
}

__global__ __launch_bounds__(kAllocThreads) void k_alloc_qmax(AllocArgs a, unsigned long long* qmax_bits)
{
    __shared__ double red[kAllocThreads];
    const uint32_t base = blockIdx.x * (uint32_t)kAllocPerBlock;
    double m = 0.0;
    for (int i = 0; i < kAllocPerThread; ++i) {
        const uint32_t h = base + threadIdx.x * kAllocPerThread + i;
        if (h < a.n_cubes) {
            const double q = pow_half_beta(a.v[h], a.beta);
            m = q > m ? q : m;
        }
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kAllocThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && red[threadIdx.x + w] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(qmax_bits, (unsigned long long)__double_as_longlong(red[0]));
}

// exclusive scan of one value per thread across the block (u64)
__device__ __forceinline__ uint64_t block_exscan(uint64_t v, uint64_t* sh, uint64_t& total)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (tid == 0) {
        uint64_t run = 0;
        for (int w = 0; w < kAllocThreads / 64; ++w) {
            const uint64_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[kAllocThreads / 64] = run;
    }
    __syncthreads();
    total = sh[kAllocThreads / 64];
    const uint64_t r = sh[wave] + x - v;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kAllocThreads) void k_alloc_sum(AllocArgs a, const unsigned long long* qmax_bits)
{
    __shared__ uint64_t sh[kAllocThreads / 64 + 1];
    const QPlan p = q_plan(a, qmax_bits);
    const uint32_t base = blockIdx.x * (uint32_t)kAllocPerBlock;
    uint64_t s = 0;
    for (int i = 0; i < kAllocPerThread; ++i) {
        const uint32_t h = base + threadIdx.x * kAllocPerThread + i;
        if (h < a.n_cubes) s += quant(a, p, h);
    }
    uint64_t total;
    block_exscan(s, sh, total);
    if (threadIdx.x == 0) a.bsum[blockIdx.x] = total;
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
    const QPlan p = q_plan(a, qmax_bits);
    const uint32_t base = blockIdx.x * (uint32_t)kAllocPerBlock;
    uint64_t Q[kAllocPerThread];
    uint64_t s = 0;
    for (int i = 0; i < kAllocPerThread; ++i) {
        const uint32_t h = base + threadIdx.x * kAllocPerThread + i;
        Q[i] = h < a.n_cubes ? quant(a, p, h) : 0ull;
        s += Q[i];
    }
    uint64_t total;
    uint64_t Cprev = a.boff[blockIdx.x] + block_exscan(s, sh, total);
    const uint64_t T = a.boff[nb];
    const uint64_t R = a.R;
    uint64_t lo = floor_mul_div(R, Cprev, T);
    for (int i = 0; i < kAllocPerThread; ++i) {
        const uint32_t h = base + threadIdx.x * kAllocPerThread + i;
        if (h >= a.n_cubes) break;
        const uint64_t C = Cprev + Q[i];
        const uint64_t hi = floor_mul_div(R, C, T);
        const uint32_t start = h * a.n_min + (uint32_t)lo;
        const uint32_t nh = a.n_min + (uint32_t)(hi - lo);
        a.start[h] = start;
        // tiles whose first sample lies in this cube
        const uint64_t end = (uint64_t)start + nh;
        for (uint64_t j = ((uint64_t)start + (uint64_t)a.tile - 1u) >> a.tile_shift; (j << a.tile_shift) < end; ++j)
            a.tile_first[j] = h;
        if (h == a.n_cubes - 1u) {
            a.start[a.n_cubes] = a.n_eval;
            a.tile_first[a.n_tiles] = a.n_cubes;
        }
        Cprev = C;
        lo = hi;
    }
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

// ---------------------------------------------------------------------------
// map refinement: one workgroup per axis
// ---------------------------------------------------------------------------
__device__ __forceinline__ double damp(double e, double alpha)
{
    if (e == 0.0) return 0.0;
    if (e == 1.0) return 1.0;
    const double t = (1.0 - e) / (-dlog(e));
    if (alpha == 0.5) return sqrt(t);
    if (alpha == 1.0) return t;
    if (alpha == 1.5) return t * sqrt(t);
    return dexp(alpha * dlog(t));
}

__global__ __launch_bounds__(1024) void k_map_update(MapArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int ng = a.ng;
    const int d = blockIdx.x;
    const int tid = threadIdx.x;
    double* x = reinterpret_cast<double*>(smem);
    double* A = x + (ng + 1);
    double* B = A + (ng + 1);
    __shared__ double S_sh;
    const int row = ng + 1;
    const int nbins = a.D * ng;
    for (int i = tid; i <= ng; i += 1024) x[i] = a.grid64[d * row + i];
    int any = 0;
    for (int i = tid; i < ng; i += 1024) {
        double H = 0.0;
        uint64_t C = 0;
        const int bi = d * ng + i;
        for (int w = 0; w < a.n_slots; ++w) {
            H += a.hist_H[(size_t)w * nbins + bi];
            C += a.hist_C[(size_t)w * nbins + bi];
        }
        a.Hsum[bi] = H;
        a.Csum[bi] = (double)C;
        A[i] = C > 0 ? H / (double)C : 0.0;
        any |= (H != 0.0);
    }
    any = __syncthreads_or(any);
    if (a.alpha == 0.0 || !any) return;
    for (int i = tid; i < ng; i += 1024) {
        double e;
        if (ng == 1) e = A[0];
        else if (i == 0) e = (7.0 * A[0] + A[1]) / 8.0;
        else if (i == ng - 1) e = (A[ng - 2] + 7.0 * A[ng - 1]) / 8.0;
        else e = ((A[i - 1] + 6.0 * A[i]) + A[i + 1]) / 8.0;
        B[i] = e;
    }
    __syncthreads();
    if (tid == 0) {
        double S = 0.0;
        for (int i = 0; i < ng; ++i) S += B[i];
        S_sh = S;
    }
    __syncthreads();
    const double S = S_sh;
    if (!(S > 0.0)) return;
    for (int i = tid; i < ng; i += 1024) A[i] = damp(B[i] / S, a.alpha);
    __syncthreads();
    if (tid == 0) {
        double c = 0.0;
        B[0] = 0.0;
        for (int i = 0; i < ng; ++i) {
            c = c + A[i];
            B[i + 1] = c;
        }
    }
    __syncthreads();
    const double G = B[ng];
    const double dg = G / (double)ng;
    for (int j = tid + 1; j < ng; j += 1024) {
        const double tau = (double)j * dg;
        int lo = 0, hi = ng;      // B[lo] <= tau < B[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (B[mid] <= tau) lo = mid; else hi = mid;
        }
        const double xn = fma((tau - B[lo]) / A[lo], x[lo + 1] - x[lo], x[lo]);
        a.grid64[d * row + j] = xn;
        a.grid32[d * row + j] = (float)xn;
    }
}

hipError_t launch_map_update(const MapArgs& a, hipStream_t st)
{
    const size_t lds = (size_t)3 * (a.ng + 1) * sizeof(double);
    hipFuncSetAttribute((const void*)k_map_update, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_map_update, dim3(a.D), dim3(1024), lds, st, a);
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
