// Device bodies of the set-up and of the update half of an iteration
// (allocation, map refinement), shared by the single-problem and the batched kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "launch.hpp"
#include "layout.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// set-up: derived integrand constants and the uniform initial grid
// ---------------------------------------------------------------------------
// derived constants of one problem and (grid64 non-null) its uniform grid;
// thread tid of nth
__device__ __forceinline__ void prep_problem(const PrepArgs& a, int tid, int nth)
{
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

// ---------------------------------------------------------------------------
// allocation
// ---------------------------------------------------------------------------
// floor(R C / T) exactly, R < 2^32, C <= T < 2^63.  rT = R/T rounded to
// double: the estimate C rT is within a few 2^-53 relative of R C/T < 2^32,
// so within one of the answer; 128-bit products settle it.
__device__ __forceinline__ uint64_t floor_mul_div(uint64_t R, uint64_t C, uint64_t T, double rT)
{
    const double est = (double)C * rT;
    // est = R C / T within five roundings, so within 2^-18.6 of it (R C / T
    // <= R < 2^32): a fraction at least 2^-16 away from both integers
    // settles the floor without the 128-bit check
    const double fl = floor(est);
    const double fr = est - fl;
    if (fr > 0x1p-16 && fr < 1.0 - 0x1p-16) return (uint64_t)fl;
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
        // a zero, infinite or NaN maximum (an overflowed variance) leaves no
        // usable weights: fall back to the uniform allocation, so T > 0
        if (!(p.qmax > 0.0) || !(p.qmax <= 1.7976931348623157e308)) p.uniform = 1;
    }
    return p;
}

// Q = floor(q / q_max 2^32) of a variance v
__device__ __forceinline__ uint64_t quant_v(double v, double beta, double qmax)
{
    const double q = pow_half_beta(v, beta);
    const double r = q / qmax;
    // r is in [0, 1] for finite variances; a NaN weight counts as 0
    return r >= 0.0 ? (uint64_t)floor(fmin(r, 1.0) * 4294967296.0) : 0ull;
}

__device__ __forceinline__ uint64_t quant(const AllocArgs& a, const QPlan& p, uint32_t h)
{
    if (p.uniform) return 1ull;
    return quant_v(a.v[h], a.beta, p.qmax);
}

// block blk of a problem's cubes: the block's largest q into qmax_bits
__device__ __forceinline__ void alloc_qmax_block(const AllocArgs& a, uint32_t blk, unsigned long long* qmax_bits,
                                                 double* red)
{
    const uint32_t base = blk * (uint32_t)kAllocPerBlock;
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
    __syncthreads();
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

// the Q_h of the kPerThread consecutive cubes h0.. of one thread (cubes past
// the end give 0); v is read 16 bytes at a time when all are in range
__device__ __forceinline__ void quant_run(const AllocArgs& a, const QPlan& p, uint32_t h0, uint64_t (&Q)[kAllocPerThread])
{
    static_assert(kAllocPerThread == 4, "two 16-byte loads per thread");
    if (p.uniform) {
        for (int i = 0; i < kAllocPerThread; ++i) Q[i] = h0 + (uint32_t)i < a.n_cubes ? 1ull : 0ull;
        return;
    }
    if (h0 + (uint32_t)kAllocPerThread <= a.n_cubes) {
        const double2 v01 = *reinterpret_cast<const double2*>(a.v + h0);
        const double2 v23 = *reinterpret_cast<const double2*>(a.v + h0 + 2);
        const double v[4] = {v01.x, v01.y, v23.x, v23.y};
        for (int i = 0; i < kAllocPerThread; ++i) Q[i] = quant_v(v[i], a.beta, p.qmax);
        return;
    }
    for (int i = 0; i < kAllocPerThread; ++i) Q[i] = h0 + (uint32_t)i < a.n_cubes ? quant(a, p, h0 + i) : 0ull;
}

// block blk: the sum of its Q_h into *bsum; Q_h (saturated) into qbuf
__device__ __forceinline__ void alloc_sum_block(const AllocArgs& a, const unsigned long long* qmax_bits, uint32_t blk,
                                                unsigned long long* bsum, uint64_t* sh)
{
    const QPlan p = q_plan(a, qmax_bits);
    const uint32_t h0 = blk * (uint32_t)kAllocPerBlock + threadIdx.x * kAllocPerThread;
    uint64_t Q[kAllocPerThread];
    quant_run(a, p, h0, Q);
    uint64_t s = 0;
    for (int i = 0; i < kAllocPerThread; ++i) s += Q[i];
    if (a.qbuf && !p.uniform) {
        uint32_t q32[kAllocPerThread];
        for (int i = 0; i < kAllocPerThread; ++i) q32[i] = Q[i] > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)Q[i];
        if (h0 + (uint32_t)kAllocPerThread <= a.n_cubes)
            *reinterpret_cast<uint4*>(a.qbuf + h0) = make_uint4(q32[0], q32[1], q32[2], q32[3]);
        else
            for (int i = 0; i < kAllocPerThread; ++i)
                if (h0 + (uint32_t)i < a.n_cubes) a.qbuf[h0 + i] = q32[i];
    }
    uint64_t total;
    block_exscan(s, sh, total);
    if (threadIdx.x == 0) *bsum = total;
}

// block blk: n_h, first samples and tile table from the exclusive offset
// boff of the block and the total T.  Q_h comes from qbuf (written by the
// sum pass), recomputed exactly where it saturated.
__device__ __forceinline__ void alloc_write_block(const AllocArgs& a, const unsigned long long* qmax_bits, uint32_t blk,
                                                  uint64_t boff, uint64_t T, uint64_t* sh)
{
    const QPlan p = q_plan(a, qmax_bits);
    const uint32_t h0 = blk * (uint32_t)kAllocPerBlock + threadIdx.x * kAllocPerThread;
    const bool full = h0 + (uint32_t)kAllocPerThread <= a.n_cubes;
    uint64_t Q[kAllocPerThread];
    if (a.qbuf && !p.uniform) {
        uint32_t q32[kAllocPerThread] = {0u, 0u, 0u, 0u};
        if (full) {
            const uint4 v = *reinterpret_cast<const uint4*>(a.qbuf + h0);
            q32[0] = v.x;
            q32[1] = v.y;
            q32[2] = v.z;
            q32[3] = v.w;
        } else {
            for (int i = 0; i < kAllocPerThread; ++i)
                if (h0 + (uint32_t)i < a.n_cubes) q32[i] = a.qbuf[h0 + i];
        }
        for (int i = 0; i < kAllocPerThread; ++i)
            Q[i] = q32[i] == 0xFFFFFFFFu ? quant(a, p, h0 + i) : (uint64_t)q32[i];
    } else {
        quant_run(a, p, h0, Q);
    }
    uint64_t s = 0;
    for (int i = 0; i < kAllocPerThread; ++i) s += Q[i];
    uint64_t total;
    uint64_t Cprev = boff + block_exscan(s, sh, total);
    const uint64_t R = a.R;
    const double rT = (double)R / (double)T;
    uint64_t lo = floor_mul_div(R, Cprev, T, rT);
    uint32_t st[kAllocPerThread];
    for (int i = 0; i < kAllocPerThread; ++i) {
        const uint32_t h = h0 + (uint32_t)i;
        if (h >= a.n_cubes) break;
        const uint64_t C = Cprev + Q[i];
        const uint64_t hi = floor_mul_div(R, C, T, rT);
        const uint32_t start = h * a.n_min + (uint32_t)lo;
        const uint32_t nh = a.n_min + (uint32_t)(hi - lo);
        st[i] = start;
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
    if (full) {
        *reinterpret_cast<uint4*>(a.start + h0) = make_uint4(st[0], st[1], st[2], st[3]);
    } else {
        for (int i = 0; i < kAllocPerThread; ++i)
            if (h0 + (uint32_t)i < a.n_cubes) a.start[h0 + i] = st[i];
    }
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

// axis d of a problem (one 1024-lane workgroup); smem holds 3 (N_g+1)
// doubles, S_sh one shared double
constexpr int kSeqChunk = 16;           // LDS reads in flight in the sequential sums

__device__ __forceinline__ void map_update_axis(const MapArgs& a, int d, unsigned char* smem, double& S_sh)
{
    const int ng = a.ng;
    const int tid = threadIdx.x;
    double* x = reinterpret_cast<double*>(smem);
    double* A = x + (ng + 1);
    double* B = A + (ng + 1);
    const int row = ng + 1;
    const int nbins = a.D * ng;
    for (int i = tid; i <= ng; i += 1024) x[i] = a.grid64[d * row + i];
    // slot groups: one lane per (group, interval) adds its group's slots in
    // order into LDS (after x, A, B: parts x N_g doubles, then as many u32)
    double* Hp = B + (ng + 1);
    uint32_t* Cp = reinterpret_cast<uint32_t*>(Hp + (size_t)a.parts * ng);
    if (a.parts > 0) {
        const int per = (a.n_slots + a.parts - 1) / a.parts;
        for (int idx = tid; idx < a.parts * ng; idx += 1024) {
            const int p = idx / ng;
            const int bi = d * ng + (idx - p * ng);
            const int w1 = min((p + 1) * per, a.n_slots);
            double h = 0.0;
            uint32_t c = 0;
            int w = p * per;
            // four loads in flight, the adds in slot order
            for (; w + 4 <= w1; w += 4) {
                const double h0 = a.hist_H[(size_t)w * nbins + bi];
                const double h1 = a.hist_H[(size_t)(w + 1) * nbins + bi];
                const double h2 = a.hist_H[(size_t)(w + 2) * nbins + bi];
                const double h3 = a.hist_H[(size_t)(w + 3) * nbins + bi];
                c += a.hist_C[(size_t)w * nbins + bi] + a.hist_C[(size_t)(w + 1) * nbins + bi] +
                     a.hist_C[(size_t)(w + 2) * nbins + bi] + a.hist_C[(size_t)(w + 3) * nbins + bi];
                h = (((h + h0) + h1) + h2) + h3;
            }
            for (; w < w1; ++w) {
                h += a.hist_H[(size_t)w * nbins + bi];
                c += a.hist_C[(size_t)w * nbins + bi];
            }
            Hp[idx] = h;
            Cp[idx] = c;
        }
        __syncthreads();
    }
    int any = 0;
    for (int i = tid; i < ng; i += 1024) {
        double H = 0.0;
        uint64_t C = 0;
        const int bi = d * ng + i;
        if (a.hist_Cw) {
            // an iteration through the learned warp: importance-weighted sums
            const double Cw = a.hist_Cw[bi];
            H = a.hist_H[bi];
            if (a.Hsum) {
                a.Hsum[bi] = H;
                a.Csum[bi] = Cw;
            }
            A[i] = Cw > 0.0 ? H / Cw : 0.0;
            any |= (H != 0.0);
            continue;
        }
        if (a.parts > 0) {
            for (int p = 0; p < a.parts; ++p) {
                H += Hp[p * ng + i];
                C += Cp[p * ng + i];
            }
        } else {
            for (int w = 0; w < a.n_slots; ++w) {
                H += a.hist_H[(size_t)w * nbins + bi];
                C += a.hist_C[(size_t)w * nbins + bi];
            }
        }
        if (a.Hsum) {
            a.Hsum[bi] = H;
            a.Csum[bi] = (double)C;
        }
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
        // in interval order; the reads go ahead in chunks, the adds do not
        double S = 0.0;
        int i = 0;
        for (; i + kSeqChunk <= ng; i += kSeqChunk) {
            double v[kSeqChunk];
#pragma unroll
            for (int k = 0; k < kSeqChunk; ++k) v[k] = B[i + k];
#pragma unroll
            for (int k = 0; k < kSeqChunk; ++k) S += v[k];
        }
        for (; i < ng; ++i) S += B[i];
        S_sh = S;
    }
    __syncthreads();
    const double S = S_sh;
    if (!(S > 0.0)) return;
    for (int i = tid; i < ng; i += 1024) A[i] = damp(B[i] / S, a.alpha);
    __syncthreads();
    if (tid == 0) {
        // sequential prefix; a chunk of A is read before its prefixes are
        // written (A and B do not overlap), so the LDS reads do not wait on
        // the writes one by one
        double c = 0.0;
        B[0] = 0.0;
        int i = 0;
        for (; i + kSeqChunk <= ng; i += kSeqChunk) {
            double v[kSeqChunk];
#pragma unroll
            for (int k = 0; k < kSeqChunk; ++k) v[k] = A[i + k];
#pragma unroll
            for (int k = 0; k < kSeqChunk; ++k) {
                c = c + v[k];
                B[i + 1 + k] = c;
            }
        }
        for (; i < ng; ++i) {
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

}  // namespace vg
