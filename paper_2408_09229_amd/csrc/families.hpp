// Built-in integrand families (vegas.h VEGAS_* ids; Tab. 3 and the benchmark
// workloads).  Each is a functor fed one coordinate at a time, so the sample
// path never stores a coordinate vector:
//   setup(sc, aux)  per-thread constants from the raw parameters and the
//                   derived per-term / per-axis table aux (in the sample
//                   path's precision; the fill kernel passes a copy in LDS)
//   begin()      reset the per-sample accumulators
//   axis(d, x)   fold in coordinate d
//   finish()     f(x)
// FP64 variants evaluate in double with libm-quality exp (parity path);
// FP32 variants use the hardware exp2 and fold constants so that the
// per-term work is a few VALU operations.
#pragma once
#ifndef __HIPCC_RTC__   // hipRTC provides the HIP device runtime itself
#include <hip/hip_runtime.h>
#endif
#include <type_traits>

#include "layout.hpp"

namespace vg {

enum : int { F_GAUSS_DIAG = 1, F_GENZ_PPEAK = 2, F_GENZ_GAUSS = 3, F_GAUSS_CORR = 4,
             F_LINEAR = 5, F_ROOS = 6, F_CONST = 7, F_COSINE = 8, F_SIN_EXP = 9, F_EXP_SQ = 10,
             F_MOROKOFF = 11, F_USER = 12 };

constexpr double kLn2 = 0.69314718055994530942;

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

template <typename R, int FAM>
struct Fn;

// Mean of Gaussians centred on the diagonal (GAUSS_DIAG):
//   A sum_j exp(-sum_d (x_d - c_j)^2 / (2 s^2))
// uses sum_d (x_d - c)^2 = S + D (m - c)^2, m the coordinate mean,
// S = sum_d (x_d - m)^2 accumulated relative to the first coordinate.
template <typename R>
struct Fn<R, F_GAUSS_DIAG> {
    R A, h, Dr, invD, x0, a1, a2;
    int M;
    const R* cj;         // FP64: c_j; FP32: K c_j with K = sqrt(D / (2 s^2 ln 2))
    R K;
    // FP32 with at most kRegTerms terms: K c_j held in registers, read once
    // from global memory, so the per-sample work issues no LDS read (an LDS
    // read would wait for the histogram atomics still in flight)
    static constexpr int kRegTerms = 4;
    float cr[kRegTerms];
    __device__ __forceinline__ void setup(const SampleConst& sc, const R* aux)
    {
        const double s = sc.prm[1];
        A = (R)sc.prm[0];
        M = (int)sc.prm[2];
        cj = aux;
        Dr = (R)sc.D;
        invD = (R)(1.0 / (double)sc.D);
        if constexpr (std::is_same<R, double>::value) {
            h = 1.0 / (2.0 * s * s);
            K = 0;
        } else {
            const double L = 1.0 / (2.0 * s * s * kLn2);
            h = (float)L;
            K = (float)sqrt((double)sc.D * L);
#pragma unroll
            for (int q = 0; q < kRegTerms; ++q) cr[q] = q < M ? sc.aux_f[q] : 0.f;
        }
    }
    __device__ __forceinline__ void begin() { x0 = 0; a1 = 0; a2 = 0; }
    __device__ __forceinline__ void axis(int d, R x)
    {
        if (d == 0) {
            x0 = x;
        } else {
            const R u = x - x0;
            a1 = a1 + u;
            a2 = fma(u, u, a2);
        }
    }
    __device__ __forceinline__ R finish() const
    {
        const R m = x0 + a1 * invD;
        R S = a2 - a1 * (a1 * invD);
        S = S > (R)0 ? S : (R)0;
        if constexpr (std::is_same<R, double>::value) {
            double acc = 0.0;
            const double dh = Dr * h;
            for (int j = 0; j < M; ++j) {
                const double u = m - cj[j];
                acc += exp(-(dh * u) * u);
            }
            return A * exp(-S * h) * acc;
        } else {
            const float Km = K * m;
            if (M <= kRegTerms) {
                // the association of the general loop below: one sum for
                // M < 4, two pairs for M = 4
                float e[kRegTerms];
#pragma unroll
                for (int q = 0; q < kRegTerms; ++q) {
                    const float g = Km - cr[q];
                    e[q] = q < M ? exp2_fast(-(g * g)) : 0.f;
                }
                const float acc = M == kRegTerms ? (e[0] + e[1]) + (e[2] + e[3]) : (e[0] + e[1]) + e[2];
                return A * exp2_fast(-S * h) * acc;
            }
            // per term: difference, square, exp2, add (4 independent sums)
            float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
            int j = 0;
            // eight terms a pass (two table reads, one wait), each sum still
            // taking every fourth term in order
            for (; j + 7 < M; j += 8) {
                float e[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float g = Km - cj[j + q];
                    e[q] = exp2_fast(-(g * g));
                }
                acc0 += e[0];
                acc1 += e[1];
                acc2 += e[2];
                acc3 += e[3];
                acc0 += e[4];
                acc1 += e[5];
                acc2 += e[6];
                acc3 += e[7];
            }
            for (; j + 3 < M; j += 4) {
                const float g0 = Km - cj[j];
                const float g1 = Km - cj[j + 1];
                const float g2 = Km - cj[j + 2];
                const float g3 = Km - cj[j + 3];
                acc0 += exp2_fast(-(g0 * g0));
                acc1 += exp2_fast(-(g1 * g1));
                acc2 += exp2_fast(-(g2 * g2));
                acc3 += exp2_fast(-(g3 * g3));
            }
            for (; j < M; ++j) {
                const float g0 = Km - cj[j];
                acc0 += exp2_fast(-(g0 * g0));
            }
            return A * exp2_fast(-S * h) * ((acc0 + acc1) + (acc2 + acc3));
        }
    }
};

// Genz product peak: A prod_d 1 / (a_d^-2 + (x_d - u_d)^2)
template <typename R>
struct Fn<R, F_GENZ_PPEAK> {
    R A, p;
    const R* ax;         // [1/a^2 .., u ..]
    int D;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R* aux)
    {
        A = (R)sc.prm[0];
        ax = aux;
        D = sc.D;
    }
    __device__ __forceinline__ void begin() { p = 1; }
    __device__ __forceinline__ void axis(int d, R x)
    {
        const R ia2 = ax[d], u0 = ax[D + d];
        const R u = x - u0;
        p = p * fma(u, u, ia2);
    }
    __device__ __forceinline__ R finish() const { return A / p; }
};

// Genz Gaussian: A exp(-sum_d a_d^2 (x_d - u_d)^2)
template <typename R>
struct Fn<R, F_GENZ_GAUSS> {
    R A, q;
    const R* ax;         // FP64: [a^2 .., u ..]; FP32: [a^2 / ln 2 .., u ..]
    int D;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R* aux)
    {
        A = (R)sc.prm[0];
        ax = aux;
        D = sc.D;
    }
    __device__ __forceinline__ void begin() { q = 0; }
    __device__ __forceinline__ void axis(int d, R x)
    {
        const R a2 = ax[d], u0 = ax[D + d];
        const R u = x - u0;
        q = fma(a2 * u, u, q);
    }
    __device__ __forceinline__ R finish() const
    {
        if constexpr (std::is_same<R, double>::value) return A * exp(-q);
        else return A * exp2_fast(-q);
    }
};

// Correlated Gaussian density N(x; mu 1, s^2 ((1-rho) I + rho 1 1^T)).
// With v = x - mu 1, vbar its mean and S = sum (v_d - vbar)^2,
// v^T Sigma^-1 v = S/(s^2 (1-rho)) + D vbar^2/(s^2 (1 + (D-1) rho)),
// which has no cancellation; log-normaliser folded into one constant.
template <typename R>
struct Fn<R, F_GAUSS_CORR> {
    R mu, c1, c2, z, x0, a1, a2, invD;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*)
    {
        const double m = sc.prm[0], s = sc.prm[1], rho = sc.prm[2];
        const int D = sc.D;
        const double k1 = 1.0 / (s * s * (1.0 - rho));
        const double k2 = (double)D / (s * s * (1.0 + (D - 1) * rho));
        const double logdet = 2.0 * D * log(s) + (D - 1) * log(1.0 - rho) + log(1.0 + (D - 1) * rho);
        const double lz = 0.5 * D * log(2.0 * 3.14159265358979323846) + 0.5 * logdet;
        mu = (R)m;
        invD = (R)(1.0 / D);
        if constexpr (std::is_same<R, double>::value) {
            c1 = 0.5 * k1; c2 = 0.5 * k2; z = lz;
        } else {
            c1 = (float)(0.5 * k1 / kLn2); c2 = (float)(0.5 * k2 / kLn2); z = (float)(lz / kLn2);
        }
    }
    __device__ __forceinline__ void begin() { x0 = 0; a1 = 0; a2 = 0; }
    __device__ __forceinline__ void axis(int d, R x)
    {
        if (d == 0) {
            x0 = x;
        } else {
            const R u = x - x0;
            a1 = a1 + u;
            a2 = fma(u, u, a2);
        }
    }
    __device__ __forceinline__ R finish() const
    {
        const R vbar = (x0 - mu) + a1 * invD;
        R S = a2 - a1 * (a1 * invD);
        S = S > (R)0 ? S : (R)0;
        const R e = fma(c1, S, fma(c2 * vbar, vbar, z));
        if constexpr (std::is_same<R, double>::value) return exp(-e);
        else return exp2_fast(-e);
    }
};

template <typename R>
struct Fn<R, F_LINEAR> {
    R A, s;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*) { A = (R)sc.prm[0]; }
    __device__ __forceinline__ void begin() { s = 0; }
    __device__ __forceinline__ void axis(int, R x) { s = s + x; }
    __device__ __forceinline__ R finish() const { return A * s; }
};

template <typename R>
struct Fn<R, F_ROOS> {
    R A, p;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*) { A = (R)sc.prm[0]; }
    __device__ __forceinline__ void begin() { p = 1; }
    __device__ __forceinline__ void axis(int, R x) { p = p * fabs((R)4 * x - (R)2); }
    __device__ __forceinline__ R finish() const { return A * p; }
};

template <typename R>
struct Fn<R, F_CONST> {
    R A;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*) { A = (R)sc.prm[0]; }
    __device__ __forceinline__ void begin() {}
    __device__ __forceinline__ void axis(int, R) {}
    __device__ __forceinline__ R finish() const { return A; }
};

// Tab. 3 #1: A (sin x_0 + exp x_1); the other axes do not enter
template <typename R>
struct Fn<R, F_SIN_EXP> {
    R A, a, b;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*) { A = (R)sc.prm[0]; }
    __device__ __forceinline__ void begin() { a = 0; b = 0; }
    __device__ __forceinline__ void axis(int d, R x)
    {
        if constexpr (std::is_same<R, double>::value) {
            if (d == 0) a = sin(x);
            else if (d == 1) b = exp(x);
        } else {
            if (d == 0) a = sinf(x);
            else if (d == 1) b = exp2_fast(x * 1.44269504088896341f);
        }
    }
    __device__ __forceinline__ R finish() const { return A * (a + b); }
};

// Tab. 3 #4: A exp(sum_d x_d^2)
template <typename R>
struct Fn<R, F_EXP_SQ> {
    R A, q;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*) { A = (R)sc.prm[0]; }
    __device__ __forceinline__ void begin() { q = 0; }
    __device__ __forceinline__ void axis(int, R x)
    {
        if constexpr (std::is_same<R, double>::value) q = q + x * x;
        else q = fmaf(x, x, q);
    }
    __device__ __forceinline__ R finish() const
    {
        if constexpr (std::is_same<R, double>::value) return A * exp(q);
        else return A * exp2_fast(q * 1.44269504088896341f);
    }
};

// Tab. 3 #6 (Morokoff & Caflisch): A (1 + 1/D)^D prod_d x_d^(1/D).  FP64
// factor by factor with pow; FP32 as 2^(sum_d log2 x_d / D) on the
// hardware log2 and exp2.
template <typename R>
struct Fn<R, F_MOROKOFF> {
    R c, e, p;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*)
    {
        const double D = (double)sc.D;
        c = (R)(sc.prm[0] * pow(1.0 + 1.0 / D, D));
        e = (R)(1.0 / D);
    }
    __device__ __forceinline__ void begin()
    {
        if constexpr (std::is_same<R, double>::value) p = c;
        else p = 0.f;
    }
    __device__ __forceinline__ void axis(int, R x)
    {
        if constexpr (std::is_same<R, double>::value) p = p * pow(x, e);
        else p = p + __builtin_amdgcn_logf(x);
    }
    __device__ __forceinline__ R finish() const
    {
        if constexpr (std::is_same<R, double>::value) return p;
        else return c * exp2_fast(p * e);
    }
};

template <typename R>
struct Fn<R, F_COSINE> {
    R A, p;
    __device__ __forceinline__ void setup(const SampleConst& sc, const R*) { A = (R)sc.prm[0]; }
    __device__ __forceinline__ void begin() { p = 1; }
    __device__ __forceinline__ void axis(int, R x) { p = p * cos(x); }
    __device__ __forceinline__ R finish() const { return A * p; }
};

}  // namespace vg
