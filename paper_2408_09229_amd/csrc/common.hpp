// Device building blocks of the VEGAS+ iteration for gfx950.
//
// Philox4x32-10 (Salmon et al., SC'11), the fixed-point stratified point and
// bin index (Sec. 2.1.1 Eq. 3, Sec. 2.1.2), the deterministic log/exp used by
// the map damping and the allocation power, and the built-in integrand
// families (Tab. 3 and the benchmark workloads).
#pragma once
#ifndef __HIPCC_RTC__   // hipRTC provides the HIP device runtime itself
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

#include "layout.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of two 32x32->64 products and an xor/permute,
// Weyl key bumps between rounds.  The key is uniform across a launch, so the
// compiler keeps the schedule in scalar registers.
// ---------------------------------------------------------------------------
struct W4 {
    uint32_t v[4];
};

// Round keys k + r W (r = 0..9) of one launch.  Kept in vector registers:
// as scalars the twenty of them do not fit beside the other uniform values
// and the compiler spills them to VGPR lanes, paying a readlane per use.
struct PhiloxKeys {
    uint32_t k0[10], k1[10];
};

// VG: pin the keys in vector registers (when the kernel has VGPRs to spare).
template <bool VG>
__device__ __forceinline__ PhiloxKeys philox_keys(uint32_t key0, uint32_t key1)
{
    PhiloxKeys K;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = key0 + (uint32_t)r * 0x9E3779B9u;
        const uint32_t b = key1 + (uint32_t)r * 0xBB67AE85u;
        if constexpr (VG) {
            asm volatile("v_mov_b32 %0, %1" : "=v"(K.k0[r]) : "s"(a));
            asm volatile("v_mov_b32 %0, %1" : "=v"(K.k1[r]) : "s"(b));
        } else {
            K.k0[r] = a;
            K.k1[r] = b;
        }
    }
    return K;
}

__device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       const PhiloxKeys& K)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        // three-input xor in one v_bitop3_b32 (truth table 0x96)
        const uint32_t y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, K.k0[r], 0x96);
        const uint32_t y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, K.k1[r], 0x96);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = y0;
        c2 = y2;
    }
    W4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// ---------------------------------------------------------------------------
// Exact division of q < 2^31 by a divisor d < 2^20 with a multiply-high:
// floor(q/d) = (q * M) >> (31 + l), M = ceil(2^(31+l)/d), l = ceil(log2 d).
// The error q*(M - 2^(31+l)/d)/2^(31+l) stays below 2^-l <= 1/d, so the floor
// never moves.  d = 1 is the identity.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t div_magic(uint32_t q, uint32_t magic, int shift)
{
    return shift < 0 ? q : (__umulhi(q, magic) >> shift);
}

// ---------------------------------------------------------------------------
// Stratified point and bin index.  The stratum digit s and the 32-bit word r
// give y = (s + (2r+1)/2^33)/N_st strictly inside (0,1).  Writing
// N_g (2r+1) = a 2^33 + b with a < N_g and q = N_g s + a, the bin is
// i = floor(q/N_st), and the offset inside the bin is
// delta = ((q mod N_st) 2^33 + b) / (N_st 2^33).  Integer-exact up to the
// final rounding of delta; requires N_st N_g < 2^31 and N_st < 2^20.
// ---------------------------------------------------------------------------
struct BinSplit {
    uint32_t bin;
    uint32_t c2;      // 2 (q mod N_st)
    uint32_t p_lo;    // N_g (2r+1) = p_hi 2^32 + p_lo
    uint32_t p_hi;
};

// q is carried doubled, q2 = 2q < 2^32.  Then floor(q / N_st) =
// floor(floor(q2 magic / 2^32) / 2^(shift+1)), the same nested floors as
// umulhi(q, magic) >> shift, and one formula covers N_st = 1 as well (magic
// 2^31, shift -1), so the split has no branch.  The remainder comes back
// doubled too, 2 (q mod N_st) = q2 - bin (2 N_st), in one 24-bit
// multiply-add.
__device__ __forceinline__ BinSplit bin_split(uint32_t s, uint32_t r, uint32_t ng, uint32_t nst,
                                              uint32_t nst_magic, int nst_shift)
{
    // N_g (2r+1) = r (2 N_g) + N_g in one 32x32+64 multiply-add
    const uint64_t P = (uint64_t)r * (2u * ng) + ng;
    BinSplit o;
    o.p_lo = (uint32_t)P;
    o.p_hi = (uint32_t)(P >> 32);
    // 2 floor(P / 2^33) = p_hi with its low bit cleared; N_g, N_st < 2^24
    // and 2 N_g s < 2^32: the 24-bit products are exact
    const uint32_t q2 = __umul24(2u * ng, s) + (o.p_hi & ~1u);
    o.bin = __umulhi(q2, nst_magic) >> (uint32_t)(nst_shift + 1);
    o.c2 = (uint32_t)((int32_t)q2 + __mul24((int32_t)o.bin, -2 * (int32_t)nst));
    return o;
}

// delta = rho / (N_st 2^33) with rho = c 2^33 + (P mod 2^33), rounded once:
// rho 2^-32 = 2c + (P mod 2^33) 2^-32 is exact in FP64 when 2 rho < 2^53,
// and dividing that exact value by 2 N_st rounds once (to the same double as
// rho 2^-33 / N_st).
__device__ __forceinline__ double delta_f64(const BinSplit& p, double nst2_d)
{
    const double b = (double)(p.p_hi & 1u) * 4294967296.0 + (double)p.p_lo;
    const double num2 = (double)p.c2 + b * 0x1p-32;
    return num2 / nst2_d;
}

// FP32 path: delta to float precision from the top 32 of the 33 fractional
// bits, (P mod 2^33) >> 1, with the doubled remainder: fma(frac, 2^-31, 2c)
// is exactly twice fma(frac, 2^-32, c), and half_inv_nst = (1/N_st)/2.
__device__ __forceinline__ float delta_f32(const BinSplit& p, float half_inv_nst)
{
    const uint32_t frac = __builtin_amdgcn_alignbit(p.p_hi, p.p_lo, 1);
    return fmaf((float)frac, 0x1p-31f, (float)p.c2) * half_inv_nst;
}

// ---------------------------------------------------------------------------
// Deterministic log/exp from IEEE +,-,*,/, fma, frexp, ldexp, rint only, so
// that the map and allocation updates reproduce bit for bit on any machine
// following the same order of operations.
//  log x: x = m 2^e with m in [sqrt(1/2), sqrt 2); ln m = 2 atanh(s),
//         s = (m-1)/(m+1), series sum_{k<=11} z^k/(2k+1) in z = s^2 (Horner,
//         fma); result e ln2_hi + (e ln2_lo + 2 s p).
//  exp x: k = rint(x/ln 2), r = (x - k ln2_hi) - k ln2_lo, Taylor series to
//         degree 13 (Horner, fma), scaled by 2^k.
// ln2_hi is ln 2 rounded to double with its low 11 mantissa bits cleared, so
// k ln2_hi is exact for |k| < 2^11; ln2_lo = ln 2 - ln2_hi rounded.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dlog(double x)
{
    if (!(x >= 0.0)) return __builtin_nan("");
    if (x == 0.0) return -__builtin_inf();
    if (__builtin_isinf(x)) return x;
    int e;
    double m = frexp(x, &e);
    if (m < 0x1.6a09e667f3bcdp-1) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
#pragma unroll
    for (int k = 10; k >= 0; --k) p = fma(p, z, 1.0 / (double)(2 * k + 1));
    const double de = (double)e;
    const double hi = de * 0x1.62e42fefa3800p-1;
    const double lo = de * 0x1.ef35793c76730p-45;
    const double tail = (2.0 * s) * p;
    return hi + (lo + tail);
}

__device__ __forceinline__ double dexp(double x)
{
    if (x != x) return x;
    if (x > 709.8) return __builtin_inf();
    if (x < -745.2) return 0.0;
    const double k = rint(x * 0x1.71547652b82fep+0);
    const double r = (x - k * 0x1.62e42fefa3800p-1) - k * 0x1.ef35793c76730p-45;
    double f[14];
    f[0] = 1.0;
#pragma unroll
    for (int j = 1; j < 14; ++j) f[j] = f[j - 1] * (double)j;
    double p = 1.0 / f[13];
#pragma unroll
    for (int j = 12; j >= 0; --j) p = fma(p, r, 1.0 / f[j]);
    return ldexp(p, (int)k);
}

// v^(beta/2): the allocation weight q_h of Eq. 7 (n_h ~ sigma_h^beta with
// sigma_h = sqrt(v_h)).  Square-root chains for the common betas, the
// deterministic exp/log otherwise.
__device__ __forceinline__ double pow_half_beta(double v, double beta)
{
    if (v == 0.0) return 0.0;
    if (beta == 0.75) {
        const double a = sqrt(v);
        const double b = sqrt(a);
        const double c = sqrt(b);
        return b * c;
    }
    if (beta == 1.0) return sqrt(v);
    if (beta == 0.5) return sqrt(sqrt(v));
    if (beta == 2.0) return v;
    return dexp((0.5 * beta) * dlog(v));
}

__host__ __device__ __forceinline__ bool beta_monotone(double beta)
{
    return beta == 0.75 || beta == 1.0 || beta == 0.5 || beta == 2.0;
}

}  // namespace vg
