// Device helpers of the learned warp shared by its sampling and training
// kernels: the BF16 MFMA product and its output layout, the log-scale, the
// Gaussian distribution function, and the conditioner MLP.
#pragma once
#include <hip/hip_runtime.h>

#include "flow.hpp"

namespace vg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma(const bf16x8& a, const bf16x8& b, const f32x16& c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// output layout of the 32x32 product: register r of lane l holds row
// mrow(l, r), column l % 32
__device__ __forceinline__ int mrow(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// log-scale of a moved axis from its raw conditioner output:
// s = S tanh(a/S) = S (1 - 2 / (e^{2a/S} + 1)), from the hardware exp2 and
// reciprocal (a few ulps of S; exact 0 at a = 0, and +-S in the limits)
__device__ __forceinline__ float flow_scale(float a)
{
    const float e = __builtin_amdgcn_exp2f(a * (2.f / kFlowSMax * 1.44269504088896341f));
    return kFlowSMax * fmaf(-2.f, __builtin_amdgcn_rcpf(e + 1.f), 1.f);
}
// e^x for the log-scales, |x| <= S: the hardware exp2 of x log2 e
__device__ __forceinline__ float flow_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// Lower tail h(a) = Phi(-a), a >= 0: h = t 2^(Q(s) - a^2 log2(e) / 2) with
// t = 1 / (1 + 0.4 a), s = 2t - 1, Q a degree-10 polynomial fitted here
// (fit_phi.py).  The exponent's roundings (a^2, its product by log2(e)/2
// with that constant's own remainder, and the difference with Q) are
// carried as the factor 1 + ln2 dy, so the result stays within about 6
// ulps (plus the hardware exp2's and reciprocal's) for all a; beyond
// a = 13.5 it underflows toward 0.
__device__ __forceinline__ float phi_lower(float a)
{
    const float t = __builtin_amdgcn_rcpf(fmaf(0.4f, a, 1.f));
    const float s = fmaf(2.f, t, -1.f);
    float q = -2.496585366e-04f;
    q = fmaf(q, s, 3.146245726e-04f);
    q = fmaf(q, s, 1.360302093e-03f);
    q = fmaf(q, s, -2.809225582e-03f);
    q = fmaf(q, s, -3.100826871e-03f);
    q = fmaf(q, s, 1.396346372e-02f);
    q = fmaf(q, s, 3.256450873e-03f);
    q = fmaf(q, s, -7.306771725e-02f);
    q = fmaf(q, s, -2.237056615e-03f);
    q = fmaf(q, s, 8.854163885e-01f);
    q = fmaf(q, s, -1.822846770e+00f);
    constexpr float kHi = 0.72134752f;                         // log2(e) / 2, rounded
    constexpr float kLo = (float)(0.72134752044448170 - (double)kHi);
    const float sq = a * a;
    const float u = kHi * sq;
    float corr = fmaf(kHi, sq, -u);                            // u's rounding
    corr = fmaf(kHi, fmaf(a, a, -sq), corr);                   // sq's
    corr = fmaf(kLo, sq, corr);                                // the constant's
    const float y = q - u;
    const float ylo = q - (y + u);                             // y's (u >= |q| beyond a = 1.6)
    const float f = fmaf(ylo - corr, 0.69314718f, 1.f);
    return t * __builtin_amdgcn_exp2f(y) * f;
}
// Gaussian distribution function in FP32
__device__ __forceinline__ float flow_phi(float z)
{
    const float h = phi_lower(fabsf(z));
    return z < 0.f ? h : 1.f - h;
}

// Phi^-1(m) = -sqrt(2) erfinv(1 - 2m) <= 0 for 0 < m <= 1/2, in M. Giles'
// two-piece form ("Approximating the erfinv function", GPU Computing Gems,
// 2011): erfinv(x) = x p(w) with w = -ln(4m(1 - m)) = -ln(1 - x^2), p a
// polynomial in w - 2.5 for w < 5 and in sqrt(w) - 3 for 5 <= w <= 16.2
// (m >= 1e-7).  The coefficients are fitted here (fit_phi.py): within
// 2.1e-7 relative (3.5 ulps) over that range.  Below m = 1e-7 (a rare,
// divergent branch) the device library's erfcinv takes over.
__device__ __forceinline__ float phi_inv_lower(float m)
{
    if (m < 1e-7f) return -1.41421356237309505f * erfcinvf(2.f * m);
    const float w = -0.693147180559945309f * __builtin_amdgcn_logf(4.f * m * (1.f - m));
    float p;
    if (w < 5.f) {
        const float t = w - 2.5f;
        p = 2.859876425e-08f;
        p = fmaf(p, t, 3.433422080e-07f);
        p = fmaf(p, t, -3.529890137e-06f);
        p = fmaf(p, t, -4.392980372e-06f);
        p = fmaf(p, t, 2.186072816e-04f);
        p = fmaf(p, t, -1.253717928e-03f);
        p = fmaf(p, t, -4.177715629e-03f);
        p = fmaf(p, t, 2.466407269e-01f);
        p = fmaf(p, t, 1.501409411e+00f);
    } else {
        const float t = __builtin_amdgcn_sqrtf(w) - 3.f;
        p = -1.941565133e-04f;
        p = fmaf(p, t, 1.017520699e-04f);
        p = fmaf(p, t, 1.340063871e-03f);
        p = fmaf(p, t, -3.675155109e-03f);
        p = fmaf(p, t, 5.743755959e-03f);
        p = fmaf(p, t, -7.621584926e-03f);
        p = fmaf(p, t, 9.438302368e-03f);
        p = fmaf(p, t, 1.001674056e+00f);
        p = fmaf(p, t, 2.832976818e+00f);
    }
    return -1.41421356237309505f * p * (1.f - 2.f * m);
}
// Phi^-1(y) from m = min(y, 1 - y) and upper = (y > 1/2), by the symmetry
// Phi^-1(1 - m) = -Phi^-1(m), so that the upper tail keeps its relative
// precision
__device__ __forceinline__ float flow_phi_inv(float m, bool upper)
{
    const float z = phi_inv_lower(m);
    return upper ? -z : z;
}

// ---------------------------------------------------------------------------
// operand packing
// ---------------------------------------------------------------------------
// Entry r of layer l's packed operands (flow.hpp) from the layer's FP32
// parameters P (global memory or LDS).
__device__ inline bf16x8 flow_pack_entry(int l, int r, const float* __restrict__ P)
{
    bf16x8 o;
    for (int j = 0; j < 8; ++j) {
        const int src = flow_pack_src(l, r, j);
        o[j] = (__bf16)(src >= 0 ? P[src] : src == -2 ? 1.f : 0.f);
    }
    return o;
}

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------
constexpr int kFlowWaves = 4;
constexpr int kFlowThreads = 64 * kFlowWaves;
constexpr int kFlowSampleWaves = 8;                    // the sampling pass: independent waves
constexpr int kFlowSampleThreads = 64 * kFlowSampleWaves;
// ---------------------------------------------------------------------------
// the conditioner MLP with the samples as columns
// ---------------------------------------------------------------------------
// The products run as W . act^T, so each one's output registers (register r
// of lane l: unit 8 (r/4) + 4 (l/32) + r % 4 of its tile, sample l % 32) are
// the next one's B operand as they stand, with the weights' k order packed
// to match (T2, T3).  Nothing passes through LDS between the products and
// no barrier is needed; the forward weights of all layers are staged in LDS
// once per workgroup.
struct __align__(16) FlowFwdLds {
    bf16x8 w[kFlowLayers][kPFwdT];                         // F1, T2, T3
    float b[kFlowLayers][2 * kFlowHidden + kFlowOut];      // b1, b2, b3
};

// Copies the forward operands and biases into LDS (every thread of the
// workgroup takes part; the caller synchronises afterwards).
__device__ __forceinline__ void flow_stage_fwd(FlowFwdLds& S, const bf16x8* __restrict__ pk,
                                               const float* __restrict__ theta)
{
    for (int e = threadIdx.x; e < kFlowLayers * kPFwdT; e += blockDim.x) {
        const int l = e / kPFwdT;
        const int r = e - l * kPFwdT;
        // F1 first, then T2 and T3, which are adjacent in the packed layer
        S.w[l][r] = pk[(size_t)l * kPLayer + (r < 2 * 64 ? kPF1 + r : kPT2 + (r - 2 * 64))];
    }
    constexpr int nb = 2 * kFlowHidden + kFlowOut;
    for (int e = threadIdx.x; e < kFlowLayers * nb; e += blockDim.x) {
        const int l = e / nb;
        const int r = e - l * nb;
        const int src = r < kFlowHidden ? kFB1 + r : r < 2 * kFlowHidden ? kFB2 + (r - kFlowHidden)
                                                                         : kFB3 + (r - 2 * kFlowHidden);
        S.b[l][r] = theta[(size_t)l * kFLayer + src];
    }
}

// the 8 values of register-order k-step q of a product's output (registers
// 8 (q % 2) .. + 7 of tile q / 2), through relu, as a BF16 operand
// 8 FP32 values to BF16 (round to nearest even), two per instruction
__device__ __forceinline__ bf16x8 cvt_bf16x8(float v0, float v1, float v2, float v3, float v4, float v5, float v6,
                                             float v7)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const f32x2 a = {v0, v1}, b = {v2, v3}, c = {v4, v5}, d = {v6, v7};
    const u32x4 w = {__builtin_bit_cast(unsigned, __builtin_convertvector(a, bf16x2)),
                     __builtin_bit_cast(unsigned, __builtin_convertvector(b, bf16x2)),
                     __builtin_bit_cast(unsigned, __builtin_convertvector(c, bf16x2)),
                     __builtin_bit_cast(unsigned, __builtin_convertvector(d, bf16x2))};
    return __builtin_bit_cast(bf16x8, w);
}

// registers 8 q2 .. + 7 of a product's output as BF16
__device__ __forceinline__ bf16x8 to_bf16(const f32x16& acc, int q2)
{
    const int b = 8 * q2;
    return cvt_bf16x8(acc[b], acc[b + 1], acc[b + 2], acc[b + 3], acc[b + 4], acc[b + 5], acc[b + 6], acc[b + 7]);
}

__device__ __forceinline__ bf16x8 relu_bf16(const f32x16& acc, int q2)
{
    const bf16x8 o = to_bf16(acc, q2);
    // relu on the rounded values' bit patterns, two per instruction: a BF16
    // with its sign bit set is a negative 16-bit integer (-0 included), so
    // max(v, 0) as integers maps it to +0 and keeps every positive value
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 zero = {};
    const s16x8 v = __builtin_elementwise_max(__builtin_bit_cast(s16x8, o), zero);
    return __builtin_bit_cast(bf16x8, v);
}

// start of an accumulator with the bias of the product's rows: register
// group q holds rows 32 tile + 8 q + 4 half + 0..3, contiguous in the bias
__device__ __forceinline__ f32x16 bias_rows(const float* __restrict__ b, int half)
{
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = *reinterpret_cast<const float4*>(b + 8 * q + 4 * half);
        acc[4 * q] = v.x;
        acc[4 * q + 1] = v.y;
        acc[4 * q + 2] = v.z;
        acc[4 * q + 3] = v.w;
    }
    return acc;
}

// Conditioner of layer L for the wave's 32 samples; lane l holds axes
// 8 (l/32) + j of sample l % 32 in z.  W: the layer's packed operands (F1,
// T2, T3 first), B: its biases b1, b2, b3.  Returns the last product's
// registers: j < 8 the raw log-scale of the lane's axis j, 8 + j its shift
// (meaningful where that axis moves in layer L).  x, h1 and h2 receive the
// BF16 product inputs (register order, after relu).
template <int L>
__device__ __forceinline__ f32x16 flow_mlp_t(const float (&z)[8], const bf16x8* __restrict__ W,
                                             const float* __restrict__ B, bf16x8& x, bf16x8 (&h1)[4],
                                             bf16x8 (&h2)[4])
{
    // the weights in LDS do not change inside the callers' loops: this
    // compiler-only fence keeps their loads here instead of hoisted (and
    // held in registers) across all layers and iterations
    __asm__ volatile("" ::: "memory");
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    float xs[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) xs[j] = flow_reg_in_a(L, j) ? kFlowXScale * z[j] : 0.f;
    x = cvt_bf16x8(xs[0], xs[1], xs[2], xs[3], xs[4], xs[5], xs[6], xs[7]);
    // h1 = relu(W1 x + b1)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = bias_rows(B + 32 * mt, half);
        acc = mfma(W[kPF1 + mt * 64 + lane], x, acc);
        h1[2 * mt] = relu_bf16(acc, 0);
        h1[2 * mt + 1] = relu_bf16(acc, 1);
    }
    // h2 = relu(W2 h1 + b2)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = bias_rows(B + kFlowHidden + 32 * mt, half);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma(W[kPT2 + (mt * 4 + ks) * 64 + lane], h1[ks], acc);
        h2[2 * mt] = relu_bf16(acc, 0);
        h2[2 * mt + 1] = relu_bf16(acc, 1);
    }
    // outputs = W3 h2 + b3, rows placed by flow_t3_row
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int o = flow_t3_row(L, mrow(lane, r));
        acc[r] = o >= 0 ? B[2 * kFlowHidden + o] : 0.f;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = mfma(W[kPT3 + ks * 64 + lane], h2[ks], acc);
    return acc;
}

template <int L>
__device__ __forceinline__ f32x16 flow_mlp_t(const float (&z)[8], const FlowFwdLds& S)
{
    bf16x8 x, h1[4], h2[4];
    return flow_mlp_t<L>(z, S.w[L], S.b[L], x, h1, h2);
}

// Forward coupling layer L on the lane's axes: z_B -> z_B e^s + t; adds the
// log-scales to lj.
template <int L>
__device__ __forceinline__ void flow_layer_fwd(float (&z)[8], float& lj, const FlowFwdLds& S)
{
    const f32x16 o = flow_mlp_t<L>(z, S);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (flow_reg_in_a(L, j)) continue;
        const float s = flow_scale(o[j]);
        z[j] = fmaf(z[j], flow_exp(s), o[8 + j]);
        lj += s;
    }
}

// Inverse coupling layer L: u_B -> (u_B - t) e^-s.
template <int L>
__device__ __forceinline__ void flow_layer_inv(float (&z)[8], const FlowFwdLds& S)
{
    const f32x16 o = flow_mlp_t<L>(z, S);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (flow_reg_in_a(L, j)) continue;
        const float s = flow_scale(o[j]);
        z[j] = (z[j] - o[8 + j]) * flow_exp(-s);
    }
}

}  // namespace vg
