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

// log-scale of a moved axis from its raw conditioner output: s = S tanh(a/S)
__device__ __forceinline__ float flow_scale(float a) { return kFlowSMax * tanhf(a * (1.f / kFlowSMax)); }

// Gaussian distribution function and its inverse in FP32 (the device
// library's erfc and erfcinv).  phi_inv takes min(y, 1 - y) separately, so
// that the upper tail keeps its relative precision.
__device__ __forceinline__ float flow_phi(float z)
{
    const float h = 0.5f * erfcf(fabsf(z) * 0.70710678118654752f);
    return z < 0.f ? h : 1.f - h;
}
// Phi^-1(y) from m = min(y, 1 - y) and upper = (y > 1/2): Phi^-1(m) =
// -sqrt(2) erfcinv(2 m) <= 0, and Phi^-1(1 - m) = -Phi^-1(m)
__device__ __forceinline__ float flow_phi_inv(float m, bool upper)
{
    const float z = 1.41421356237309505f * erfcinvf(2.f * m);
    return upper ? z : -z;
}

// ---------------------------------------------------------------------------
// one coupling layer for the 32 samples of a wavefront
// ---------------------------------------------------------------------------
constexpr int kFlowWaves = 4;
constexpr int kFlowThreads = 64 * kFlowWaves;
struct __align__(16) FlowLds {
    __bf16 h[kFlowWaves][32 * kFlowHidden];            // hidden activations [sample][unit]
    float o[kFlowWaves][32 * kFlowOut];                // conditioner outputs [sample][a(8), t(8)]
};

// MLP of layer l for the wave's 32 samples: outputs into ob[sample][16].
// z: the lane's 8 Gaussian coordinates (axes 8 (lane/32) + j of sample
// lane % 32).  h1 goes to hb, h2 to h2b (may be hb); xb (if not null) keeps
// the BF16 product input x [sample][axis].  Called by every lane of the
// workgroup (it synchronises it).
__device__ __forceinline__ void flow_mlp(int l, const float (&z)[8], const float* __restrict__ P,
                                         const bf16x8* __restrict__ pk, __bf16* hb, float* ob,
                                         __bf16* h2b = nullptr, __bf16* xb = nullptr)
{
    if (!h2b) h2b = hb;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int n32 = lane & 31;
    bf16x8 xa;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        xa[j] = flow_in_a(l, 8 * half + j) ? (__bf16)(kFlowXScale * z[j]) : (__bf16)0.f;
    if (xb) *reinterpret_cast<bf16x8*>(xb + n32 * kFlowDim + 8 * half) = xa;
    // h1 = relu(W1 x + b1)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc = {};
        acc = mfma(xa, pk[kPF1 + nt * 64 + lane], acc);
        const float bias = P[kFB1 + nt * 32 + n32];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float v = acc[r] + bias;
            hb[mrow(lane, r) * kFlowHidden + nt * 32 + n32] = (__bf16)(v > 0.f ? v : 0.f);
        }
    }
    __syncthreads();
    // h2 = relu(W2 h1 + b2)
    bf16x8 ha[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) ha[ks] = *reinterpret_cast<const bf16x8*>(hb + n32 * kFlowHidden + ks * 16 + 8 * half);
    f32x16 acc2[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma(ha[ks], pk[kPF2 + (nt * 4 + ks) * 64 + lane], acc);
        acc2[nt] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const float bias = P[kFB2 + nt * 32 + n32];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float v = acc2[nt][r] + bias;
            h2b[mrow(lane, r) * kFlowHidden + nt * 32 + n32] = (__bf16)(v > 0.f ? v : 0.f);
        }
    }
    __syncthreads();
    // outputs = W3 h2 + b3 (columns 16..31 of the product are zero padding)
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) ha[ks] = *reinterpret_cast<const bf16x8*>(h2b + n32 * kFlowHidden + ks * 16 + 8 * half);
    {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma(ha[ks], pk[kPF3 + ks * 64 + lane], acc);
        if (n32 < kFlowOut) {
            const float bias = P[kFB3 + n32];
#pragma unroll
            for (int r = 0; r < 16; ++r) ob[mrow(lane, r) * kFlowOut + n32] = acc[r] + bias;
        }
    }
    __syncthreads();
}

}  // namespace vg
