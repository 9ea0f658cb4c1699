// Training of the learned warp on the samples of one iteration.
//
// Loss L = sum_k c_k log J_F(F^-1(w_k)) with c_k = |omega_k|^gamma / sum
// |omega|^gamma.  gamma = 2: its gradient is a positive multiple of the
// gradient of the estimator's variance (the warp's density at w is
// 1 / J_F(F^-1(w))); gamma = 1: of the KL divergence from the normalised
// |f| to the warp's density, whose sample gradient has lighter tails.  The
// gradient goes through the inverse chain in Gaussian coordinates,
// u_4 = z_4 -> u_3 -> u_2 -> u_1 -> u_0, where log J_F depends on the
// parameters through each layer's log-scales and through u_0 (the term
// u_0^2 / 2):
//   k_flow_sumsq    sum of |omega|^gamma (block partials, then in order)
//   k_flow_inverse  u_3, u_2, u_1 of every training sample (MLP on MFMA) and
//                   the upstream gradient dL/du_0 = c u_0
//   k_flow_grad     the coupling layers l = 0..3 in turn: from g = dL/du_l,
//                   the layer's log-scales and inverse transform give
//                   dL/d(a, t); the MLP backward runs on MFMA (dO W3, dA2 W2,
//                   dA1 W1); the weight gradients dW = sum_samples delta^T
//                   activation are MFMA products over the workgroup's 128
//                   samples, each wave owning some output tiles,
//                   accumulated across the workgroup's chunks
//   k_flow_reduce   per-workgroup gradients summed in a fixed order, and
//                   Adam on the FP32 parameters (then the BF16 repack)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "flow.hpp"
#include "flow_dev.hpp"
#include "launch.hpp"

namespace vg {

constexpr int kSumThreads = 256;
constexpr int kSumBlocks = 256;

// sum of |omega|^gamma, gamma = 2 (variance loss) or 1 (KL loss): block
// partials (strided samples), then the partials in block order
__global__ __launch_bounds__(kSumThreads) void k_flow_sumsq(const float* om, uint32_t n, uint32_t stride, uint32_t off,
                                                            int gamma, double* part)
{
    __shared__ double red[kSumThreads];
    double s = 0.0;
    for (uint32_t i = blockIdx.x * kSumThreads + threadIdx.x; i < n; i += kSumThreads * kSumBlocks) {
        const double v = fabs((double)om[(size_t)off + (size_t)i * stride]);
        s += gamma == 2 ? v * v : v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[1 + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kSumThreads) void k_flow_sumsq_final(double* part)
{
    __shared__ double red[kSumThreads];
    red[threadIdx.x] = threadIdx.x < kSumBlocks ? part[1 + threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[0] = red[0];
}

// ---------------------------------------------------------------------------
// inverse pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load8(const float* p, float (&v)[8])
{
    const float4* q = reinterpret_cast<const float4*>(p);
    const float4 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ __forceinline__ void store8(float* p, const float (&v)[8])
{
    float4* q = reinterpret_cast<float4*>(p);
    q[0] = make_float4(v[0], v[1], v[2], v[3]);
    q[1] = make_float4(v[4], v[5], v[6], v[7]);
}

// c_k of a training sample in double, rounded to FP32: tiny weights (an
// integrand that underflows almost everywhere) put 1/sum beyond FP32
__device__ __forceinline__ float train_coef(const FlowTrainArgs& a, uint32_t k, bool valid)
{
    const double ss = *a.sumsq;
    const double inv_ss = ss > 0.0 && ss < INFINITY ? 1.0 / ss : 0.0;
    const double om = valid ? fabs((double)a.om[(size_t)a.off + (size_t)k * a.stride]) : 0.0;
    return (float)((a.gamma == 2 ? om * om : om) * inv_ss);
}

__global__ __launch_bounds__(kFlowSampleThreads) void k_flow_inverse(FlowTrainArgs a)
{
    __shared__ FlowFwdLds S;
    flow_stage_fwd(S, reinterpret_cast<const bf16x8*>(a.packed), a.theta);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int n32 = lane & 31;
    const uint32_t N = a.n;
    const uint32_t chunks = (N + 31u) / 32u;
    const uint32_t n_waves = gridDim.x * kFlowSampleWaves;
    // waves run independently: no barrier inside the loop
    for (uint32_t chunk = blockIdx.x * kFlowSampleWaves + (threadIdx.x >> 6); chunk < chunks; chunk += n_waves) {
        const uint32_t k = min(chunk * 32u + (uint32_t)n32, N - 1u);
        const bool valid = chunk * 32u + (uint32_t)n32 < N;
        float z[8];
        load8(a.zf + ((size_t)a.off + (size_t)k * a.stride) * kFlowDim + 8 * half, z);
        float* U = a.U + (size_t)k * kFlowDim + 8 * half;
        const size_t lay = (size_t)N * kFlowDim;
        flow_layer_inv<3>(z, S);
        if (valid) store8(U + 2 * lay, z);
        flow_layer_inv<2>(z, S);
        if (valid) store8(U + lay, z);
        flow_layer_inv<1>(z, S);
        if (valid) store8(U, z);
        flow_layer_inv<0>(z, S);
        // dL/du_0 = c u_0 (the term u_0^2 / 2 of log J_F)
        if (valid) {
            const float c = train_coef(a, k, true);
            float g[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) g[j] = c * z[j];
            store8(a.g_out + (size_t)k * kFlowDim + 8 * half, g);
        }
    }
}

// ---------------------------------------------------------------------------
// backward pass of one coupling layer
// ---------------------------------------------------------------------------
struct __align__(16) FlowGradLds {
    float o[kFlowWaves][32 * kFlowOut];                // conditioner outputs, then dL/d(a, t) (FP32)
    __bf16 h1[kFlowWaves][32 * kFlowHidden];
    __bf16 h2[kFlowWaves][32 * kFlowHidden];
    __bf16 da2[kFlowWaves][32 * kFlowHidden];
    __bf16 da1[kFlowWaves][32 * kFlowHidden];
    __bf16 x[kFlowWaves][32 * kFlowDim];
    float dx[kFlowWaves][32 * 32];
    float red[2][kFlowWaves][kFlowHidden];
};

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__global__ __launch_bounds__(kFlowThreads) void k_flow_grad(FlowTrainArgs a)
{
    __shared__ FlowGradLds S;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int n32 = lane & 31;
    const uint32_t N = a.n;
    const uint32_t chunks = (N + 31u) / 32u;
    const uint32_t per_round = gridDim.x * kFlowWaves;
    const uint32_t rounds = (chunks + per_round - 1u) / per_round;
    // dL/du_l passes between the layers through two buffers: the inverse
    // pass left dL/du_0 in g_in; a sample's gradient is written and read
    // again by the same lane, as every layer maps chunks to waves alike
    float* const gbuf[2] = {const_cast<float*>(a.g_in), a.g_out};
    for (int l = 0; l < kFlowLayers; ++l) {
        const float* g_in = gbuf[l & 1];
        float* g_out = gbuf[(l & 1) ^ 1];
        const float* P = a.theta + (size_t)l * kFLayer;
        const bf16x8* pk = reinterpret_cast<const bf16x8*>(a.packed) + (size_t)l * kPLayer;
        // the layer's input in the inverse direction, u_{l+1}: z_4 itself for
        // the last layer (at the training samples), else the inverse pass's
        // compact output
        const bool from_z = l == kFlowLayers - 1;
        const float* uin = from_z ? a.zf : a.U + (size_t)l * N * kFlowDim;
        f32x16 acc3 = {}, acc2 = {}, acc1 = {};
        float db3 = 0.f, db2[2] = {0.f, 0.f}, db1[2] = {0.f, 0.f};
        for (uint32_t rd = 0; rd < rounds; ++rd) {
            const uint32_t chunk = rd * per_round + blockIdx.x * kFlowWaves + wave;
            const bool live = chunk < chunks;
            const uint32_t k = live ? min(chunk * 32u + (uint32_t)n32, N - 1u) : 0u;
            const bool valid = live && chunk * 32u + (uint32_t)n32 < N;
            float u[8], g[8];
            load8(uin + (from_z ? (size_t)a.off + (size_t)k * a.stride : (size_t)k) * kFlowDim + 8 * half, u);
            if (valid) {
                load8(g_in + (size_t)k * kFlowDim + 8 * half, g);
            } else {
    #pragma unroll
                for (int j = 0; j < 8; ++j) g[j] = 0.f;
            }
            const float coef = train_coef(a, k, valid);

            // ---- recompute the conditioner of this layer -----------------------
            flow_mlp(l, u, P, pk, S.h1[wave], S.o[wave], S.h2[wave], S.x[wave]);

            // ---- inverse transform and log-scale: dL/d(a, t) -------------------
            // u_l,B = (u_{l+1},B - t) e^-s: dL/ds = c - g_B u_l,B (the log-scale
            // is a term of log J_F), dL/dt = -g_B e^-s, dL/du_{l+1},B = g_B e^-s;
            // s = S tanh(a/S), ds/da = 1 - (s/S)^2
            float gn[8];
    #pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c = 8 * half + j;
                gn[j] = g[j];
                if (flow_in_a(l, c)) continue;
                float* ob = S.o[wave] + n32 * kFlowOut + flow_pos(l, c);
                const float s = flow_scale(ob[0]);
                const float es = expf(-s);
                const float ub = (u[j] - ob[kFlowHalf]) * es;
                const float ds = valid ? coef - g[j] * ub : 0.f;
                const float rs = s * (1.f / kFlowSMax);
                ob[0] = ds * (1.f - rs * rs);
                ob[kFlowHalf] = -g[j] * es;
                gn[j] = g[j] * es;
            }
            __syncthreads();

            // ---- dH2 = dO W3; dA2 = dH2 (h2 > 0) -------------------------------
            {
                f32x16 t[2] = {};
                const float* orow = S.o[wave] + n32 * kFlowOut + 8 * half;
                bf16x8 av;
    #pragma unroll
                for (int j = 0; j < 8; ++j) av[j] = (__bf16)orow[j];
    #pragma unroll
                for (int nt = 0; nt < 2; ++nt) t[nt] = mfma(av, pk[kPR3 + nt * 64 + lane], t[nt]);
    #pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
    #pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int idx = mrow(lane, r) * kFlowHidden + nt * 32 + n32;
                        const float d = (float)S.h2[wave][idx] > 0.f ? t[nt][r] : 0.f;
                        db2[nt] += d;
                        S.da2[wave][idx] = (__bf16)d;
                    }
                }
            }
            __syncthreads();

            // ---- dH1 = dA2 W2; dA1 = dH1 (h1 > 0) ------------------------------
            {
                f32x16 t[2] = {};
    #pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const bf16x8 av = ld8(S.da2[wave] + n32 * kFlowHidden + ks * 16 + 8 * half);
    #pragma unroll
                    for (int nt = 0; nt < 2; ++nt) t[nt] = mfma(av, pk[kPR2 + (nt * 4 + ks) * 64 + lane], t[nt]);
                }
    #pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
    #pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int idx = mrow(lane, r) * kFlowHidden + nt * 32 + n32;
                        const float d = (float)S.h1[wave][idx] > 0.f ? t[nt][r] : 0.f;
                        db1[nt] += d;
                        S.da1[wave][idx] = (__bf16)d;
                    }
                }
            }
            __syncthreads();

            // ---- dX = dA1 W1 (columns = axes) ---------------------------------
            {
                f32x16 t = {};
    #pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    t = mfma(ld8(S.da1[wave] + n32 * kFlowHidden + ks * 16 + 8 * half), pk[kPR1 + ks * 64 + lane], t);
    #pragma unroll
                for (int r = 0; r < 16; ++r) S.dx[wave][mrow(lane, r) * 32 + n32] = t[r];
            }
            __syncthreads();

            // ---- dL/du_{l+1}: conditioning axes add the MLP's input gradient ----
    #pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c = 8 * half + j;
                if (flow_in_a(l, c)) gn[j] = g[j] + kFlowXScale * S.dx[wave][n32 * 32 + c];
            }
            if (valid) store8(g_out + (size_t)k * kFlowDim + 8 * half, gn);

            // ---- weight gradients over the workgroup's 128 samples ------------
            // dW3[o][h] += sum_s dO[s][o] h2[s][h]: one 32-row tile (rows o < 16
            // used), waves 0 and 1 take the two column tiles
            if (wave < 2) {
    #pragma unroll 1
                for (int ks = 0; ks < 8; ++ks) {
                    const int ws = ks >> 1;
                    const int s0 = (ks & 1) * 16 + 8 * half;
                    bf16x8 av, bv;
    #pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        av[j] = n32 < kFlowOut ? (__bf16)S.o[ws][(s0 + j) * kFlowOut + n32] : (__bf16)0.f;
                        bv[j] = S.h2[ws][(s0 + j) * kFlowHidden + wave * 32 + n32];
                    }
                    acc3 = mfma(av, bv, acc3);
                }
            }
            // dW2[n2][n1] += sum_s dA2[s][n2] h1[s][n1]: one tile per wave
            {
                const int mt = wave >> 1, nt = wave & 1;
    #pragma unroll 1
                for (int ks = 0; ks < 8; ++ks) {
                    const int ws = ks >> 1;
                    const int s0 = (ks & 1) * 16 + 8 * half;
                    bf16x8 av, bv;
    #pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        av[j] = S.da2[ws][(s0 + j) * kFlowHidden + mt * 32 + n32];
                        bv[j] = S.h1[ws][(s0 + j) * kFlowHidden + nt * 32 + n32];
                    }
                    acc2 = mfma(av, bv, acc2);
                }
            }
            // dW1[h][axis] += sum_s dA1[s][h] x[s][axis]: waves 2 and 3
            if (wave >= 2) {
                const int mt = wave - 2;
    #pragma unroll 1
                for (int ks = 0; ks < 8; ++ks) {
                    const int ws = ks >> 1;
                    const int s0 = (ks & 1) * 16 + 8 * half;
                    bf16x8 av, bv;
    #pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        av[j] = S.da1[ws][(s0 + j) * kFlowHidden + mt * 32 + n32];
                        bv[j] = n32 < kFlowDim ? S.x[ws][(s0 + j) * kFlowDim + n32] : (__bf16)0.f;
                    }
                    acc1 = mfma(av, bv, acc1);
                }
            }
            // db3: one output per thread, FP32
            if (threadIdx.x < kFlowOut) {
                for (int ws = 0; ws < kFlowWaves; ++ws)
                    for (int s = 0; s < 32; ++s) db3 += S.o[ws][s * kFlowOut + threadIdx.x];
            }
            __syncthreads();
        }

        // ---- this workgroup's gradient of layer l ------------------------------
        float* out = a.part + (size_t)blockIdx.x * kFParams + (size_t)l * kFLayer;
        if (wave < 2) {
    #pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int o = mrow(lane, r);
                if (o < kFlowOut) out[kFW3 + o * kFlowHidden + wave * 32 + n32] = acc3[r];
            }
        }
        {
            const int mt = wave >> 1, nt = wave & 1;
    #pragma unroll
            for (int r = 0; r < 16; ++r)
                out[kFW2 + (mt * 32 + mrow(lane, r)) * kFlowHidden + nt * 32 + n32] = acc2[r];
        }
        if (wave >= 2 && n32 < kFlowDim && flow_in_a(l, n32)) {
    #pragma unroll
            for (int r = 0; r < 16; ++r)
                out[kFW1 + ((wave - 2) * 32 + mrow(lane, r)) * kFlowHalf + flow_pos(l, n32)] = acc1[r];
        }
        if (threadIdx.x < kFlowOut) out[kFB3 + threadIdx.x] = db3;
    #pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            db2[nt] += __shfl_xor(db2[nt], 32, 64);
            db1[nt] += __shfl_xor(db1[nt], 32, 64);
            if (half == 0) {
                S.red[0][wave][nt * 32 + n32] = db2[nt];
                S.red[1][wave][nt * 32 + n32] = db1[nt];
            }
        }
        __syncthreads();
        if (threadIdx.x < kFlowHidden) {
            float s2 = 0.f, s1 = 0.f;
            for (int w = 0; w < kFlowWaves; ++w) {
                s2 += S.red[0][w][threadIdx.x];
                s1 += S.red[1][w][threadIdx.x];
            }
            out[kFB2 + threadIdx.x] = s2;
            out[kFB1 + threadIdx.x] = s1;
        }
        // S.red and the activations are reused by the next layer
        __syncthreads();
    }
}

// per-workgroup gradients summed in a fixed order: segments of consecutive
// workgroups first (one thread per parameter and segment), then the
// segments in order
constexpr int kRedSegs = 16;

__global__ void k_flow_reduce_seg(const float* part, int n_wg, float* seg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kFParams) return;
    const int per = (n_wg + kRedSegs - 1) / kRedSegs;
    const int w0 = blockIdx.y * per;
    const int w1 = min(w0 + per, n_wg);
    float s = 0.f;
    for (int w = w0; w < w1; ++w) s += part[(size_t)w * kFParams + i];
    seg[(size_t)blockIdx.y * kFParams + i] = s;
}

__device__ __forceinline__ void adam_update(float* theta, float* m, float* v, int i, float gi, float lr, float c1,
                                            float c2)
{
    const float mi = fmaf(0.9f, m[i], 0.1f * gi);
    const float vi = fmaf(0.999f, v[i], 0.001f * gi * gi);
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// the segments in order into grad; with theta set, the Adam step too
__global__ void k_flow_reduce(const float* seg, float* grad, float* theta, float* m, float* v, float lr, float c1,
                              float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kFParams) return;
    float s = 0.f;
    for (int g = 0; g < kRedSegs; ++g) s += seg[(size_t)g * kFParams + i];
    grad[i] = s;
    if (theta) adam_update(theta, m, v, i, s, lr, c1, c2);
}

__global__ void k_flow_adam(float* theta, const float* grad, float* m, float* v, float lr, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kFParams) return;
    adam_update(theta, m, v, i, grad[i], lr, c1, c2);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
// Adam's bias corrections in double: 1 - 0.999^t in FP32 (from the FP32
// constant 0.999f) is off by 1.3e-5 relative at t = 1
void adam_corrections(int step, float* c1, float* c2)
{
    *c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)step)));
    *c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)step)));
}
}  // namespace

hipError_t launch_flow_gradient(const FlowTrainArgs& base, int n_wg, float* G0, float* G1, float* grad,
                                float* seg, const FlowAdamArgs* adam, hipStream_t st)
{
    double* ss = const_cast<double*>(base.sumsq);
    hipLaunchKernelGGL(k_flow_sumsq, dim3(kSumBlocks), dim3(kSumThreads), 0, st, base.om, base.n, base.stride,
                       base.off, base.gamma, ss);
    hipLaunchKernelGGL(k_flow_sumsq_final, dim3(1), dim3(kSumThreads), 0, st, ss);
    // the inverse pass writes u_1..u_3 and dL/du_0 (into G1); then every
    // layer's backward pass in one launch, alternating G1 and G0
    FlowTrainArgs a = base;
    a.g_in = G1;
    a.g_out = G1;
    hipLaunchKernelGGL(k_flow_inverse, dim3(2 * n_wg), dim3(kFlowSampleThreads), 0, st, a);
    a.g_out = G0;
    hipLaunchKernelGGL(k_flow_grad, dim3(n_wg), dim3(kFlowThreads), 0, st, a);
    hipLaunchKernelGGL(k_flow_reduce_seg, dim3((kFParams + 255) / 256, kRedSegs), dim3(256), 0, st,
                       (const float*)a.part, n_wg, seg);
    float c1 = 0.f, c2 = 0.f;
    if (adam) adam_corrections(adam->step, &c1, &c2);
    hipLaunchKernelGGL(k_flow_reduce, dim3((kFParams + 255) / 256), dim3(256), 0, st, (const float*)seg, grad,
                       adam ? adam->theta : nullptr, adam ? adam->m : nullptr, adam ? adam->v : nullptr,
                       adam ? adam->lr : 0.f, c1, c2);
    return hipGetLastError();
}

hipError_t launch_flow_adam(float* theta, const float* grad, float* m, float* v, float lr, int step, hipStream_t st)
{
    float c1, c2;
    adam_corrections(step, &c1, &c2);
    hipLaunchKernelGGL(k_flow_adam, dim3((kFParams + 255) / 256), dim3(256), 0, st, theta, grad, m, v, lr, c1, c2);
    return hipGetLastError();
}

}  // namespace vg
