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
//   k_flow_sumsq    sum of |omega|^gamma (block partials; the gradient
//                   kernel adds them in order)
//   k_flow_grad     first the inverse pass: u_3, u_2, u_1 of the
//                   workgroup's training samples (MLP on MFMA) and the
//                   upstream gradient dL/du_0 = c u_0; then the coupling
//                   layers l = 0..3 in turn: from g = dL/du_l, the layer's
//                   log-scales and inverse transform give dL/d(a, t); the
//                   MLP backward and the weight gradients dW = sum_samples
//                   delta^T activation run on MFMA with every activation
//                   and delta in registers, each wave summing its samples,
//                   the waves added in LDS
//   k_flow_update   per-workgroup gradients summed in a fixed order, Adam
//                   on the FP32 parameters, and each weight's two BF16
//                   copies in the packed operands written in place (the
//                   full repack, k_flow_pack in flow.hip, runs when the
//                   parameters are set)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

#include "flow.hpp"
#include "flow_dev.hpp"
#include "launch.hpp"

namespace vg {

constexpr int kSumThreads = 256;
constexpr int kSumBlocks = kFlowSumBlocks;

// sum of |omega|^gamma, gamma = 2 (variance loss) or 1 (KL loss), over the
// samples off, off + stride, ... of each slice y = blockIdx.y (off =
// (off0 + y) mod stride): block partials (strided samples) into
// part[y kFlowSumRecord + 1 + block], which the gradient kernel adds in
// block order
__global__ __launch_bounds__(kSumThreads) void k_flow_sumsq(const float* om, uint32_t n_eval, uint32_t stride,
                                                            uint32_t off0, int gamma, double* part)
{
    __shared__ double red[kSumThreads];
    const uint32_t off = (off0 + blockIdx.y) % stride;
    const uint32_t n = (n_eval - off + stride - 1) / stride;
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
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * kFlowSumRecord + 1 + blockIdx.x] = red[0];
}

// c_k of a training sample in double, rounded to FP32: tiny weights (an
// integrand that underflows almost everywhere) put 1/sum beyond FP32
__device__ __forceinline__ float train_coef(const FlowTrainArgs& a, uint32_t k, bool valid, double ss)
{
    const double inv_ss = ss > 0.0 && ss < INFINITY ? 1.0 / ss : 0.0;
    const double om = valid ? fabs((double)a.om[(size_t)a.off + (size_t)k * a.stride]) : 0.0;
    return (float)((a.gamma == 2 ? om * om : om) * inv_ss);
}

// ---------------------------------------------------------------------------
// backward pass of the coupling layers
// ---------------------------------------------------------------------------
// Per wave and 32 samples, all in registers: the conditioner forward with
// samples as columns (h1, h2 and the outputs in register order); the inverse
// transform's derivatives per lane; the deltas back through the MLP with
// samples as columns (U3, U2, U1), which give the next dL/du in the lanes of
// their axes; the same activations and deltas with samples as rows (the
// column products read as B operands, and the 0/1 products P and I), whose
// output registers hold 16 samples per lane; and the weight gradients as
// products over samples with both operands in that layout.  Each wave sums
// its samples' gradients in registers; at the end of a layer the waves add
// theirs in LDS and the workgroup writes its part.
struct __align__(16) FlowBwdLds {
    bf16x8 w[kPLayer];                         // this layer's operands
    float b[2 * kFlowHidden + kFlowOut];       // b1, b2, b3
    union {
        float red[kFlowWaves][kFLayer];        // per-wave gradients of the layer
        FlowFwdLds fwd;                        // the inverse pass: every layer's forward operands
    };
    double sum[kSumThreads];                   // the total of the sums' block partials
};
static_assert(kFlowThreads == kSumThreads, "one partial per thread");

// sum of a lane's 16 registers
__device__ __forceinline__ float reg_sum(const f32x16& a)
{
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) s += a[r];
    return s;
}

// relu mask of a register-order tile: where the activation (BF16, k-steps
// 2 t and 2 t + 1 of a register-order input) is positive.  The activations
// come out of relu_bf16, so each is +0 or positive: positive exactly where
// its 16 bits are not zero (one 16-bit compare, no conversion to FP32).
__device__ __forceinline__ void mask_by(f32x16& d, const bf16x8& a0, const bf16x8& a1)
{
    typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
    const u16x8 b0 = __builtin_bit_cast(u16x8, a0), b1 = __builtin_bit_cast(u16x8, a1);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (b0[i] == 0) d[i] = 0.f;
        if (b1[i] == 0) d[8 + i] = 0.f;
    }
}

// per-wave gradient of one layer, in registers
struct LayerGrad {
    f32x16 w3[2];          // dW3[o][32 nt + column], rows o < 16
    f32x16 w2[2][2];       // dW2[32 mt + row][32 nt + column]
    f32x16 w1[2];          // dW1[32 mt + row][axis = column]
    float b3, b2[2], b1[2];
};

// one layer's backward pass for the wave's 32 samples; g holds dL/du_l of
// the lane's axes and receives dL/du_{l+1}.  FIRST: the wave's first chunk
// of the layer, whose sums start G (the products then start from the
// constant zero, with no accumulator to clear).
template <int L, bool FIRST>
__device__ __forceinline__ void grad_chunk(const float (&u)[8], float (&g)[8], float coef, const bf16x8* __restrict__ W,
                                           const float* __restrict__ B, LayerGrad& G)
{
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    bf16x8 x, h1[4], h2[4];
    const f32x16 o = flow_mlp_t<L>(u, W, B, x, h1, h2);

    // ---- inverse transform and log-scale: dL/d(a, t) ----------------------
    // u_l,B = (u_{l+1},B - t) e^-s: dL/ds = c - g_B u_l,B (the log-scale is
    // a term of log J_F), dL/dt = -g_B e^-s, dL/du_{l+1},B = g_B e^-s;
    // s = S tanh(a/S), ds/da = 1 - (s/S)^2.  dO in T3's row order.
    f32x16 dO;
#pragma unroll
    for (int r = 0; r < 16; ++r) dO[r] = 0.f;
    float gn[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        gn[j] = g[j];
        if (flow_reg_in_a(L, j)) continue;
        const float s = flow_scale(o[j]);
        const float es = flow_exp(-s);
        const float ub = (u[j] - o[8 + j]) * es;
        const float ds = coef - g[j] * ub;
        const float rs = s * (1.f / kFlowSMax);
        dO[j] = ds * (1.f - rs * rs);
        dO[8 + j] = -g[j] * es;
        gn[j] = g[j] * es;
    }
    const bf16x8 dOb[2] = {to_bf16(dO, 0), to_bf16(dO, 1)};

    // ---- deltas with samples as columns ------------------------------------
    bf16x8 dA2[4], dA1[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) acc = mfma(W[kPU3 + (mt * 2 + ks) * 64 + lane], dOb[ks], acc);
        mask_by(acc, h2[2 * mt], h2[2 * mt + 1]);
        dA2[2 * mt] = to_bf16(acc, 0);
        dA2[2 * mt + 1] = to_bf16(acc, 1);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma(W[kPU2 + (mt * 4 + ks) * 64 + lane], dA2[ks], acc);
        mask_by(acc, h1[2 * mt], h1[2 * mt + 1]);
        dA1[2 * mt] = to_bf16(acc, 0);
        dA1[2 * mt + 1] = to_bf16(acc, 1);
    }
    {
        // dX: register j < 8 is the lane's conditioning axis j
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma(W[kPU1 + ks * 64 + lane], dA1[ks], acc);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (flow_reg_in_a(L, j)) gn[j] = g[j] + kFlowXScale * acc[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) g[j] = gn[j];

    // ---- the same with samples as rows (16 samples in each lane's registers)
    const int n32 = lane & 31;
    bf16x8 h1r[2][2], h2r[2][2], dA2r[2][2], dA1r[2][2], dOr[2], xr[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc;
        const float b1 = B[32 * nt + n32];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = b1;
        acc = mfma(x, W[kPF1 + nt * 64 + lane], acc);
        h1r[nt][0] = relu_bf16(acc, 0);
        h1r[nt][1] = relu_bf16(acc, 1);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc;
        const float b2 = B[kFlowHidden + 32 * nt + n32];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = b2;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma(h1[ks], W[kPT2 + (nt * 4 + ks) * 64 + lane], acc);
        h2r[nt][0] = relu_bf16(acc, 0);
        h2r[nt][1] = relu_bf16(acc, 1);
    }
    {
        // dO with samples as rows through the 0/1 product P: its BF16 part
        // (the weight gradient's operand) and, for the bias sum, the
        // rounding remainder too (dO = hi + lo to about 16 bits)
        f32x16 acc = {}, rem = {};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            float r[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) r[i] = dO[8 * ks + i] - (float)dOb[ks][i];
            const bf16x8 lo = cvt_bf16x8(r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7]);
            acc = mfma(dOb[ks], W[kPP + ks * 64 + lane], acc);
            rem = mfma(lo, W[kPP + ks * 64 + lane], rem);
        }
        G.b3 = (FIRST ? 0.f : G.b3) + (reg_sum(acc) + reg_sum(rem));
        dOr[0] = to_bf16(acc, 0);
        dOr[1] = to_bf16(acc, 1);
    }
    {
        f32x16 acc = {};
        acc = mfma(x, W[kPI + lane], acc);
        xr[0] = to_bf16(acc, 0);
        xr[1] = to_bf16(acc, 1);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) acc = mfma(dOb[ks], W[kPU3 + (nt * 2 + ks) * 64 + lane], acc);
        mask_by(acc, h2r[nt][0], h2r[nt][1]);
        G.b2[nt] = (FIRST ? 0.f : G.b2[nt]) + reg_sum(acc);
        dA2r[nt][0] = to_bf16(acc, 0);
        dA2r[nt][1] = to_bf16(acc, 1);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) acc = mfma(dA2[ks], W[kPU2 + (nt * 4 + ks) * 64 + lane], acc);
        mask_by(acc, h1r[nt][0], h1r[nt][1]);
        G.b1[nt] = (FIRST ? 0.f : G.b1[nt]) + reg_sum(acc);
        dA1r[nt][0] = to_bf16(acc, 0);
        dA1r[nt][1] = to_bf16(acc, 1);
    }

    // ---- weight gradients: sums over the samples ---------------------------
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            G.w3[nt] = mfma(dOr[ks], h2r[nt][ks], FIRST && ks == 0 ? f32x16{} : G.w3[nt]);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                G.w2[mt][nt] = mfma(dA2r[mt][ks], h1r[nt][ks], FIRST && ks == 0 ? f32x16{} : G.w2[mt][nt]);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            G.w1[mt] = mfma(dA1r[mt][ks], xr[ks], FIRST && ks == 0 ? f32x16{} : G.w1[mt]);
}

// this wave's gradient of layer L into its LDS slice (every entry written)
template <int L>
__device__ __forceinline__ void grad_to_lds(const LayerGrad& G, float* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int n32 = lane & 31;
    const int half = lane >> 5;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = mrow(lane, r);
            if (o < kFlowOut) out[kFW3 + o * kFlowHidden + 32 * nt + n32] = G.w3[nt][r];
        }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                out[kFW2 + (32 * mt + mrow(lane, r)) * kFlowHidden + 32 * nt + n32] = G.w2[mt][nt][r];
    if (n32 < kFlowDim && flow_in_a(L, n32)) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                out[kFW1 + (32 * mt + mrow(lane, r)) * kFlowHalf + flow_pos(L, n32)] = G.w1[mt][r];
    }
    // bias sums: each lane holds 16 samples of its column; the other half
    // holds the other 16
    const float b3 = G.b3 + __shfl_xor(G.b3, 32, 64);
    float b2[2], b1[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        b2[nt] = G.b2[nt] + __shfl_xor(G.b2[nt], 32, 64);
        b1[nt] = G.b1[nt] + __shfl_xor(G.b1[nt], 32, 64);
    }
    if (half == 0) {
        if (n32 < kFlowOut) out[kFB3 + n32] = b3;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            out[kFB2 + 32 * nt + n32] = b2[nt];
            out[kFB1 + 32 * nt + n32] = b1[nt];
        }
    }
}

// layer L: every chunk of the workgroup, then its part of the gradient
// SINGLE: every wave has one chunk at most (the grid covers the samples),
// so no gradient accumulator lives across chunks: the kernel then fits the
// architectural registers.
template <int L, bool SINGLE>
__device__ void grad_layer(const FlowTrainArgs& a, FlowBwdLds& S, float* const (&gbuf)[2], double ss)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int n32 = lane & 31;
    const uint32_t N = a.n;
    const float* g_in = gbuf[L & 1];
    float* g_out = gbuf[(L & 1) ^ 1];
    // this layer's operands and biases into LDS (the previous layer's
    // reduction is done with them)
    {
        const bf16x8* pk = reinterpret_cast<const bf16x8*>(a.packed) + (size_t)L * kPLayer;
        for (int e = threadIdx.x; e < kPLayer; e += kFlowThreads) S.w[e] = pk[e];
        const float* P = a.theta + (size_t)L * kFLayer;
        for (int e = threadIdx.x; e < 2 * kFlowHidden + kFlowOut; e += kFlowThreads)
            S.b[e] = P[e < kFlowHidden ? kFB1 + e : e < 2 * kFlowHidden ? kFB2 + (e - kFlowHidden)
                                                                          : kFB3 + (e - 2 * kFlowHidden)];
    }
    __syncthreads();
    // the layer's input in the inverse direction, u_{l+1}: z_4 itself for
    // the last layer (at the training samples), else the inverse pass's
    // compact output
    constexpr bool from_z = L == kFlowLayers - 1;
    const float* uin = from_z ? a.zf : a.U + (size_t)L * N * kFlowDim;
    LayerGrad G;
    const uint32_t chunks = (N + 31u) / 32u;
    const uint32_t n_waves = gridDim.x * kFlowWaves;
    // waves run independently: no barrier inside the loop.  A sample's
    // dL/du is written and read again by the same lane, as every layer maps
    // chunks to waves alike.
    auto run = [&](uint32_t chunk, auto first) {
        const uint32_t k = min(chunk * 32u + (uint32_t)n32, N - 1u);
        const bool valid = chunk * 32u + (uint32_t)n32 < N;
        // lanes past the end take u = 0 and g = 0 (finite: their zero
        // deltas then add nothing to the sums over samples)
        float u[8], g[8];
        if (valid) {
            flow_lane_load(uin + (from_z ? (size_t)a.off + (size_t)k * a.stride : (size_t)k) * kFlowDim, half, u);
            flow_lane_load(g_in + (size_t)k * kFlowDim, half, g);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) u[j] = g[j] = 0.f;
        }
        const float coef = train_coef(a, k, valid, ss);
        grad_chunk<L, decltype(first)::value>(u, g, coef, S.w, S.b, G);
        if (valid) flow_lane_store(g_out + (size_t)k * kFlowDim, half, g);
    };
    const uint32_t c0 = blockIdx.x * kFlowWaves + wave;
    if (c0 < chunks) {
        run(c0, std::true_type{});
        if (!SINGLE)
            for (uint32_t chunk = c0 + n_waves; chunk < chunks; chunk += n_waves) run(chunk, std::false_type{});
    } else {
        // no chunk: a zero gradient
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            G.w3[t] = {};
            G.w1[t] = {};
            G.w2[t][0] = {};
            G.w2[t][1] = {};
            G.b2[t] = 0.f;
            G.b1[t] = 0.f;
        }
        G.b3 = 0.f;
    }
    grad_to_lds<L>(G, S.red[wave]);
    __syncthreads();
    float* out = a.part + (size_t)blockIdx.x * kFParams + (size_t)L * kFLayer;
    for (int i = threadIdx.x; i < kFLayer; i += kFlowThreads) {
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < kFlowWaves; ++w) s += S.red[w][i];
        out[i] = s;
    }
    __syncthreads();
}

// The inverse pass of the workgroup's training samples, with the chunk of
// every wave the one it takes in each layer of the backward pass, so that
// u_1..u_3 and dL/du_0 are read back by the lanes that wrote them.  Returns
// the total of the sums' block partials, added by every workgroup in the
// same order (workgroup 0 keeps it).
__device__ double inverse_pass(const FlowTrainArgs& a, FlowBwdLds& S, float* g0)
{
    flow_stage_fwd(S.fwd, reinterpret_cast<const bf16x8*>(a.packed), a.theta);
    S.sum[threadIdx.x] = threadIdx.x < kSumBlocks ? a.sumsq[1 + threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) S.sum[threadIdx.x] += S.sum[threadIdx.x + w];
        __syncthreads();
    }
    const double ss = S.sum[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) const_cast<double*>(a.sumsq)[0] = ss;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int n32 = lane & 31;
    const uint32_t N = a.n;
    const uint32_t chunks = (N + 31u) / 32u;
    const uint32_t n_waves = gridDim.x * kFlowWaves;
    for (uint32_t chunk = blockIdx.x * kFlowWaves + (threadIdx.x >> 6); chunk < chunks; chunk += n_waves) {
        const uint32_t k = min(chunk * 32u + (uint32_t)n32, N - 1u);
        const bool valid = chunk * 32u + (uint32_t)n32 < N;
        float z[8];
        flow_lane_load(a.zf + ((size_t)a.off + (size_t)k * a.stride) * kFlowDim, half, z);
        float* U = a.U + (size_t)k * kFlowDim;
        const size_t lay = (size_t)N * kFlowDim;
        flow_layer_inv<3>(z, S.fwd);
        if (valid) flow_lane_store(U + 2 * lay, half, z);
        flow_layer_inv<2>(z, S.fwd);
        if (valid) flow_lane_store(U + lay, half, z);
        flow_layer_inv<1>(z, S.fwd);
        if (valid) flow_lane_store(U, half, z);
        flow_layer_inv<0>(z, S.fwd);
        // dL/du_0 = c u_0 (the term u_0^2 / 2 of log J_F)
        if (valid) {
            const float c = train_coef(a, k, true, ss);
            float g[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) g[j] = c * z[j];
            flow_lane_store(g0 + (size_t)k * kFlowDim, half, g);
        }
    }
    // the first layer's staging ends with a barrier before the per-wave
    // gradients (which share the forward operands' LDS) are written
    return ss;
}

template <bool SINGLE>
__global__ __launch_bounds__(kFlowThreads) void k_flow_grad(FlowTrainArgs a)
{
    __shared__ FlowBwdLds S;
    // dL/du_l passes between the layers through two buffers: the inverse
    // pass leaves dL/du_0 in g_in
    float* const gbuf[2] = {const_cast<float*>(a.g_in), a.g_out};
    const double ss = inverse_pass(a, S, gbuf[0]);
    grad_layer<0, SINGLE>(a, S, gbuf, ss);
    grad_layer<1, SINGLE>(a, S, gbuf, ss);
    grad_layer<2, SINGLE>(a, S, gbuf, ss);
    grad_layer<3, SINGLE>(a, S, gbuf, ss);
}

__device__ __forceinline__ float adam_update(float* theta, float* m, float* v, int i, float gi, float lr, float c1,
                                             float c2)
{
    const float mi = fmaf(0.9f, m[i], 0.1f * gi);
    const float vi = fmaf(0.999f, v[i], 0.001f * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float t = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    theta[i] = t;
    return t;
}

// The per-workgroup gradients summed in a fixed order into grad: 64
// parameters per workgroup of 1024 threads, each parameter summed by 16
// threads over every 16th workgroup's part (so that each load instruction
// reads 64 consecutive parameters, and a thread's 16 loads are all in
// flight at once), the 16 sums added in LDS in a fixed order; with adam
// set, the Adam step on it too, and with adam.slots the weight's two BF16
// copies written in place (else a full repack follows: a launch of its
// own, 4.8 us; done inside this kernel by the last workgroup to finish each
// layer, it made the kernel 16-20 us long).  (Two launches before: segments
// of 16 workgroups, then the segments, 6.8 + 4.9 us; one launch with 4
// threads per parameter looping over 64 workgroups each took 18.8 us.)
constexpr int kUpdSplit = 16;
constexpr int kUpdParams = 64;
constexpr int kUpdPer = 16;                    // workgroup parts per thread
constexpr int kUpdMaxWG = kUpdSplit * kUpdPer;
constexpr int kUpdBlocks = (kFParams + kUpdParams - 1) / kUpdParams;
static_assert(kUpdMaxWG >= kFlowMaxTrainWG, "one part per training workgroup");

__global__ __launch_bounds__(kUpdSplit * kUpdParams) void k_flow_update(const float* part, int n_wg, float* grad,
                                                                        FlowAdamArgs adam, float c1, float c2)
{
    __shared__ float red[kUpdSplit][kUpdParams];
    const int lp = threadIdx.x % kUpdParams;
    const int q = threadIdx.x / kUpdParams;
    const int i = blockIdx.x * kUpdParams + lp;
    float v[kUpdPer];
#pragma unroll
    for (int j = 0; j < kUpdPer; ++j) {
        const int w = q + kUpdSplit * j;
        v[j] = i < kFParams && w < n_wg ? part[(size_t)w * kFParams + i] : 0.f;
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kUpdPer; ++j) s += v[j];
    red[q][lp] = s;
    __syncthreads();
    if (q != 0 || i >= kFParams) return;
    float g = 0.f;
#pragma unroll
    for (int t = 0; t < kUpdSplit; ++t) g += red[t][lp];
    grad[i] = g;
    if (!adam.theta) return;
    const float t = adam_update(adam.theta, adam.m, adam.v, i, g, adam.lr, c1, c2);
    if (adam.slots) {
        // the weight's two BF16 copies in the packed operands, in place
        __bf16* pk = reinterpret_cast<__bf16*>(adam.packed);
        const __bf16 b = (__bf16)t;
        const int f = adam.slots[2 * i], k = adam.slots[2 * i + 1];
        if (f >= 0) pk[f] = b;
        if (k >= 0) pk[k] = b;
    }
}

__global__ void k_flow_adam(float* theta, const float* grad, float* m, float* v, float lr, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kFParams) return;
    (void)adam_update(theta, m, v, i, grad[i], lr, c1, c2);
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

hipError_t launch_flow_sums(const float* om, uint32_t n_eval, uint32_t stride, uint32_t off0, int n_slices,
                            int gamma, double* sumsq, hipStream_t st)
{
    hipLaunchKernelGGL(k_flow_sumsq, dim3(kSumBlocks, n_slices), dim3(kSumThreads), 0, st, om, n_eval, stride, off0,
                       gamma, sumsq);
    return hipGetLastError();
}

hipError_t launch_flow_gradient(const FlowTrainArgs& base, int n_wg, float* G0, float* G1, float* grad,
                                const FlowAdamArgs* adam, hipStream_t st, hipEvent_t* ev)
{
    // one launch totals those sums, runs the inverse pass (u_1..u_3, and
    // dL/du_0 into G1) and every layer's backward pass, alternating G1 and G0
    FlowTrainArgs a = base;
    a.g_in = G1;
    a.g_out = G0;
    if (ev) {
        const hipError_t r = hipEventRecord(ev[0], st);
        if (r != hipSuccess) return r;
    }
    // one chunk of 32 samples per wave when the grid covers them all
    if ((a.n + 31u) / 32u <= (uint32_t)n_wg * kFlowWaves)
        hipLaunchKernelGGL(k_flow_grad<true>, dim3(n_wg), dim3(kFlowThreads), 0, st, a);
    else
        hipLaunchKernelGGL(k_flow_grad<false>, dim3(n_wg), dim3(kFlowThreads), 0, st, a);
    if (ev) {
        const hipError_t r = hipEventRecord(ev[1], st);
        if (r != hipSuccess) return r;
    }
    if (n_wg > kUpdMaxWG) return hipErrorInvalidValue;
    FlowAdamArgs none = {};
    float c1 = 0.f, c2 = 0.f;
    if (adam) adam_corrections(adam->step, &c1, &c2);
    hipLaunchKernelGGL(k_flow_update, dim3(kUpdBlocks), dim3(kUpdSplit * kUpdParams), 0, st, (const float*)a.part,
                       n_wg, grad, adam ? *adam : none, c1, c2);
    if (adam && !adam->slots) return launch_flow_pack(adam->theta, adam->packed, st);
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
