// The learned warp: a coupling flow F on [0,1]^16 stacked on the VEGAS map
// (stratified y -> w = F(y) -> x = map(w)); shapes, parameter layout and the
// launch records of its kernels.
//
// The flow works in Gaussian coordinates: z_0 = Phi^-1(y), four affine
// coupling layers, w = Phi(z_4).  Layer l keeps the axes A_l and moves the
// others (B_l): A = {0..7}, {8..15}, even axes, odd axes.  The conditioner of
// a layer is an MLP 8 -> 64 -> 64 -> 16 with ReLU, fed x = z_A / 2; its 16
// outputs are the raw log-scales a (8) and the shifts t (8) of the moved
// axes, s = 3 tanh(a / 3) and z_B -> z_B e^s + t.  log J_F = sum s +
// sum_d (z_0d^2 - z_4d^2) / 2, exact.  Matrix products run on BF16 MFMA with
// FP32 accumulation; everything else is FP32.
#pragma once
#include <stdint.h>

#include "layout.hpp"

namespace vg {

constexpr int kFlowDim = 16;
constexpr int kFlowHidden = 64;
constexpr int kFlowLayers = 4;
constexpr int kFlowHalf = 8;                   // |A| = |B|
constexpr int kFlowOut = 2 * kFlowHalf;        // log-scales, then shifts
constexpr float kFlowSMax = 3.f;               // |s| < 3
constexpr float kFlowXScale = 0.5f;            // conditioner input z_A / 2

// per-layer parameter offsets (floats; row-major W[out][in])
constexpr int kFW1 = 0;                                    // [64][8]
constexpr int kFB1 = kFW1 + kFlowHidden * kFlowHalf;       // [64]
constexpr int kFW2 = kFB1 + kFlowHidden;                   // [64][64]
constexpr int kFB2 = kFW2 + kFlowHidden * kFlowHidden;     // [64]
constexpr int kFW3 = kFB2 + kFlowHidden;                   // [16][64]
constexpr int kFB3 = kFW3 + kFlowOut * kFlowHidden;        // [16]
constexpr int kFLayer = kFB3 + kFlowOut;                   // 5776
constexpr int kFParams = kFlowLayers * kFLayer;

// Packed BF16 operands of one layer for v_mfma_f32_32x32x16_bf16, one
// 8-value entry per (tile, k-step, lane): lane l holds A[l % 32][8 (l/32) + j]
// of an A operand, or B[8 (l/32) + j][l % 32] of a B operand.  A product's
// output register r of lane l holds row 8 (r/4) + 4 (l/32) + r % 4, column
// l % 32 ("register order").  The forward products run as W . act^T
// (samples as columns), so each one's output registers are the next one's B
// operand as they stand, with the weights' k order packed to match:
//   F1: W1 (rows: hidden unit; k: axis, B axes zero)        [2 m-tiles]
//   T2: W2, k in the hidden units' register order           [2 m-tiles][4 k]
//   T3: W3, k likewise; rows placed where the lanes that
//       move each axis hold them (flow_t3_row)              [4 k]
// The backward products run the same way (samples as columns) on the
// transposed weights, and read as B operands with samples as rows they give
// the activations and deltas with samples in registers, which the weight
// gradients (sums over samples) take as both operands:
//   U3: W3^T (rows: hidden unit of h2; k: T3's rows)        [2 m-tiles][2 k]
//   U2: W2^T (rows: unit of h1; k: units of h2, reg. order) [2 m-tiles][4 k]
//   U1: W1^T (rows placed on the lanes holding each
//       conditioning axis, flow_dx_row; k: units of h1)    [4 k]
//   P:  0/1, T3's rows -> conditioner outputs (a transpose) [2 k]
//   I:  0/1, axes -> axes (a transpose)                     [1]
constexpr int kPF1 = 0;
constexpr int kPT2 = kPF1 + 2 * 64;
constexpr int kPT3 = kPT2 + 2 * 4 * 64;
constexpr int kPU3 = kPT3 + 4 * 64;
constexpr int kPU2 = kPU3 + 2 * 2 * 64;
constexpr int kPU1 = kPU2 + 2 * 4 * 64;
constexpr int kPP = kPU1 + 4 * 64;
constexpr int kPI = kPP + 2 * 64;
constexpr int kPLayer = kPI + 64;                // 2112 entries of 16 bytes
constexpr int kPFwdT = kPU3;                     // F1, T2, T3: the forward pass's 896 entries

// Register order of a product's 32x32 output (register r of lane l holds
// row 8 (r/4) + 4 (l/32) + r % 4): fed to the next product as its B operand,
// k-step ks takes registers 8 (ks % 2) .. + 7 of tile ks / 2, so k index
// 8 h + i of k-step ks is hidden unit flow_t_unit(ks, h, i).
__host__ __device__ inline int flow_t_unit(int ks, int h, int i)
{
    return 32 * (ks >> 1) + 16 * (ks & 1) + 8 * (i >> 2) + 4 * h + (i & 3);
}

// axis c is conditioning (in A) in layer l
__host__ __device__ constexpr bool flow_in_a(int l, int c)
{
    return l == 0 ? c < 8 : l == 1 ? c >= 8 : l == 2 ? (c & 1) == 0 : (c & 1) == 1;
}
// position of axis c inside its set (A or B) of layer l
__host__ __device__ constexpr int flow_pos(int l, int c) { return l < 2 ? (c & 7) : (c >> 1); }

// A sample's 16 axes are held by two lanes, 8 in registers each: register j
// of the lanes of half h holds axis 8 (j/4) + 4 h + j % 4 (h = 0: axes 0-3
// and 8-11; h = 1: axes 4-7 and 12-15).  Both halves then hold two axes of
// each class (c < 8 or not, c even or odd) at the same registers, so in
// every layer the moved axes sit at the same 4 registers of every lane, and
// the conditioner's per-axis work is the same for the whole wave.  Axis
// m < 16 is also the row that register j of half h holds in a product's
// output (8 (r/4) + 4 h + r % 4).
__host__ __device__ constexpr int flow_axis(int h, int j) { return 8 * (j >> 2) + 4 * h + (j & 3); }
// register j holds a conditioning axis of layer l, in both halves
__host__ __device__ constexpr bool flow_reg_in_a(int l, int j) { return flow_in_a(l, flow_axis(0, j)); }

constexpr bool flow_axis_layout_ok()
{
    for (int l = 0; l < 4; ++l)
        for (int j = 0; j < 8; ++j)
            if (flow_in_a(l, flow_axis(0, j)) != flow_in_a(l, flow_axis(1, j))) return false;
    return true;
}
static_assert(flow_axis_layout_ok(), "both lane halves move the same registers in every layer");

// Conditioner output carried by row m of the transposed last product of
// layer l, or -1 for a zero row.  Row m lands in register r = 4 (m/8) + m % 4
// of the lanes of half (m/4) % 2: register j < 8 gets the raw log-scale of
// the lane's axis flow_axis(half, j), register 8 + j its shift, where that
// axis moves in layer l.
__host__ __device__ inline int flow_t3_row(int l, int m)
{
    const int half = (m >> 2) & 1;
    const int r = 4 * (m >> 3) + (m & 3);
    const int c = flow_axis(half, r & 7);
    if (flow_in_a(l, c)) return -1;
    return (r < 8 ? 0 : kFlowHalf) + flow_pos(l, c);
}

// Conditioning axis (its position in A) carried by row m of the transposed
// input-gradient product dX^T = W1^T dA1^T of layer l, or -1: row m lands in
// register j = 4 (m/8) + m % 4 < 8 of the lanes of half (m/4) % 2, the
// lane's own axis flow_axis(half, j).
__host__ __device__ inline int flow_dx_row(int l, int m)
{
    const int half = (m >> 2) & 1;
    const int r = 4 * (m >> 3) + (m & 3);
    const int c = flow_axis(half, r & 7);
    if (r >= 8 || !flow_in_a(l, c)) return -1;
    return flow_pos(l, c);
}

// Source of value j of entry r of layer l's packed operands: the offset of
// the layer parameter it copies, or -1 for a constant 0, -2 for a constant
// 1 (the 0/1 transposes P and I).  Every weight has exactly one forward
// (F1, T2, T3) and one backward (U3, U2, U1) copy; biases have none.
__host__ __device__ inline int flow_pack_src(int l, int r, int j)
{
    const int lane = r & 63;
    const int h = lane >> 5;              // k half of this lane
    const int n32 = lane & 31;            // its row (A operand) or column (B operand)
    if (r < kPT2) {                       // F1[mt]: W1[unit][pos(axis of (h, j))], axes in A
        const int m = (r >> 6) * 32 + n32;
        const int c = flow_axis(h, j);
        return flow_in_a(l, c) ? kFW1 + m * kFlowHalf + flow_pos(l, c) : -1;
    }
    if (r < kPT3) {                       // T2[mt][ks]: W2[unit2][unit1(ks, k)]
        r -= kPT2;
        const int m = (r >> 8) * 32 + n32, ks = (r >> 6) & 3;
        return kFW2 + m * kFlowHidden + flow_t_unit(ks, h, j);
    }
    if (r < kPU3) {                       // T3[ks]: W3[row(m)][unit2(ks, k)]
        r -= kPT3;
        const int o = flow_t3_row(l, n32);
        return o >= 0 ? kFW3 + o * kFlowHidden + flow_t_unit(r >> 6, h, j) : -1;
    }
    if (r < kPU2) {                       // U3[mt][ks]: W3[row(k)][unit2 = m]
        r -= kPU3;
        const int m = (r >> 7) * 32 + n32, ks = (r >> 6) & 1;
        const int o = flow_t3_row(l, flow_t_unit(ks, h, j));
        return o >= 0 ? kFW3 + o * kFlowHidden + m : -1;
    }
    if (r < kPU1) {                       // U2[mt][ks]: W2[unit2(ks, k)][unit1 = m]
        r -= kPU2;
        const int m = (r >> 8) * 32 + n32, ks = (r >> 6) & 3;
        return kFW2 + flow_t_unit(ks, h, j) * kFlowHidden + m;
    }
    if (r < kPP) {                        // U1[ks]: W1[unit1(ks, k)][pos of row m's axis]
        r -= kPU1;
        const int p = flow_dx_row(l, n32);
        return p >= 0 ? kFW1 + flow_t_unit(r >> 6, h, j) * kFlowHalf + p : -1;
    }
    if (r < kPI) {                        // P[ks]: 1 where T3's row (ks, k) carries output n
        r -= kPP;
        return flow_t3_row(l, flow_t_unit(r >> 6, h, j)) == n32 ? -2 : -1;
    }
    return flow_axis(h, j) == n32 ? -2 : -1;   // I: 1 where the axis of (h, j) is column n
}

// the lane's 8 axes of a sample's 16 values (row: the sample's first value)
__host__ __device__ inline void flow_lane_load(const float* row, int half, float (&v)[8])
{
    const float4 a = *reinterpret_cast<const float4*>(row + 4 * half);
    const float4 b = *reinterpret_cast<const float4*>(row + 8 + 4 * half);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__host__ __device__ inline void flow_lane_store(float* row, int half, const float (&v)[8])
{
    *reinterpret_cast<float4*>(row + 4 * half) = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4*>(row + 8 + 4 * half) = make_float4(v[4], v[5], v[6], v[7]);
}

struct FlowSampleArgs {
    SampleConst sc;
    uint32_t t;
    const uint32_t* start;        // [N_c+1]
    const float* theta;           // FP32 parameters (biases are read from here)
    const void* packed;           // [4][kPLayer] x 16 bytes of BF16
    float* w;                     // [N][16] out: w = Phi(z_4)
    float* z;                     // [N][16] out: z_4 (the training data)
    float* lj;                    // [N] out: log J_F
};

// Training records.  The loss of an iteration is
// L = sum_k c_k log J_F(F^-1(w_k)), c_k = |omega_k|^gamma / sum |omega|^gamma,
// and its gradient is taken through the inverse chain u_4 = z_4 -> u_3 ->
// u_2 -> u_1 -> u_0 (Gaussian coordinates): the inverse pass stores u_1..u_3
// and the upstream gradient dL/du_0 = c z_0, then one backward pass per
// layer (l = 0, 1, 2, 3) turns g = dL/du_l into dL/du_{l+1} and the layer's
// parameter gradient.
struct FlowTrainArgs {
    uint32_t n;                   // training samples: j = 0 .. n-1 is sample off + j stride
    uint32_t stride, off;
    int32_t layer;                // backward pass: layer index
    const float* theta;
    const void* packed;
    const float* zf;              // [N_ev][16] z_4, read at the training samples
    const float* om;              // [N_ev] sample weights, read at the training samples
    const double* sumsq;          // sum of |om|^gamma
    int32_t gamma;                // 2: variance loss, 1: KL loss
    float* U;                     // [3][n][16]: u_1, u_2, u_3 of the training samples
    const float* g_in;            // [n][16] upstream gradient dL/du_layer
    float* g_out;                 // [n][16] dL/du_{layer+1}
    float* part;                  // [n_wg][kFParams] per-workgroup gradient
};

// Adam step fused into the gradient's last reduction (training), or none
// (the gradient alone)
// sums of |omega|^gamma of one training step's slice: the total, then 256
// block partials (doubles)
constexpr int kFlowSumBlocks = 256;
constexpr int kFlowSumRecord = 1 + kFlowSumBlocks;
// workgroups of the training kernel at most (their partial gradients are
// summed by a fixed-order reduction sized for this many)
constexpr int kFlowMaxTrainWG = 256;

struct FlowAdamArgs {
    float* theta;                 // null: the gradient alone
    float* m;
    float* v;
    void* packed;                 // repacked BF16 operands
    const int* slots;             // [n_params][2]: each weight's forward and backward BF16 copy in packed
                                  // (value index, -1 none); null: repack every entry after the step
    float lr;
    int step;                     // counts from 1
};

}  // namespace vg
