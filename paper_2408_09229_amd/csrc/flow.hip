// The learned warp on gfx950: packing of the BF16 MFMA operands, the
// sampling pass (stratified y -> z_0 = Phi^-1(y) -> four affine coupling
// layers -> w = Phi(z_4), log J_F), and the fill of an iteration through the
// warp (weight f(map(w)) J_map(w) J_F(y)).
//
// One wavefront evaluates the flow for 32 samples at a time, each lane
// holding 8 axes of one sample.  Its matrix products are
// v_mfma_f32_32x32x16_bf16 with the samples as columns (W . act^T), so that
// each product's output registers feed the next product directly and the
// last one's land in the lanes that move each axis; the weights are read
// from LDS, staged once per workgroup.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "fill_dev.hpp"
#include "flow.hpp"
#include "flow_dev.hpp"
#include "launch.hpp"
#include "layout.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// operand packing (after every parameter change)
// ---------------------------------------------------------------------------
__global__ void k_flow_pack(const float* __restrict__ theta, bf16x8* __restrict__ packed)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kFlowLayers * kPLayer) return;
    const int l = e / kPLayer;
    packed[e] = flow_pack_entry(l, e - l * kPLayer, theta + (size_t)l * kFLayer);
}

// ---------------------------------------------------------------------------
// starting weights: W1 and W2 uniform in +-1/sqrt(fan_in) (fan_in 8 and 64),
// every other parameter 0.  The zero last layer makes every log-scale and
// shift exactly 0, so F starts as the identity.  Parameter i draws word 0 of
// Philox4x32-10 with key = seed and counter (i, 0, 0, "FLOW"); its top 23
// bits m give the odd multiple (2m + 1 - 2^23) 2^-23 of the unit interval's
// half width, exact in FP32, which the bound then scales (one rounding).
// ---------------------------------------------------------------------------
__global__ void k_flow_init(float* __restrict__ theta, uint32_t key0, uint32_t key1)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kFParams) return;
    const int r = i % kFLayer;
    const float bound = r < kFB1 ? 0.35355339059327376f : (r >= kFW2 && r < kFB2) ? 0.125f : 0.f;
    float v = 0.f;
    if (bound != 0.f) {
        const PhiloxKeys K = philox_keys<false>(key0, key1);
        const W4 o = philox10((uint32_t)i, 0u, 0u, 0x464C4F57u, K);
        const int m = (int)(o.v[0] >> 9);
        v = (float)(2 * m + 1 - (1 << 23)) * 0x1p-23f * bound;
    }
    theta[i] = v;
}

// ---------------------------------------------------------------------------
// operand layout check: D = A B for one 32x32x16 product (A 32x16 and B
// 16x32 row-major FP32, rounded to BF16; D 32x32 FP32).  One wavefront.
// ---------------------------------------------------------------------------
__global__ void k_mfma_probe(const float* A, const float* B, float* D)
{
    const int l = threadIdx.x;
    bf16x8 a, b;
    for (int j = 0; j < 8; ++j) {
        a[j] = (__bf16)A[(l & 31) * 16 + 8 * (l >> 5) + j];
        b[j] = (__bf16)B[(8 * (l >> 5) + j) * 32 + (l & 31)];
    }
    f32x16 c = {};
    c = mfma(a, b, c);
    for (int r = 0; r < 16; ++r) D[mrow(l, r) * 32 + (l & 31)] = c[r];
}

// ---------------------------------------------------------------------------
// sampling pass: y of every sample of iteration t, pushed through F
// ---------------------------------------------------------------------------
// Cube of sample k for the wave's 32 consecutive samples k0 .. k0 + 31
// (k0 <= k < N).  A 64-way search over the start offsets finds k0's cube c0
// (one gather and a ballot per step, the same for the whole wave); then each
// lane searches the 64 starts from c0, held one per lane, by shuffles.
// Every cube holds at least n_min >= 2 samples, so the wave's samples lie in
// cubes c0 .. c0 + 16.
__device__ __forceinline__ uint32_t flow_cube(const uint32_t* __restrict__ start, uint32_t n_cubes, uint32_t k0,
                                              uint32_t k, int lane)
{
    uint32_t lo = 0, span = n_cubes;          // start[lo] <= k0 < start[lo + span]
    while (span > 1) {
        const uint32_t step = (span + 63u) >> 6;
        const uint32_t off = (uint32_t)lane * step;
        const bool ok = off < span && start[lo + off] <= k0;
        const unsigned long long m = __ballot(ok);
        const uint32_t last = 63u - (uint32_t)__clzll(m);   // lane 0 always holds
        lo += last * step;
        span = min(step, span - last * step);
    }
    const uint32_t idx = lo + (uint32_t)lane;
    const uint32_t sw = idx < n_cubes ? start[idx] : 0xFFFFFFFFu;
    int a = 0, b = 64;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        const int mid = (a + b) >> 1;
        const uint32_t v = __shfl(sw, mid, 64);
        if (v <= k) a = mid; else b = mid;
    }
    return lo + (uint32_t)a;
}

__global__ __launch_bounds__(kFlowSampleThreads, 4) void k_flow_sample(FlowSampleArgs a)
{
    __shared__ FlowFwdLds S;
    flow_stage_fwd(S, reinterpret_cast<const bf16x8*>(a.packed), a.theta);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int n32 = lane & 31;
    const SampleConst& sc = a.sc;
    const PhiloxKeys keys = philox_keys<false>(sc.key0, sc.key1);
    const uint32_t N = sc.n_eval;
    const uint32_t chunks = (N + 31u) / 32u;
    const uint32_t n_waves = gridDim.x * kFlowSampleWaves;
    const double den = (double)sc.nst * 0x1p33;
    const double inv_den = 1.0 / den;
    // N_st^16 cubes fit in 32 bits, so N_st <= 4 and every shift below is
    // at most 30
    const bool pow2 = (sc.nst & (sc.nst - 1u)) == 0u;
    const uint32_t lg = (uint32_t)__builtin_ctz(sc.nst);
    // waves run independently: no barrier inside the loop
    for (uint32_t chunk = blockIdx.x * kFlowSampleWaves + (threadIdx.x >> 6); chunk < chunks; chunk += n_waves) {
        const uint32_t k0 = chunk * 32u;
        const uint32_t k = min(k0 + (uint32_t)n32, N - 1u);
        // the stratum digits of the lane's axes (axis d sits in register
        // 4 (d / 8) + d % 4 of half (d / 4) % 2).  N_st a power of two (the
        // usual case at d = 16: 2^16 or 4^16 cubes): each digit is a shift
        // and a mask.  Otherwise division by N_st, one digit after the
        // other, each kept by the half that holds it (written per register:
        // an index into all 16 digits that depends on the lane would be a
        // 16-way select chain).
        uint32_t hc = flow_cube(a.start, sc.n_cubes, k0, k, lane), dig[8];
        if (pow2) {
            const uint32_t hb = hc >> (4u * lg * (uint32_t)half);
#pragma unroll
            for (int j = 0; j < 8; ++j) dig[j] = (hb >> ((uint32_t)flow_axis(0, j) * lg)) & (sc.nst - 1u);
        } else {
#pragma unroll
            for (int d = 0; d < kFlowDim; ++d) {
                const uint32_t q = div_magic(hc, sc.nst_magic, sc.nst_shift);
                const uint32_t digit = hc - q * sc.nst;
                hc = q;
                const int j = 4 * (d >> 3) + (d & 3);
                if ((d >> 2) & 1) {
                    if (half) dig[j] = digit;
                } else {
                    dig[j] = digit;
                }
            }
        }
        // the stratified point y = (s 2^33 + 2r + 1) / (N_st 2^33) and
        // z_0 = Phi^-1(y): numerator and den - numerator are exact in FP64
        // (s < 2^20), so min(y, 1 - y) is one FP64 product by 1/den (two
        // roundings in FP64), rounded to FP32.  Axis c takes word c % 4 of
        // counter c / 4; register block b of this lane's half holds axes
        // 8 b + 4 half + q, counter 2 b + half.
        float z0[8], z[8];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const W4 o = philox10(k, 0u, a.t, sc.ctr3 | (uint32_t)(2 * b + half), keys);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = 4 * b + q;
                const double num = fma((double)dig[j], 0x1p33, 2.0 * (double)o.v[q] + 1.0);
                const bool upper = 2.0 * num > den;
                const float m = (float)((upper ? den - num : num) * inv_den);
                z0[j] = flow_phi_inv(m, upper);
                z[j] = z0[j];
            }
        }
        float lj = 0.f;
        flow_layer_fwd<0>(z, lj, S);
        flow_layer_fwd<1>(z, lj, S);
        flow_layer_fwd<2>(z, lj, S);
        flow_layer_fwd<3>(z, lj, S);
        float wv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            lj += 0.5f * (z0[j] - z[j]) * (z0[j] + z[j]);
            wv[j] = flow_phi(z[j]);
        }
        lj += __shfl_xor(lj, 32, 64);
        if (k0 + (uint32_t)n32 < N) {
            flow_lane_store(a.w + (size_t)k * kFlowDim, half, wv);
            flow_lane_store(a.z + (size_t)k * kFlowDim, half, z);
            if (half == 0) a.lj[k] = lj;
        }
    }
}

// ---------------------------------------------------------------------------
// the fill through the warp
// ---------------------------------------------------------------------------
// Sample path of the warped fill: the point is w_k from the sampling pass
// (FP32), its map bin floor(w N_g), and the weight carries J_F = exp(lj_k).
// The stratum digits are not needed (the sampling pass used them).  The
// map's histograms weigh the sample by 1/J_F (see fill_tile).
template <int FAM>
struct WarpedPath {
    static constexpr bool kExact = true;       // D = 16 always
    static constexpr bool kWeightedHist = true;
    float jf = 1.f;                            // J_F of the last sample evaluated
    const SampleConst& sc;
    Fn<float, FAM> fn;
    float ngR;
    double ngD;
    const float* w;
    const float* lj;
    float* om;

    __device__ __forceinline__ WarpedPath(const SampleConst& c, const float* aux, const float* w_, const float* lj_,
                                          float* om_)
        : sc(c), w(w_), lj(lj_), om(om_)
    {
        fn.setup(c, aux);
        ngR = (float)c.ng;
        ngD = (double)c.ng;
    }
    __device__ __forceinline__ double last_jf() const { return (double)jf; }
    __device__ __forceinline__ void digits(uint32_t, uint32_t (&)[kFlowDim]) const {}
    __device__ __forceinline__ void next_digits(uint32_t (&)[kFlowDim]) const {}

    template <bool PROBE>
    __device__ __forceinline__ float eval(uint32_t k, uint32_t, const uint32_t (&)[kFlowDim], const float* __restrict__ g,
                                          uint32_t (&bins)[kFlowDim], float*, float*, float& J, float& f)
    {
        const float4* wk = reinterpret_cast<const float4*>(w + (size_t)k * kFlowDim);
        float wv[kFlowDim];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = wk[q];
            wv[4 * q] = v.x;
            wv[4 * q + 1] = v.y;
            wv[4 * q + 2] = v.z;
            wv[4 * q + 3] = v.w;
        }
        J = 1.f;
        fn.begin();
        const uint32_t row = sc.ng + 1u;
        const int top = (int)sc.ng - 1;
        // bin and offset of w in the map, exactly: w N_g (w FP32, N_g <=
        // 4096) is exact in FP64, so are its floor and the remainder, which
        // is rounded once to FP32
#pragma unroll
        for (int d = 0; d < kFlowDim; ++d) {
            const double u = (double)wv[d] * ngD;
            const int bin = min((int)u, top);
            const float delta = (float)(u - (double)bin);
            bins[d] = (uint32_t)bin;
            const float* gd = g + d * row;
            const float xl = gd[bin];
            const float dx = gd[bin + 1] - xl;
            J = J * (ngR * dx);
            fn.axis(d, fmaf(dx, delta, xl));
        }
        f = fn.finish();
        jf = expf(lj[k]);
        J = J * jf;
        const float wt = J * f;
        om[k] = __builtin_isfinite(wt) ? wt : 0.f;
        return wt;
    }
};

template <int FAM, bool KAHAN>
__global__ __launch_bounds__(kFillThreads) void k_fill_flow(FillArgs a, const float* w, const float* lj, float* om)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SampleConst& sc = a.sc;
    const int D = sc.D;
    const uint32_t ng = sc.ng;
    const int tid = threadIdx.x;
    const LdsPlan lp = lds_plan(D, (int)ng, 4, a.lds_hist, a.tile, sc.n_aux, 1);
    const FillLds<float> L(smem, lp);
    const int nbins = D * (int)ng;
    const float* gsrc = reinterpret_cast<const float*>(a.grid);
    for (int i = tid; i < D * (int)(ng + 1); i += kFillThreads) L.gl[i] = gsrc[i];
    for (int i = tid; i < sc.n_aux; i += kFillThreads) L.auxl[i] = sc.aux_f[i];
    if (a.lds_hist) {
        for (int i = tid; i < nbins; i += kFillThreads) {
            L.hl[i] = 0.0;
            L.cl[i] = 0u;
        }
    }
    WarpedPath<FAM> sp(sc, L.auxl, w, lj, om);
    LaneTotal<KAHAN> totI, totV;
    double vmax = 0.0;
    unsigned long long bad = 0;
    TileIO io;
    io.grid = nullptr;
    io.t = a.t;
    io.tile = a.tile;
    io.per_lane = a.per_lane;
    io.lds_hist = a.lds_hist;
    io.start = a.start;
    io.tile_first = a.tile_first;
    io.v_out = a.v_out;
    io.side = a.side;
    io.hist_H = a.hist_H;
    io.hist_C = a.hist_C;
    io.hist_Cw = a.hist_Cw;
    __syncthreads();
    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x)
        fill_tile<float, kFlowDim, KAHAN, false>(tile, io, L, sp, totI, totV, vmax, bad);
    if (a.lds_hist) {
        double* slotH = a.hist_H + (size_t)blockIdx.x * nbins;
        uint32_t* slotC = a.hist_C + (size_t)blockIdx.x * nbins;
        for (int i = tid; i < nbins; i += kFillThreads) {
            slotH[i] = L.hl[i];
            slotC[i] = L.cl[i];
        }
    }
    double sI, sV, mx;
    wg_reduce_totals(totI.value(), totV.value(), vmax, L.red, sI, sV, mx);
    if (tid == 0) {
        a.wg_part[2 * blockIdx.x] = sI;
        a.wg_part[2 * blockIdx.x + 1] = sV;
        atomicMax(a.vmax, (unsigned long long)__double_as_longlong(mx));
    }
    if (bad) atomicAdd(a.nonfinite, bad);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_flow_pack(const float* theta, void* packed, hipStream_t st)
{
    const int n = kFlowLayers * kPLayer;
    hipLaunchKernelGGL(k_flow_pack, dim3((n + 255) / 256), dim3(256), 0, st, theta, (bf16x8*)packed);
    return hipGetLastError();
}

hipError_t launch_flow_init(float* theta, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_flow_init, dim3((kFParams + 255) / 256), dim3(256), 0, st, theta, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_mfma_probe(const float* A, const float* B, float* D, hipStream_t st)
{
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, st, A, B, D);
    return hipGetLastError();
}

hipError_t launch_flow_sample(const FlowSampleArgs& a, int n_wg, hipStream_t st)
{
    hipLaunchKernelGGL(k_flow_sample, dim3(n_wg), dim3(kFlowSampleThreads), 0, st, a);
    return hipGetLastError();
}

template <int FAM>
static hipError_t launch_fill_flow_fam(const FillArgs& a, const float* w, const float* lj, float* om, int n_wg,
                                       size_t lds, hipStream_t st)
{
    if (a.accum == 1) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_fill_flow<FAM, true>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_fill_flow<FAM, true>), dim3(n_wg), dim3(kFillThreads), lds, st, a, w, lj, om);
    } else {
        const hipError_t e = hipFuncSetAttribute((const void*)k_fill_flow<FAM, false>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_fill_flow<FAM, false>), dim3(n_wg), dim3(kFillThreads), lds, st, a, w, lj, om);
    }
    return hipGetLastError();
}

hipError_t launch_fill_flow(const FillArgs& a, const float* w, const float* lj, float* om, int n_wg, size_t lds,
                            hipStream_t st)
{
    switch (a.sc.family) {
    case F_GAUSS_DIAG: return launch_fill_flow_fam<F_GAUSS_DIAG>(a, w, lj, om, n_wg, lds, st);
    case F_GENZ_PPEAK: return launch_fill_flow_fam<F_GENZ_PPEAK>(a, w, lj, om, n_wg, lds, st);
    case F_GENZ_GAUSS: return launch_fill_flow_fam<F_GENZ_GAUSS>(a, w, lj, om, n_wg, lds, st);
    case F_GAUSS_CORR: return launch_fill_flow_fam<F_GAUSS_CORR>(a, w, lj, om, n_wg, lds, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace vg
