// Host-side launchers of the VEGAS+ kernels (defined in fill.hip, update.hip,
// ordered.hip and batch.hip; called by the C ABI in api.hip and
// batch_api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "flow.hpp"
#include "layout.hpp"

namespace vg {

struct ProbeArgs {
    SampleConst sc;
    uint32_t t;
    uint64_t k0;
    int64_t n;
    const void* grid;           // FP64 or FP32 grid per precision
    const uint32_t* start;      // [N_c+1]
    uint32_t* cube;
    uint32_t* bins;
    double* delta;
    double* x;
    double* jac;
    double* f;
};

struct OrderedArgs {
    SampleConst sc;
    uint32_t t;
    const double* grid;         // FP64 [D][N_g+1]
    const uint32_t* start;      // [N_c+1]
    double* w;                  // [N_ev] sample weights
    uint32_t* bins;             // [N_ev][D]
    double* m;                  // [N_c] cube means
    double* v;                  // [N_c] cube unbiased variances
    double* hist_H;             // [D*N_g] (slot 0)
    uint32_t* hist_C;
    double* iter_out;           // (I_t, sigma_t^2)
    unsigned long long* vmax;
    unsigned long long* nonfinite;
};

struct PrepArgs {
    int32_t family;
    int32_t D;
    int32_t n_params;
    const double* prm;
    const double* lo;
    const double* hi;
    int32_t ng;
    double* aux_d;
    float* aux_f;
    double* grid64;             // non-null: write the uniform grid
    float* grid32;
};

hipError_t launch_fill(const FillArgs& a, bool fp64, int n_wg, size_t lds, hipStream_t st);
hipError_t launch_fixup(const FixupArgs& a, hipStream_t st);
hipError_t launch_final(const FinalArgs& a, hipStream_t st);
hipError_t launch_probe(const ProbeArgs& a, bool fp64, hipStream_t st);
// LDS bytes of a fill launch; map_lds = 1 for the kernels that keep the map
// in LDS (the warped fill, the persistent batch), 0 for k_fill
size_t fill_lds_bytes(int D, int ng, bool fp64, int lds_hist, int tile, int n_aux, int map_lds);

hipError_t launch_prep(const PrepArgs& a, hipStream_t st);
hipError_t launch_ordered(const OrderedArgs& a, hipStream_t st);
hipError_t launch_alloc(const AllocArgs& a, unsigned long long* qmax_bits, hipStream_t st);
hipError_t launch_map_update(const MapArgs& a, hipStream_t st);
hipError_t launch_update_small(const UpdateArgs& u, hipStream_t st);
hipError_t launch_hist_reduce(const HistReduceArgs& a, hipStream_t st);
hipError_t launch_reset(unsigned long long* p, int n, hipStream_t st);
hipError_t launch_grid32(const double* g64, float* g32, int n, hipStream_t st);

hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t st);
hipError_t launch_batch_fill(const BatchArgs& a, bool fp64, bool kahan, int n_wg, size_t lds, hipStream_t st);
hipError_t launch_batch_estimate(const BatchArgs& a, hipStream_t st);
hipError_t launch_batch_alloc(const BatchArgs& a, bool any_general_beta, hipStream_t st);
hipError_t launch_batch_map(const BatchArgs& a, int max_ng, hipStream_t st);
hipError_t launch_batch_prep(const BatchArgs& a, hipStream_t st);

hipError_t launch_flow_pack(const float* theta, void* packed, hipStream_t st);
hipError_t launch_flow_init(float* theta, uint64_t seed, hipStream_t st);
hipError_t launch_mfma_probe(const float* A, const float* B, float* D, hipStream_t st);
hipError_t launch_flow_sample(const FlowSampleArgs& a, int n_wg, hipStream_t st);
hipError_t launch_fill_flow(const FillArgs& a, const float* w, const float* lj, float* om, int n_wg, size_t lds,
                            hipStream_t st);
// Block partials of sum |omega|^gamma for n_slices slices of the samples,
// slice y holding off, off + stride, ... with off = (off0 + y) mod stride:
// sumsq[y kFlowSumRecord + 1 ..], one slice's record per training step.
hipError_t launch_flow_sums(const float* om, uint32_t n_eval, uint32_t stride, uint32_t off0, int n_slices,
                            int gamma, double* sumsq, hipStream_t st);
// One training step on the slice base.off, base.stride, whose sums'
// partials base.sumsq holds (launch_flow_sums).  ev: null, or two events
// recorded on st just before and after the gradient kernel (its own
// duration)
hipError_t launch_flow_gradient(const FlowTrainArgs& base, int n_wg, float* G0, float* G1, float* grad,
                                const FlowAdamArgs* adam, hipStream_t st, hipEvent_t* ev = nullptr);
hipError_t launch_flow_adam(float* theta, const float* grad, float* m, float* v, float lr, int step, hipStream_t st);

constexpr int kAllocThreads = 1024;
constexpr int kAllocPerThread = 4;
constexpr int kAllocPerBlock = kAllocThreads * kAllocPerThread;

}  // namespace vg
