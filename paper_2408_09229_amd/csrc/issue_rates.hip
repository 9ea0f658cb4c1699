// Issue cost of the VALU instruction kinds the VEGAS+ sample path uses, on
// the current device: eight independent dependency chains per lane keep the
// issue port, not latency, the limit.  Used to weight operations in the
// fill kernel's ALU roofline (an operation issuing at half rate occupies two
// slots).  Not part of the VEGAS+ path.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;
constexpr int kBlock = 256;

template <int OP>
__global__ __launch_bounds__(kBlock) void k_issue(float* out, int iters)
{
    float f[kChains];
    double d[kChains];
    uint32_t u[kChains];
    for (int c = 0; c < kChains; ++c) {
        f[c] = threadIdx.x * 1e-3f + c;
        d[c] = f[c];
        u[c] = threadIdx.x * 77u + c;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (OP == 0) f[c] = fmaf(f[c], 0.999f, 0.5f);                                   // 1 op
            if (OP == 1) f[c] = __builtin_amdgcn_exp2f(f[c] * -1e-3f);                      // mul + exp2
            if (OP == 2) {                                                                  // mad_u64 + xor
                const uint64_t p = (uint64_t)u[c] * 0xD2511F53u;
                u[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            }
            if (OP == 3) d[c] = fma(d[c], 0.999, 0.5);                                      // 1 op
            if (OP == 4) u[c] = __builtin_amdgcn_bitop3_b32(u[c], u[(c + 1) % kChains], 0x1234567u, 0x96);
            if (OP == 5) d[c] = __builtin_amdgcn_rcp(d[c] + 1.0);                            // add + rcp64
        }
    }
    float s = 0.f;
    for (int c = 0; c < kChains; ++c) s += f[c] + (float)d[c] + (float)u[c];
    out[blockIdx.x * kBlock + threadIdx.x] = s;
}

}  // namespace

// out[op] = wave64 instructions retired per 4 cycles per SIMD for op kind
// 0 fma_f32, 1 mul+exp2_f32, 2 mad_u64_u32+xor, 3 fma_f64, 4 bitop3,
// 5 add_f64+rcp_f64 (1.0 = one full-rate instruction every issue slot).
// Returns 0 on success, -3 on a HIP error.
extern "C" int vegas_issue_rates(double* out, int n_ops, double clock_ghz, int n_simd)
{
    const int blocks = 4096, iters = 2048;
    const int per_step[6] = {1, 2, 2, 1, 1, 2};
    float* buf = nullptr;
    if (hipMalloc(&buf, sizeof(float) * blocks * kBlock) != hipSuccess) return -3;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    for (int op = 0; op < n_ops && op < 6; ++op) {
        for (int rep = 0; rep < 2; ++rep) {
            hipEventRecord(a);
            switch (op) {
            case 0: hipLaunchKernelGGL(k_issue<0>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 1: hipLaunchKernelGGL(k_issue<1>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 2: hipLaunchKernelGGL(k_issue<2>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 3: hipLaunchKernelGGL(k_issue<3>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 4: hipLaunchKernelGGL(k_issue<4>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 5: hipLaunchKernelGGL(k_issue<5>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            }
            hipEventRecord(b);
            hipEventSynchronize(b);
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, a, b);
        const double wave_instr = (double)blocks * kBlock / 64 * iters * kChains * per_step[op];
        const double issue_slots = ms * 1e-3 * clock_ghz * 1e9 * n_simd / 4.0;
        out[op] = wave_instr / issue_slots;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(buf);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
