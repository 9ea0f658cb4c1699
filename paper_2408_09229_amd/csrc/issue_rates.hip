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
            if (OP == 6) f[c] = __builtin_amdgcn_exp2f(-f[c]);                              // exp2 alone
            if (OP == 7) {                                                                  // 2 exp2 : 6 fma
                if (c % 4 == 0) f[c] = __builtin_amdgcn_exp2f(-f[c]);
                else f[c] = fmaf(f[c], 0.999f, 0.5f);
            }
        }
    }
    float s = 0.f;
    for (int c = 0; c < kChains; ++c) s += f[c] + (float)d[c] + (float)u[c];
    out[blockIdx.x * kBlock + threadIdx.x] = s;
}

// LDS atomic adds without return: every lane adds `iters` times into
// workgroup memory.  PATTERN 0: lane l of wave w always hits word (or
// double) 64 w + l, no bank conflicts; PATTERN 1: each add goes to one of
// 1024 entries drawn by a per-lane linear congruential sequence, the way
// the fill's histogram adds land.  All indexes stay inside the arrays.
template <int OP, int PATTERN>
__global__ __launch_bounds__(kBlock) void k_lds_atomic(float* out, int iters)
{
    __shared__ uint32_t su[1024];
    __shared__ float sf[1024];
    __shared__ double sd[1024];
    for (int i = threadIdx.x; i < 1024; i += kBlock) {
        su[i] = 0u;
        sf[i] = 0.f;
        sd[i] = 0.0;
    }
    __syncthreads();
    uint32_t x = blockIdx.x * 7919u + threadIdx.x * 104729u + 1u;
    const int fixed = threadIdx.x & (kBlock - 1);        // 64 w + l, < 256
    for (int it = 0; it < iters; ++it) {
        int idx = fixed;
        if (PATTERN == 1) {
            x = x * 1664525u + 1013904223u;
            idx = (int)((x >> 16) & 1023u);
        }
        if (OP == 0) atomicAdd(&su[idx], 1u);
        if (OP == 1) unsafeAtomicAdd(&sf[idx], 1.0f);
        if (OP == 2) unsafeAtomicAdd(&sd[idx], 1.0);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (float)su[0] + sf[0] + (float)sd[0];
}

}  // namespace

// out[6 * pattern + op] = LDS atomic adds retired per cycle per CU, op 0 u32,
// 1 f32, 2 f64; pattern 0 without bank conflicts, 1 to random entries of a
// 1024-entry table (six values).  Returns 0 on success, -3 on a HIP error.
extern "C" int vegas_lds_atomic_rates(double* out, double clock_ghz, int n_cu)
{
    const int blocks = 4096, iters = 4096;
    float* buf = nullptr;
    if (hipMalloc(&buf, sizeof(float) * blocks) != hipSuccess) return -3;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    for (int k = 0; k < 6; ++k) {
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            hipEventRecord(a);
            switch (k) {
            case 0: hipLaunchKernelGGL((k_lds_atomic<0, 0>), dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 1: hipLaunchKernelGGL((k_lds_atomic<1, 0>), dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 2: hipLaunchKernelGGL((k_lds_atomic<2, 0>), dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 3: hipLaunchKernelGGL((k_lds_atomic<0, 1>), dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 4: hipLaunchKernelGGL((k_lds_atomic<1, 1>), dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 5: hipLaunchKernelGGL((k_lds_atomic<2, 1>), dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            }
            hipEventRecord(b);
            hipEventSynchronize(b);
        }
        hipEventElapsedTime(&ms, a, b);
        const double adds = (double)blocks * kBlock * iters;
        out[k] = adds / (ms * 1e-3 * clock_ghz * 1e9 * n_cu);
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(buf);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// out[op] = wave64 instructions retired per 4 cycles per SIMD for op kind
// 0 fma_f32, 1 mul+exp2_f32, 2 mad_u64_u32+xor, 3 fma_f64, 4 bitop3,
// 5 add_f64+rcp_f64, 6 exp2_f32 alone, 7 exp2_f32 and fma_f32 on
// independent chains, one exp2 to three fma (1.0 = one full-rate
// instruction every issue slot).
// Returns 0 on success, -3 on a HIP error.
extern "C" int vegas_issue_rates(double* out, int n_ops, double clock_ghz, int n_simd)
{
    const int blocks = 4096, iters = 2048;
    const int per_step[8] = {1, 2, 2, 1, 1, 2, 1, 1};
    float* buf = nullptr;
    if (hipMalloc(&buf, sizeof(float) * blocks * kBlock) != hipSuccess) return -3;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    for (int op = 0; op < n_ops && op < 8; ++op) {
        for (int rep = 0; rep < 2; ++rep) {
            hipEventRecord(a);
            switch (op) {
            case 0: hipLaunchKernelGGL(k_issue<0>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 1: hipLaunchKernelGGL(k_issue<1>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 2: hipLaunchKernelGGL(k_issue<2>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 3: hipLaunchKernelGGL(k_issue<3>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 4: hipLaunchKernelGGL(k_issue<4>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 5: hipLaunchKernelGGL(k_issue<5>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 6: hipLaunchKernelGGL(k_issue<6>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
            case 7: hipLaunchKernelGGL(k_issue<7>, dim3(blocks), dim3(kBlock), 0, 0, buf, iters); break;
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
