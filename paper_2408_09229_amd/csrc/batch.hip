// Many independent integrals advanced together: one VEGAS+ iteration of
// every problem of a batch with one launch per phase.
//
// The fill is one persistent launch.  Each problem's samples are cut into
// the same tiles the single-problem fill uses, and runs of consecutive tiles
// of one problem form work items.  Workgroups pop items from an atomic queue
// whose order puts the most expensive items first (longest processing time
// first), so problems of uneven dimension and budget share the chip with a
// short tail.  Per item the workgroup loads that problem's map and integrand
// constants into LDS, runs the tiles (Alg. 2, the same tile body as the
// single-problem fill, specialised by family and a dimension bound), and
// writes the item's histograms into a slot of its own and its partial sums
// into a record of its own.  Every later sum runs over those slots and
// records in item order, so the estimates do not depend on which workgroup
// took which item (the histogram bins themselves are LDS atomic sums, whose
// rounding follows the order of the adds, as in the single-problem fill).
//
// The update phases run per problem from block tables: the cube fix-up per
// tile, the iteration estimate per problem (one wavefront), the allocation
// (Eq. 7) per block of 4096 cubes with a per-problem scan of block sums, and
// the map refinement per (problem, axis).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "fill_dev.hpp"
#include "launch.hpp"
#include "layout.hpp"
#include "sample.hpp"
#include "update_dev.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// per-iteration reset: the problems' max-v / max-q for this iteration and the
// queue head
// ---------------------------------------------------------------------------
__global__ void k_batch_reset(BatchArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *a.next = 0u;
    if (i < a.n_inst) {
        unsigned long long* c = a.inst[i].ctr;
        c[a.t & 1u] = 0ull;
        c[2 + (a.t & 1u)] = 0ull;
    }
}

// ---------------------------------------------------------------------------
// the batched fill
// ---------------------------------------------------------------------------

// uniform (workgroup-wide) values loaded from memory the kernel also
// writes: the compiler cannot use scalar loads there, so the words are read
// with vector loads and moved to scalar registers
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int32_t uni(int32_t v) { return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v); }
template <typename T>
__device__ __forceinline__ T* uni(T* p)
{
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint64_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint64_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(uintptr_t)(lo | (hi << 32));
}
// a word-sized record, every word moved to scalar registers
template <typename T>
__device__ __forceinline__ T uni_struct(const T& src)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized records only");
    T out;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&src);
    uint32_t* d = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return out;
}
// What the fill loop hands to one work item (uniform over the workgroup).
struct ItemCall {
    uint32_t it;                // item index (problem order)
    uint32_t tile0, n_tiles;    // its tiles, local to the problem
    uint32_t t;                 // iteration
    int32_t cur;                // allocation buffer
    const BatchInst* in;
    TileSide* side;             // global side records
    double* item_part;
};

// One work item: load the problem's map and constants, run its tiles, write
// its histogram slot and partial sums.  All lanes call it.  A function of
// its own per (family, dimension bound), so that each keeps the register
// allocation of the single-problem fill; the call costs once per item.
template <typename R, int FAM, int MAXD, bool KAHAN>
__device__ __noinline__ void batch_item(ItemCall c0, unsigned char* smem)
{
    const ItemCall c = uni_struct(c0);
    const BatchInst& in = *c.in;
    const SampleConst sc = uni_struct(in.sc);
    const int D = sc.D;
    const int ng = (int)sc.ng;
    const int tid = threadIdx.x;
    const int tile_sz = uni(in.tile);
    const LdsPlan lp = lds_plan(D, ng, (int)sizeof(R), 1, tile_sz, sc.n_aux, 1);
    const FillLds<R> L(smem, lp);
    const int nbins = D * ng;
    const R* gsrc = std::is_same<R, double>::value ? reinterpret_cast<const R*>(uni(in.grid64))
                                                   : reinterpret_cast<const R*>(uni(in.grid32));
    for (int i = tid; i < D * (ng + 1); i += kFillThreads) L.gl[i] = gsrc[i];
    const R* asrc = std::is_same<R, double>::value ? reinterpret_cast<const R*>(sc.aux_d)
                                                   : reinterpret_cast<const R*>(sc.aux_f);
    for (int i = tid; i < sc.n_aux; i += kFillThreads) L.auxl[i] = asrc[i];
    for (int i = tid; i < nbins; i += kFillThreads) {
        L.hl[i] = 0.0;
        L.cl[i] = 0u;
    }
    __syncthreads();

    SamplePath<R, FAM, MAXD> sp(sc, L.auxl);
    LaneTotal<KAHAN> totI, totV;
    double vmax = 0.0;
    unsigned long long bad = 0;
    TileIO io;
    io.grid = nullptr;
    io.t = c.t;
    io.tile = tile_sz;
    io.per_lane = uni(in.per_lane);
    io.lds_hist = 1;
    io.start = uni(in.start[c.cur]);
    io.tile_first = uni(in.tfirst[c.cur]);
    io.v_out = uni(in.v);
    io.side = c.side + uni(in.tile0);
    io.hist_H = nullptr;
    io.hist_C = nullptr;
    io.hist_Cw = nullptr;
    for (uint32_t j = 0; j < c.n_tiles; ++j)
        fill_tile<R, MAXD, KAHAN, false>((int)(c.tile0 + j), io, L, sp, totI, totV, vmax, bad);

    // histograms into the item's slot
    const size_t slot = (size_t)(c.it - uni(in.item0)) * (size_t)nbins;
    double* hH = uni(in.hist_H) + slot;
    uint32_t* hC = uni(in.hist_C) + slot;
    for (int i = tid; i < nbins; i += kFillThreads) {
        hH[i] = L.hl[i];
        hC[i] = L.cl[i];
    }
    double sI, sV, mx;
    wg_reduce_totals(totI.value(), totV.value(), vmax, L.red, sI, sV, mx);
    unsigned long long* ctr = uni(in.ctr);
    if (tid == 0) {
        c.item_part[2 * (size_t)c.it] = sI;
        c.item_part[2 * (size_t)c.it + 1] = sV;
        atomicMax(ctr + (c.t & 1u), (unsigned long long)__double_as_longlong(mx));
    }
    if (bad) atomicAdd(ctr + 4, bad);
}

template <typename R, int FAM, bool KAHAN>
__device__ __forceinline__ void batch_item_dim(const ItemCall& c, int D, unsigned char* smem)
{
    if (D <= 4) batch_item<R, FAM, 4, KAHAN>(c, smem);
    else if (D <= 8) batch_item<R, FAM, 8, KAHAN>(c, smem);
    else batch_item<R, FAM, 12, KAHAN>(c, smem);
}

template <typename R, bool KAHAN>
__global__ __launch_bounds__(kFillThreads) void k_batch_fill(BatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t pop;
    for (;;) {
        if (threadIdx.x == 0) pop = atomicAdd(a.next, 1u);
        __syncthreads();
        // the item index is uniform over the workgroup: keep it (and the
        // records it selects) in scalar registers
        const uint32_t q = __builtin_amdgcn_readfirstlane(pop);
        __syncthreads();
        if (q >= (uint32_t)a.n_items) break;
        const uint32_t it = __builtin_amdgcn_readfirstlane(a.order[q]);
        const BatchItem bi = uni_struct(a.items[it]);
        const BatchInst& in = a.inst[bi.inst];
        ItemCall c;
        c.it = it;
        c.tile0 = bi.tile0;
        c.n_tiles = bi.n_tiles;
        c.t = a.t;
        c.cur = a.cur;
        c.in = &in;
        c.side = a.side;
        c.item_part = a.item_part;
        const int D = uni(in.sc.D);
        switch (uni(in.sc.family)) {
        case F_GENZ_PPEAK: batch_item_dim<R, F_GENZ_PPEAK, KAHAN>(c, D, smem); break;
        case F_GENZ_GAUSS: batch_item_dim<R, F_GENZ_GAUSS, KAHAN>(c, D, smem); break;
        default: batch_item_dim<R, F_GAUSS_DIAG, KAHAN>(c, D, smem); break;
        }
    }
}

// ---------------------------------------------------------------------------
// cubes crossing tiles, then the per-problem iteration estimate
// ---------------------------------------------------------------------------
__global__ void k_batch_fixup(BatchArgs a)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n_tiles) return;
    const BatchInst& in = a.inst[a.tile_inst[g]];
    fixup_chain(a.side + in.tile0, in.n_tiles, g - (int)in.tile0, in.v, in.ctr + (a.t & 1u), a.fix_part + 2 * (size_t)g);
}

// one wavefront per problem: item partials then tile fix-ups, each lane
// striding in order, lanes combined by a fixed shuffle tree
__global__ __launch_bounds__(256) void k_batch_final(BatchArgs a)
{
    const int w = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= a.n_inst) return;
    const BatchInst& in = a.inst[w];
    double sI = 0.0, sV = 0.0;
    for (uint32_t i = lane; i < in.n_items; i += 64) {
        sI += a.item_part[2 * (size_t)(in.item0 + i)];
        sV += a.item_part[2 * (size_t)(in.item0 + i) + 1];
    }
    for (uint32_t j = lane; j < (uint32_t)in.n_tiles; j += 64) {
        sI += a.fix_part[2 * (size_t)(in.tile0 + j)];
        sV += a.fix_part[2 * (size_t)(in.tile0 + j) + 1];
    }
    for (int o = 32; o > 0; o >>= 1) {
        sI += __shfl_down(sI, o, 64);
        sV += __shfl_down(sV, o, 64);
    }
    if (lane == 0) {
        const double nc = (double)in.sc.n_cubes;
        in.iter[2 * (size_t)a.t] = sI / nc;
        in.iter[2 * (size_t)a.t + 1] = sV / (nc * nc);
    }
}

// ---------------------------------------------------------------------------
// allocation (Eq. 7), per problem, into start buffer 1 - cur
// ---------------------------------------------------------------------------
__device__ __forceinline__ AllocArgs inst_alloc(const BatchArgs& a, const BatchInst& in)
{
    AllocArgs r;
    r.n_cubes = in.sc.n_cubes;
    r.n_min = in.n_min;
    r.R = in.R;
    r.n_eval = in.sc.n_eval;
    r.beta = in.beta;
    r.uniform = (a.force_uniform || !in.adapt_strat || !(in.beta > 0.0)) ? 1 : 0;
    r.tile = in.tile;
    r.tile_shift = in.tile_shift;
    r.n_tiles = in.n_tiles;
    r.per_block = kAllocPerBlock;
    r.v = in.v;
    r.vmax = in.ctr + (a.t & 1u);
    r.qmax_buf = nullptr;
    r.bsum = in.bsum;
    r.boff = in.boff;
    r.start = in.start[1 - a.cur];
    r.tile_first = in.tfirst[1 - a.cur];
    r.qbuf = nullptr;
    return r;
}

__global__ __launch_bounds__(kAllocThreads) void k_batch_alloc_qmax(BatchArgs a)
{
    __shared__ double red[kAllocThreads];
    const BatchInst& in = a.inst[a.blk_inst[blockIdx.x]];
    const AllocArgs r = inst_alloc(a, in);
    if (r.uniform || beta_monotone(r.beta)) return;
    alloc_qmax_block(r, blockIdx.x - in.blk0, in.ctr + 2 + (a.t & 1u), red);
}

__global__ __launch_bounds__(kAllocThreads) void k_batch_alloc_sum(BatchArgs a)
{
    __shared__ uint64_t sh[kAllocThreads / 64 + 1];
    const BatchInst& in = a.inst[a.blk_inst[blockIdx.x]];
    const AllocArgs r = inst_alloc(a, in);
    const uint32_t b = blockIdx.x - in.blk0;
    alloc_sum_block(r, in.ctr + 2 + (a.t & 1u), b, in.bsum + b, sh);
}

// one wavefront per problem: exclusive scan of its block sums in order
__global__ __launch_bounds__(256) void k_batch_alloc_scan(BatchArgs a)
{
    const int w = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= a.n_inst) return;
    const BatchInst& in = a.inst[w];
    uint64_t carry = 0;
    for (uint32_t base = 0; base < in.n_blk; base += 64) {
        const uint32_t i = base + (uint32_t)lane;
        const uint64_t v = i < in.n_blk ? (uint64_t)in.bsum[i] : 0ull;
        uint64_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (i < in.n_blk) in.boff[i] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    if (lane == 0) in.boff[in.n_blk] = carry;
}

__global__ __launch_bounds__(kAllocThreads) void k_batch_alloc_write(BatchArgs a)
{
    __shared__ uint64_t sh[kAllocThreads / 64 + 1];
    const BatchInst& in = a.inst[a.blk_inst[blockIdx.x]];
    const AllocArgs r = inst_alloc(a, in);
    const uint32_t b = blockIdx.x - in.blk0;
    alloc_write_block(r, in.ctr + 2 + (a.t & 1u), b, in.boff[b], in.boff[in.n_blk], sh);
}

// ---------------------------------------------------------------------------
// map refinement: one workgroup per (problem, axis); the item slots of the
// problem are added in item order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_batch_map(BatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double S_sh;
    const uint32_t e = a.axis_inst[blockIdx.x];
    const BatchInst& in = a.inst[e >> 4];
    MapArgs m;
    m.D = in.sc.D;
    m.ng = (int)in.sc.ng;
    m.n_slots = (int)in.n_items;
    m.parts = 0;
    m.alpha = in.adapt_map ? in.alpha : 0.0;
    m.hist_H = in.hist_H;
    m.hist_C = in.hist_C;
    m.grid64 = in.grid64;
    m.grid32 = in.grid32;
    m.Hsum = nullptr;
    m.Csum = nullptr;
    map_update_axis(m, (int)(e & 15u), smem, S_sh);
}

// ---------------------------------------------------------------------------
// set-up: derived constants and the uniform grid, one workgroup per problem
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_prep(BatchArgs a)
{
    const BatchInst& in = a.inst[blockIdx.x];
    PrepArgs p;
    p.family = in.sc.family;
    p.D = in.sc.D;
    p.n_params = in.sc.n_params;
    p.prm = in.sc.prm;
    p.lo = in.lo;
    p.hi = in.hi;
    p.ng = (int)in.sc.ng;
    p.aux_d = const_cast<double*>(in.sc.aux_d);
    p.aux_f = const_cast<float*>(in.sc.aux_f);
    p.grid64 = in.grid64;
    p.grid32 = in.grid32;
    prep_problem(p, threadIdx.x, blockDim.x);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t st)
{
    const int n = a.n_inst > 1 ? a.n_inst : 1;
    hipLaunchKernelGGL(k_batch_reset, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename R, bool KAHAN>
static hipError_t launch_batch_fill_k(const BatchArgs& a, int n_wg, size_t lds, hipStream_t st)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_batch_fill<R, KAHAN>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_batch_fill<R, KAHAN>), dim3(n_wg), dim3(kFillThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_fill(const BatchArgs& a, bool fp64, bool kahan, int n_wg, size_t lds, hipStream_t st)
{
    if (fp64) return launch_batch_fill_k<double, false>(a, n_wg, lds, st);
    if (kahan) return launch_batch_fill_k<float, true>(a, n_wg, lds, st);
    return launch_batch_fill_k<float, false>(a, n_wg, lds, st);
}

hipError_t launch_batch_estimate(const BatchArgs& a, hipStream_t st)
{
    if (a.n_tiles > 0)
        hipLaunchKernelGGL(k_batch_fixup, dim3((a.n_tiles + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_final, dim3((a.n_inst + 3) / 4), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_alloc(const BatchArgs& a, bool any_general_beta, hipStream_t st)
{
    if (any_general_beta && !a.force_uniform)
        hipLaunchKernelGGL(k_batch_alloc_qmax, dim3(a.n_blk), dim3(kAllocThreads), 0, st, a);
    hipLaunchKernelGGL(k_batch_alloc_sum, dim3(a.n_blk), dim3(kAllocThreads), 0, st, a);
    hipLaunchKernelGGL(k_batch_alloc_scan, dim3((a.n_inst + 3) / 4), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_alloc_write, dim3(a.n_blk), dim3(kAllocThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_map(const BatchArgs& a, int max_ng, hipStream_t st)
{
    const size_t lds = (size_t)3 * (max_ng + 1) * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)k_batch_map, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_map, dim3(a.n_axes), dim3(1024), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_prep(const BatchArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_prep, dim3(a.n_inst), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace vg
