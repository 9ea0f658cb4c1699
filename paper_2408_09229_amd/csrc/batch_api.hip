// C ABI of the batched VEGAS+ path (include/vegas.h, vegas_batch_*).
//
// A batch holds n independent problems (each with its own dimension,
// intervals, budget, integrand and Philox stream) that advance one
// iteration at a time together, under one of two launch schedules:
//  - streams: one single-problem context per problem (the kernels of one
//    problem are the single-problem kernels), the problems spread over a
//    few streams of the batch, longest first onto the least loaded stream;
//    fork from and join to the caller's stream around every iteration.  An
//    autotuner times the fill of all problems under each stream count and
//    keeps the fastest in a text cache.
//  - persistent: one persistent fill launch for all problems, then batched
//    estimate, allocation and map kernels (batch.hip).  Switched off: its
//    first device run faulted and the cause is not yet found.
//
// Host work of the persistent schedule: validation, the work layout (tile
// size per problem, tiles per work item, the longest-first queue order),
// workspace carving, its autotuner over layouts, and the Eq. 8-9
// combination per problem on request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/vegas.h"
#include "common.hpp"
#include "host.hpp"
#include "launch.hpp"

using namespace vg;
using namespace vgh;

namespace {

constexpr int kBatchMaxDim = 12;
constexpr int kBatchDefaultLog = 256;      // iteration log capacity when max_iter = 0
constexpr bool kPersistentDisabled = true;

// streams schedule: candidate stream counts (the first entry after the
// default is timed first) and the default without tuning
const int kStreamCandidates[] = {1, 2, 4, 8};
constexpr int kDefaultStreams = 4;
constexpr int kMaxStreams = 8;

// A work layout: samples per lane (upper bound; small problems use fewer)
// and the target number of samples in one work item.
struct Layout {
    int per_lane;
    int64_t item_samples;
};

// Layouts the autotuner times; the first is the default without tuning.
const Layout kCandidates[] = {
    {8, 1 << 18}, {4, 1 << 18}, {2, 1 << 18}, {8, 1 << 20}, {4, 1 << 16}, {2, 1 << 16},
};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);

// per-problem tile layout under a Layout
struct InstLayout {
    int per_lane, tile, tile_shift, n_tiles, tiles_per_item, n_items, n_blk;
};

InstLayout inst_layout(const Geometry& g, const Layout& L)
{
    InstLayout r;
    int p = L.per_lane;
    while (p > 1 && (int64_t)g.n_eval < (int64_t)2 * kFillThreads * p) p >>= 1;
    r.per_lane = p;
    r.tile = kFillThreads * p;
    r.tile_shift = 0;
    while ((1 << r.tile_shift) < r.tile) ++r.tile_shift;
    r.n_tiles = (int)(((int64_t)g.n_eval + r.tile - 1) / r.tile);
    r.tiles_per_item = (int)std::max<int64_t>(1, L.item_samples / r.tile);
    r.n_items = (r.n_tiles + r.tiles_per_item - 1) / r.tiles_per_item;
    r.n_blk = (int)(((int64_t)g.n_cubes + kAllocPerBlock - 1) / kAllocPerBlock);
    return r;
}

// Workspace offsets.  Global arrays first, then per problem.
struct BatchPlan {
    size_t inst, items, order, tile_inst, blk_inst, axis_inst, next, item_part, side, fix_part, consts, iter, ctr;
    std::vector<size_t> aux_d, aux_f, grid64, grid32, start0, start1, tf0, tf1, v, histH, histC, bsum, boff;
    std::vector<size_t> c_prm, c_lo, c_hi;      // element offsets into consts (doubles)
    std::vector<InstLayout> il;
    int64_t n_items, n_tiles, n_blk, n_axes;
    size_t total;
};

BatchPlan batch_plan(const std::vector<Geometry>& gs, const Layout& L, int max_iter)
{
    BatchPlan p;
    const size_t n = gs.size();
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    p.il.resize(n);
    p.n_items = p.n_tiles = p.n_blk = p.n_axes = 0;
    size_t nconst = 0;
    p.c_prm.resize(n);
    p.c_lo.resize(n);
    p.c_hi.resize(n);
    for (size_t i = 0; i < n; ++i) {
        p.il[i] = inst_layout(gs[i], L);
        p.n_items += p.il[i].n_items;
        p.n_tiles += p.il[i].n_tiles;
        p.n_blk += p.il[i].n_blk;
        p.n_axes += gs[i].D;
        p.c_prm[i] = nconst;
        nconst += gs[i].n_params;
        p.c_lo[i] = nconst;
        nconst += gs[i].D;
        p.c_hi[i] = nconst;
        nconst += gs[i].D;
    }
    p.inst = take(sizeof(BatchInst) * n);
    p.items = take(sizeof(BatchItem) * p.n_items);
    p.order = take(sizeof(uint32_t) * p.n_items);
    p.tile_inst = take(sizeof(uint32_t) * p.n_tiles);
    p.blk_inst = take(sizeof(uint32_t) * p.n_blk);
    p.axis_inst = take(sizeof(uint32_t) * p.n_axes);
    p.next = take(sizeof(unsigned int) * 4);
    p.item_part = take(sizeof(double) * 2 * p.n_items);
    p.side = take(sizeof(TileSide) * p.n_tiles);
    p.fix_part = take(sizeof(double) * 2 * p.n_tiles);
    p.consts = take(sizeof(double) * nconst);
    p.iter = take(sizeof(double) * 2 * (size_t)max_iter * n);
    p.ctr = take(sizeof(unsigned long long) * 8 * n);
    for (auto* v : {&p.aux_d, &p.aux_f, &p.grid64, &p.grid32, &p.start0, &p.start1, &p.tf0, &p.tf1, &p.v, &p.histH,
                    &p.histC, &p.bsum, &p.boff})
        v->resize(n);
    for (size_t i = 0; i < n; ++i) {
        const Geometry& g = gs[i];
        const InstLayout& il = p.il[i];
        const size_t row = (size_t)g.D * (g.ng + 1);
        const size_t nb = (size_t)g.D * g.ng;
        p.aux_d[i] = take(sizeof(double) * g.n_aux);
        p.aux_f[i] = take(sizeof(float) * g.n_aux);
        p.grid64[i] = take(sizeof(double) * row);
        p.grid32[i] = take(sizeof(float) * row);
        p.start0[i] = take(sizeof(uint32_t) * ((size_t)g.n_cubes + 1));
        p.start1[i] = take(sizeof(uint32_t) * ((size_t)g.n_cubes + 1));
        p.tf0[i] = take(sizeof(uint32_t) * ((size_t)il.n_tiles + 1));
        p.tf1[i] = take(sizeof(uint32_t) * ((size_t)il.n_tiles + 1));
        p.v[i] = take(sizeof(double) * g.n_cubes);
        p.histH[i] = take(sizeof(double) * nb * il.n_items);
        p.histC[i] = take(sizeof(uint32_t) * nb * il.n_items);
        p.bsum[i] = take(sizeof(unsigned long long) * il.n_blk);
        p.boff[i] = take(sizeof(unsigned long long) * ((size_t)il.n_blk + 1));
    }
    p.total = o;
    return p;
}

// validation of the batch as a whole; fills gs
vegas_status batch_geometry(int32_t n, const vegas_config* cfgs, const vegas_integrand* fs, int32_t schedule,
                            std::vector<Geometry>& gs, int* max_iter)
{
    if (n < 1 || n > (1 << 20)) return fail(VEGAS_EINVAL, "batch size must be 1..2^20");
    if (!cfgs || !fs) return fail(VEGAS_EINVAL, "null configs or integrands");
    if (schedule != VEGAS_BATCH_STREAMS && schedule != VEGAS_BATCH_PERSISTENT)
        return fail(VEGAS_EINVAL, "unknown batch schedule %d", schedule);
    gs.resize(n);
    int mi = 0;
    for (int i = 0; i < n; ++i) {
        const vegas_config& c = cfgs[i];
        const bool ordered_ok = schedule == VEGAS_BATCH_STREAMS && c.accum == VEGAS_ACC_ORDERED;
        if (c.accum != VEGAS_ACC_FP64 && c.accum != VEGAS_ACC_KAHAN && !ordered_ok)
            return fail(VEGAS_EUNSUPPORTED, "problem %d: a batch accumulates in FP64 or KAHAN form (or ORDERED "
                                            "under the streams schedule)", i);
        if (c.precision != cfgs[0].precision || c.accum != cfgs[0].accum)
            return fail(VEGAS_EINVAL, "problem %d: precision and accumulation must agree across the batch", i);
        const vegas_status s = geometry(&c, &fs[i], &gs[i]);
        if (s != VEGAS_OK) {
            std::string m = vegas_last_error();
            return fail(s, "problem %d: %s", i, m.c_str());
        }
        const int fam = fs[i].family;
        if (fam != VEGAS_GENZ_PPEAK && fam != VEGAS_GENZ_GAUSS && fam != VEGAS_GAUSS_DIAG)
            return fail(VEGAS_EUNSUPPORTED, "problem %d: batched families are GENZ_PPEAK, GENZ_GAUSS, GAUSS_DIAG", i);
        if (c.dim > kBatchMaxDim) return fail(VEGAS_EUNSUPPORTED, "problem %d: batched problems have dim <= %d", i, kBatchMaxDim);
        const bool fp64 = c.precision == VEGAS_PREC_FP64;
        const int tile_max = kFillThreads * 8;
        if (fill_lds_bytes(gs[i].D, gs[i].ng, fp64, 1, tile_max, gs[i].n_aux, 1) > kLdsLimit)
            return fail(VEGAS_EUNSUPPORTED, "problem %d: map and histograms of %d x %d intervals exceed LDS", i,
                        gs[i].D, gs[i].ng);
        mi = std::max(mi, c.max_iter);
    }
    *max_iter = mi > 0 ? mi : kBatchDefaultLog;
    return VEGAS_OK;
}

size_t batch_bytes(const std::vector<Geometry>& gs, int max_iter)
{
    size_t b = 0;
    for (const Layout& L : kCandidates) b = std::max(b, batch_plan(gs, L, max_iter).total);
    return b;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n)
{
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

}  // namespace

struct vegas_batch {
    int n;
    std::vector<vegas_config> cfg;
    std::vector<Geometry> g;
    std::vector<double> consts;        // params, lo, hi of every problem (plan order)
    bool fp64, kahan, any_general_beta;
    int max_ng;
    int max_iter;
    hipStream_t stream;
    unsigned char* ws;
    size_t ws_bytes;
    int n_wg;
    int cur;
    int n_run;
    std::vector<uint8_t> combined;
    Layout layout;
    BatchPlan p;
    size_t lds;
    int tuned;                         // 0 default layout, 1 timed now, 2 from the cache
    double tune_ms;
    bool timing;
    std::vector<hipEvent_t> events;

    // streams schedule
    bool streams = false;
    std::vector<vegas_ctx*> ctx;           // one per problem
    std::vector<size_t> ctx_off;           // its workspace slice
    std::vector<hipStream_t> lanes;        // kMaxStreams streams of the batch
    std::vector<hipEvent_t> joins;         // one per stream
    hipEvent_t fork = nullptr;
    int n_lanes = 0;                       // streams in use
    std::vector<uint32_t> order;           // problems, most expensive first

    ~vegas_batch()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (vegas_ctx* c : ctx)
            if (c) vegas_destroy(c);
        for (hipEvent_t e : joins) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        for (hipStream_t q : lanes) (void)hipStreamDestroy(q);
    }
    hipError_t mark()
    {
        if (!timing) return hipSuccess;
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        events.push_back(e);
        return hipEventRecord(e, stream);
    }
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

BatchArgs batch_args(const vegas_batch* b, uint32_t t, int force_uniform)
{
    BatchArgs a;
    a.n_inst = b->n;
    a.n_items = (int32_t)b->p.n_items;
    a.n_tiles = (int32_t)b->p.n_tiles;
    a.n_blk = (int32_t)b->p.n_blk;
    a.n_axes = (int32_t)b->p.n_axes;
    a.t = t;
    a.cur = b->cur;
    a.force_uniform = force_uniform;
    a.inst = b->at<BatchInst>(b->p.inst);
    a.items = b->at<BatchItem>(b->p.items);
    a.order = b->at<uint32_t>(b->p.order);
    a.tile_inst = b->at<uint32_t>(b->p.tile_inst);
    a.blk_inst = b->at<uint32_t>(b->p.blk_inst);
    a.axis_inst = b->at<uint32_t>(b->p.axis_inst);
    a.next = b->at<unsigned int>(b->p.next);
    a.item_part = b->at<double>(b->p.item_part);
    a.side = b->at<TileSide>(b->p.side);
    a.fix_part = b->at<double>(b->p.fix_part);
    a.nonfinite = nullptr;
    return a;
}

// Carve the workspace for layout L, upload the tables, set up every problem
// (constants, uniform map, uniform allocation into buffer 0) and clear the
// counters.  Valid only before the first iteration.
vegas_status apply_layout(vegas_batch* b, const Layout& L)
{
    BatchPlan p = batch_plan(b->g, L, b->max_iter);
    if (p.total > b->ws_bytes) return fail(VEGAS_ENOMEM, "workspace has %zu bytes, layout needs %zu", b->ws_bytes, p.total);
    if (p.n_tiles >= INT32_MAX || p.n_items >= INT32_MAX || p.n_blk >= INT32_MAX)
        return fail(VEGAS_EUNSUPPORTED, "batch too large for 32-bit tile and block tables");
    const int n = b->n;
    std::vector<BatchInst> inst(n);
    std::vector<BatchItem> items(p.n_items);
    std::vector<uint32_t> tile_inst(p.n_tiles), blk_inst(p.n_blk), axis_inst(p.n_axes);
    std::vector<double> cost(p.n_items);
    double* consts = b->at<double>(p.consts);
    uint32_t item0 = 0, tile0 = 0, blk0 = 0, ax = 0;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        const Geometry& g = b->g[i];
        const vegas_config& c = b->cfg[i];
        const InstLayout& il = p.il[i];
        BatchInst& r = inst[i];
        std::memset(&r, 0, sizeof r);
        SampleConst& s = r.sc;
        s.D = g.D;
        s.ng = (uint32_t)g.ng;
        s.nst = g.nst;
        s.nst_magic = g.magic;
        s.nst_shift = g.shift;
        s.n_eval = g.n_eval;
        s.n_cubes = g.n_cubes;
        s.key0 = (uint32_t)c.seed;
        s.key1 = (uint32_t)(c.seed >> 32);
        s.ctr3 = c.instance << 8;
        s.family = g.family;
        s.n_params = g.n_params;
        s.prm = consts + p.c_prm[i];
        s.aux_d = b->at<double>(p.aux_d[i]);
        s.aux_f = b->at<float>(p.aux_f[i]);
        s.n_aux = g.n_aux;
        r.alpha = c.alpha;
        r.beta = c.beta;
        r.R = g.R;
        r.n_min = (uint32_t)g.n_min;
        r.adapt_strat = c.adapt_strat;
        r.adapt_map = c.adapt_map;
        r.per_lane = il.per_lane;
        r.tile = il.tile;
        r.tile_shift = il.tile_shift;
        r.n_tiles = il.n_tiles;
        r.tile0 = tile0;
        r.item0 = item0;
        r.n_items = (uint32_t)il.n_items;
        r.blk0 = blk0;
        r.n_blk = (uint32_t)il.n_blk;
        r.lo = consts + p.c_lo[i];
        r.hi = consts + p.c_hi[i];
        r.grid64 = b->at<double>(p.grid64[i]);
        r.grid32 = b->at<float>(p.grid32[i]);
        r.start[0] = b->at<uint32_t>(p.start0[i]);
        r.start[1] = b->at<uint32_t>(p.start1[i]);
        r.tfirst[0] = b->at<uint32_t>(p.tf0[i]);
        r.tfirst[1] = b->at<uint32_t>(p.tf1[i]);
        r.v = b->at<double>(p.v[i]);
        r.hist_H = b->at<double>(p.histH[i]);
        r.hist_C = b->at<uint32_t>(p.histC[i]);
        r.bsum = b->at<unsigned long long>(p.bsum[i]);
        r.boff = b->at<unsigned long long>(p.boff[i]);
        r.ctr = b->at<unsigned long long>(p.ctr) + 8 * (size_t)i;
        r.iter = b->at<double>(p.iter) + 2 * (size_t)b->max_iter * i;
        // items: runs of tiles_per_item tiles; cost ~ samples x per-sample work
        const double per_sample = 16.0 + 6.0 * g.D;
        for (int j = 0; j < il.n_items; ++j) {
            BatchItem& it = items[item0 + j];
            it.inst = (uint32_t)i;
            it.tile0 = (uint32_t)(j * il.tiles_per_item);
            it.n_tiles = (uint32_t)std::min(il.tiles_per_item, il.n_tiles - j * il.tiles_per_item);
            it.pad = 0;
            const int64_t k0 = (int64_t)it.tile0 * il.tile;
            const int64_t k1 = std::min<int64_t>((int64_t)(it.tile0 + it.n_tiles) * il.tile, g.n_eval);
            cost[item0 + j] = (double)(k1 - k0) * per_sample + 4096.0 * it.n_tiles;
        }
        for (int j = 0; j < il.n_tiles; ++j) tile_inst[tile0 + j] = (uint32_t)i;
        for (int j = 0; j < il.n_blk; ++j) blk_inst[blk0 + j] = (uint32_t)i;
        for (int d = 0; d < g.D; ++d) axis_inst[ax++] = ((uint32_t)i << 4) | (uint32_t)d;
        item0 += il.n_items;
        tile0 += il.n_tiles;
        blk0 += il.n_blk;
        lds = std::max(lds, fill_lds_bytes(g.D, g.ng, b->fp64, 1, il.tile, g.n_aux, 1));
    }
    // queue order: longest first; ties by item index, so the order is fixed
    std::vector<uint32_t> order(p.n_items);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });

    hipStream_t st = b->stream;
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(b->at<void>(p.inst), inst.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->at<void>(p.items), items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->at<void>(p.order), order.data(), sizeof(uint32_t) * order.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->at<void>(p.tile_inst), tile_inst.data(), sizeof(uint32_t) * tile_inst.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->at<void>(p.blk_inst), blk_inst.data(), sizeof(uint32_t) * blk_inst.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->at<void>(p.axis_inst), axis_inst.data(), sizeof(uint32_t) * axis_inst.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(consts, b->consts.data(), sizeof(double) * b->consts.size(), hipMemcpyHostToDevice));
    b->p = std::move(p);
    b->layout = L;
    b->lds = lds;
    HIPCHK(launch_reset(b->at<unsigned long long>(b->p.ctr), 8 * n, st));
    BatchArgs a = batch_args(b, 0, 1);
    HIPCHK(launch_batch_prep(a, st));
    // uniform allocation into buffer 0
    b->cur = 1;
    a = batch_args(b, 0, 1);
    HIPCHK(launch_batch_alloc(a, false, st));
    b->cur = 0;
    HIPCHK(hipStreamSynchronize(st));
    return VEGAS_OK;
}

// one fill of iteration 0 under the current layout, timed with events
vegas_status time_fill(vegas_batch* b, float* ms)
{
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    BatchArgs a = batch_args(b, 0, 0);
    hipError_t r = launch_batch_reset(a, b->stream);
    if (r == hipSuccess) r = hipEventRecord(e0, b->stream);
    if (r == hipSuccess) r = launch_batch_fill(a, b->fp64, b->kahan, b->n_wg, b->lds, b->stream);
    if (r == hipSuccess) r = hipEventRecord(e1, b->stream);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    if (r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(r);
    return VEGAS_OK;
}

uint64_t batch_key(const vegas_batch* b)
{
    uint64_t h = 0xcbf29ce484222325ull;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
        h = fnv1a(h, &prop.multiProcessorCount, sizeof prop.multiProcessorCount);
    }
    const int32_t head[3] = {b->n, b->fp64 ? 1 : 0, b->kahan ? 1 : 0};
    h = fnv1a(h, head, sizeof head);
    for (int i = 0; i < b->n; ++i) {
        const Geometry& g = b->g[i];
        const int64_t v[6] = {g.D, g.family, g.ng, (int64_t)g.n_eval, (int64_t)g.nst, g.n_aux};
        h = fnv1a(h, v, sizeof v);
    }
    return h;
}

bool cache_lookup(const char* path, uint64_t key, Layout* L, double* ms)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool hit = false;
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long k;
        int pl;
        long long is;
        double t;
        if (std::sscanf(line, "%llx %d %lld %lf", &k, &pl, &is, &t) != 4 || k != key) continue;
        for (const Layout& c : kCandidates)
            if (c.per_lane == pl && c.item_samples == is) {
                *L = c;
                *ms = t;
                hit = true;
            }
    }
    std::fclose(f);
    return hit;
}

void cache_store(const char* path, uint64_t key, const Layout& L, double ms)
{
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%016llx %d %lld %.6f\n", (unsigned long long)key, L.per_lane, (long long)L.item_samples, ms);
    std::fclose(f);
}

// time every candidate layout (one warm-up fill, best of two timed fills)
// and keep the fastest
vegas_status autotune(vegas_batch* b, Layout* best, double* best_ms)
{
    double bm = INFINITY;
    Layout bl = kCandidates[0];
    for (const Layout& L : kCandidates) {
        vegas_status s = apply_layout(b, L);
        if (s == VEGAS_ENOMEM) continue;
        if (s != VEGAS_OK) return s;
        float t0 = 0.f, t1 = 0.f, t2 = 0.f;
        if ((s = time_fill(b, &t0)) != VEGAS_OK) return s;
        if ((s = time_fill(b, &t1)) != VEGAS_OK) return s;
        if ((s = time_fill(b, &t2)) != VEGAS_OK) return s;
        const double t = std::min(t1, t2);
        if (t < bm) {
            bm = t;
            bl = L;
        }
    }
    *best = bl;
    *best_ms = bm;
    return VEGAS_OK;
}

vegas_status batch_iteration(vegas_batch* b, bool integrate)
{
    if (b->n_run >= b->max_iter) return fail(VEGAS_ESTATE, "iteration log full (max_iter = %d)", b->max_iter);
    const uint32_t t = (uint32_t)b->n_run;
    hipStream_t st = b->stream;
    BatchArgs a = batch_args(b, t, 0);
    HIPCHK(launch_batch_reset(a, st));
    HIPCHK(b->mark());
    HIPCHK(launch_batch_fill(a, b->fp64, b->kahan, b->n_wg, b->lds, st));
    HIPCHK(b->mark());
    HIPCHK(launch_batch_estimate(a, st));
    HIPCHK(b->mark());
    HIPCHK(launch_batch_alloc(a, b->any_general_beta, st));
    b->cur = 1 - b->cur;
    HIPCHK(b->mark());
    HIPCHK(launch_batch_map(a, b->max_ng, st));
    HIPCHK(b->mark());
    b->n_run = (int)t + 1;
    b->combined.push_back(integrate ? 1 : 0);
    return VEGAS_OK;
}


// ---------------------------------------------------------------------------
// streams schedule
// ---------------------------------------------------------------------------

// workspace slices: problem i as a single context whose log holds max_iter
vegas_status streams_layout(int32_t n, const vegas_config* cfgs, const vegas_integrand* fs, int max_iter,
                            std::vector<size_t>* off, size_t* total)
{
    size_t o = 0;
    if (off) off->resize(n);
    for (int i = 0; i < n; ++i) {
        vegas_config c = cfgs[i];
        c.max_iter = max_iter;
        size_t bytes = 0;
        const vegas_status s = vegas_workspace_size(&c, &fs[i], &bytes);
        if (s != VEGAS_OK) {
            std::string m = vegas_last_error();
            return fail(s, "problem %d: %s", i, m.c_str());
        }
        if (off) (*off)[i] = o;
        o += (bytes + 255) & ~(size_t)255;
    }
    *total = o;
    return VEGAS_OK;
}

// relative cost of one iteration of a problem: samples times per-sample
// work, plus the fixed cost of its dozen small launches
double problem_cost(const Geometry& g) { return (double)g.n_eval * (16.0 + 6.0 * g.D) + 2.0e6; }

// spread the problems over S streams: most expensive first, each onto the
// stream with the least work so far (ties to the lower index).  Only between
// iterations, with every stream idle.
void assign_lanes(vegas_batch* b, int S)
{
    std::vector<double> load(S, 0.0);
    for (uint32_t i : b->order) {
        int q = 0;
        for (int r = 1; r < S; ++r)
            if (load[r] < load[q]) q = r;
        load[q] += problem_cost(b->g[i]);
        ctx_set_stream(b->ctx[i], b->lanes[q]);
    }
    b->n_lanes = S;
}

// the streams in use start after the work queued on the caller's stream ...
vegas_status fork_lanes(vegas_batch* b)
{
    HIPCHK(hipEventRecord(b->fork, b->stream));
    for (int q = 0; q < b->n_lanes; ++q) HIPCHK(hipStreamWaitEvent(b->lanes[q], b->fork, 0));
    return VEGAS_OK;
}

// ... and the caller's stream waits for all of them
vegas_status join_lanes(vegas_batch* b)
{
    for (int q = 0; q < b->n_lanes; ++q) {
        HIPCHK(hipEventRecord(b->joins[q], b->lanes[q]));
        HIPCHK(hipStreamWaitEvent(b->stream, b->joins[q], 0));
    }
    return VEGAS_OK;
}

vegas_status sync_lanes(vegas_batch* b)
{
    for (hipStream_t q : b->lanes) HIPCHK(hipStreamSynchronize(q));
    HIPCHK(hipStreamSynchronize(b->stream));
    return VEGAS_OK;
}

vegas_status streams_iteration(vegas_batch* b, bool integrate)
{
    if (b->n_run >= b->max_iter) return fail(VEGAS_ESTATE, "iteration log full (max_iter = %d)", b->max_iter);
    HIPCHK(b->mark());
    vegas_status s = fork_lanes(b);
    if (s != VEGAS_OK) return s;
    for (uint32_t i : b->order) {
        s = integrate ? vegas_integrate(b->ctx[i], 1) : vegas_adapt(b->ctx[i], 1);
        if (s != VEGAS_OK) {
            std::string m = vegas_last_error();
            return fail(s, "problem %u: %s", i, m.c_str());
        }
    }
    s = join_lanes(b);
    if (s != VEGAS_OK) return s;
    HIPCHK(b->mark());
    b->n_run += 1;
    b->combined.push_back(integrate ? 1 : 0);
    return VEGAS_OK;
}

// the fill of the next iteration of every problem under S streams, timed
// on the caller's stream
vegas_status time_streams(vegas_batch* b, int S, float* ms)
{
    assign_lanes(b, S);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    hipError_t r = hipEventRecord(e0, b->stream);
    vegas_status s = r == hipSuccess ? fork_lanes(b) : VEGAS_EDEVICE;
    for (size_t j = 0; s == VEGAS_OK && j < b->order.size(); ++j) s = ctx_fill_pass(b->ctx[b->order[j]]);
    if (s == VEGAS_OK) s = join_lanes(b);
    if (s == VEGAS_OK) r = hipEventRecord(e1, b->stream);
    if (s == VEGAS_OK && r == hipSuccess) r = hipEventSynchronize(e1);
    if (s == VEGAS_OK && r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != VEGAS_OK) return s;
    HIPCHK(r);
    return VEGAS_OK;
}

// one warm-up and the better of two timed passes per stream count
// The fill pass is what can be timed without changing a problem's state;
// the update kernels after each fill (fix-up, estimate, allocation, map) are
// short and latency-bound, and gain from more streams more than the fills
// do (whole iterations of the 4096-problem workload: 371, 253, 200, 201 ms
// at 1, 2, 4, 8 streams, while the fill passes alone were within a few
// percent from 2 streams on).  So the largest stream count whose fill pass
// is within kStreamSlack of the fastest is taken.
constexpr double kStreamSlack = 1.10;

vegas_status tune_streams(vegas_batch* b, int* best, double* best_ms)
{
    double t_of[16];
    int n = 0;
    double bm = INFINITY;
    for (int S : kStreamCandidates) {
        float t0 = 0.f, t1 = 0.f, t2 = 0.f;
        vegas_status s;
        if ((s = time_streams(b, S, &t0)) != VEGAS_OK) return s;
        if ((s = time_streams(b, S, &t1)) != VEGAS_OK) return s;
        if ((s = time_streams(b, S, &t2)) != VEGAS_OK) return s;
        t_of[n++] = std::min(t1, t2);
        bm = std::min(bm, t_of[n - 1]);
    }
    int bs = kDefaultStreams;
    double bt = INFINITY;
    n = 0;
    for (int S : kStreamCandidates) {
        const double t = t_of[n++];
        if (t <= kStreamSlack * bm && (bt == INFINITY || S > bs)) {
            bs = S;
            bt = t;
        }
    }
    *best = bs;
    *best_ms = bt;
    return VEGAS_OK;
}

bool streams_cache_lookup(const char* path, uint64_t key, int* S, double* ms)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool hit = false;
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long k;
        int q;
        double t;
        if (std::sscanf(line, "%llx streams %d %lf", &k, &q, &t) != 3 || k != key) continue;
        for (int c : kStreamCandidates)
            if (c == q) {
                *S = q;
                *ms = t;
                hit = true;
            }
    }
    std::fclose(f);
    return hit;
}

void streams_cache_store(const char* path, uint64_t key, int S, double ms)
{
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%016llx streams %d %.6f\n", (unsigned long long)key, S, ms);
    std::fclose(f);
}

// set up every problem as a context in its slice of the workspace, then
// choose the stream count
vegas_status create_streams(vegas_batch* b, const vegas_config* cfgs, const vegas_integrand* fs,
                            const char* tune_cache)
{
    const int n = b->n;
    size_t total = 0;
    vegas_status s = streams_layout(n, cfgs, fs, b->max_iter, &b->ctx_off, &total);
    if (s != VEGAS_OK) return s;
    if (b->ws_bytes < total) return fail(VEGAS_ENOMEM, "workspace has %zu bytes, needs %zu", b->ws_bytes, total);
    b->ws_bytes = total;
    b->lanes.resize(kMaxStreams);
    b->joins.resize(kMaxStreams);
    for (int q = 0; q < kMaxStreams; ++q) {
        HIPCHK(hipStreamCreateWithFlags(&b->lanes[q], hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&b->joins[q], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    b->order.resize(n);
    std::iota(b->order.begin(), b->order.end(), 0u);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](uint32_t x, uint32_t y) { return problem_cost(b->g[x]) > problem_cost(b->g[y]); });
    b->n_lanes = kMaxStreams;
    if ((s = fork_lanes(b)) != VEGAS_OK) return s;
    b->ctx.assign(n, nullptr);
    for (int i = 0; i < n; ++i) {
        vegas_config c = cfgs[i];
        c.max_iter = b->max_iter;
        const size_t end = i + 1 < n ? b->ctx_off[i + 1] : total;
        s = vegas_create(&c, &fs[i], b->ws + b->ctx_off[i], end - b->ctx_off[i], b->lanes[i % kMaxStreams],
                         &b->ctx[i]);
        if (s != VEGAS_OK) {
            std::string m = vegas_last_error();
            return fail(s, "problem %d: %s", i, m.c_str());
        }
    }
    if ((s = sync_lanes(b)) != VEGAS_OK) return s;
    int S = kDefaultStreams;
    // (the bare fill pass the tuner times has no ORDERED form)
    if (tune_cache && cfgs[0].accum != VEGAS_ACC_ORDERED) {
        const uint64_t key = fnv1a(batch_key(b), "streams", 7);
        double ms = 0.0;
        if (streams_cache_lookup(tune_cache, key, &S, &ms)) {
            b->tuned = 2;
            b->tune_ms = ms;
        } else {
            if ((s = tune_streams(b, &S, &ms)) != VEGAS_OK) return s;
            b->tuned = 1;
            b->tune_ms = ms;
            streams_cache_store(tune_cache, key, S, ms);
        }
    }
    assign_lanes(b, S);
    return sync_lanes(b);
}

}  // namespace

extern "C" {

vegas_status vegas_batch_workspace_size(int32_t n, const vegas_config* cfgs, const vegas_integrand* fs,
                                        int32_t schedule, size_t* bytes)
{
    std::vector<Geometry> gs;
    int max_iter = 0;
    const vegas_status s = batch_geometry(n, cfgs, fs, schedule, gs, &max_iter);
    if (s != VEGAS_OK) return s;
    if (!bytes) return fail(VEGAS_EINVAL, "null bytes");
    if (schedule == VEGAS_BATCH_STREAMS) return streams_layout(n, cfgs, fs, max_iter, nullptr, bytes);
    *bytes = batch_bytes(gs, max_iter);
    return VEGAS_OK;
}

vegas_status vegas_batch_create(int32_t n, const vegas_config* cfgs, const vegas_integrand* fs, void* d_workspace,
                                size_t bytes, void* hip_stream, int32_t schedule, const char* tune_cache,
                                vegas_batch** out)
{
    if (!out) return fail(VEGAS_EINVAL, "null out");
    *out = nullptr;
    std::vector<Geometry> gs;
    int max_iter = 0;
    vegas_status s = batch_geometry(n, cfgs, fs, schedule, gs, &max_iter);
    if (s != VEGAS_OK) return s;
    if (!d_workspace) return fail(VEGAS_EINVAL, "null workspace");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(VEGAS_EINVAL, "workspace must be 256-byte aligned");
    if (schedule == VEGAS_BATCH_STREAMS) {
        vegas_batch* b = new vegas_batch();
        b->n = n;
        b->cfg.assign(cfgs, cfgs + n);
        b->g = gs;
        b->fp64 = cfgs[0].precision == VEGAS_PREC_FP64;
        b->kahan = cfgs[0].accum == VEGAS_ACC_KAHAN;
        b->any_general_beta = false;
        b->max_ng = 1;
        b->max_iter = max_iter;
        b->stream = (hipStream_t)hip_stream;
        b->ws = (unsigned char*)d_workspace;
        b->ws_bytes = bytes;
        b->n_wg = 0;
        b->cur = 0;
        b->n_run = 0;
        b->tuned = 0;
        b->tune_ms = 0.0;
        b->timing = false;
        b->lds = 0;
        b->streams = true;
        s = create_streams(b, cfgs, fs, tune_cache);
        if (s != VEGAS_OK) {
            (void)sync_lanes(b);
            delete b;
            return s;
        }
        *out = b;
        return VEGAS_OK;
    }
    // Switched off: the first device run of the batched iteration ended in a
    // memory fault whose cause is not found (a CPU emulation of the same
    // kernels is clean and matches the oracle).  Validation and sizing stay
    // available.
    if (kPersistentDisabled)
        return fail(VEGAS_EUNSUPPORTED, "the persistent batch schedule is switched off: its device run faulted "
                                        "and the cause is not yet found");
    const size_t need = batch_bytes(gs, max_iter);
    if (bytes < need) return fail(VEGAS_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, need);
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));

    vegas_batch* b = new vegas_batch();
    b->n = n;
    b->cfg.assign(cfgs, cfgs + n);
    b->g = gs;
    b->fp64 = cfgs[0].precision == VEGAS_PREC_FP64;
    b->kahan = cfgs[0].accum == VEGAS_ACC_KAHAN;
    b->any_general_beta = false;
    b->max_ng = 1;
    for (int i = 0; i < n; ++i) {
        const vegas_config& c = cfgs[i];
        if (c.adapt_strat && c.beta > 0.0 && !beta_monotone(c.beta)) b->any_general_beta = true;
        b->max_ng = std::max(b->max_ng, gs[i].ng);
        const vegas_integrand& f = fs[i];
        b->consts.insert(b->consts.end(), f.params, f.params + gs[i].n_params);
        for (int d = 0; d < gs[i].D; ++d) b->consts.push_back(f.lo ? f.lo[d] : 0.0);
        for (int d = 0; d < gs[i].D; ++d) b->consts.push_back(f.hi ? f.hi[d] : 1.0);
    }
    b->max_iter = max_iter;
    b->stream = (hipStream_t)hip_stream;
    b->ws = (unsigned char*)d_workspace;
    b->ws_bytes = bytes;
    b->n_wg = std::max(1, cus);
    b->cur = 0;
    b->n_run = 0;
    b->tuned = 0;
    b->tune_ms = 0.0;
    b->timing = false;
    b->lds = 0;

    Layout L = kCandidates[0];
    if (tune_cache) {
        const uint64_t key = batch_key(b);
        double ms = 0.0;
        if (cache_lookup(tune_cache, key, &L, &ms)) {
            b->tuned = 2;
            b->tune_ms = ms;
        } else {
            s = autotune(b, &L, &ms);
            if (s != VEGAS_OK) {
                delete b;
                return s;
            }
            b->tuned = 1;
            b->tune_ms = ms;
            cache_store(tune_cache, key, L, ms);
        }
    }
    s = apply_layout(b, L);
    if (s != VEGAS_OK) {
        delete b;
        return s;
    }
    *out = b;
    return VEGAS_OK;
}

void vegas_batch_destroy(vegas_batch* b)
{
    if (!b) return;
    if (b->streams) (void)sync_lanes(b);
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

vegas_status vegas_batch_set_streams(vegas_batch* b, int32_t n_streams)
{
    if (!b) return fail(VEGAS_EINVAL, "null batch");
    if (!b->streams) return fail(VEGAS_EUNSUPPORTED, "the stream count belongs to the streams schedule");
    if (b->n_run != 0) return fail(VEGAS_ESTATE, "the stream count is fixed once iterations have run");
    if (n_streams < 1 || n_streams > kMaxStreams) return fail(VEGAS_EINVAL, "n_streams must be 1..%d", kMaxStreams);
    vegas_status s = sync_lanes(b);
    if (s != VEGAS_OK) return s;
    assign_lanes(b, n_streams);
    return VEGAS_OK;
}

vegas_status vegas_batch_set_layout(vegas_batch* b, int32_t per_lane, int64_t item_samples)
{
    if (!b) return fail(VEGAS_EINVAL, "null batch");
    if (b->streams) return fail(VEGAS_EUNSUPPORTED, "layouts belong to the persistent schedule");
    if (b->n_run != 0) return fail(VEGAS_ESTATE, "the layout is fixed once iterations have run");
    for (const Layout& c : kCandidates)
        if (c.per_lane == per_lane && c.item_samples == item_samples) return apply_layout(b, c);
    return fail(VEGAS_EINVAL, "(%d, %lld) is not one of the tuned layouts", per_lane, (long long)item_samples);
}

vegas_status vegas_batch_adapt(vegas_batch* b, int32_t n_iter)
{
    if (!b || n_iter < 0) return fail(VEGAS_EINVAL, "bad arguments");
    for (int i = 0; i < n_iter; ++i) {
        const vegas_status s = b->streams ? streams_iteration(b, false) : batch_iteration(b, false);
        if (s != VEGAS_OK) return s;
    }
    return VEGAS_OK;
}

vegas_status vegas_batch_integrate(vegas_batch* b, int32_t n_iter)
{
    if (!b || n_iter < 0) return fail(VEGAS_EINVAL, "bad arguments");
    for (int i = 0; i < n_iter; ++i) {
        const vegas_status s = b->streams ? streams_iteration(b, true) : batch_iteration(b, true);
        if (s != VEGAS_OK) return s;
    }
    return VEGAS_OK;
}

vegas_status vegas_batch_results(vegas_batch* b, vegas_estimate* out)
{
    if (!b || !out) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    if (b->streams) {
        int64_t bad = 0;
        for (int i = 0; i < b->n; ++i) {
            const vegas_status s = vegas_result(b->ctx[i], &out[i]);
            if (s != VEGAS_OK && s != VEGAS_ENONFINITE) return s;
            bad += out[i].n_nonfinite;
        }
        if (bad) return fail(VEGAS_ENONFINITE, "%lld sample weights were NaN/Inf and counted as 0", (long long)bad);
        return VEGAS_OK;
    }
    const size_t n = (size_t)b->n;
    std::vector<double> it(2 * (size_t)b->max_iter * n);
    std::vector<unsigned long long> ctr(8 * n);
    HIPCHK(hipMemcpy(it.data(), b->at<double>(b->p.iter), sizeof(double) * it.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ctr.data(), b->at<unsigned long long>(b->p.ctr), sizeof(unsigned long long) * ctr.size(),
                     hipMemcpyDeviceToHost));
    unsigned long long bad_total = 0;
    for (size_t i = 0; i < n; ++i) {
        std::vector<double> Ic, s2c;
        for (int t = 0; t < b->n_run; ++t)
            if (b->combined[t]) {
                Ic.push_back(it[2 * ((size_t)b->max_iter * i + t)]);
                s2c.push_back(it[2 * ((size_t)b->max_iter * i + t) + 1]);
            }
        vegas_estimate& e = out[i];
        combine(Ic, s2c, &e.integral, &e.sigma2, &e.chi2_dof);
        e.n_iter_combined = (int32_t)Ic.size();
        e.n_iter_total = b->n_run;
        e.n_eval_total = (int64_t)b->n_run * (int64_t)b->g[i].n_eval;
        e.n_nonfinite = (int64_t)ctr[8 * i + 4];
        bad_total += ctr[8 * i + 4];
    }
    if (bad_total) return fail(VEGAS_ENONFINITE, "%llu sample weights were NaN/Inf and counted as 0", bad_total);
    return VEGAS_OK;
}

vegas_status vegas_batch_get_iterations(vegas_batch* b, int32_t i, double* I, double* sigma2, int32_t cap, int32_t* n)
{
    if (!b || i < 0 || i >= b->n || cap < 0 || (cap > 0 && (!I || !sigma2))) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    if (b->streams) {
        int32_t m = 0;
        const vegas_status s = vegas_get_iterations(b->ctx[i], I, sigma2, cap, &m);
        if (s == VEGAS_OK && n) *n = m;
        return s;
    }
    const int m = std::min(cap, b->n_run);
    std::vector<double> buf(2 * (size_t)std::max(m, 1));
    if (m > 0)
        HIPCHK(hipMemcpy(buf.data(), b->at<double>(b->p.iter) + 2 * (size_t)b->max_iter * i, sizeof(double) * 2 * m,
                         hipMemcpyDeviceToHost));
    for (int t = 0; t < m; ++t) {
        I[t] = buf[2 * t];
        sigma2[t] = buf[2 * t + 1];
    }
    if (n) *n = b->n_run;
    return VEGAS_OK;
}

vegas_status vegas_batch_get_map(vegas_batch* b, int32_t i, double* grid)
{
    if (!b || i < 0 || i >= b->n || !grid) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    if (b->streams) return vegas_get_map(b->ctx[i], grid);
    const Geometry& g = b->g[i];
    HIPCHK(hipMemcpy(grid, b->at<double>(b->p.grid64[i]), sizeof(double) * g.D * (g.ng + 1), hipMemcpyDeviceToHost));
    return VEGAS_OK;
}

vegas_status vegas_batch_get_nh(vegas_batch* b, int32_t i, uint32_t* nh)
{
    if (!b || i < 0 || i >= b->n || !nh) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    if (b->streams) return vegas_get_nh(b->ctx[i], nh);
    const Geometry& g = b->g[i];
    std::vector<uint32_t> st((size_t)g.n_cubes + 1);
    HIPCHK(hipMemcpy(st.data(), b->at<uint32_t>(b->cur ? b->p.start1[i] : b->p.start0[i]),
                     sizeof(uint32_t) * st.size(), hipMemcpyDeviceToHost));
    for (uint32_t h = 0; h < g.n_cubes; ++h) nh[h] = st[h + 1] - st[h];
    return VEGAS_OK;
}

vegas_status vegas_batch_get_info(const vegas_batch* b, vegas_batch_info* out)
{
    if (!b || !out) return fail(VEGAS_EINVAL, "bad arguments");
    out->n = b->n;
    out->schedule = b->streams ? VEGAS_BATCH_STREAMS : VEGAS_BATCH_PERSISTENT;
    out->n_streams = b->streams ? b->n_lanes : 0;
    if (b->streams) {
        out->per_lane = 0;
        out->item_samples = 0;
        out->n_items = b->n;
        int64_t tiles = 0, ne = 0, nc = 0;
        int32_t wg = 0;
        size_t lds = 0;
        for (int i = 0; i < b->n; ++i) {
            const Geometry& g = b->g[i];
            vegas_info ci;
            const vegas_status s = vegas_get_info(b->ctx[i], &ci);
            if (s != VEGAS_OK) return s;
            tiles += g.n_tiles;
            wg += ci.n_workgroups;
            ne += g.n_eval;
            nc += g.n_cubes;
            lds = std::max(lds, fill_lds_bytes(g.D, g.ng, b->fp64, ci.lds_hist, g.tile, g.n_aux, 0));
        }
        out->n_tiles = tiles;
        out->n_workgroups = wg;
        out->tuned = b->tuned;
        out->tune_ms = b->tune_ms;
        out->lds_bytes = lds;
        out->workspace_bytes = b->ws_bytes;
        out->n_eval_total = ne;
        out->n_cubes_total = nc;
        return VEGAS_OK;
    }
    out->per_lane = b->layout.per_lane;
    out->item_samples = b->layout.item_samples;
    out->n_items = b->p.n_items;
    out->n_tiles = b->p.n_tiles;
    out->n_workgroups = b->n_wg;
    out->tuned = b->tuned;
    out->tune_ms = b->tune_ms;
    out->lds_bytes = b->lds;
    out->workspace_bytes = b->p.total;
    int64_t ne = 0, nc = 0;
    for (const Geometry& g : b->g) {
        ne += g.n_eval;
        nc += g.n_cubes;
    }
    out->n_eval_total = ne;
    out->n_cubes_total = nc;
    return VEGAS_OK;
}

vegas_status vegas_batch_set_timing(vegas_batch* b, int32_t on)
{
    if (!b) return fail(VEGAS_EINVAL, "bad arguments");
    if (b->streams) {
        const vegas_status s = sync_lanes(b);
        if (s != VEGAS_OK) return s;
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    b->events.clear();
    b->timing = on != 0;
    return VEGAS_OK;
}

vegas_status vegas_batch_get_timing(vegas_batch* b, double* ms, int32_t* n_iter)
{
    if (!b || !ms) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int i = 0; i < 4; ++i) ms[i] = 0.0;
    size_t i = 0;
    int n = 0;
    if (b->streams) {
        // two marks per iteration: before the fork, after the join
        for (; i + 2 <= b->events.size(); i += 2, ++n) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, b->events[i], b->events[i + 1]));
            ms[0] += t;
        }
        if (n_iter) *n_iter = n;
        return VEGAS_OK;
    }
    while (i + 5 <= b->events.size()) {
        for (int q = 0; q < 4; ++q) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, b->events[i + q], b->events[i + q + 1]));
            ms[q] += t;
        }
        i += 5;
        ++n;
    }
    if (n_iter) *n_iter = n;
    return VEGAS_OK;
}

}  // extern "C"
