// C ABI of the VEGAS+ iteration library (include/vegas.h).
//
// Host orchestration of Alg. 1: per iteration the fill (Alg. 2), the cube
// fix-up and the fixed-order estimate, the allocation update (Eq. 7) and the
// map refinement, all launched on the caller's stream.  The only host work
// is validation, workspace carving, and the Eq. 8-9 combination of the
// per-iteration estimates when a result is requested.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vegas.h"
#include "common.hpp"
#include "host.hpp"
#include "launch.hpp"

using namespace vg;

namespace vgh {

thread_local std::string g_err;

vegas_status fail(vegas_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

constexpr int kMaxWG = 256;            // fill workgroups at most (one per CU of the 256); histogram slots

// largest m with m^D <= lim, without overflow
bool pow_at_most(uint64_t m, int D, uint64_t lim, uint64_t* out)
{
    uint64_t v = 1;
    for (int d = 0; d < D; ++d) {
        if (m != 0 && v > lim / m) return false;
        v *= m;
    }
    if (v > lim) return false;
    if (out) *out = v;
    return true;
}

int family_params(int fam, int D, const vegas_integrand* f)
{
    switch (fam) {
    case VEGAS_GAUSS_DIAG:
        if (f->n_params < 3 || !f->params || !(f->params[2] >= 1.0 && f->params[2] <= 4096.0) ||
            f->params[2] != std::floor(f->params[2]))
            return -1;
        return 3 + (int)f->params[2];
    case VEGAS_GENZ_PPEAK:
    case VEGAS_GENZ_GAUSS: return 1 + 2 * D;
    case VEGAS_GAUSS_CORR: return 3;
    case VEGAS_LINEAR:
    case VEGAS_ROOS:
    case VEGAS_CONST:
    case VEGAS_COSINE:
    case VEGAS_SIN_EXP:
    case VEGAS_EXP_SQ:
    case VEGAS_MOROKOFF: return 1;
    case VEGAS_USER:
        return f->n_params >= 0 && f->n_params <= 4096 && (f->n_params == 0 || f->params) ? f->n_params : -1;
    default: return -1;
    }
}

vegas_status geometry(const vegas_config* c, const vegas_integrand* f, Geometry* g)
{
    if (!c || !f) return fail(VEGAS_EINVAL, "null config or integrand");
    if (c->dim < 1 || c->dim > kMaxDim) return fail(VEGAS_EINVAL, "dim must be 1..%d", kMaxDim);
    if (c->n_intervals < 1 || c->n_intervals > kMaxNg)
        return fail(VEGAS_EINVAL, "n_intervals must be 1..%d", kMaxNg);
    if (c->n_eval < 2 || c->n_eval >= (int64_t)UINT32_MAX) return fail(VEGAS_EINVAL, "n_eval must be in [2, 2^32-1)");
    if (c->n_min < 2) return fail(VEGAS_EINVAL, "n_min must be >= 2");
    if (!(c->alpha >= 0.0) || !std::isfinite(c->alpha)) return fail(VEGAS_EINVAL, "alpha must be finite and >= 0");
    if (!(c->beta >= 0.0) || !std::isfinite(c->beta)) return fail(VEGAS_EINVAL, "beta must be finite and >= 0");
    if (c->precision != VEGAS_PREC_FP64 && c->precision != VEGAS_PREC_FP32)
        return fail(VEGAS_EINVAL, "unknown precision %d", c->precision);
    if (c->accum != VEGAS_ACC_FP64 && c->accum != VEGAS_ACC_ORDERED && c->accum != VEGAS_ACC_KAHAN)
        return fail(VEGAS_EINVAL, "unknown accumulation mode %d", c->accum);
    if (c->accum == VEGAS_ACC_KAHAN && c->precision != VEGAS_PREC_FP32)
        return fail(VEGAS_EINVAL, "KAHAN accumulation is for the FP32 sample path");
    if (c->accum == VEGAS_ACC_ORDERED) {
        if (c->precision != VEGAS_PREC_FP64) return fail(VEGAS_EINVAL, "ORDERED accumulation runs in FP64");
        if ((double)c->n_eval * c->dim * c->n_intervals > (double)(1ull << 28) || c->n_eval > (1 << 24))
            return fail(VEGAS_EUNSUPPORTED, "ORDERED accumulation is for n_eval*dim*n_intervals <= 2^28");
    }
    if (c->instance >= (1u << 24)) return fail(VEGAS_EINVAL, "instance must be < 2^24");
    if (c->max_iter < 0) return fail(VEGAS_EINVAL, "max_iter must be >= 0");
    const int np = family_params(f->family, c->dim, f);
    if (np < 0) return fail(VEGAS_EINVAL, "unknown integrand family %d or bad parameters (GAUSS_DIAG: 1..4096 terms)", f->family);
    if (f->n_params != np || (np > 0 && !f->params))
        return fail(VEGAS_EINVAL, "family %d expects %d parameters, got %d", f->family, np, f->n_params);
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(f->params[i])) return fail(VEGAS_EINVAL, "parameter %d is not finite", i);
    for (int d = 0; d < c->dim; ++d) {
        const double lo = f->lo ? f->lo[d] : 0.0, hi = f->hi ? f->hi[d] : 1.0;
        if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi)) return fail(VEGAS_EINVAL, "bad box on axis %d", d);
    }
    if (f->family == VEGAS_GAUSS_DIAG && !(f->params[1] > 0.0)) return fail(VEGAS_EINVAL, "GAUSS_DIAG needs s > 0");
    if (f->family == VEGAS_SIN_EXP && c->dim < 2) return fail(VEGAS_EINVAL, "SIN_EXP needs dim >= 2");
    if (f->family == VEGAS_MOROKOFF)
        for (int d = 0; d < c->dim; ++d)
            if (f->lo && !(f->lo[d] >= 0.0)) return fail(VEGAS_EINVAL, "MOROKOFF needs a box in x >= 0");
    if (f->family == VEGAS_GAUSS_CORR) {
        const double s = f->params[1], rho = f->params[2];
        if (!(s > 0.0) || !(rho < 1.0) || !(1.0 + (c->dim - 1) * rho > 0.0))
            return fail(VEGAS_EINVAL, "GAUSS_CORR covariance not positive definite");
    }

    g->D = c->dim;
    g->ng = c->n_intervals;
    g->n_min = c->n_min;
    g->family = f->family;
    g->n_params = np;
    g->n_eval = (uint32_t)c->n_eval;
    uint64_t m;
    if (c->n_strat > 0) {
        m = (uint64_t)c->n_strat;
    } else {
        m = 1;
        while (pow_at_most(m + 1, c->dim, (uint64_t)c->n_eval / 4, nullptr)) ++m;
    }
    uint64_t nc = 0;
    for (;;) {
        if (pow_at_most(m, c->dim, (uint64_t)INT32_MAX - 1, &nc) && (uint64_t)c->n_min * nc <= (uint64_t)c->n_eval)
            break;
        if (c->n_strat > 0 || m == 1) return fail(VEGAS_EINVAL, "n_eval cannot give n_min samples to every hypercube");
        --m;
    }
    if (m >= (1u << 20)) return fail(VEGAS_EINVAL, "strata per axis must be < 2^20");
    if (m * (uint64_t)g->ng >= (1ull << 31)) return fail(VEGAS_EINVAL, "n_strat * n_intervals must be < 2^31");
    g->nst = (uint32_t)m;
    g->n_cubes = (uint32_t)nc;
    g->R = (uint64_t)c->n_eval - (uint64_t)c->n_min * nc;
    if (m == 1) {
        g->magic = 0x80000000u;      // q2 2^31 / 2^32 = q, with shift -1
        g->shift = -1;
    } else {
        int l = 0;
        while ((1ull << l) < m) ++l;
        const unsigned __int128 num = (unsigned __int128)1 << (31 + l);
        g->magic = (uint32_t)((num + m - 1) / m);
        g->shift = l - 1;
    }
    const bool fp64 = c->precision == VEGAS_PREC_FP64;
    g->n_aux = std::max(f->family == VEGAS_GAUSS_DIAG ? (int)f->params[2] : 2 * g->D, 1);
    // the warped fill (dimension kFlowDim only) keeps the map in LDS as well
    const int map_lds = g->D == kFlowDim ? 1 : 0;
    // samples per lane: long enough runs for large budgets (the tile's
    // set-up, binary search and cross-lane scan are paid once per tile),
    // enough tiles to keep every CU busy for small ones; 16 and 32 only
    // where the tile's cube starts still fit in LDS beside the histograms
    const uint64_t ne = g->n_eval;
    auto fits = [&](int per_lane) {
        return fill_lds_bytes(g->D, g->ng, fp64, 1, kLanesPerTile * per_lane, g->n_aux, map_lds) <= kLdsLimit;
    };
    g->per_lane = 1;
    if (ne >= (uint64_t)256 * kLanesPerTile * 4 * 2) g->per_lane = 4;
    if (ne >= (uint64_t)256 * kLanesPerTile * 8 * 8) g->per_lane = 8;
    // longer runs only with at least 8 tiles per workgroup on 256 CUs
    for (int pl = 16; pl * kLanesPerTile <= kMaxTile; pl *= 2)
        if (ne >= (uint64_t)256 * kLanesPerTile * pl * 8 && fits(pl)) g->per_lane = pl;
    g->tile = kLanesPerTile * g->per_lane;
    g->n_tiles = (int)((ne + g->tile - 1) / g->tile);
    g->lds_hist_ok = fill_lds_bytes(g->D, g->ng, fp64, 1, g->tile, g->n_aux, map_lds) <= kLdsLimit;
    if (!g->lds_hist_ok && fill_lds_bytes(g->D, g->ng, fp64, 0, g->tile, g->n_aux, map_lds) > kLdsLimit)
        return fail(VEGAS_EUNSUPPORTED, "map of %d x %d intervals does not fit in LDS", g->D, g->ng);
    if ((size_t)3 * (g->ng + 1) * 8 > kLdsLimit) return fail(VEGAS_EUNSUPPORTED, "n_intervals too large for the map update");
    return VEGAS_OK;
}

}  // namespace vgh

using namespace vgh;

namespace {

// Workspace carving: offsets of every device array (256-byte aligned).
struct Plan {
    size_t prm, lo, hi, aux_d, aux_f, grid64, grid32, start[2], tfirst[2], v, qbuf, wg_part, side, fix_part,
        histH, histC, histCw, partH, partC, Hsum, Csum, counters, bsum, boff, iter, ord_w, ord_bins, ord_m, total;
};

Plan plan(const Geometry& g, int max_iter, bool ordered)
{
    Plan p;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t nb = (size_t)g.D * g.ng;
    const size_t row = (size_t)g.D * (g.ng + 1);
    const size_t nblk = (g.n_cubes + kAllocPerBlock - 1) / kAllocPerBlock;
    p.prm = take(sizeof(double) * g.n_params);
    p.lo = take(sizeof(double) * g.D);
    p.hi = take(sizeof(double) * g.D);
    p.aux_d = take(sizeof(double) * g.n_aux);
    p.aux_f = take(sizeof(float) * g.n_aux);
    p.grid64 = take(sizeof(double) * row);
    p.grid32 = take(sizeof(float) * row);
    for (int b = 0; b < 2; ++b) {
        p.start[b] = take(sizeof(uint32_t) * ((size_t)g.n_cubes + 1));
        p.tfirst[b] = take(sizeof(uint32_t) * ((size_t)g.n_tiles + 1));
    }
    p.v = take(sizeof(double) * g.n_cubes);
    p.qbuf = take(sizeof(uint32_t) * g.n_cubes);
    p.wg_part = take(sizeof(double) * 2 * kMaxWG);
    p.side = take(sizeof(TileSide) * g.n_tiles);
    p.fix_part = take(sizeof(double) * 2 * g.n_tiles);
    // one slot per fill workgroup; a problem never runs more workgroups
    // than tiles
    // one histogram slot per workgroup in both modes (LDS histograms are
    // copied out into them; global ones are added into them directly)
    const size_t slots = (size_t)std::min(kMaxWG, g.n_tiles);
    p.histH = take(sizeof(double) * nb * slots);
    p.histC = take(sizeof(uint32_t) * nb * slots);
    // the learned warp's iterations (dimension 16): FP64 count weights
    p.histCw = g.D == kFlowDim ? take(sizeof(double) * nb) : 0;
    p.partH = take(sizeof(double) * nb * kHistParts);
    p.partC = take(sizeof(uint32_t) * nb * kHistParts);
    p.Hsum = take(sizeof(double) * nb);
    p.Csum = take(sizeof(double) * nb);
    p.counters = take(sizeof(unsigned long long) * 8);   // vmax[2], qmax[2], nonfinite
    p.bsum = take(sizeof(unsigned long long) * nblk);
    p.boff = take(sizeof(unsigned long long) * (nblk + 1));
    p.iter = take(sizeof(double) * 2 * (size_t)max_iter);
    p.ord_w = p.ord_bins = p.ord_m = 0;
    if (ordered) {
        p.ord_w = take(sizeof(double) * g.n_eval);
        p.ord_bins = take(sizeof(uint32_t) * (size_t)g.n_eval * g.D);
        p.ord_m = take(sizeof(double) * g.n_cubes);
    }
    p.total = o;
    return p;
}

}  // namespace

struct vegas_ctx {
    vegas_config cfg;
    Geometry g;
    Plan p;
    std::vector<double> params, lo, hi;
    hipStream_t stream;
    unsigned char* ws;
    int n_wg;
    int cur;
    int max_iter;
    int n_run;
    std::vector<uint8_t> combined;     // per iteration: 1 = integrate
    int slots_last;                    // histogram slots written by the last fill
    bool have_prev;                    // previous estimate valid (FP32 histogram scale)
    bool hist_weighted = false;        // the last fill wrote importance-weighted histograms (warp)
    const vegas_user_fn* user = nullptr;   // integrand compiled at run time (family VEGAS_USER)
    bool timing;
    std::vector<hipEvent_t> events;    // 5 per timed iteration

    // learned warp (vegas_flow_*): its own workspace, carved by flow_plan
    bool flow_attached = false;
    bool flow_on = false;
    vegas_flow_config fcfg{};
    unsigned char* fws = nullptr;
    size_t f_theta = 0, f_packed = 0, f_w = 0, f_z = 0, f_lj = 0, f_om = 0, f_U = 0, f_G0 = 0, f_G1 = 0, f_part = 0,
           f_grad = 0, f_m = 0, f_v = 0, f_sumsq = 0, f_slots = 0;
    int f_nwg = 0;                     // workgroups of the training passes
    int f_step = 0;                    // Adam steps taken
    size_t f_acc = 0;                  // last accepted parameters
    int n_cus = 1;
    bool fused = false;                // small problem: one launch after the fill
    std::vector<uint8_t> warped;       // per iteration: 0 plain, 1 through the warp, 2 plain control
    // the judge: iterations since the warp was enabled, GPU time of each
    // iteration while the warp is on (event pairs in a ring), the log
    // entries already read, and its running records
    int f_phase = 0;
    std::vector<hipEvent_t> f_ev;      // [kJudgeRing][2]
    std::vector<int> f_ev_iter;        // iteration held by each ring slot, -1 none
    std::vector<double> f_ms;          // per iteration: GPU ms, NaN when unknown
    std::vector<double> log_I, log_s2; // host copy of the iteration log
    std::vector<double> kept_rv;       // relative variances of kept warped iterations
    std::vector<double> warp_eff, ctrl_eff;   // relative variance x GPU ms
    double kw_sum = 0.0, kw_w = 0.0;   // kept warped iterations of the cost phase: sum I/s2, sum 1/s2
    bool f_timing = false;             // events around the sampling pass and the training
    std::vector<hipEvent_t> f_tev;     // 4 per timed warped iteration
    std::vector<hipEvent_t> f_gev;     // 2 per timed launch of the gradient kernel
    int strikes = 0;                   // consecutive control checks the warp lost
    int rejects = 0;                   // consecutive rejected warped iterations
    int n_accepted = 0, n_rejected = 0, n_control = 0;

    ~vegas_ctx()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipEvent_t e : f_ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : f_tev) (void)hipEventDestroy(e);
        for (hipEvent_t e : f_gev) (void)hipEventDestroy(e);
    }
    hipError_t fmark()
    {
        if (!f_timing) return hipSuccess;
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        f_tev.push_back(e);
        return hipEventRecord(e, stream);
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
    unsigned long long* vmax(int t) const { return at<unsigned long long>(p.counters) + (t & 1); }
    unsigned long long* qmax(int t) const { return at<unsigned long long>(p.counters) + 2 + (t & 1); }
    unsigned long long* nonfinite() const { return at<unsigned long long>(p.counters) + 4; }
};

namespace {

SampleConst sample_const(const vegas_ctx* c)
{
    SampleConst s;
    s.D = c->g.D;
    s.ng = (uint32_t)c->g.ng;
    s.nst = c->g.nst;
    s.nst_magic = c->g.magic;
    s.nst_shift = c->g.shift;
    s.n_eval = c->g.n_eval;
    s.n_cubes = c->g.n_cubes;
    s.key0 = (uint32_t)c->cfg.seed;
    s.key1 = (uint32_t)(c->cfg.seed >> 32);
    s.ctr3 = c->cfg.instance << 8;
    s.family = c->g.family;
    s.n_params = c->g.n_params;
    s.prm = c->at<double>(c->p.prm);
    s.aux_d = c->at<double>(c->p.aux_d);
    s.aux_f = c->at<float>(c->p.aux_f);
    s.n_aux = c->g.n_aux;
    return s;
}

AllocArgs alloc_args(vegas_ctx* c, int t, int uniform)
{
    AllocArgs a;
    a.n_cubes = c->g.n_cubes;
    a.n_min = (uint32_t)c->g.n_min;
    a.R = c->g.R;
    a.n_eval = c->g.n_eval;
    a.beta = c->cfg.beta;
    a.uniform = uniform;
    a.tile = c->g.tile;
    a.tile_shift = 0;
    while ((1 << a.tile_shift) < c->g.tile) ++a.tile_shift;
    a.n_tiles = c->g.n_tiles;
    a.per_block = kAllocPerBlock;
    a.v = c->at<double>(c->p.v);
    a.vmax = c->vmax(t);
    a.qmax_buf = nullptr;
    a.bsum = c->at<unsigned long long>(c->p.bsum);
    a.boff = c->at<unsigned long long>(c->p.boff);
    a.start = c->at<uint32_t>(c->p.start[1 - c->cur]);
    a.tile_first = c->at<uint32_t>(c->p.tfirst[1 - c->cur]);
    a.qbuf = c->at<uint32_t>(c->p.qbuf);
    return a;
}

// the map refinement's record over n_slots histogram slots added in order
MapArgs map_args(vegas_ctx* c, int n_slots)
{
    MapArgs m;
    m.D = c->g.D;
    m.ng = c->g.ng;
    m.n_slots = n_slots;
    m.parts = 0;
    m.alpha = c->cfg.adapt_map ? c->cfg.alpha : 0.0;
    m.hist_H = c->at<double>(c->p.histH);
    m.hist_C = c->at<uint32_t>(c->p.histC);
    m.hist_Cw = c->hist_weighted ? c->at<double>(c->p.histCw) : nullptr;
    m.grid64 = c->at<double>(c->p.grid64);
    m.grid32 = c->at<float>(c->p.grid32);
    m.Hsum = c->at<double>(c->p.Hsum);
    m.Csum = c->at<double>(c->p.Csum);
    return m;
}

// allocation then map refinement from the accumulators of "slot set" t
vegas_status run_update(vegas_ctx* c, int t, int n_slots, bool timed)
{
    const bool adapt_strat = c->cfg.adapt_strat && c->cfg.beta > 0.0;
    AllocArgs aa = alloc_args(c, t, adapt_strat ? 0 : 1);
    HIPCHK(launch_alloc(aa, c->qmax(t), c->stream));
    c->cur = 1 - c->cur;
    if (timed) HIPCHK(c->mark());
    MapArgs m = map_args(c, n_slots);
    if (n_slots > kHistParts) {
        // many workgroup slots: a wide first-level reduce, then the map
        // kernel adds kHistParts partials in order
        HistReduceArgs hr;
        hr.nbins = c->g.D * c->g.ng;
        hr.n_slots = n_slots;
        hr.parts = kHistParts;
        hr.hist_H = m.hist_H;
        hr.hist_C = m.hist_C;
        hr.part_H = c->at<double>(c->p.partH);
        hr.part_C = c->at<uint32_t>(c->p.partC);
        HIPCHK(launch_hist_reduce(hr, c->stream));
        m.n_slots = kHistParts;
        m.hist_H = hr.part_H;
        m.hist_C = hr.part_C;
    }
    HIPCHK(launch_map_update(m, c->stream));
    if (timed) HIPCHK(c->mark());
    return VEGAS_OK;
}

vegas_status flow_train_step(vegas_ctx* c, int slice = -1);
hipError_t flow_step_sums(vegas_ctx* c, int n_steps);
constexpr int kFlowSumSlices = 32;       // training steps of an iteration whose sums are taken together
vegas_status flow_judge(vegas_ctx* c, int t, bool* keep);
hipError_t judge_mark(vegas_ctx* c, int t, int end);

// the fill's launch record for iteration t over the current map and
// allocation; non-finite weights are counted into *nonfinite
FillArgs fill_args(vegas_ctx* c, int t, unsigned long long* nonfinite)
{
    const bool fp64 = c->cfg.precision == VEGAS_PREC_FP64;
    FillArgs a;
    a.sc = sample_const(c);
    a.t = (uint32_t)t;
    a.tile = c->g.tile;
    a.per_lane = c->g.per_lane;
    a.n_tiles = c->g.n_tiles;
    a.lds_hist = c->g.lds_hist_ok ? 1 : 0;
    a.accum = c->cfg.accum;
    a.grid = fp64 ? (const void*)c->at<double>(c->p.grid64) : (const void*)c->at<float>(c->p.grid32);
    a.start = c->at<uint32_t>(c->p.start[c->cur]);
    a.tile_first = c->at<uint32_t>(c->p.tfirst[c->cur]);
    a.v_out = c->at<double>(c->p.v);
    a.wg_part = c->at<double>(c->p.wg_part);
    a.side = c->at<TileSide>(c->p.side);
    a.hist_H = c->at<double>(c->p.histH);
    a.hist_C = c->at<uint32_t>(c->p.histC);
    a.hist_Cw = nullptr;
    a.vmax = c->vmax(t);
    a.nonfinite = nonfinite;
    a.hist_slots = c->g.lds_hist_ok ? 0 : 1;
    return a;
}

vegas_status run_iteration(vegas_ctx* c, bool integrate)
{
    if (c->n_run >= c->max_iter) return fail(VEGAS_ESTATE, "iteration log full (max_iter = %d)", c->max_iter);
    const int t = c->n_run;
    const bool fp64 = c->cfg.precision == VEGAS_PREC_FP64;
    const int nb = c->g.D * c->g.ng;
    HIPCHK(launch_reset(c->vmax(t), 1, c->stream));
    HIPCHK(launch_reset(c->qmax(t), 1, c->stream));
    if (c->cfg.accum == VEGAS_ACC_ORDERED) {
        c->hist_weighted = false;
        OrderedArgs o;
        o.sc = sample_const(c);
        o.t = (uint32_t)t;
        o.grid = c->at<double>(c->p.grid64);
        o.start = c->at<uint32_t>(c->p.start[c->cur]);
        o.w = c->at<double>(c->p.ord_w);
        o.bins = c->at<uint32_t>(c->p.ord_bins);
        o.m = c->at<double>(c->p.ord_m);
        o.v = c->at<double>(c->p.v);
        o.hist_H = c->at<double>(c->p.histH);
        o.hist_C = c->at<uint32_t>(c->p.histC);
        o.iter_out = c->at<double>(c->p.iter) + 2 * t;
        o.vmax = c->vmax(t);
        o.nonfinite = c->nonfinite();
        HIPCHK(c->mark());
        HIPCHK(launch_ordered(o, c->stream));
        HIPCHK(c->mark());
        HIPCHK(c->mark());
        const vegas_status s = run_update(c, t, 1, true);
        if (s != VEGAS_OK) return s;
        c->n_run = t + 1;
        c->combined.push_back(integrate ? 1 : 0);
        c->warped.push_back(0);
        c->f_ms.push_back(NAN);
        c->have_prev = true;
        return VEGAS_OK;
    }
    // with the judge on, every control_period-th iteration of the warp's
    // phase samples plain VEGAS+ (the control)
    const bool control = c->flow_on && c->fcfg.judge > 0 && (c->f_phase + 1) % c->fcfg.control_period == 0;
    const bool warp_now = c->flow_on && !control;
    // the warped fill's histograms are importance-weighted FP64 sums in
    // global memory (one slot)
    const int lds_hist = warp_now ? 0 : (c->g.lds_hist_ok ? 1 : 0);
    // while the map is held a warped fill writes no histograms
    const bool warp_hist = warp_now && c->cfg.adapt_map;
    // a plain fill with global histograms adds into one slot per workgroup
    const bool slotted = !lds_hist && !warp_now;
    const size_t nbr = slotted ? (size_t)nb * c->n_wg : (size_t)nb;
    if (!lds_hist && (!warp_now || warp_hist)) {
        HIPCHK(launch_reset(c->at<unsigned long long>(c->p.histH), (int)nbr, c->stream));
        if (warp_now) HIPCHK(launch_reset(c->at<unsigned long long>(c->p.histCw), (int)nbr, c->stream));
        else HIPCHK(launch_reset(c->at<unsigned long long>(c->p.histC), (int)((nbr + 1) / 2), c->stream));
    }
    FillArgs a = fill_args(c, t, c->nonfinite());
    a.lds_hist = lds_hist;
    a.hist_slots = slotted ? 1 : 0;
    if (warp_hist) a.hist_Cw = c->at<double>(c->p.histCw);
    c->hist_weighted = warp_hist;
    if (c->flow_on) HIPCHK(judge_mark(c, t, 0));
    // the warped fill keeps the map in LDS; k_fill reads it through the cache
    const size_t lds = fill_lds_bytes(c->g.D, c->g.ng, fp64, lds_hist, c->g.tile, c->g.n_aux, warp_now ? 1 : 0);
    HIPCHK(c->mark());
    if (warp_now) {
        // the warp: y -> w = F(y) for every sample, then the fill on w
        FlowSampleArgs fa;
        fa.sc = a.sc;
        fa.t = a.t;
        fa.start = a.start;
        fa.theta = reinterpret_cast<const float*>(c->fws + c->f_theta);
        fa.packed = c->fws + c->f_packed;
        fa.w = reinterpret_cast<float*>(c->fws + c->f_w);
        fa.z = reinterpret_cast<float*>(c->fws + c->f_z);
        fa.lj = reinterpret_cast<float*>(c->fws + c->f_lj);
        HIPCHK(c->fmark());
        HIPCHK(launch_flow_sample(fa, 2 * c->n_wg, c->stream));
        HIPCHK(c->fmark());
        HIPCHK(launch_fill_flow(a, fa.w, fa.lj, reinterpret_cast<float*>(c->fws + c->f_om), c->n_wg, lds, c->stream));
    } else if (c->user) {
        HIPCHK(launch_user_fill(c->user, a, c->n_wg, lds, c->stream));
    } else {
        HIPCHK(launch_fill(a, fp64, c->n_wg, lds, c->stream));
    }
    HIPCHK(c->mark());
    FixupArgs fx;
    fx.n_tiles = c->g.n_tiles;
    fx.side = a.side;
    fx.v_out = a.v_out;
    fx.fix_part = c->at<double>(c->p.fix_part);
    fx.vmax = a.vmax;
    FinalArgs fa;
    fa.n_wg = c->n_wg;
    fa.n_tiles = c->g.n_tiles;
    fa.n_cubes = (double)c->g.n_cubes;
    fa.wg_part = a.wg_part;
    fa.fix_part = fx.fix_part;
    fa.iter_out = c->at<double>(c->p.iter) + 2 * t;
    const int n_slots = lds_hist || slotted ? c->n_wg : 1;
    if (c->fused) {
        // small problem: fix-up, estimate and map in one launch, then the
        // allocation (the timing puts the map into the estimate phase)
        UpdateArgs u;
        u.fx = fx;
        u.fin = fa;
        u.map = map_args(c, n_slots);
        u.map.parts = n_slots > kHistParts ? kHistParts : 0;
        HIPCHK(launch_update_small(u, c->stream));
        HIPCHK(c->mark());
        const bool adapt_strat = c->cfg.adapt_strat && c->cfg.beta > 0.0;
        const AllocArgs aa = alloc_args(c, t, adapt_strat ? 0 : 1);
        HIPCHK(launch_alloc(aa, c->qmax(t), c->stream));
        c->cur = 1 - c->cur;
        HIPCHK(c->mark());
        HIPCHK(c->mark());
    } else {
        HIPCHK(launch_fixup(fx, c->stream));
        HIPCHK(launch_final(fa, c->stream));
        HIPCHK(c->mark());
        const vegas_status s = run_update(c, t, n_slots, true);
        if (s != VEGAS_OK) return s;
    }
    const bool phase = c->flow_on;
    c->n_run = t + 1;
    // control iterations measure plain VEGAS+ for the judge and are not
    // combined: on the workloads the warp is for, a separable density's
    // weights can be so heavy-tailed that its own variance estimate is
    // far too small, and Eq. 8-9 would then let it decide the result
    c->combined.push_back(integrate && !control ? 1 : 0);
    c->warped.push_back(warp_now ? 1 : control ? 2 : 0);
    c->f_ms.push_back(NAN);
    c->have_prev = true;
    if (phase) c->f_phase += 1;
    if (warp_now) {
        bool keep = true;
        if (c->fcfg.judge > 0) {
            const vegas_status js = flow_judge(c, t, &keep);
            if (js != VEGAS_OK) return js;
        }
        HIPCHK(c->fmark());
        if (keep && c->flow_on && c->fcfg.train) {
            // the sums of every step's slice in one launch (omega is fixed
            // for the iteration), each step reading its own
            const int n = c->fcfg.steps_per_iter;
            const bool together = n <= kFlowSumSlices;
            if (together) HIPCHK(flow_step_sums(c, n));
            for (int st = 0; st < n; ++st) {
                const vegas_status s = flow_train_step(c, together ? st : -1);
                if (s != VEGAS_OK) return s;
            }
        }
        HIPCHK(c->fmark());
    }
    if (phase) HIPCHK(judge_mark(c, t, 1));
    return VEGAS_OK;
}

// host-side start / tile table from an injected allocation
vegas_status upload_nh(vegas_ctx* c, const uint32_t* nh, int buf)
{
    const uint32_t nc = c->g.n_cubes;
    std::vector<uint32_t> st(nc + 1), tf(c->g.n_tiles + 1);
    uint64_t run = 0;
    for (uint32_t h = 0; h < nc; ++h) {
        if (nh[h] < (uint32_t)c->g.n_min) return fail(VEGAS_EINVAL, "n_h[%u] = %u below n_min", h, nh[h]);
        st[h] = (uint32_t)run;
        run += nh[h];
    }
    if (run != c->g.n_eval) return fail(VEGAS_EINVAL, "n_h sums to %llu, not n_eval", (unsigned long long)run);
    st[nc] = c->g.n_eval;
    uint32_t h = 0;
    for (int j = 0; j < c->g.n_tiles; ++j) {
        const uint64_t k = (uint64_t)j * c->g.tile;
        while (st[h + 1] <= k) ++h;
        tf[j] = h;
    }
    tf[c->g.n_tiles] = nc;
    HIPCHK(hipMemcpyAsync(c->at<uint32_t>(c->p.start[buf]), st.data(), sizeof(uint32_t) * st.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->at<uint32_t>(c->p.tfirst[buf]), tf.data(), sizeof(uint32_t) * tf.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return VEGAS_OK;
}

}  // namespace

namespace vgh {

void combine(const std::vector<double>& I, const std::vector<double>& s2, double* Ib, double* s2b, double* chi)
{
    // Eq. 8-9.  An iteration with sigma^2 = 0 is exact and decides the
    // result; one with I = 0 and sigma^2 = 0 had only zero weights (its
    // samples missed the integrand, or it underflowed) and is left out
    // whenever another iteration has a nonzero estimate.
    const size_t n = I.size();
    if (n == 0) {
        *Ib = 0.0;
        *s2b = INFINITY;
        *chi = 0.0;
        return;
    }
    auto empty = [&](size_t t) { return I[t] == 0.0 && s2[t] == 0.0; };
    size_t n_empty = 0;
    for (size_t t = 0; t < n; ++t) n_empty += empty(t) ? 1 : 0;
    if (n_empty == n) {
        *Ib = 0.0;
        *s2b = 0.0;
        *chi = 0.0;
        return;
    }
    int nz = 0;
    size_t m = 0;
    double zs = 0.0;
    for (size_t t = 0; t < n; ++t) {
        if (empty(t)) continue;
        ++m;
        if (s2[t] == 0.0) {
            ++nz;
            zs += I[t];
        }
    }
    if (nz > 0) {
        *Ib = zs / nz;
        *s2b = 0.0;
        *chi = 0.0;
        return;
    }
    double w = 0.0, wi = 0.0;
    for (size_t t = 0; t < n; ++t) {
        if (s2[t] == 0.0) continue;
        w += 1.0 / s2[t];
        wi += I[t] / s2[t];
    }
    const double mean = wi / w;
    double c2 = 0.0;
    for (size_t t = 0; t < n; ++t) {
        if (s2[t] == 0.0) continue;
        const double u = I[t] - mean;
        c2 += u * u / s2[t];
    }
    *Ib = mean;
    *s2b = 1.0 / w;
    *chi = m > 1 ? c2 / (double)(m - 1) : 0.0;
}

void ctx_set_stream(vegas_ctx* c, hipStream_t s) { c->stream = s; }

vegas_status ctx_fill_pass(vegas_ctx* c)
{
    if (c->flow_on || c->user || c->cfg.accum == VEGAS_ACC_ORDERED)
        return fail(VEGAS_EUNSUPPORTED, "a bare fill pass is for the plain FP64 / Kahan iteration");
    const int t = c->n_run;
    const bool fp64 = c->cfg.precision == VEGAS_PREC_FP64;
    const int lds_hist = c->g.lds_hist_ok ? 1 : 0;
    const int nb = c->g.D * c->g.ng;
    HIPCHK(launch_reset(c->vmax(t), 1, c->stream));
    if (!lds_hist) {
        const size_t nbr = (size_t)nb * c->n_wg;
        HIPCHK(launch_reset(c->at<unsigned long long>(c->p.histH), (int)nbr, c->stream));
        HIPCHK(launch_reset(c->at<unsigned long long>(c->p.histC), (int)((nbr + 1) / 2), c->stream));
    }
    // non-finite weights of this pass go to a spare counter, so the
    // iteration's own count is not touched
    const FillArgs a = fill_args(c, t, c->nonfinite() + 1);
    const size_t lds = fill_lds_bytes(c->g.D, c->g.ng, fp64, lds_hist, c->g.tile, c->g.n_aux, 0);
    HIPCHK(launch_fill(a, fp64, c->n_wg, lds, c->stream));
    return VEGAS_OK;
}

}  // namespace vgh

extern "C" {

const char* vegas_status_string(vegas_status s)
{
    switch (s) {
    case VEGAS_OK: return "ok";
    case VEGAS_EINVAL: return "invalid argument";
    case VEGAS_ENOMEM: return "workspace too small";
    case VEGAS_EDEVICE: return "HIP error";
    case VEGAS_ESTATE: return "invalid state";
    case VEGAS_ENONFINITE: return "non-finite integrand values";
    case VEGAS_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* vegas_last_error(void) { return g_err.c_str(); }

vegas_status vegas_workspace_size(const vegas_config* cfg, const vegas_integrand* f, size_t* bytes)
{
    Geometry g;
    const vegas_status s = geometry(cfg, f, &g);
    if (s != VEGAS_OK) return s;
    if (!bytes) return fail(VEGAS_EINVAL, "null bytes");
    *bytes = plan(g, cfg->max_iter > 0 ? cfg->max_iter : 4096, cfg->accum == VEGAS_ACC_ORDERED).total;
    return VEGAS_OK;
}

}  // extern "C"

namespace vgh {

// a context on the caller's workspace; user: the compiled integrand of
// family VEGAS_USER (else null)
vegas_status create_ctx(const vegas_config* cfg, const vegas_integrand* f, const vegas_user_fn* user,
                        void* d_workspace, size_t bytes, void* hip_stream, vegas_ctx** out)
{
    if (!out) return fail(VEGAS_EINVAL, "null out");
    *out = nullptr;
    Geometry g;
    vegas_status s = geometry(cfg, f, &g);
    if (s != VEGAS_OK) return s;
    if ((f->family == VEGAS_USER) != (user != nullptr))
        return fail(VEGAS_EINVAL, "family VEGAS_USER goes with a compiled integrand (vegas_create_user)");
    if (user) {
        if (user_fn_dim(user) != cfg->dim || user_fn_precision(user) != cfg->precision)
            return fail(VEGAS_EINVAL, "the compiled integrand is for dim %d precision %d, the config has %d and %d",
                        user_fn_dim(user), user_fn_precision(user), cfg->dim, cfg->precision);
        if (cfg->accum == VEGAS_ACC_ORDERED)
            return fail(VEGAS_EUNSUPPORTED, "ORDERED accumulation does not take compiled integrands");
    }
    const int max_iter = cfg->max_iter > 0 ? cfg->max_iter : 4096;
    const Plan p = plan(g, max_iter, cfg->accum == VEGAS_ACC_ORDERED);
    if (!d_workspace) return fail(VEGAS_EINVAL, "null workspace");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(VEGAS_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < p.total) return fail(VEGAS_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, p.total);
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    vegas_ctx* c = new vegas_ctx();
    c->cfg = *cfg;
    c->cfg.max_iter = max_iter;
    c->g = g;
    c->p = p;
    c->user = user;
    c->params.assign(f->params, f->params + g.n_params);
    c->lo.resize(g.D);
    c->hi.resize(g.D);
    for (int d = 0; d < g.D; ++d) {
        c->lo[d] = f->lo ? f->lo[d] : 0.0;
        c->hi[d] = f->hi ? f->hi[d] : 1.0;
    }
    c->stream = (hipStream_t)hip_stream;
    c->ws = (unsigned char*)d_workspace;
    c->n_wg = std::max(1, std::min({cus, kMaxWG, g.n_tiles}));
    c->n_cus = std::max(1, cus);
    // one launch for the fix-up, estimate and map where the map is cheap
    // against a launch (few intervals); larger maps keep their own kernel
    c->fused = cfg->accum != VEGAS_ACC_ORDERED && g.n_tiles <= 4096 && g.ng <= 512;
    c->cur = 0;
    c->max_iter = max_iter;
    c->n_run = 0;
    c->slots_last = 0;
    c->have_prev = false;
    c->timing = false;
    auto cleanup = [&](vegas_status st) {
        delete c;
        return st;
    };
#define HIPCHK_C(expr)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return cleanup(fail(VEGAS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    HIPCHK_C(hipMemcpyAsync(c->at<double>(p.prm), c->params.data(), sizeof(double) * g.n_params,
                            hipMemcpyHostToDevice, c->stream));
    HIPCHK_C(hipMemcpyAsync(c->at<double>(p.lo), c->lo.data(), sizeof(double) * g.D, hipMemcpyHostToDevice,
                            c->stream));
    HIPCHK_C(hipMemcpyAsync(c->at<double>(p.hi), c->hi.data(), sizeof(double) * g.D, hipMemcpyHostToDevice,
                            c->stream));
    HIPCHK_C(launch_reset(c->at<unsigned long long>(p.counters), 8, c->stream));
    PrepArgs pa;
    pa.family = g.family;
    pa.D = g.D;
    pa.n_params = g.n_params;
    pa.prm = c->at<double>(p.prm);
    pa.lo = c->at<double>(p.lo);
    pa.hi = c->at<double>(p.hi);
    pa.ng = g.ng;
    pa.aux_d = c->at<double>(p.aux_d);
    pa.aux_f = c->at<float>(p.aux_f);
    pa.grid64 = c->at<double>(p.grid64);
    pa.grid32 = c->at<float>(p.grid32);
    HIPCHK_C(launch_prep(pa, c->stream));
    // uniform initial allocation into buffer 0
    c->cur = 1;
    AllocArgs aa = alloc_args(c, 0, 1);
    HIPCHK_C(launch_alloc(aa, c->qmax(0), c->stream));
    c->cur = 0;
#undef HIPCHK_C
    *out = c;
    return VEGAS_OK;
}

}  // namespace vgh

extern "C" {

vegas_status vegas_create(const vegas_config* cfg, const vegas_integrand* f, void* d_workspace, size_t bytes,
                          void* hip_stream, vegas_ctx** out)
{
    return create_ctx(cfg, f, nullptr, d_workspace, bytes, hip_stream, out);
}

vegas_status vegas_create_user(const vegas_config* cfg, const vegas_integrand* f, const vegas_user_fn* fn,
                               void* d_workspace, size_t bytes, void* hip_stream, vegas_ctx** out)
{
    if (out) *out = nullptr;
    if (!fn) return fail(VEGAS_EINVAL, "null compiled integrand");
    if (!f || f->family != VEGAS_USER) return fail(VEGAS_EINVAL, "vegas_create_user takes family VEGAS_USER");
    return create_ctx(cfg, f, fn, d_workspace, bytes, hip_stream, out);
}

void vegas_destroy(vegas_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The library-held workspace of vegas_create_static, for callers that cannot
// allocate device memory.  Each device that runs the library holds its own
// copy of this array, at its own address, until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device memory: host
// code uses only the per-device address hipGetSymbolAddress returns.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[VEGAS_STATIC_SCRATCH_BYTES];

namespace vgh {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// the current device's address of `scratch`, looked up once per device with
// that device current
vegas_status scratch_address(void** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(VEGAS_EUNSUPPORTED, "device %d: the static workspace is kept for devices 0..%d", dev,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(VEGAS_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return VEGAS_OK;
}

}  // namespace vgh

extern "C" {

vegas_status vegas_create_static(const vegas_config* cfg, const vegas_integrand* f, void* hip_stream,
                                 vegas_ctx** out)
{
    if (!out) return fail(VEGAS_EINVAL, "null out");
    *out = nullptr;
    size_t need = 0;
    const vegas_status s = vegas_workspace_size(cfg, f, &need);
    if (s != VEGAS_OK) return s;
    if (need > (size_t)VEGAS_STATIC_SCRATCH_BYTES)
        return fail(VEGAS_ENOMEM, "the problem needs %zu bytes of workspace; the static workspace holds %zu",
                    need, (size_t)VEGAS_STATIC_SCRATCH_BYTES);
    void* ws = nullptr;
    const vegas_status a = scratch_address(&ws);
    if (a != VEGAS_OK) return a;
    // the same set-up as a caller workspace: every array an iteration reads
    // before writing it (counters, map, allocation, constants) is written
    // here, so what an earlier context left in the array does not matter
    return vegas_create(cfg, f, ws, (size_t)VEGAS_STATIC_SCRATCH_BYTES, hip_stream, out);
}

vegas_status vegas_adapt(vegas_ctx* ctx, int32_t n_iter)
{
    if (!ctx || n_iter < 0) return fail(VEGAS_EINVAL, "bad arguments");
    for (int i = 0; i < n_iter; ++i) {
        const vegas_status s = run_iteration(ctx, false);
        if (s != VEGAS_OK) return s;
    }
    return VEGAS_OK;
}

vegas_status vegas_integrate(vegas_ctx* ctx, int32_t n_iter)
{
    if (!ctx || n_iter < 0) return fail(VEGAS_EINVAL, "bad arguments");
    for (int i = 0; i < n_iter; ++i) {
        const vegas_status s = run_iteration(ctx, true);
        if (s != VEGAS_OK) return s;
    }
    return VEGAS_OK;
}

vegas_status vegas_get_iterations(vegas_ctx* c, double* I, double* sigma2, int32_t cap, int32_t* n)
{
    if (!c || !n) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    *n = c->n_run;
    const int m = std::min(cap, c->n_run);
    if (m > 0) {
        std::vector<double> buf(2 * (size_t)m);
        HIPCHK(hipMemcpy(buf.data(), c->at<double>(c->p.iter), sizeof(double) * buf.size(), hipMemcpyDeviceToHost));
        for (int t = 0; t < m; ++t) {
            if (I) I[t] = buf[2 * t];
            if (sigma2) sigma2[t] = buf[2 * t + 1];
        }
    }
    return VEGAS_OK;
}

vegas_status vegas_result(vegas_ctx* c, vegas_estimate* out)
{
    if (!c || !out) return fail(VEGAS_EINVAL, "bad arguments");
    std::vector<double> I(c->n_run), s2(c->n_run);
    int32_t n = 0;
    const vegas_status s = vegas_get_iterations(c, I.data(), s2.data(), c->n_run, &n);
    if (s != VEGAS_OK) return s;
    std::vector<double> Ic, s2c;
    for (int t = 0; t < n; ++t)
        if (c->combined[t]) {
            Ic.push_back(I[t]);
            s2c.push_back(s2[t]);
        }
    combine(Ic, s2c, &out->integral, &out->sigma2, &out->chi2_dof);
    out->n_iter_combined = (int32_t)Ic.size();
    out->n_iter_total = c->n_run;
    out->n_eval_total = (int64_t)c->n_run * (int64_t)c->g.n_eval;
    unsigned long long bad = 0;
    HIPCHK(hipMemcpy(&bad, c->nonfinite(), sizeof bad, hipMemcpyDeviceToHost));
    out->n_nonfinite = (int64_t)bad;
    if (bad) return fail(VEGAS_ENONFINITE, "%llu sample weights were NaN/Inf and counted as 0", bad);
    for (int t = 0; t < n; ++t)
        if (!std::isfinite(I[t]) || !std::isfinite(s2[t]))
            return fail(VEGAS_ENONFINITE, "iteration %d: estimate %g, variance %g are not finite (with KAHAN "
                                          "accumulation the sums are FP32: |w| must stay below about 1e19)",
                        t, I[t], s2[t]);
    return VEGAS_OK;
}

vegas_status vegas_get_info(const vegas_ctx* c, vegas_info* out)
{
    if (!c || !out) return fail(VEGAS_EINVAL, "bad arguments");
    out->n_strat = c->g.nst;
    out->n_cubes = c->g.n_cubes;
    out->n_rest = (int64_t)c->g.R;
    out->tile = c->g.tile;
    out->n_tiles = c->g.n_tiles;
    out->n_workgroups = c->n_wg;
    out->lds_hist = c->g.lds_hist_ok;
    out->workspace_bytes = c->p.total;
    return VEGAS_OK;
}

vegas_status vegas_get_map(vegas_ctx* c, double* grid)
{
    if (!c || !grid) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(grid, c->at<double>(c->p.grid64), sizeof(double) * c->g.D * (c->g.ng + 1),
                     hipMemcpyDeviceToHost));
    return VEGAS_OK;
}

vegas_status vegas_set_map(vegas_ctx* c, const double* grid)
{
    if (!c || !grid) return fail(VEGAS_EINVAL, "bad arguments");
    const int row = c->g.ng + 1;
    for (int d = 0; d < c->g.D; ++d)
        for (int i = 0; i < row; ++i) {
            const double v = grid[d * row + i];
            if (!std::isfinite(v) || (i > 0 && v < grid[d * row + i - 1]))
                return fail(VEGAS_EINVAL, "grid axis %d is not finite and non-decreasing", d);
        }
    const size_t n = (size_t)c->g.D * row;
    HIPCHK(hipMemcpyAsync(c->at<double>(c->p.grid64), grid, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(launch_grid32(c->at<double>(c->p.grid64), c->at<float>(c->p.grid32), (int)n, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return VEGAS_OK;
}

vegas_status vegas_set_params(vegas_ctx* c, const double* params)
{
    if (!c || !params) return fail(VEGAS_EINVAL, "bad arguments");
    // validate as a new problem of the same family and shape
    vegas_integrand f;
    f.family = c->g.family;
    f.n_params = c->g.n_params;
    f.params = params;
    f.lo = c->lo.data();
    f.hi = c->hi.data();
    Geometry g;
    const vegas_status s = geometry(&c->cfg, &f, &g);
    if (s != VEGAS_OK) return s;
    if (g.n_aux != c->g.n_aux) return fail(VEGAS_EINVAL, "new parameters change the size of the integrand's tables");
    c->params.assign(params, params + g.n_params);
    HIPCHK(hipMemcpyAsync(c->at<double>(c->p.prm), c->params.data(), sizeof(double) * g.n_params,
                          hipMemcpyHostToDevice, c->stream));
    PrepArgs pa;
    pa.family = g.family;
    pa.D = g.D;
    pa.n_params = g.n_params;
    pa.prm = c->at<double>(c->p.prm);
    pa.lo = c->at<double>(c->p.lo);
    pa.hi = c->at<double>(c->p.hi);
    pa.ng = g.ng;
    pa.aux_d = c->at<double>(c->p.aux_d);
    pa.aux_f = c->at<float>(c->p.aux_f);
    pa.grid64 = nullptr;                  // the map stays
    pa.grid32 = nullptr;
    HIPCHK(launch_prep(pa, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return VEGAS_OK;
}

vegas_status vegas_set_adapt(vegas_ctx* c, int32_t adapt_map, int32_t adapt_strat)
{
    if (!c || (adapt_map != 0 && adapt_map != 1) || (adapt_strat != 0 && adapt_strat != 1))
        return fail(VEGAS_EINVAL, "bad arguments");
    c->cfg.adapt_map = adapt_map;
    c->cfg.adapt_strat = adapt_strat;
    return VEGAS_OK;
}

vegas_status vegas_get_nh(vegas_ctx* c, uint32_t* nh)
{
    if (!c || !nh) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<uint32_t> st(c->g.n_cubes + 1);
    HIPCHK(hipMemcpy(st.data(), c->at<uint32_t>(c->p.start[c->cur]), sizeof(uint32_t) * st.size(),
                     hipMemcpyDeviceToHost));
    for (uint32_t h = 0; h < c->g.n_cubes; ++h) nh[h] = st[h + 1] - st[h];
    return VEGAS_OK;
}

vegas_status vegas_set_nh(vegas_ctx* c, const uint32_t* nh)
{
    if (!c || !nh) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    return upload_nh(c, nh, c->cur);
}

vegas_status vegas_get_accumulators(vegas_ctx* c, double* H, double* C, double* v)
{
    if (!c) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    const size_t nb = (size_t)c->g.D * c->g.ng;
    if (H) HIPCHK(hipMemcpy(H, c->at<double>(c->p.Hsum), sizeof(double) * nb, hipMemcpyDeviceToHost));
    if (C) HIPCHK(hipMemcpy(C, c->at<double>(c->p.Csum), sizeof(double) * nb, hipMemcpyDeviceToHost));
    if (v) HIPCHK(hipMemcpy(v, c->at<double>(c->p.v), sizeof(double) * c->g.n_cubes, hipMemcpyDeviceToHost));
    return VEGAS_OK;
}

vegas_status vegas_set_accumulators(vegas_ctx* c, const double* H, const double* C, const double* v)
{
    if (!c || !H || !C || !v) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    const size_t nb = (size_t)c->g.D * c->g.ng;
    std::vector<uint32_t> cu(nb);
    for (size_t i = 0; i < nb; ++i) {
        if (!(C[i] >= 0.0) || C[i] != std::floor(C[i]) || C[i] > 4294967295.0)
            return fail(VEGAS_EINVAL, "counts must be non-negative integers");
        cu[i] = (uint32_t)C[i];
    }
    double vmax = 0.0;
    for (uint32_t h = 0; h < c->g.n_cubes; ++h) {
        if (!(v[h] >= 0.0) || !std::isfinite(v[h])) return fail(VEGAS_EINVAL, "v must be finite and >= 0");
        vmax = std::max(vmax, v[h]);
    }
    unsigned long long bits;
    std::memcpy(&bits, &vmax, sizeof bits);
    const unsigned long long zero = 0;
    const int t = c->n_run;
    c->hist_weighted = false;
    HIPCHK(hipMemcpy(c->at<double>(c->p.histH), H, sizeof(double) * nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->at<uint32_t>(c->p.histC), cu.data(), sizeof(uint32_t) * nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->at<double>(c->p.v), v, sizeof(double) * c->g.n_cubes, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->vmax(t), &bits, sizeof bits, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->qmax(t), &zero, sizeof zero, hipMemcpyHostToDevice));
    c->slots_last = -1;      // injected: a single slot
    return VEGAS_OK;
}

vegas_status vegas_update(vegas_ctx* c)
{
    if (!c) return fail(VEGAS_EINVAL, "bad arguments");
    if (c->slots_last != -1) return fail(VEGAS_ESTATE, "vegas_update needs injected accumulators");
    const vegas_status s = run_update(c, c->n_run, 1, false);
    c->slots_last = 0;
    return s;
}

vegas_status vegas_set_timing(vegas_ctx* c, int32_t on)
{
    if (!c) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    c->events.clear();
    c->timing = on != 0;
    return VEGAS_OK;
}

vegas_status vegas_get_timing(vegas_ctx* c, double* ms, int32_t* n_iter)
{
    if (!c || !ms) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < 4; ++i) ms[i] = 0.0;
    // iterations record 5 marks; a lone vegas_update records 2 (alloc, map)
    size_t i = 0;
    int n = 0;
    while (i + 5 <= c->events.size()) {
        for (int p = 0; p < 4; ++p) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, c->events[i + p], c->events[i + p + 1]));
            ms[p] += t;
        }
        i += 5;
        ++n;
    }
    if (n_iter) *n_iter = n;
    return VEGAS_OK;
}

vegas_status vegas_sample_probe(vegas_ctx* c, uint32_t t, uint64_t k0, int64_t n, uint32_t* d_cube,
                                uint32_t* d_bins, double* d_delta, double* d_x, double* d_jac, double* d_f)
{
    if (!c || n < 0) return fail(VEGAS_EINVAL, "bad arguments");
    if (c->user) return fail(VEGAS_EUNSUPPORTED, "the sample probe does not take compiled integrands");
    if (n == 0) return VEGAS_OK;
    if (k0 + (uint64_t)n > c->g.n_eval) return fail(VEGAS_EINVAL, "sample range beyond n_eval");
    const bool fp64 = c->cfg.precision == VEGAS_PREC_FP64;
    ProbeArgs a;
    a.sc = sample_const(c);
    a.t = t;
    a.k0 = k0;
    a.n = n;
    a.grid = fp64 ? (const void*)c->at<double>(c->p.grid64) : (const void*)c->at<float>(c->p.grid32);
    a.start = c->at<uint32_t>(c->p.start[c->cur]);
    a.cube = d_cube;
    a.bins = d_bins;
    a.delta = d_delta;
    a.x = d_x;
    a.jac = d_jac;
    a.f = d_f;
    HIPCHK(launch_probe(a, fp64, c->stream));
    return VEGAS_OK;
}

// state image: header, grid, n_h, iteration log, flags, counters
}  // extern "C"

// ---------------------------------------------------------------------------
// learned warp
// ---------------------------------------------------------------------------
namespace {

struct FlowPlan {
    size_t theta, packed, slots, w, z, lj, om, U, G0, G1, part, grad, m, v, sumsq, acc, total;
};

// Each weight's forward and backward BF16 copy in the packed operands
// (value index, -1 none), from the packing's source map, which must give
// every weight exactly one of each and the biases none (checked once).
const std::vector<int32_t>* flow_slot_table()
{
    static const std::vector<int32_t> table = [] {
        std::vector<int32_t> t(2 * (size_t)kFParams, -1);
        std::vector<int> count(2 * (size_t)kFParams, 0);
        for (int l = 0; l < kFlowLayers; ++l)
            for (int r = 0; r < kPLayer; ++r)
                for (int j = 0; j < 8; ++j) {
                    const int src = flow_pack_src(l, r, j);
                    if (src < 0) continue;
                    const size_t at = 2 * ((size_t)l * kFLayer + src) + (r >= kPFwdT ? 1 : 0);
                    t[at] = (int32_t)(((size_t)l * kPLayer + r) * 8 + j);
                    count[at] += 1;
                }
        for (int l = 0; l < kFlowLayers; ++l)
            for (int i = 0; i < kFLayer; ++i) {
                const bool bias = (i >= kFB1 && i < kFW2) || (i >= kFB2 && i < kFW3) || i >= kFB3;
                for (int d = 0; d < 2; ++d)
                    if (count[2 * ((size_t)l * kFLayer + i) + d] != (bias ? 0 : 1)) return std::vector<int32_t>();
            }
        return t;
    }();
    return table.empty() ? nullptr : &table;
}

FlowPlan flow_plan(uint32_t n_eval, int n_wg)
{
    FlowPlan p;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    p.theta = take(sizeof(float) * kFParams);
    p.packed = take((size_t)16 * kFlowLayers * kPLayer);
    p.slots = take(sizeof(int32_t) * 2 * kFParams);
    p.w = take(sizeof(float) * kFlowDim * (size_t)n_eval);
    p.z = take(sizeof(float) * kFlowDim * (size_t)n_eval);
    p.lj = take(sizeof(float) * (size_t)n_eval);
    p.om = take(sizeof(float) * (size_t)n_eval);
    p.U = take(sizeof(float) * 3 * kFlowDim * (size_t)n_eval);
    p.G0 = take(sizeof(float) * kFlowDim * (size_t)n_eval);
    p.G1 = take(sizeof(float) * kFlowDim * (size_t)n_eval);
    p.part = take(sizeof(float) * kFParams * (size_t)n_wg);
    p.grad = take(sizeof(float) * kFParams);
    p.m = take(sizeof(float) * kFParams);
    p.v = take(sizeof(float) * kFParams);
    p.sumsq = take(sizeof(double) * kFlowSumRecord * kFlowSumSlices);
    p.acc = take(sizeof(float) * kFParams);
    p.total = o;
    return p;
}

// one training workgroup per CU (the gradient kernel takes 129 KB of LDS),
// at most the 256 whose parts the update kernel sums
int flow_train_wg(const vegas_ctx* c)
{
    const int chunks = (int)((c->g.n_eval + 127) / 128);
    return std::max(1, std::min({c->n_cus, chunks, kFlowMaxTrainWG}));
}

// the training samples are off, off + stride, ... of the iteration's samples
FlowTrainArgs flow_train_args(vegas_ctx* c, uint32_t stride, uint32_t off)
{
    FlowTrainArgs a;
    a.n = (c->g.n_eval - off + stride - 1) / stride;
    a.stride = stride;
    a.off = off;
    a.layer = 0;
    a.theta = reinterpret_cast<const float*>(c->fws + c->f_theta);
    a.packed = c->fws + c->f_packed;
    a.zf = reinterpret_cast<const float*>(c->fws + c->f_z);
    a.om = reinterpret_cast<const float*>(c->fws + c->f_om);
    a.sumsq = reinterpret_cast<const double*>(c->fws + c->f_sumsq);
    a.gamma = c->fcfg.loss == 1 ? 1 : 2;
    a.U = reinterpret_cast<float*>(c->fws + c->f_U);
    a.g_in = nullptr;
    a.g_out = nullptr;
    a.part = reinterpret_cast<float*>(c->fws + c->f_part);
    return a;
}

uint32_t flow_train_stride(const vegas_ctx* c)
{
    return (uint32_t)std::min<int64_t>(c->fcfg.train_stride, c->g.n_eval);
}

// the sums of the next n_steps training steps' slices (flow_train_step's
// offsets), one record each
hipError_t flow_step_sums(vegas_ctx* c, int n_steps)
{
    const uint32_t stride = flow_train_stride(c);
    return launch_flow_sums(reinterpret_cast<const float*>(c->fws + c->f_om), (uint32_t)c->g.n_eval, stride,
                            (uint32_t)(c->f_step % stride), n_steps, c->fcfg.loss == 1 ? 1 : 2,
                            reinterpret_cast<double*>(c->fws + c->f_sumsq), c->stream);
}

// gradient of the warp's loss on the last warped iteration's samples
// off, off + stride, ...; with adam set, the Adam step on it too.  slice:
// the record of flow_step_sums holding this slice's sums, or -1 to take
// them here.
vegas_status flow_gradient(vegas_ctx* c, uint32_t stride, uint32_t off, const FlowAdamArgs* adam, int slice = -1)
{
    FlowTrainArgs a = flow_train_args(c, stride, off);
    double* sums = reinterpret_cast<double*>(c->fws + c->f_sumsq);
    if (slice < 0) {
        HIPCHK(launch_flow_sums(a.om, (uint32_t)c->g.n_eval, stride, off, 1, a.gamma, sums, c->stream));
    } else {
        a.sumsq = sums + (size_t)slice * kFlowSumRecord;
    }
    hipEvent_t* ev = nullptr;
    if (c->f_timing) {
        for (int i = 0; i < 2; ++i) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            c->f_gev.push_back(e);
        }
        ev = c->f_gev.data() + c->f_gev.size() - 2;
    }
    HIPCHK(launch_flow_gradient(a, c->f_nwg, reinterpret_cast<float*>(c->fws + c->f_G0),
                                reinterpret_cast<float*>(c->fws + c->f_G1), reinterpret_cast<float*>(c->fws + c->f_grad),
                                adam, c->stream, ev));
    return VEGAS_OK;
}

constexpr int kJudgeRing = 64;           // iterations whose GPU time can be pending
constexpr double kJudgeGuard = 10.0;     // a warped iteration is rejected above this x the reference

double rel_var(double I, double s2) { return I != 0.0 ? s2 / (I * I) : INFINITY; }

double median_tail(const std::vector<double>& v, size_t m)
{
    if (v.empty()) return NAN;
    std::vector<double> t(v.end() - (ptrdiff_t)std::min(m, v.size()), v.end());
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

// Reads the GPU time of every finished iteration in the ring (both events
// complete) and files its efficiency, relative variance x ms, under warped
// or control.  Returns whether a new control efficiency arrived.
bool judge_read_times(vegas_ctx* c, int upto)
{
    bool new_ctrl = false;
    for (int slot = 0; slot < kJudgeRing; ++slot) {
        const int it = c->f_ev_iter[slot];
        if (it < 0 || it >= upto || it >= (int)c->log_I.size()) continue;
        float ms = 0.f;
        if (hipEventQuery(c->f_ev[2 * slot + 1]) != hipSuccess) continue;
        if (hipEventElapsedTime(&ms, c->f_ev[2 * slot], c->f_ev[2 * slot + 1]) != hipSuccess) continue;
        c->f_ev_iter[slot] = -1;
        c->f_ms[it] = ms;
        const double rv = rel_var(c->log_I[it], c->log_s2[it]);
        if (c->warped[it] == 1 && std::isfinite(rv)) c->warp_eff.push_back(rv * ms);
        if (c->warped[it] == 2) {
            // a control whose estimate lies beyond 5 sigma of the kept warped
            // estimate has missed the integrand's mass: plain VEGAS+ fails
            double e = rv * ms;
            if (c->kw_w > 0.0) {
                const double Iw = c->kw_sum / c->kw_w;
                if (std::fabs(c->log_I[it] - Iw) > 5.0 * std::sqrt(c->log_s2[it] + 1.0 / c->kw_w)) e = INFINITY;
            }
            if (!std::isfinite(rv)) e = INFINITY;
            c->ctrl_eff.push_back(e);
            new_ctrl = true;
        }
    }
    return new_ctrl;
}

// Event at the start (end = 0) or the end (end = 1) of iteration t while the
// warp is on; the pair of an iteration lives in ring slot t mod kJudgeRing.
hipError_t judge_mark(vegas_ctx* c, int t, int end)
{
    if (c->f_ev.empty()) {
        c->f_ev.assign(2 * kJudgeRing, nullptr);
        c->f_ev_iter.assign(kJudgeRing, -1);
        for (auto& e : c->f_ev) {
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
    }
    const int slot = t % kJudgeRing;
    if (end == 0) c->f_ev_iter[slot] = t;
    return hipEventRecord(c->f_ev[2 * slot + end], c->stream);
}

// The judge of warped iteration t (its estimate is read after a stream
// synchronisation):
//  guard: rejected when its estimate or variance is not finite, or its
//    relative variance sigma^2/I^2 exceeds kJudgeGuard x the median of the
//    last (up to 4) kept warped iterations (before any was kept: of the
//    last plain iterations).  A rejected iteration restores the last kept
//    parameters and restarts Adam; three rejections in a row switch the
//    warp off.  Kept: its parameters become the kept ones.
//  cost (judge = 2), after each control iteration: the warp's efficiency,
//    the median relative variance x GPU ms of its last (up to 8) warped
//    iterations, against the same for the last (up to 3) controls.  Not
//    better twice in a row: the warp is switched off and plain VEGAS+
//    continues.
vegas_status flow_judge(vegas_ctx* c, int t, bool* keep)
{
    HIPCHK(hipStreamSynchronize(c->stream));
    const int from = (int)c->log_I.size();
    if (t + 1 > from) {
        std::vector<double> buf(2 * (size_t)(t + 1 - from));
        HIPCHK(hipMemcpy(buf.data(), c->at<double>(c->p.iter) + 2 * from, sizeof(double) * buf.size(),
                         hipMemcpyDeviceToHost));
        for (int i = 0; i < t + 1 - from; ++i) {
            c->log_I.push_back(buf[2 * i]);
            c->log_s2.push_back(buf[2 * i + 1]);
        }
    }
    const double I = c->log_I[t], s2 = c->log_s2[t];
    const double rv = rel_var(I, s2);
    double ref = median_tail(c->kept_rv, 4);
    if (!(ref >= 0.0)) {
        std::vector<double> prv;
        for (int i = t - 1; i >= 0 && prv.size() < 4; --i)
            if (c->warped[i] != 1 && std::isfinite(rel_var(c->log_I[i], c->log_s2[i])))
                prv.push_back(rel_var(c->log_I[i], c->log_s2[i]));
        ref = median_tail(prv, 4);
    }
    bool ok = std::isfinite(I) && std::isfinite(s2) && std::isfinite(rv);
    if (ok && ref >= 0.0 && std::isfinite(ref)) ok = rv <= kJudgeGuard * ref;
    float* th = reinterpret_cast<float*>(c->fws + c->f_theta);
    float* acc = reinterpret_cast<float*>(c->fws + c->f_acc);
    if (ok) {
        c->rejects = 0;
        c->n_accepted += 1;
        c->kept_rv.push_back(rv);
        if (c->fcfg.judge == 2 && s2 > 0.0) {
            c->kw_sum += I / s2;
            c->kw_w += 1.0 / s2;
        }
        HIPCHK(hipMemcpyAsync(acc, th, sizeof(float) * kFParams, hipMemcpyDeviceToDevice, c->stream));
    } else {
        c->rejects += 1;
        c->n_rejected += 1;
        HIPCHK(hipMemcpyAsync(th, acc, sizeof(float) * kFParams, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(launch_flow_pack(th, c->fws + c->f_packed, c->stream));
        HIPCHK(launch_reset(reinterpret_cast<unsigned long long*>(c->fws + c->f_m), kFParams / 2, c->stream));
        HIPCHK(launch_reset(reinterpret_cast<unsigned long long*>(c->fws + c->f_v), kFParams / 2, c->stream));
        c->f_step = 0;
        if (c->rejects >= 3) c->flow_on = false;
    }
    const bool new_ctrl = judge_read_times(c, t);
    if (c->fcfg.judge == 2 && new_ctrl && !c->warp_eff.empty() && c->flow_on) {
        const double ew = median_tail(c->warp_eff, 8), ep = median_tail(c->ctrl_eff, 3);
        c->strikes = ew < ep ? 0 : c->strikes + 1;
        if (c->strikes >= 2) c->flow_on = false;
    }
    *keep = ok;
    return VEGAS_OK;
}

// one training step: gradient, Adam and the BF16 repack; slice as in
// flow_gradient
vegas_status flow_train_step(vegas_ctx* c, int slice)
{
    // a strided subset of the samples, its offset turning with the steps
    const uint32_t stride = flow_train_stride(c);
    float* th = reinterpret_cast<float*>(c->fws + c->f_theta);
    FlowAdamArgs adam;
    adam.theta = th;
    adam.m = reinterpret_cast<float*>(c->fws + c->f_m);
    adam.v = reinterpret_cast<float*>(c->fws + c->f_v);
    adam.packed = c->fws + c->f_packed;
    adam.slots = reinterpret_cast<const int32_t*>(c->fws + c->f_slots);
    adam.lr = c->fcfg.lr;
    adam.step = (int)(c->f_step + 1);
    vegas_status s = flow_gradient(c, stride, (uint32_t)(c->f_step % stride), &adam, slice);
    if (s != VEGAS_OK) return s;
    c->f_step += 1;
    return VEGAS_OK;
}

// validated copy of a warp configuration, defaults filled in
vegas_status flow_config_check(const vegas_flow_config* cfg, vegas_flow_config* out)
{
    if (!(cfg->lr >= 0.f) || !std::isfinite(cfg->lr)) return fail(VEGAS_EINVAL, "lr must be finite and >= 0");
    if (cfg->loss != 0 && cfg->loss != 1) return fail(VEGAS_EINVAL, "loss must be 0 (variance) or 1 (KL)");
    if (cfg->judge < 0 || cfg->judge > 2) return fail(VEGAS_EINVAL, "judge must be 0, 1 or 2");
    if (cfg->steps_per_iter < 0 || cfg->steps_per_iter > 64) return fail(VEGAS_EINVAL, "steps_per_iter must be 0..64");
    if (cfg->control_period != 0 && (cfg->control_period < 2 || cfg->control_period > 32))
        return fail(VEGAS_EINVAL, "control_period must be 0 or 2..32");
    if (cfg->train_stride < 0 || cfg->train_stride > 1024) return fail(VEGAS_EINVAL, "train_stride must be 0..1024");
    *out = *cfg;
    if (out->steps_per_iter == 0) out->steps_per_iter = 1;
    if (out->train_stride == 0) out->train_stride = 1;
    if (out->control_period == 0) out->control_period = 16;
    return VEGAS_OK;
}

vegas_status flow_check(const vegas_ctx* c)
{
    if (c->g.D != kFlowDim) return fail(VEGAS_EUNSUPPORTED, "the learned warp is built for dim %d", kFlowDim);
    if (c->cfg.precision != VEGAS_PREC_FP32) return fail(VEGAS_EUNSUPPORTED, "the learned warp runs the FP32 sample path");
    if (c->cfg.accum == VEGAS_ACC_ORDERED) return fail(VEGAS_EUNSUPPORTED, "no learned warp in ORDERED accumulation");
    const int f = c->g.family;
    if (f != VEGAS_GAUSS_DIAG && f != VEGAS_GENZ_PPEAK && f != VEGAS_GENZ_GAUSS && f != VEGAS_GAUSS_CORR)
        return fail(VEGAS_EUNSUPPORTED, "family %d has no warped fill", f);
    return VEGAS_OK;
}

}  // namespace

extern "C" {

int32_t vegas_flow_n_params(void) { return kFParams; }

vegas_status vegas_flow_workspace_size(const vegas_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return fail(VEGAS_EINVAL, "bad arguments");
    const vegas_status s = flow_check(c);
    if (s != VEGAS_OK) return s;
    *bytes = flow_plan(c->g.n_eval, flow_train_wg(c)).total;
    return VEGAS_OK;
}

vegas_status vegas_flow_attach(vegas_ctx* c, const vegas_flow_config* cfg, const float* params, void* d_ws,
                               size_t bytes)
{
    if (!c || !cfg || !d_ws) return fail(VEGAS_EINVAL, "bad arguments");
    vegas_status s = flow_check(c);
    if (s != VEGAS_OK) return s;
    if (((uintptr_t)d_ws & 255u) != 0) return fail(VEGAS_EINVAL, "flow workspace must be 256-byte aligned");
    const int nwg = flow_train_wg(c);
    const FlowPlan p = flow_plan(c->g.n_eval, nwg);
    if (bytes < p.total) return fail(VEGAS_ENOMEM, "flow workspace has %zu bytes, needs %zu", bytes, p.total);
    vegas_flow_config fc;
    s = flow_config_check(cfg, &fc);
    if (s != VEGAS_OK) return s;
    if (params)
        for (int i = 0; i < kFParams; ++i)
            if (!std::isfinite(params[i])) return fail(VEGAS_EINVAL, "flow parameter %d is not finite", i);
    c->fcfg = fc;
    c->fws = (unsigned char*)d_ws;
    c->f_theta = p.theta;
    c->f_packed = p.packed;
    c->f_slots = p.slots;
    c->f_w = p.w;
    c->f_z = p.z;
    c->f_lj = p.lj;
    c->f_om = p.om;
    c->f_U = p.U;
    c->f_G0 = p.G0;
    c->f_G1 = p.G1;
    c->f_part = p.part;
    c->f_grad = p.grad;
    c->f_m = p.m;
    c->f_v = p.v;
    c->f_sumsq = p.sumsq;
    c->f_acc = p.acc;
    c->f_nwg = nwg;
    c->f_step = 0;
    c->flow_attached = true;
    c->flow_on = false;
    HIPCHK(launch_reset(reinterpret_cast<unsigned long long*>(c->fws + p.m), kFParams / 2, c->stream));
    HIPCHK(launch_reset(reinterpret_cast<unsigned long long*>(c->fws + p.v), kFParams / 2, c->stream));
    HIPCHK(launch_reset(reinterpret_cast<unsigned long long*>(c->fws + p.om), (int)((c->g.n_eval + 1) / 2), c->stream));
    const std::vector<int32_t>* slots = flow_slot_table();
    if (!slots) return fail(VEGAS_EUNSUPPORTED, "warp operand packing: a weight without exactly one copy per direction");
    HIPCHK(hipMemcpyAsync(c->fws + p.slots, slots->data(), sizeof(int32_t) * slots->size(), hipMemcpyHostToDevice,
                          c->stream));
    if (params) return vegas_flow_set_params(c, params);
    // the library's own starting weights
    float* th = reinterpret_cast<float*>(c->fws + c->f_theta);
    HIPCHK(launch_flow_init(th, fc.init_seed, c->stream));
    HIPCHK(launch_flow_pack(th, c->fws + c->f_packed, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return VEGAS_OK;
}

vegas_status vegas_flow_set_config(vegas_ctx* c, const vegas_flow_config* cfg)
{
    if (!c || !cfg) return fail(VEGAS_EINVAL, "bad arguments");
    if (!c->flow_attached) return fail(VEGAS_ESTATE, "no flow attached");
    vegas_flow_config fc;
    const vegas_status s = flow_config_check(cfg, &fc);
    if (s != VEGAS_OK) return s;
    if (fc.judge != c->fcfg.judge) {
        // a new judge mode starts its cost records afresh
        c->warp_eff.clear();
        c->ctrl_eff.clear();
        c->kw_sum = c->kw_w = 0.0;
        c->strikes = 0;
    }
    if (fc.control_period != c->fcfg.control_period) c->f_phase = 0;
    c->fcfg = fc;
    return VEGAS_OK;
}

vegas_status vegas_flow_enable(vegas_ctx* c, int32_t on)
{
    if (!c) return fail(VEGAS_EINVAL, "bad arguments");
    if (on && !c->flow_attached) return fail(VEGAS_ESTATE, "no flow attached");
    if (on && !c->flow_on) {
        // the parameters now in place are the kept ones
        c->rejects = 0;
        c->strikes = 0;
        c->f_phase = 0;
        HIPCHK(hipMemcpyAsync(c->fws + c->f_acc, c->fws + c->f_theta, sizeof(float) * kFParams,
                              hipMemcpyDeviceToDevice, c->stream));
    }
    c->flow_on = on != 0;
    return VEGAS_OK;
}

vegas_status vegas_flow_set_timing(vegas_ctx* c, int32_t on)
{
    if (!c) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    for (hipEvent_t e : c->f_tev) (void)hipEventDestroy(e);
    c->f_tev.clear();
    for (hipEvent_t e : c->f_gev) (void)hipEventDestroy(e);
    c->f_gev.clear();
    c->f_timing = on != 0;
    return VEGAS_OK;
}

vegas_status vegas_flow_get_timing(vegas_ctx* c, double* ms, int32_t* n_iter)
{
    if (!c || !ms) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    ms[0] = ms[1] = 0.0;
    int n = 0;
    for (size_t i = 0; i + 4 <= c->f_tev.size(); i += 4, ++n) {
        float a = 0.f, b = 0.f;
        HIPCHK(hipEventElapsedTime(&a, c->f_tev[i], c->f_tev[i + 1]));
        HIPCHK(hipEventElapsedTime(&b, c->f_tev[i + 2], c->f_tev[i + 3]));
        ms[0] += a;
        ms[1] += b;
    }
    if (n_iter) *n_iter = n;
    return VEGAS_OK;
}

vegas_status vegas_flow_get_grad_timing(vegas_ctx* c, double* ms, int32_t* n_launch)
{
    if (!c || !ms) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(c->stream));
    *ms = 0.0;
    int n = 0;
    for (size_t i = 0; i + 2 <= c->f_gev.size(); i += 2, ++n) {
        float a = 0.f;
        HIPCHK(hipEventElapsedTime(&a, c->f_gev[i], c->f_gev[i + 1]));
        *ms += a;
    }
    if (n_launch) *n_launch = n;
    return VEGAS_OK;
}

vegas_status vegas_flow_get_kinds(vegas_ctx* c, int32_t* kinds, int32_t cap, int32_t* n)
{
    if (!c || !n) return fail(VEGAS_EINVAL, "bad arguments");
    *n = c->n_run;
    for (int t = 0; t < std::min(cap, c->n_run) && kinds; ++t) kinds[t] = c->warped[t];
    return VEGAS_OK;
}

vegas_status vegas_flow_status(const vegas_ctx* c, int32_t* on, int32_t* accepted, int32_t* rejected)
{
    if (!c) return fail(VEGAS_EINVAL, "bad arguments");
    if (on) *on = c->flow_on ? 1 : 0;
    if (accepted) *accepted = c->n_accepted;
    if (rejected) *rejected = c->n_rejected;
    return VEGAS_OK;
}

vegas_status vegas_flow_set_params(vegas_ctx* c, const float* params)
{
    if (!c || !params) return fail(VEGAS_EINVAL, "bad arguments");
    if (!c->flow_attached) return fail(VEGAS_ESTATE, "no flow attached");
    HIPCHK(hipMemcpyAsync(c->fws + c->f_theta, params, sizeof(float) * kFParams, hipMemcpyHostToDevice, c->stream));
    HIPCHK(launch_flow_pack(reinterpret_cast<const float*>(c->fws + c->f_theta), c->fws + c->f_packed, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return VEGAS_OK;
}

vegas_status vegas_flow_get_params(vegas_ctx* c, float* params)
{
    if (!c || !params) return fail(VEGAS_EINVAL, "bad arguments");
    if (!c->flow_attached) return fail(VEGAS_ESTATE, "no flow attached");
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(params, c->fws + c->f_theta, sizeof(float) * kFParams, hipMemcpyDeviceToHost));
    return VEGAS_OK;
}

vegas_status vegas_flow_get_samples(vegas_ctx* c, float* w, float* lj, float* om, float* z)
{
    if (!c) return fail(VEGAS_EINVAL, "bad arguments");
    if (!c->flow_attached) return fail(VEGAS_ESTATE, "no flow attached");
    HIPCHK(hipStreamSynchronize(c->stream));
    const size_t n = c->g.n_eval;
    if (w) HIPCHK(hipMemcpy(w, c->fws + c->f_w, sizeof(float) * kFlowDim * n, hipMemcpyDeviceToHost));
    if (lj) HIPCHK(hipMemcpy(lj, c->fws + c->f_lj, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (om) HIPCHK(hipMemcpy(om, c->fws + c->f_om, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (z) HIPCHK(hipMemcpy(z, c->fws + c->f_z, sizeof(float) * kFlowDim * n, hipMemcpyDeviceToHost));
    return VEGAS_OK;
}

vegas_status vegas_flow_grad(vegas_ctx* c, float* grad)
{
    if (!c || !grad) return fail(VEGAS_EINVAL, "bad arguments");
    if (!c->flow_attached) return fail(VEGAS_ESTATE, "no flow attached");
    const vegas_status s = flow_gradient(c, 1, 0, nullptr);
    if (s != VEGAS_OK) return s;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(grad, c->fws + c->f_grad, sizeof(float) * kFParams, hipMemcpyDeviceToHost));
    return VEGAS_OK;
}

vegas_status vegas_flow_adam_step(vegas_ctx* c, const float* grad)
{
    if (!c || !grad) return fail(VEGAS_EINVAL, "bad arguments");
    if (!c->flow_attached) return fail(VEGAS_ESTATE, "no flow attached");
    for (int i = 0; i < kFParams; ++i)
        if (!std::isfinite(grad[i])) return fail(VEGAS_EINVAL, "gradient entry %d is not finite", i);
    HIPCHK(hipMemcpyAsync(c->fws + c->f_grad, grad, sizeof(float) * kFParams, hipMemcpyHostToDevice, c->stream));
    c->f_step += 1;
    float* th = reinterpret_cast<float*>(c->fws + c->f_theta);
    HIPCHK(launch_flow_adam(th, reinterpret_cast<const float*>(c->fws + c->f_grad), reinterpret_cast<float*>(c->fws + c->f_m),
                            reinterpret_cast<float*>(c->fws + c->f_v), c->fcfg.lr, c->f_step, c->stream));
    HIPCHK(launch_flow_pack(th, c->fws + c->f_packed, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return VEGAS_OK;
}

vegas_status vegas_mfma_probe(const float* d_A, const float* d_B, float* d_D)
{
    if (!d_A || !d_B || !d_D) return fail(VEGAS_EINVAL, "bad arguments");
    HIPCHK(launch_mfma_probe(d_A, d_B, d_D, nullptr));
    HIPCHK(hipDeviceSynchronize());
    return VEGAS_OK;
}

}  // extern "C"

extern "C" {

struct StateHeader {
    uint64_t magic;
    int32_t D, ng;
    uint32_t n_cubes, n_eval;
    int32_t n_run, have_prev;
    uint64_t nonfinite;
};
static const uint64_t kStateMagic = 0x5645474153535431ull;   // "VEGASST1"

vegas_status vegas_get_state(vegas_ctx* c, void* buf, size_t* bytes)
{
    if (!c || !bytes) return fail(VEGAS_EINVAL, "bad arguments");
    const size_t ng = (size_t)c->g.D * (c->g.ng + 1);
    const size_t need = sizeof(StateHeader) + sizeof(double) * ng + sizeof(uint32_t) * c->g.n_cubes +
                        sizeof(double) * 2 * c->n_run + c->n_run;
    if (!buf) {
        *bytes = need;
        return VEGAS_OK;
    }
    if (*bytes < need) return fail(VEGAS_ENOMEM, "state buffer needs %zu bytes", need);
    HIPCHK(hipStreamSynchronize(c->stream));
    unsigned char* o = (unsigned char*)buf;
    StateHeader h;
    h.magic = kStateMagic;
    h.D = c->g.D;
    h.ng = c->g.ng;
    h.n_cubes = c->g.n_cubes;
    h.n_eval = c->g.n_eval;
    h.n_run = c->n_run;
    h.have_prev = c->have_prev;
    unsigned long long bad = 0;
    HIPCHK(hipMemcpy(&bad, c->nonfinite(), sizeof bad, hipMemcpyDeviceToHost));
    h.nonfinite = bad;
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    HIPCHK(hipMemcpy(o, c->at<double>(c->p.grid64), sizeof(double) * ng, hipMemcpyDeviceToHost));
    o += sizeof(double) * ng;
    const vegas_status s = vegas_get_nh(c, (uint32_t*)o);
    if (s != VEGAS_OK) return s;
    o += sizeof(uint32_t) * c->g.n_cubes;
    if (c->n_run > 0)
        HIPCHK(hipMemcpy(o, c->at<double>(c->p.iter), sizeof(double) * 2 * c->n_run, hipMemcpyDeviceToHost));
    o += sizeof(double) * 2 * c->n_run;
    std::memcpy(o, c->combined.data(), c->n_run);
    *bytes = need;
    return VEGAS_OK;
}

vegas_status vegas_set_state(vegas_ctx* c, const void* buf, size_t bytes)
{
    if (!c || !buf || bytes < sizeof(StateHeader)) return fail(VEGAS_EINVAL, "bad arguments");
    StateHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (h.magic != kStateMagic || h.D != c->g.D || h.ng != c->g.ng || h.n_cubes != c->g.n_cubes ||
        h.n_eval != c->g.n_eval)
        return fail(VEGAS_EINVAL, "state image does not match this context");
    const size_t ng = (size_t)c->g.D * (c->g.ng + 1);
    const size_t need = sizeof(StateHeader) + sizeof(double) * ng + sizeof(uint32_t) * c->g.n_cubes +
                        sizeof(double) * 2 * h.n_run + h.n_run;
    if (bytes < need || h.n_run > c->max_iter) return fail(VEGAS_EINVAL, "state image truncated or too long");
    const unsigned char* o = (const unsigned char*)buf + sizeof h;
    vegas_status s = vegas_set_map(c, (const double*)o);
    if (s != VEGAS_OK) return s;
    o += sizeof(double) * ng;
    s = vegas_set_nh(c, (const uint32_t*)o);
    if (s != VEGAS_OK) return s;
    o += sizeof(uint32_t) * c->g.n_cubes;
    if (h.n_run > 0)
        HIPCHK(hipMemcpy(c->at<double>(c->p.iter), o, sizeof(double) * 2 * h.n_run, hipMemcpyHostToDevice));
    o += sizeof(double) * 2 * h.n_run;
    c->combined.assign(o, o + h.n_run);
    c->warped.assign(h.n_run, 0);
    c->f_ms.assign(h.n_run, NAN);
    c->log_I.clear();
    c->log_s2.clear();
    if (!c->f_ev_iter.empty()) c->f_ev_iter.assign(c->f_ev_iter.size(), -1);
    c->n_run = h.n_run;
    c->have_prev = h.have_prev != 0;
    unsigned long long bad = h.nonfinite;
    HIPCHK(hipMemcpy(c->nonfinite(), &bad, sizeof bad, hipMemcpyHostToDevice));
    return VEGAS_OK;
}

}  // extern "C"
