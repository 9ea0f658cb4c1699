// VegasFill (Alg. 2) for gfx950: the data-parallel half of one VEGAS+
// iteration.
//
// Layout of the work.  Samples k = 0 .. N_ev-1 of an iteration are ordered by
// hypercube: cube h owns the contiguous range [start_h, start_{h+1}) (its
// n_h samples, Sec. 2.1.2).  The fill is a persistent kernel, one 1024-lane
// workgroup per CU, that walks tiles of `tile` consecutive samples; lane l of
// a tile owns `per_lane` consecutive samples.  Every sample costs the same
// whatever the allocation (the balance requirement of Sec. 3.1), and a lane
// meets the cubes of its range in order, so most cubes are summed inside one
// lane with no atomics.
//
// Per sample (Alg. 2): its cube (getCube) from the tile's cube starts in
// LDS; its stratum digits; Philox4x32-10 words keyed by (k, t, instance);
// the fixed-point point and bin index (getPoint, Eq. 3); x and the Jacobian
// J = prod N_g dx from the map held in LDS (getJac, Eq. 2-4); f(x); w = J f.
// Then w^2 and a count go to the per-axis histograms (LDS-privatised,
// flushed per workgroup) and w to the running shifted sums of its cube.
//
// Per cube (Eq. 5-6): runs of a cube that cross lanes merge in LDS with
// Chan's pairwise formula; runs that cross tiles go to a side record and a
// fix-up kernel merges them in tile order.  Each finished cube yields its
// mean m_h and unbiased variance v_h; the iteration estimate is
// I = sum m_h / N_c and sigma^2 = sum v_h / (N_c^2 n_h), reduced in a fixed
// order so that a run is reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "layout.hpp"
#include "launch.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// merging partial moments (Chan, Golub, LeVeque 1983)
// ---------------------------------------------------------------------------
__device__ __forceinline__ Partial merge(const Partial& a, const Partial& b)
{
    Partial o;
    o.h = a.h;
    o.n = a.n + b.n;
    const double na = (double)a.n, nb = (double)b.n, n = (double)o.n;
    const double dm = b.mean - a.mean;
    o.mean = a.mean + dm * (nb / n);
    o.m2 = a.m2 + b.m2 + (dm * dm) * (na * nb / n);
    return o;
}

__device__ __forceinline__ double unbiased_var(const Partial& p)
{
    const double m2 = p.m2 > 0.0 ? p.m2 : 0.0;
    return m2 / (double)(p.n - 1u);
}

// ---------------------------------------------------------------------------
// the per-sample path shared by the fill and the probe
// ---------------------------------------------------------------------------
template <typename R, int FAM, int MAXD>
struct SamplePath {
    const SampleConst& sc;
    Fn<R, FAM> fn;
    R ngR;
    double nst_d;
    float inv_nst_f;

    __device__ __forceinline__ explicit SamplePath(const SampleConst& c) : sc(c)
    {
        fn.setup(c);
        ngR = (R)c.ng;
        nst_d = (double)c.nst;
        inv_nst_f = (float)(1.0 / (double)c.nst);
    }

    // digits of cube h in base N_st, axis 0 fastest
    __device__ __forceinline__ void digits(uint32_t h, uint32_t (&s)[MAXD]) const
    {
#pragma unroll
        for (int d = 0; d < MAXD; ++d) {
            const uint32_t q = div_magic(h, sc.nst_magic, sc.nst_shift);
            s[d] = h - q * sc.nst;
            h = q;
        }
    }

    __device__ __forceinline__ void next_digits(uint32_t (&s)[MAXD]) const
    {
        bool carry = true;
#pragma unroll
        for (int d = 0; d < MAXD; ++d) {
            if (carry) {
                const uint32_t v = s[d] + 1u;
                carry = (v == sc.nst);
                s[d] = carry ? 0u : v;
            }
        }
    }

    // Evaluate sample k (iteration t) of the cube with digits s against the
    // grid g (row stride N_g+1).  Returns w = J f; bins and (optionally)
    // delta / x / J / f are reported through the out-parameters.
    template <bool PROBE>
    __device__ __forceinline__ R eval(uint32_t k, uint32_t t, const uint32_t (&s)[MAXD],
                                      const R* __restrict__ g, uint32_t (&bins)[MAXD],
                                      R* delta_out, R* x_out, R& J, R& f)
    {
        uint32_t wd[MAXD];
#pragma unroll
        for (int b = 0; b < (MAXD + 3) / 4; ++b) {
            if (4 * b < sc.D) {
                const W4 o = philox10(k, 0u, t, sc.ctr3 | (uint32_t)b, sc.key0, sc.key1);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * b + q < MAXD) wd[4 * b + q] = o.v[q];
            }
        }
        J = (R)1;
        fn.begin();
        const uint32_t row = sc.ng + 1u;
#pragma unroll
        for (int d = 0; d < MAXD; ++d) {
            if (d < sc.D) {
                const BinSplit p = bin_split(s[d], wd[d], sc.ng, sc.nst, sc.nst_magic, sc.nst_shift);
                bins[d] = p.bin;
                R delta;
                if constexpr (std::is_same<R, double>::value) delta = delta_f64(p, nst_d);
                else delta = delta_f32(p, inv_nst_f);
                const R* gd = g + d * row;
                const R xl = gd[p.bin];
                const R dx = gd[p.bin + 1] - xl;
                const R x = fma(dx, delta, xl);
                J = J * (ngR * dx);
                fn.axis(d, x);
                if constexpr (PROBE) {
                    delta_out[d] = delta;
                    x_out[d] = x;
                }
            }
        }
        f = fn.finish();
        return J * f;
    }
};

// ---------------------------------------------------------------------------
// the fill kernel
// ---------------------------------------------------------------------------
struct LdsPlan {
    uint32_t grid_off, h_off, c_off, st_off, hp_off, tp_off, fl_off, misc_off, total;
};

__host__ __device__ inline LdsPlan lds_plan(int D, int ng, int real_bytes, int lds_hist, int tile, int n_min)
{
    LdsPlan p;
    uint32_t o = 0;
    auto al = [](uint32_t v) { return (v + 15u) & ~15u; };
    p.grid_off = o; o = al(o + (uint32_t)(D * (ng + 1) * real_bytes));
    p.h_off = o;
    if (lds_hist) o = al(o + (uint32_t)(D * ng * real_bytes));
    p.c_off = o;
    if (lds_hist) o = al(o + (uint32_t)(((D * ng + 1) / 2) * 4));
    p.st_off = o; o = al(o + (uint32_t)((tile / n_min + 4) * 4));
    p.hp_off = o; o = al(o + (uint32_t)(kLanesPerTile * sizeof(Partial)));
    p.tp_off = o; o = al(o + (uint32_t)(kLanesPerTile * sizeof(Partial)));
    p.fl_off = o; o = al(o + (uint32_t)kLanesPerTile);
    p.misc_off = o; o = al(o + 2 * sizeof(Partial) + 64);
    p.total = o;
    return p;
}

template <typename R>
__device__ __forceinline__ void lds_fadd(R* p, R v)
{
    atomicAdd(p, v);
}

template <typename R, int FAM, int MAXD>
__global__ __launch_bounds__(kFillThreads) void k_fill(FillArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SampleConst& sc = a.sc;
    const int D = sc.D;
    const uint32_t ng = sc.ng;
    const int tid = threadIdx.x;
    const int S = a.per_lane;
    const LdsPlan lp = lds_plan(D, (int)ng, (int)sizeof(R), a.lds_hist, a.tile, 2);
    R* gl = reinterpret_cast<R*>(smem + lp.grid_off);
    R* hl = reinterpret_cast<R*>(smem + lp.h_off);
    uint32_t* cl = reinterpret_cast<uint32_t*>(smem + lp.c_off);
    uint32_t* st = reinterpret_cast<uint32_t*>(smem + lp.st_off);
    Partial* HP = reinterpret_cast<Partial*>(smem + lp.hp_off);
    Partial* TP = reinterpret_cast<Partial*>(smem + lp.tp_off);
    uint8_t* FL = smem + lp.fl_off;
    Partial* tside = reinterpret_cast<Partial*>(smem + lp.misc_off);     // [0] head, [1] tail
    uint32_t* tflags = reinterpret_cast<uint32_t*>(smem + lp.misc_off + 2 * sizeof(Partial));

    const int nbins = D * (int)ng;
    const int nwords = (nbins + 1) / 2;
    const R* gsrc = reinterpret_cast<const R*>(a.grid);
    for (int i = tid; i < D * (int)(ng + 1); i += kFillThreads) gl[i] = gsrc[i];
    if (a.lds_hist) {
        for (int i = tid; i < nbins; i += kFillThreads) hl[i] = (R)0;
        for (int i = tid; i < nwords; i += kFillThreads) cl[i] = 0u;
    }

    // power-of-two scale for the FP32 histogram (keeps (J f)^2 in range)
    R hs = (R)1;
    double inv_hs2 = 1.0;
    if (std::is_same<R, float>::value && a.prev_iter != nullptr) {
        const double Ip = fabs(a.prev_iter[0]);
        if (Ip > 0.0 && Ip < 1e300) {
            int e = ilogb(Ip);
            e = e < -60 ? -60 : (e > 60 ? 60 : e);
            hs = (R)ldexp(1.0, -e);
            inv_hs2 = ldexp(1.0, 2 * e);
        }
    }

    SamplePath<R, FAM, MAXD> sp(sc);
    double accI = 0.0, accV = 0.0, vmax = 0.0;
    unsigned long long bad = 0;
    const double* hslotH = nullptr;
    (void)hslotH;
    double* slotH = a.lds_hist ? a.hist_H + (size_t)blockIdx.x * nbins : a.hist_H;
    uint32_t* slotC = a.lds_hist ? a.hist_C + (size_t)blockIdx.x * nbins : a.hist_C;
    bool first_flush = true;
    int since_flush = 0;

    auto flush = [&]() {
        // called by all threads between barriers
        for (int wi = tid; wi < nwords; wi += kFillThreads) {
            const uint32_t cw = cl[wi];
            cl[wi] = 0u;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int i = 2 * wi + q;
                if (i < nbins) {
                    const double hv = (double)hl[i] * inv_hs2;
                    hl[i] = (R)0;
                    const uint32_t cv = (cw >> (16 * q)) & 0xFFFFu;
                    if (first_flush) {
                        slotH[i] = hv;
                        slotC[i] = cv;
                    } else {
                        slotH[i] += hv;
                        slotC[i] += cv;
                    }
                }
            }
        }
        first_flush = false;
    };

    __syncthreads();

    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const uint32_t t0 = (uint32_t)tile * (uint32_t)a.tile;
        const uint32_t t1 = min(t0 + (uint32_t)a.tile, sc.n_eval);
        const uint32_t h_lo = a.tile_first[tile];
        const uint32_t h_nx = a.tile_first[tile + 1];
        const uint32_t h_top = min(h_nx, sc.n_cubes - 1u);
        const int nst_load = (int)(h_top - h_lo) + 2;   // starts of h_lo .. h_top+1
        for (int i = tid; i < nst_load; i += kFillThreads) st[i] = a.start[h_lo + i];
        if (tid == 0) *tflags = 0u;
        __syncthreads();

        const uint32_t k0 = t0 + (uint32_t)(tid * S);
        const uint32_t k1 = min(k0 + (uint32_t)S, t1);
        const int n_active = (int)((t1 - t0 + (uint32_t)S - 1u) / (uint32_t)S);
        uint8_t fl = 0;
        if (k0 < k1) {
            // largest idx with st[idx] <= k0
            int lo = 0, hi = nst_load - 1;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (st[mid] <= k0) lo = mid; else hi = mid;
            }
            int idx = lo;
            uint32_t h = h_lo + (uint32_t)idx;
            uint32_t nxt = st[idx + 1];
            bool head = st[idx] < k0;
            uint32_t s[MAXD];
            sp.digits(h, s);
            uint32_t n = 0;
            double c = 0.0, S1 = 0.0, S2 = 0.0;

            auto close_run = [&]() {
                Partial p;
                p.h = h;
                p.n = n;
                const double dn = (double)n;
                p.mean = c + S1 / dn;
                p.m2 = S2 - S1 * (S1 / dn);
                if (head) {
                    HP[tid] = p;
                    fl |= (uint8_t)kHasHead;
                } else {
                    const double v = unbiased_var(p);
                    a.v_out[h] = v;
                    accI += p.mean;
                    accV += v / dn;
                    vmax = v > vmax ? v : vmax;
                }
            };

            for (int j = 0; j < S; ++j) {
                const uint32_t k = k0 + (uint32_t)j;
                if (k >= k1) break;
                if (k == nxt) {
                    close_run();
                    ++idx;
                    ++h;
                    nxt = st[idx + 1];
                    head = false;
                    n = 0;
                    S1 = 0.0;
                    S2 = 0.0;
                    sp.next_digits(s);
                }
                uint32_t bins[MAXD];
                R J, f;
                R w = sp.template eval<false>(k, a.t, s, gl, bins, nullptr, nullptr, J, f);
                if (!__builtin_isfinite(w)) {
                    w = (R)0;
                    ++bad;
                }
                if (a.lds_hist) {
                    const R ws = w * hs;
                    const R w2 = ws * ws;
#pragma unroll
                    for (int d = 0; d < MAXD; ++d) {
                        if (d < D) {
                            const uint32_t bi = (uint32_t)d * ng + bins[d];
                            lds_fadd(hl + bi, w2);
                            atomicAdd(cl + (bi >> 1), 1u << ((bi & 1u) << 4));
                        }
                    }
                } else {
                    const double wd = (double)w;
                    const double w2 = wd * wd;
#pragma unroll
                    for (int d = 0; d < MAXD; ++d) {
                        if (d < D) {
                            const uint32_t bi = (uint32_t)d * ng + bins[d];
                            unsafeAtomicAdd(a.hist_H + bi, w2);
                            atomicAdd(a.hist_C + bi, 1u);
                        }
                    }
                }
                const double wd = (double)w;
                if (n == 0) c = wd;
                const double u = wd - c;
                S1 += u;
                S2 = fma(u, u, S2);
                ++n;
            }
            if (nxt > k1) {
                Partial p;
                p.h = h;
                p.n = n;
                const double dn = (double)n;
                p.mean = c + S1 / dn;
                p.m2 = S2 - S1 * (S1 / dn);
                TP[tid] = p;
                fl |= (uint8_t)(head ? (kHasTail | kSpan) : kHasTail);
            } else {
                close_run();
            }
        }
        FL[tid] = fl;
        __syncthreads();

        // ---- merge runs of cubes that cross lanes -------------------------
        if ((fl & kHasTail) && !(fl & kSpan)) {
            Partial cur = TP[tid];
            int m = tid + 1;
            for (;;) {
                if (m >= n_active) {          // continues into the next tile
                    tside[1] = cur;
                    atomicOr(tflags, kHasTail);
                    break;
                }
                const uint8_t fm = FL[m];
                if (fm & kSpan) {
                    cur = merge(cur, TP[m]);
                    ++m;
                    continue;
                }
                cur = merge(cur, HP[m]);
                const double v = unbiased_var(cur);
                a.v_out[cur.h] = v;
                accI += cur.mean;
                accV += v / (double)cur.n;
                vmax = v > vmax ? v : vmax;
                break;
            }
        }
        if (tid == 0 && (fl & (kHasHead | kSpan))) {
            // the tile's first cube began in an earlier tile
            if (fl & kSpan) {
                Partial cur = TP[0];
                int m = 1;
                uint32_t f2 = kHasHead;
                for (;;) {
                    if (m >= n_active) {
                        f2 = kHasHead | kHasTail | kSpan;
                        break;
                    }
                    const uint8_t fm = FL[m];
                    if (fm & kSpan) {
                        cur = merge(cur, TP[m]);
                        ++m;
                        continue;
                    }
                    cur = merge(cur, HP[m]);
                    break;
                }
                tside[0] = cur;
                atomicOr(tflags, f2);
            } else {
                tside[0] = HP[0];
                atomicOr(tflags, kHasHead);
            }
        }
        __syncthreads();
        if (tid == 0) {
            TileSide ts;
            ts.flags = *tflags;
            ts.head = tside[0];
            ts.tail = (ts.flags & kSpan) ? tside[0] : tside[1];
            ts.pad = 0;
            a.side[tile] = ts;
        }
        if (a.lds_hist && ++since_flush >= a.flush_every) {
            flush();
            since_flush = 0;
        }
        __syncthreads();
    }
    if (a.lds_hist) {
        flush();
    }

    // ---- fixed-order workgroup reduction of the lane partials -------------
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem + lp.hp_off);
    red[tid] = accI;
    red[kFillThreads + tid] = accV;
    red[2 * kFillThreads + tid] = vmax;
    __syncthreads();
    for (int w = kFillThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[tid] += red[tid + w];
            red[kFillThreads + tid] += red[kFillThreads + tid + w];
            const double o = red[2 * kFillThreads + tid + w];
            if (o > red[2 * kFillThreads + tid]) red[2 * kFillThreads + tid] = o;
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.wg_part[2 * blockIdx.x] = red[0];
        a.wg_part[2 * blockIdx.x + 1] = red[kFillThreads];
        atomicMax(a.vmax, (unsigned long long)__double_as_longlong(red[2 * kFillThreads]));
    }
    if (bad) atomicAdd(a.nonfinite, bad);
}

// ---------------------------------------------------------------------------
// cubes that cross tiles: merge their runs in tile order
// ---------------------------------------------------------------------------
__global__ void k_fixup(FixupArgs a)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n_tiles) return;
    double mI = 0.0, mV = 0.0;
    const uint32_t f = a.side[j].flags;
    if ((f & kHasTail) && !(f & kSpan)) {
        Partial cur = a.side[j].tail;
        int m = j + 1;
        while (m < a.n_tiles) {
            const TileSide& ts = a.side[m];
            cur = merge(cur, ts.head);
            if (!(ts.flags & kSpan)) break;
            ++m;
        }
        const double v = unbiased_var(cur);
        a.v_out[cur.h] = v;
        mI = cur.mean;
        mV = v / (double)cur.n;
        atomicMax(a.vmax, (unsigned long long)__double_as_longlong(v));
    }
    a.fix_part[2 * j] = mI;
    a.fix_part[2 * j + 1] = mV;
}

// ---------------------------------------------------------------------------
// iteration estimate: fixed-order sum of workgroup and fix-up partials
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_final(FinalArgs a)
{
    __shared__ double rI[1024], rV[1024];
    const int tid = threadIdx.x;
    double sI = 0.0, sV = 0.0;
    for (int i = tid; i < a.n_wg; i += 1024) {
        sI += a.wg_part[2 * i];
        sV += a.wg_part[2 * i + 1];
    }
    for (int i = tid; i < a.n_tiles; i += 1024) {
        sI += a.fix_part[2 * i];
        sV += a.fix_part[2 * i + 1];
    }
    rI[tid] = sI;
    rV[tid] = sV;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) {
            rI[tid] += rI[tid + w];
            rV[tid] += rV[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.iter_out[0] = rI[0] / a.n_cubes;
        a.iter_out[1] = rV[0] / (a.n_cubes * a.n_cubes);
    }
}

// ---------------------------------------------------------------------------
// probe: the per-sample path for a range of samples, outputs widened to FP64
// ---------------------------------------------------------------------------
template <typename R, int FAM, int MAXD>
__global__ void k_probe(ProbeArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t k = (uint32_t)(a.k0 + (uint64_t)i);
    // cube of k: largest h with start[h] <= k
    uint32_t lo = 0, hi = a.sc.n_cubes;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.start[mid] <= k) lo = mid; else hi = mid;
    }
    SamplePath<R, FAM, MAXD> sp(a.sc);
    uint32_t s[MAXD], bins[MAXD];
    R delta[MAXD], x[MAXD], J, f;
    sp.digits(lo, s);
    sp.template eval<true>(k, a.t, s, reinterpret_cast<const R*>(a.grid), bins, delta, x, J, f);
    const int D = a.sc.D;
    if (a.cube) a.cube[i] = lo;
#pragma unroll
    for (int d = 0; d < MAXD; ++d) {
        if (d < D) {
            if (a.bins) a.bins[i * D + d] = bins[d];
            if (a.delta) a.delta[i * D + d] = (double)delta[d];
            if (a.x) a.x[i * D + d] = (double)x[d];
        }
    }
    if (a.jac) a.jac[i] = (double)J;
    if (a.f) a.f[i] = (double)f;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <typename R, int FAM>
static hipError_t launch_fill_fam(const FillArgs& a, int n_wg, size_t lds, hipStream_t st)
{
    const int D = a.sc.D;
    if (D <= 4) {
        hipFuncSetAttribute((const void*)k_fill<R, FAM, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_fill<R, FAM, 4>), dim3(n_wg), dim3(kFillThreads), lds, st, a);
    } else if (D <= 8) {
        hipFuncSetAttribute((const void*)k_fill<R, FAM, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_fill<R, FAM, 8>), dim3(n_wg), dim3(kFillThreads), lds, st, a);
    } else if (D <= 12) {
        hipFuncSetAttribute((const void*)k_fill<R, FAM, 12>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_fill<R, FAM, 12>), dim3(n_wg), dim3(kFillThreads), lds, st, a);
    } else {
        hipFuncSetAttribute((const void*)k_fill<R, FAM, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_fill<R, FAM, 16>), dim3(n_wg), dim3(kFillThreads), lds, st, a);
    }
    return hipGetLastError();
}

template <typename R, int FAM>
static hipError_t launch_probe_fam(const ProbeArgs& a, hipStream_t st)
{
    const int D = a.sc.D;
    const int bs = 256;
    const unsigned nb = (unsigned)((a.n + bs - 1) / bs);
    if (D <= 4) hipLaunchKernelGGL((k_probe<R, FAM, 4>), dim3(nb), dim3(bs), 0, st, a);
    else if (D <= 8) hipLaunchKernelGGL((k_probe<R, FAM, 8>), dim3(nb), dim3(bs), 0, st, a);
    else if (D <= 12) hipLaunchKernelGGL((k_probe<R, FAM, 12>), dim3(nb), dim3(bs), 0, st, a);
    else hipLaunchKernelGGL((k_probe<R, FAM, 16>), dim3(nb), dim3(bs), 0, st, a);
    return hipGetLastError();
}

#define VG_FAMILY_SWITCH(R, CALL, ...)                                          \
    switch (fam) {                                                             \
    case F_GAUSS_DIAG: return CALL<R, F_GAUSS_DIAG>(__VA_ARGS__);              \
    case F_GENZ_PPEAK: return CALL<R, F_GENZ_PPEAK>(__VA_ARGS__);              \
    case F_GENZ_GAUSS: return CALL<R, F_GENZ_GAUSS>(__VA_ARGS__);              \
    case F_GAUSS_CORR: return CALL<R, F_GAUSS_CORR>(__VA_ARGS__);              \
    case F_LINEAR: return CALL<R, F_LINEAR>(__VA_ARGS__);                      \
    case F_ROOS: return CALL<R, F_ROOS>(__VA_ARGS__);                          \
    case F_CONST: return CALL<R, F_CONST>(__VA_ARGS__);                        \
    case F_COSINE: return CALL<R, F_COSINE>(__VA_ARGS__);                      \
    default: return hipErrorInvalidValue;                                      \
    }

hipError_t launch_fill(const FillArgs& a, bool fp64, int n_wg, size_t lds, hipStream_t st)
{
    const int fam = a.sc.family;
    if (fp64) {
        VG_FAMILY_SWITCH(double, launch_fill_fam, a, n_wg, lds, st)
    } else {
        VG_FAMILY_SWITCH(float, launch_fill_fam, a, n_wg, lds, st)
    }
}

hipError_t launch_probe(const ProbeArgs& a, bool fp64, hipStream_t st)
{
    const int fam = a.sc.family;
    if (fp64) {
        VG_FAMILY_SWITCH(double, launch_probe_fam, a, st)
    } else {
        VG_FAMILY_SWITCH(float, launch_probe_fam, a, st)
    }
}

hipError_t launch_fixup(const FixupArgs& a, hipStream_t st)
{
    const int bs = 256;
    hipLaunchKernelGGL(k_fixup, dim3((a.n_tiles + bs - 1) / bs), dim3(bs), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_final(const FinalArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

size_t fill_lds_bytes(int D, int ng, bool fp64, int lds_hist, int tile)
{
    return lds_plan(D, ng, fp64 ? 8 : 4, lds_hist, tile, 2).total;
}

}  // namespace vg
