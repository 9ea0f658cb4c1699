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
// Then w^2 and a count go to the per-axis histograms (privatised in LDS,
// written once per workgroup) and w to the running shifted sums of its cube.
//
// Per cube (Eq. 5-6): runs of a cube that cross lanes merge with Chan's
// pairwise formula in a segmented scan over wavefront shuffles, with one
// carry per wave through LDS; runs that cross tiles go to a side record and
// a fix-up kernel merges them in tile order.  Each finished cube yields its
// mean m_h and unbiased variance v_h; the iteration estimate is
// I = sum m_h / N_c and sigma^2 = sum v_h / (N_c^2 n_h), reduced in a fixed
// order so that a run is reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "layout.hpp"
#include "launch.hpp"
#include "sample.hpp"

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
// runs of one cube: count, mean, sum of squared deviations
// ---------------------------------------------------------------------------
struct Run {
    uint32_t n;
    double mean;
    double m2;
};

__device__ __forceinline__ Run run_empty()
{
    Run r;
    r.n = 0;
    r.mean = 0.0;
    r.m2 = 0.0;
    return r;
}

__device__ __forceinline__ Run run_merge(const Run& a, const Run& b)
{
    if (a.n == 0) return b;
    if (b.n == 0) return a;
    Run o;
    o.n = a.n + b.n;
    const double na = (double)a.n, nb = (double)b.n, n = (double)o.n;
    const double dm = b.mean - a.mean;
    o.mean = a.mean + dm * (nb / n);
    o.m2 = a.m2 + b.m2 + (dm * dm) * (na * nb / n);
    return o;
}

__device__ __forceinline__ Run run_shfl_up(const Run& r, int o)
{
    Run u;
    u.n = __shfl_up(r.n, o, 64);
    u.mean = __shfl_up(r.mean, o, 64);
    u.m2 = __shfl_up(r.m2, o, 64);
    return u;
}

// 1/n to double precision: hardware reciprocal plus one Newton step
__device__ __forceinline__ double recip(double n)
{
    double y = __builtin_amdgcn_rcp(n);
    y = fma(fma(-n, y, 1.0), y, y);
    return fma(fma(-n, y, 1.0), y, y);
}

// shifted sums (c, S1 = sum (w - c), S2 = sum (w - c)^2) of n samples -> run
__device__ __forceinline__ Run run_from_sums(uint32_t n, double c, double S1, double S2)
{
    Run r;
    r.n = n;
    const double inv = recip((double)n);
    const double m1 = S1 * inv;
    r.mean = c + m1;
    r.m2 = fma(-S1, m1, S2);
    return r;
}

// unbiased variance of a finished cube and its share v/n of sigma^2
__device__ __forceinline__ void run_finish(const Run& r, double& v, double& v_over_n)
{
    const double dn = (double)r.n;
    const double m2 = r.m2 > 0.0 ? r.m2 : 0.0;
    v = m2 * recip(dn - 1.0);
    v_over_n = v * recip(dn);
}

__device__ __forceinline__ Partial to_partial(const Run& r, uint32_t h)
{
    Partial p;
    p.h = h;
    p.n = r.n;
    p.mean = r.mean;
    p.m2 = r.m2;
    return p;
}

// ---------------------------------------------------------------------------
// the fill kernel
// ---------------------------------------------------------------------------
constexpr int kWaves = kFillThreads / 64;

struct WaveRec {
    Run s;            // scanned run at the wave's last lane
    uint32_t tail;    // last lane ends in a cube that continues
    uint32_t open;    // that run reaches back past the wave's first lane
};

struct LdsPlan {
    uint32_t grid_off, aux_off, h_off, c_off, st_off, wave_off, cin_off, side_off, red_off, total;
};

// LDS: map [D][N_g+1] in the sample path's precision; histogram weights
// [D][N_g] in FP64 (the FP32 LDS atomic add is an order of magnitude slower
// than the FP64 one on gfx950) and u32 counts; the tile's cube starts;
// per-wave carry records; the tile's side record; a reduction area.
__host__ __device__ inline LdsPlan lds_plan(int D, int ng, int real_bytes, int lds_hist, int tile, int n_aux)
{
    LdsPlan p;
    uint32_t o = 0;
    auto al = [](uint32_t v) { return (v + 15u) & ~15u; };
    p.grid_off = o; o = al(o + (uint32_t)(D * (ng + 1) * real_bytes));
    p.aux_off = o; o = al(o + (uint32_t)(n_aux * real_bytes));
    p.h_off = o;
    if (lds_hist) o = al(o + (uint32_t)(D * ng * 8));
    p.c_off = o;
    if (lds_hist) o = al(o + (uint32_t)(D * ng * 4));
    p.st_off = o; o = al(o + (uint32_t)((tile / 2 + 4) * 4));
    p.wave_off = o; o = al(o + (uint32_t)(kWaves * sizeof(WaveRec)));
    p.cin_off = o; o = al(o + (uint32_t)(kWaves * sizeof(WaveRec)));
    p.side_off = o; o = al(o + (uint32_t)(2 * sizeof(Partial) + 16));
    p.red_off = o; o = al(o + (uint32_t)(kWaves * 3 * sizeof(double)));
    p.total = o;
    return p;
}

template <typename R, int FAM, int MAXD>
__global__ __launch_bounds__(kFillThreads) void k_fill(FillArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SampleConst& sc = a.sc;
    const int D = sc.D;
    const uint32_t ng = sc.ng;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int S = a.per_lane;
    const LdsPlan lp = lds_plan(D, (int)ng, (int)sizeof(R), a.lds_hist, a.tile, sc.n_aux);
    R* gl = reinterpret_cast<R*>(smem + lp.grid_off);
    R* auxl = reinterpret_cast<R*>(smem + lp.aux_off);
    double* hl = reinterpret_cast<double*>(smem + lp.h_off);
    uint32_t* cl = reinterpret_cast<uint32_t*>(smem + lp.c_off);
    uint32_t* st = reinterpret_cast<uint32_t*>(smem + lp.st_off);
    WaveRec* wrec = reinterpret_cast<WaveRec*>(smem + lp.wave_off);
    WaveRec* cin = reinterpret_cast<WaveRec*>(smem + lp.cin_off);     // open = tile-head chain
    Partial* tside = reinterpret_cast<Partial*>(smem + lp.side_off);  // [0] head, [1] tail
    uint32_t* tflags = reinterpret_cast<uint32_t*>(smem + lp.side_off + 2 * sizeof(Partial));
    double* red = reinterpret_cast<double*>(smem + lp.red_off);

    const int nbins = D * (int)ng;
    const R* gsrc = reinterpret_cast<const R*>(a.grid);
    for (int i = tid; i < D * (int)(ng + 1); i += kFillThreads) gl[i] = gsrc[i];
    {
        const R* asrc = std::is_same<R, double>::value ? reinterpret_cast<const R*>(sc.aux_d)
                                                       : reinterpret_cast<const R*>(sc.aux_f);
        for (int i = tid; i < sc.n_aux; i += kFillThreads) auxl[i] = asrc[i];
    }
    if (a.lds_hist) {
        for (int i = tid; i < nbins; i += kFillThreads) {
            hl[i] = 0.0;
            cl[i] = 0u;
        }
    }

    SamplePath<R, FAM, MAXD> sp(sc, auxl);
    double accI = 0.0, accV = 0.0, vmax = 0.0;
    unsigned long long bad = 0;

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
        // per lane: the run of its first cube when that cube began earlier
        // (head), and the run of its last cube when it continues (tail)
        bool has_head = false, has_tail = false, span = false;
        Run hrun = run_empty(), trun = run_empty();
        uint32_t h_first = 0, h_last = 0;
        if (k0 < k1) {
            int lo = 0, hi = nst_load - 1;          // largest idx with st[idx] <= k0
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (st[mid] <= k0) lo = mid; else hi = mid;
            }
            int idx = lo;
            uint32_t h = h_lo + (uint32_t)idx;
            h_first = h;
            uint32_t nxt = st[idx + 1];
            bool head = st[idx] < k0;
            uint32_t s[MAXD];
            sp.digits(h, s);
            uint32_t n = 0;
            double c = 0.0, S1 = 0.0, S2 = 0.0;

            for (int j = 0; j < S; ++j) {
                const uint32_t k = k0 + (uint32_t)j;
                if (k >= k1) break;
                if (k == nxt) {
                    // the current cube ends: shifted sums -> (mean, m2)
                    const Run r = run_from_sums(n, c, S1, S2);
                    if (head) {
                        hrun = r;
                        has_head = true;
                    } else {
                        double v, vn;
                        run_finish(r, v, vn);
                        a.v_out[h] = v;
                        accI += r.mean;
                        accV += vn;
                        vmax = v > vmax ? v : vmax;
                    }
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
                const double wd = (double)w;
                const double w2 = wd * wd;
                if (a.lds_hist) {
#pragma unroll
                    for (int d = 0; d < MAXD; ++d) {
                        if (d < D) {
                            const uint32_t bi = (uint32_t)d * ng + bins[d];
                            atomicAdd(hl + bi, w2);
                            atomicAdd(cl + bi, 1u);
                        }
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < MAXD; ++d) {
                        if (d < D) {
                            const uint32_t bi = (uint32_t)d * ng + bins[d];
                            unsafeAtomicAdd(a.hist_H + bi, w2);
                            atomicAdd(a.hist_C + bi, 1u);
                        }
                    }
                }
                if (n == 0) c = wd;
                const double u = wd - c;
                S1 += u;
                S2 = fma(u, u, S2);
                ++n;
            }
            h_last = h;
            const Run r = run_from_sums(n, c, S1, S2);
            if (nxt > k1) {                 // continues into the next lane
                trun = r;
                has_tail = true;
                span = head;
            } else if (head) {
                hrun = r;
                has_head = true;
            } else {
                double v, vn;
                run_finish(r, v, vn);
                a.v_out[h] = v;
                accI += r.mean;
                accV += vn;
                vmax = v > vmax ? v : vmax;
            }
        }

        // ---- runs that cross lanes: segmented scan inside the wavefront ---
        // S_l = merge(S_{l-1}, tail_l) while lane l continues the cube of
        // lane l-1 (span), else tail_l.  Hillis-Steele over shuffles, stopping
        // as soon as every chain has reached its first lane.
        Run sv = has_tail ? trun : run_empty();
        int sf = (has_tail && span) ? 0 : 1;       // 1: a chain starts here
        for (int o = 1; o < 64; o <<= 1) {
            const Run u = run_shfl_up(sv, o);
            const int fu = __shfl_up(sf, o, 64);
            if (lane >= o && !sf) {
                sv = run_merge(u, sv);
                sf = fu;
            }
            if (__ballot(!sf && lane >= 2 * o) == 0ull) break;
        }
        if (lane == 63) {
            wrec[wave].s = sv;
            wrec[wave].tail = has_tail ? 1u : 0u;
            wrec[wave].open = sf ? 0u : 1u;
        }
        const Run prev = run_shfl_up(sv, 1);
        const int prev_f = __shfl_up(sf, 1, 64);
        __syncthreads();
        if (tid == 0) {
            // carries between waves; the chain entering wave 0 is the tile's
            // first cube, which began in an earlier tile
            Run c = run_empty();
            uint32_t th = 1u;
            for (int w = 0; w < kWaves; ++w) {
                cin[w].s = c;
                cin[w].open = th;
                const WaveRec& r = wrec[w];
                if (r.tail) {
                    if (r.open) {
                        c = run_merge(c, r.s);
                    } else {
                        c = r.s;
                        th = 0u;
                    }
                } else {
                    c = run_empty();
                    th = 0u;
                }
            }
        }
        __syncthreads();
        if (has_head && !span) {
            Run pre;
            uint32_t th;
            if (lane == 0 || !prev_f) {
                pre = lane == 0 ? cin[wave].s : run_merge(cin[wave].s, prev);
                th = cin[wave].open;
            } else {
                pre = prev;
                th = 0u;
            }
            const Run fin = run_merge(pre, hrun);
            if (th) {
                tside[0] = to_partial(fin, h_lo);
                atomicOr(tflags, kHasHead);
            } else {
                double v, vn;
                run_finish(fin, v, vn);
                a.v_out[h_first] = v;
                accI += fin.mean;
                accV += vn;
                vmax = v > vmax ? v : vmax;
            }
        }
        if (tid == n_active - 1 && has_tail) {
            Run t = sv;
            uint32_t th = 0u;
            if (!sf) {
                t = run_merge(cin[wave].s, sv);
                th = cin[wave].open;
            }
            if (th) {
                tside[0] = to_partial(t, h_lo);
                atomicOr(tflags, kHasHead | kHasTail | kSpan);
            } else {
                tside[1] = to_partial(t, h_last);
                atomicOr(tflags, kHasTail);
            }
        }
        __syncthreads();
        if (tid == 0) {
            const uint32_t fl = *tflags;
            TileSide* ts = a.side + tile;
            ts->flags = fl;
            ts->head = tside[0];
            ts->tail = (fl & kSpan) ? tside[0] : tside[1];
        }
        __syncthreads();
    }
    if (a.lds_hist) {
        // this workgroup's histograms into its slot (reduced in slot order by
        // the map kernel)
        double* slotH = a.hist_H + (size_t)blockIdx.x * nbins;
        uint32_t* slotC = a.hist_C + (size_t)blockIdx.x * nbins;
        for (int i = tid; i < nbins; i += kFillThreads) {
            slotH[i] = hl[i];
            slotC[i] = cl[i];
        }
    }

    // ---- fixed-order workgroup reduction of the lane partials -------------
    for (int o = 32; o > 0; o >>= 1) {
        accI += __shfl_down(accI, o, 64);
        accV += __shfl_down(accV, o, 64);
        const double m = __shfl_down(vmax, o, 64);
        vmax = m > vmax ? m : vmax;
    }
    if (lane == 0) {
        red[3 * wave] = accI;
        red[3 * wave + 1] = accV;
        red[3 * wave + 2] = vmax;
    }
    __syncthreads();
    if (tid == 0) {
        double sI = 0.0, sV = 0.0, mx = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            sI += red[3 * w];
            sV += red[3 * w + 1];
            mx = red[3 * w + 2] > mx ? red[3 * w + 2] : mx;
        }
        a.wg_part[2 * blockIdx.x] = sI;
        a.wg_part[2 * blockIdx.x + 1] = sV;
        atomicMax(a.vmax, (unsigned long long)__double_as_longlong(mx));
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
    const R* aux = std::is_same<R, double>::value ? reinterpret_cast<const R*>(a.sc.aux_d)
                                                  : reinterpret_cast<const R*>(a.sc.aux_f);
    SamplePath<R, FAM, MAXD> sp(a.sc, aux);
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

size_t fill_lds_bytes(int D, int ng, bool fp64, int lds_hist, int tile, int n_aux)
{
    return lds_plan(D, ng, fp64 ? 8 : 4, lds_hist, tile, n_aux).total;
}

}  // namespace vg
