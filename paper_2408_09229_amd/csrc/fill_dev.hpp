// Device building blocks of the fill (Alg. 2): per-cube moment runs and
// their merges, per-lane accumulators, the LDS plan, and one tile of the
// fill.  Shared by the single-problem and the batched fill kernels.
#pragma once
#ifndef __HIPCC_RTC__   // hipRTC provides the HIP device runtime itself
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>
#include <type_traits>

#include "common.hpp"
#include "families.hpp"
#include "layout.hpp"
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
// per-lane accumulators.  FP64: shifted sums in double.  Kahan: shifted sums
// and lane totals in compensated FP32 (each add carries its rounding error
// forward; contraction is off, so the compensation is not folded away).
// ---------------------------------------------------------------------------
template <bool KAHAN>
struct CubeSums;

template <>
struct CubeSums<false> {
    double c, s1, s2;
    __device__ __forceinline__ void reset() { s1 = 0.0; s2 = 0.0; }
    template <typename R>
    __device__ __forceinline__ void add(R w, bool first)
    {
        const double wd = (double)w;
        if (first) c = wd;
        const double u = wd - c;
        s1 += u;
        s2 = fma(u, u, s2);
    }
    __device__ __forceinline__ Run run(uint32_t n) const { return run_from_sums(n, c, s1, s2); }
};

template <>
struct CubeSums<true> {
    float c, s1, k1, s2, k2;
    __device__ __forceinline__ void reset() { s1 = 0.f; k1 = 0.f; s2 = 0.f; k2 = 0.f; }
    template <typename R>
    __device__ __forceinline__ void add(R w, bool first)
    {
        const float wf = (float)w;
        if (first) c = wf;
        const float u = wf - c;
        const float y1 = u - k1;
        const float t1 = s1 + y1;
        k1 = (t1 - s1) - y1;
        s1 = t1;
        const float y2 = u * u - k2;
        const float t2 = s2 + y2;
        k2 = (t2 - s2) - y2;
        s2 = t2;
    }
    __device__ __forceinline__ Run run(uint32_t n) const
    {
        return run_from_sums(n, (double)c, (double)s1 - (double)k1, (double)s2 - (double)k2);
    }
};

template <bool KAHAN>
struct LaneTotal;

template <>
struct LaneTotal<false> {
    double s = 0.0;
    __device__ __forceinline__ void add(double v) { s += v; }
    __device__ __forceinline__ double value() const { return s; }
};

template <>
struct LaneTotal<true> {
    float s = 0.f, k = 0.f;
    __device__ __forceinline__ void add(double v)
    {
        const float y = (float)v - k;
        const float t = s + y;
        k = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)k; }
};

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

// LDS: map [D][N_g+1] in the sample path's precision (map_lds = 1; the
// plain fill reads the map through the vector cache instead, whose loads do
// not queue behind the histogram atomics in the LDS pipe); histogram weights
// [D][N_g] in FP64 (the FP32 LDS atomic add is about 25 times slower than the
// FP64 one on gfx950) and u32 counts; the tile's cube starts; per-wave carry
// records; the tile's side record; a reduction area.
__host__ __device__ inline LdsPlan lds_plan(int D, int ng, int real_bytes, int lds_hist, int tile, int n_aux,
                                            int map_lds)
{
    LdsPlan p;
    uint32_t o = 0;
    auto al = [](uint32_t v) { return (v + 15u) & ~15u; };
    p.grid_off = o;
    if (map_lds) o = al(o + (uint32_t)(D * (ng + 1) * real_bytes));
    p.aux_off = o; o = al(o + (uint32_t)(n_aux * real_bytes));
    p.h_off = o;
    if (lds_hist) o = al(o + (uint32_t)(D * ng * 8));
    p.c_off = o;
    if (lds_hist) o = al(o + (uint32_t)(D * ng * 4));
    p.st_off = o; o = al(o + (uint32_t)((tile / 2 + 4) * 2));
    p.wave_off = o; o = al(o + (uint32_t)(kWaves * sizeof(WaveRec)));
    p.cin_off = o; o = al(o + (uint32_t)(kWaves * sizeof(WaveRec)));
    p.side_off = o; o = al(o + (uint32_t)(2 * sizeof(Partial) + 16));
    p.red_off = o; o = al(o + (uint32_t)(kWaves * 3 * sizeof(double)));
    p.total = o;
    return p;
}

// What one tile of the fill reads and writes outside LDS.
struct TileIO {
    uint32_t t;                   // iteration (Philox counter word 2)
    int32_t tile;                 // samples per tile
    int32_t per_lane;
    int32_t lds_hist;
    const uint32_t* start;        // [N_c+1]
    const uint32_t* tile_first;   // [n_tiles+1]
    double* v_out;                // [N_c]
    TileSide* side;               // [n_tiles]
    double* hist_H;               // global histogram (when not in LDS)
    uint32_t* hist_C;
    double* hist_Cw;              // paths with weighted histograms: FP64 count weights
    const void* grid;             // the map in global memory (null: read the LDS copy)
};

// LDS views of the fill (see lds_plan).
template <typename R>
struct FillLds {
    R* gl;
    R* auxl;
    double* hl;
    uint32_t* cl;
    uint16_t* st;
    WaveRec* wrec;
    WaveRec* cin;
    Partial* tside;
    uint32_t* tflags;
    double* red;

    __device__ __forceinline__ FillLds(unsigned char* smem, const LdsPlan& lp)
    {
        gl = reinterpret_cast<R*>(smem + lp.grid_off);
        auxl = reinterpret_cast<R*>(smem + lp.aux_off);
        hl = reinterpret_cast<double*>(smem + lp.h_off);
        cl = reinterpret_cast<uint32_t*>(smem + lp.c_off);
        st = reinterpret_cast<uint16_t*>(smem + lp.st_off);
        wrec = reinterpret_cast<WaveRec*>(smem + lp.wave_off);
        cin = reinterpret_cast<WaveRec*>(smem + lp.cin_off);
        tside = reinterpret_cast<Partial*>(smem + lp.side_off);
        tflags = reinterpret_cast<uint32_t*>(smem + lp.side_off + 2 * sizeof(Partial));
        red = reinterpret_cast<double*>(smem + lp.red_off);
    }
};

// One tile of `io.tile` consecutive samples: every lane walks its
// `per_lane` samples (Alg. 2), cubes finished inside a lane are finalised
// there, runs crossing lanes merge by the wavefront scan, and the tile's
// boundary runs go to its side record.  Called by all lanes of the
// workgroup; ends with a barrier.
// Path: the per-sample path (SamplePath, or the warped path of the learned
// warp), with digits / next_digits / eval and the problem constants sc.
// The map a tile reads: GMAP reads it from global memory through the vector
// cache (typed as a global pointer, so its loads are waited on by the vector
// counter alone and never by the LDS atomics in flight); otherwise the copy
// in LDS.
template <bool GMAP, typename R>
__device__ __forceinline__ auto tile_map(const TileIO& io, const R* gl)
{
    typedef const __attribute__((address_space(1))) R GlobalR;
    if constexpr (GMAP) return (GlobalR*)(io.grid);
    else return gl;
}

template <typename R, int MAXD, bool KAHAN, bool GMAP, typename Path>
__device__ __forceinline__ void fill_tile(int tile, const TileIO& io, const FillLds<R>& L, Path& sp,
                                          LaneTotal<KAHAN>& totI, LaneTotal<KAHAN>& totV, double& vmax,
                                          unsigned long long& bad)
{
    const SampleConst& sc = sp.sc;
    const int D = sc.D;
    const uint32_t ng = sc.ng;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int S = io.per_lane;
    R* gl = L.gl;
    const auto gmap = tile_map<GMAP>(io, gl);
    double* hl = L.hl;
    uint32_t* cl = L.cl;
    uint16_t* st = L.st;
    WaveRec* wrec = L.wrec;
    WaveRec* cin = L.cin;
    Partial* tside = L.tside;
    uint32_t* tflags = L.tflags;
        const uint32_t t0 = (uint32_t)tile * (uint32_t)io.tile;
        const uint32_t t1 = min(t0 + (uint32_t)io.tile, sc.n_eval);
        const uint32_t h_lo = io.tile_first[tile];
        const uint32_t h_nx = io.tile_first[tile + 1];
        const uint32_t h_top = min(h_nx, sc.n_cubes - 1u);
        const int nst_load = (int)(h_top - h_lo) + 2;   // starts of h_lo .. h_top+1
        // the starts relative to the tile, plus one, clamped to [0, tile + 2]:
        // 16 bits hold them (tile <= kMaxTile), and every comparison below
        // with a sample of the tile keeps its outcome
        for (int i = tid; i < nst_load; i += kFillThreads) {
            const int64_t r = (int64_t)io.start[h_lo + i] - (int64_t)t0 + 1;
            st[i] = (uint16_t)(r < 0 ? 0 : (r > io.tile + 2 ? io.tile + 2 : r));
        }
        if (tid == 0) *tflags = 0u;
        __syncthreads();

        const uint32_t k0 = t0 + (uint32_t)(tid * S);
        const uint32_t k1 = min(k0 + (uint32_t)S, t1);
        const uint32_t kr = k0 - t0 + 1u;           // k0 in the frame of st
        const int n_active = (int)((t1 - t0 + (uint32_t)S - 1u) / (uint32_t)S);
        // per lane: the run of its first cube when that cube began earlier
        // (head), and the run of its last cube when it continues (tail)
        bool has_head = false, has_tail = false, span = false;
        Run hrun = run_empty(), trun = run_empty();
        uint32_t h_first = 0, h_last = 0;
        if (k0 < k1) {
            int lo = 0, hi = nst_load - 1;          // largest idx with start <= k0
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (st[mid] <= kr) lo = mid; else hi = mid;
            }
            int idx = lo;
            uint32_t h = h_lo + (uint32_t)idx;
            h_first = h;
            uint32_t nxt = t0 - 1u + st[idx + 1];
            bool head = st[idx] < kr;
            uint32_t s[MAXD];
            sp.digits(h, s);
            uint32_t n = 0;
            CubeSums<KAHAN> cs;
            cs.reset();

            for (int j = 0; j < S; ++j) {
                const uint32_t k = k0 + (uint32_t)j;
                if (k >= k1) break;
                if (k == nxt) {
                    // the current cube ends: shifted sums -> (mean, m2)
                    const Run r = cs.run(n);
                    if (head) {
                        hrun = r;
                        has_head = true;
                    } else {
                        double v, vn;
                        run_finish(r, v, vn);
                        io.v_out[h] = v;
                        totI.add(r.mean);
                        totV.add(vn);
                        vmax = v > vmax ? v : vmax;
                    }
                    ++h;
                    // from global memory: an LDS read here would be waited
                    // on behind this lane's histogram atomics
                    nxt = io.start[h + 1];
                    head = false;
                    n = 0;
                    cs.reset();
                    sp.next_digits(s);
                }
                uint32_t bins[MAXD];
                R J, f;
                R w = sp.template eval<false>(k, io.t, s, gmap, bins, nullptr, nullptr, J, f);
                if (!__builtin_isfinite(w)) {
                    w = (R)0;
                    ++bad;
                }
                const double wd = (double)w;
                const double w2 = wd * wd;
                if constexpr (Path::kWeightedHist) {
                    // the warped path's samples have density q = 1/J_F in w:
                    // the map's bin averages of w^2 over uniform points are
                    // sum (w^2 / J_F) / sum J_F (global memory); none while
                    // the map is held (null hist_Cw)
                    const double jf = sp.last_jf();
                    if (io.hist_Cw && jf > 0.0 && __builtin_isfinite(jf)) {
                        const double h = w2 / jf;
#pragma unroll
                        for (int d = 0; d < MAXD; ++d) {
                            const uint32_t bi = (uint32_t)d * ng + bins[d];
                            unsafeAtomicAdd(io.hist_H + bi, h);
                            unsafeAtomicAdd(io.hist_Cw + bi, jf);
                        }
                    }
                } else if (io.lds_hist) {
#pragma unroll
                    for (int d = 0; d < MAXD; ++d) {
                        if (Path::kExact || d < D) {
                            const uint32_t bi = (uint32_t)d * ng + bins[d];
                            atomicAdd(hl + bi, w2);
                            atomicAdd(cl + bi, 1u);
                        }
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < MAXD; ++d) {
                        if (Path::kExact || d < D) {
                            const uint32_t bi = (uint32_t)d * ng + bins[d];
                            unsafeAtomicAdd(io.hist_H + bi, w2);
                            atomicAdd(io.hist_C + bi, 1u);
                        }
                    }
                }
                cs.add(w, n == 0);
                ++n;
            }
            h_last = h;
            const Run r = cs.run(n);
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
                io.v_out[h] = v;
                totI.add(r.mean);
                totV.add(vn);
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
                io.v_out[h_first] = v;
                totI.add(fin.mean);
                totV.add(vn);
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
            TileSide* ts = io.side + tile;
            ts->flags = fl;
            ts->head = tside[0];
            ts->tail = (fl & kSpan) ? tside[0] : tside[1];
        }
        __syncthreads();
}


// Fixed-order workgroup reduction of the lane totals: sum of cube means and
// of v/n over the lanes (wave shuffles, then waves in order), max of v.
// Results are valid in thread 0.  Uses red[3 * kWaves]; ends with a barrier.
__device__ __forceinline__ void wg_reduce_totals(double accI, double accV, double vmax, double* red, double& sI,
                                                 double& sV, double& mx)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
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
    sI = 0.0;
    sV = 0.0;
    mx = 0.0;
    if (tid == 0) {
        for (int w = 0; w < kWaves; ++w) {
            sI += red[3 * w];
            sV += red[3 * w + 1];
            mx = red[3 * w + 2] > mx ? red[3 * w + 2] : mx;
        }
    }
    __syncthreads();
}

// A cube whose runs cross tiles, owned by the tile where it starts (tile j
// has a tail that does not span the whole tile): merge the heads of the
// following tiles in tile order until the cube ends.  Writes v of the cube
// and returns (mean, v/n) in out[0..1]; zeros for tiles that own none.
constexpr int kFixAhead = 8;            // side records in flight in the fix-up

// iteration estimate: fixed-order sum of the workgroup and fix-up partials
// (per thread strided, then a tree over the 1024 threads); rI, rV hold 1024
// doubles each; called by 1024 threads
__device__ __forceinline__ void final_reduce(const FinalArgs& a, double* rI, double* rV)
{
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

// Tile j's tail run merged with the heads of the tiles it reaches into; the
// finished cube's variance goes to v_out and its partials to out[0..1].
// Returns the variance's bit pattern for the maximum (0 when tile j
// finishes no cube).
__device__ __forceinline__ unsigned long long fixup_chain_v(const TileSide* side, int n_tiles, int j, double* v_out,
                                                            double* out)
{
    double mI = 0.0, mV = 0.0;
    unsigned long long vb = 0ull;
    const uint32_t f = side[j].flags;
    if ((f & kHasTail) && !(f & kSpan)) {
        Partial cur = side[j].tail;
        // the heads of the following tiles, merged in tile order up to the
        // first tile the cube does not span; their loads go out kFixAhead at
        // a time, since a cube can span many tiles
        int m = j + 1;
        bool open = true;
        while (open && m < n_tiles) {
            Partial hd[kFixAhead];
            uint32_t fl[kFixAhead];
#pragma unroll
            for (int q = 0; q < kFixAhead; ++q) {
                if (m + q < n_tiles) {
                    hd[q] = side[m + q].head;
                    fl[q] = side[m + q].flags;
                }
            }
#pragma unroll
            for (int q = 0; q < kFixAhead; ++q) {
                if (open && m + q < n_tiles) {
                    cur = merge(cur, hd[q]);
                    if (!(fl[q] & kSpan)) open = false;
                }
            }
            m += kFixAhead;
        }
        const double v = unbiased_var(cur);
        v_out[cur.h] = v;
        mI = cur.mean;
        mV = v / (double)cur.n;
        vb = (unsigned long long)__double_as_longlong(v);
    }
    out[0] = mI;
    out[1] = mV;
    return vb;
}

__device__ __forceinline__ void fixup_chain(const TileSide* side, int n_tiles, int j, double* v_out,
                                            unsigned long long* vmax, double* out)
{
    const unsigned long long vb = fixup_chain_v(side, n_tiles, j, v_out, out);
    if (vb) atomicMax(vmax, vb);
}

// the largest of the wavefront's bit patterns into *p with one atomic (the
// same maximum as one atomicMax per lane); all 64 lanes call it
__device__ __forceinline__ void wave_atomic_max(unsigned long long b, unsigned long long* p)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(b, o, 64);
        b = y > b ? y : b;
    }
    if ((threadIdx.x & 63) == 0 && b) atomicMax(p, b);
}

// The whole fill of one workgroup (Alg. 2): the integrand's table and the
// histograms into LDS, the workgroup's tiles (static round-robin), its
// histogram slot and its fixed-order partial sums.  The body of the built-in
// fill kernels and of a runtime-compiled integrand's fill kernel; smem is
// the kernel's dynamic LDS.
template <typename R, int FAM, int MAXD, bool KAHAN, bool EXACT>
__device__ __forceinline__ void fill_body(const FillArgs& a, unsigned char* smem)
{
    const SampleConst& sc = a.sc;
    const int D = sc.D;
    const uint32_t ng = sc.ng;
    const int tid = threadIdx.x;
    const LdsPlan lp = lds_plan(D, (int)ng, (int)sizeof(R), a.lds_hist, a.tile, sc.n_aux, 0);
    const FillLds<R> L(smem, lp);

    const int nbins = D * (int)ng;
    {
        const R* asrc = std::is_same<R, double>::value ? reinterpret_cast<const R*>(sc.aux_d)
                                                       : reinterpret_cast<const R*>(sc.aux_f);
        for (int i = tid; i < sc.n_aux; i += kFillThreads) L.auxl[i] = asrc[i];
    }
    if (a.lds_hist) {
        for (int i = tid; i < nbins; i += kFillThreads) {
            L.hl[i] = 0.0;
            L.cl[i] = 0u;
        }
    }

    SamplePath<R, FAM, MAXD, EXACT> sp(sc, L.auxl);
    LaneTotal<KAHAN> totI, totV;
    double vmax = 0.0;
    unsigned long long bad = 0;
    TileIO io;
    io.t = a.t;
    io.tile = a.tile;
    io.per_lane = a.per_lane;
    io.lds_hist = a.lds_hist;
    io.start = a.start;
    io.tile_first = a.tile_first;
    io.v_out = a.v_out;
    io.side = a.side;
    // global mode: with hist_slots each workgroup adds into a slot of its
    // own, so a histogram line stays in one XCD's L2 instead of moving
    // between the XCDs that add to it (the map kernel adds the slots in
    // order)
    const size_t slot = !a.lds_hist && a.hist_slots ? (size_t)blockIdx.x * nbins : 0;
    io.hist_H = a.hist_H + slot;
    io.hist_C = a.hist_C + slot;
    io.hist_Cw = nullptr;
    io.grid = a.grid;

    __syncthreads();

    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x)
        fill_tile<R, MAXD, KAHAN, true>(tile, io, L, sp, totI, totV, vmax, bad);

    if (a.lds_hist) {
        // this workgroup's histograms into its slot (reduced in slot order by
        // the map kernel)
        double* slotH = a.hist_H + (size_t)blockIdx.x * nbins;
        uint32_t* slotC = a.hist_C + (size_t)blockIdx.x * nbins;
        for (int i = tid; i < nbins; i += kFillThreads) {
            slotH[i] = L.hl[i];
            slotC[i] = L.cl[i];
        }
    }

    // ---- fixed-order workgroup reduction of the lane partials -------------
    double sI, sV, mx;
    wg_reduce_totals(totI.value(), totV.value(), vmax, L.red, sI, sV, mx);
    if (tid == 0) {
        a.wg_part[2 * blockIdx.x] = sI;
        a.wg_part[2 * blockIdx.x + 1] = sV;
        atomicMax(a.vmax, (unsigned long long)__double_as_longlong(mx));
    }
    if (bad) atomicAdd(a.nonfinite, bad);
}

}  // namespace vg
