// The per-sample path of Alg. 2 shared by the fill, the ordered mode and
// the probe: stratum digits of a cube, Philox words, fixed-point point and
// bin, map and Jacobian, integrand.
#pragma once
#ifndef __HIPCC_RTC__   // hipRTC provides the HIP device runtime itself
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>
#include <type_traits>

#include "common.hpp"
#include "families.hpp"
#include "layout.hpp"

namespace vg {

// ---------------------------------------------------------------------------
// the per-sample path shared by the fill and the probe
// ---------------------------------------------------------------------------
// MAXD bounds the dimension; EXACT says D == MAXD, which drops the per-axis
// guards (and the register moves and lane-mask copies they cost).
template <typename R, int FAM, int MAXD, bool EXACT = false>
struct SamplePath {
    static constexpr bool kExact = EXACT;
    static constexpr bool kWeightedHist = false;
    const SampleConst& sc;
    Fn<R, FAM> fn;
    PhiloxKeys keys;
    R ngR;
    double nst2_d;        // 2 N_st
    float half_inv_nst_f; // (1 / N_st) / 2

    // aux: the family's derived table in the path's precision (LDS in the
    // fill, global memory in the probe)
    __device__ __forceinline__ SamplePath(const SampleConst& c, const R* aux) : sc(c)
    {
        fn.setup(c, aux);
        keys = philox_keys<std::is_same<R, float>::value && MAXD <= 8>(c.key0, c.key1);
        ngR = (R)c.ng;
        nst2_d = 2.0 * (double)c.nst;
        half_inv_nst_f = 0.5f * (float)(1.0 / (double)c.nst);
    }

    __device__ __forceinline__ bool has(int d) const { return EXACT || d < sc.D; }

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

    // digits of h+1 from those of h; the carry reaches axis d once every
    // N_st^d cubes, so the nested branches are rarely taken past axis 0
    __device__ __forceinline__ void next_digits(uint32_t (&s)[MAXD]) const
    {
        next_digit_from<0>(s);
    }
    template <int d>
    __device__ __forceinline__ void next_digit_from(uint32_t (&s)[MAXD]) const
    {
        if constexpr (d < MAXD) {
            const uint32_t v = s[d] + 1u;
            if (v == sc.nst) {
                s[d] = 0u;
                next_digit_from<d + 1>(s);
            } else {
                s[d] = v;
            }
        }
    }

    // Evaluate sample k (iteration t) of the cube with digits s against the
    // grid g (row stride N_g+1).  Returns w = J f; bins and (optionally)
    // delta / x / J / f are reported through the out-parameters.
    template <bool PROBE, typename GP>
    __device__ __forceinline__ R eval(uint32_t k, uint32_t t, const uint32_t (&s)[MAXD],
                                      GP __restrict__ g, uint32_t (&bins)[MAXD],
                                      R* delta_out, R* x_out, R& J, R& f)
    {
        uint32_t wd[MAXD];
#pragma unroll
        for (int b = 0; b < (MAXD + 3) / 4; ++b) {
            if (has(4 * b)) {
                const W4 o = philox10(k, 0u, t, sc.ctr3 | (uint32_t)b, keys);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * b + q < MAXD) wd[4 * b + q] = o.v[q];
            }
        }
        // every axis's bin and map interval first, so that the map loads are
        // all in flight before the first of them is used
        const uint32_t row = sc.ng + 1u;
        R lo[MAXD], hi[MAXD], dl[MAXD];
#pragma unroll
        for (int d = 0; d < MAXD; ++d) {
            if (has(d)) {
                const BinSplit p = bin_split(s[d], wd[d], sc.ng, sc.nst, sc.nst_magic, sc.nst_shift);
                bins[d] = p.bin;
                if constexpr (std::is_same<R, double>::value) dl[d] = delta_f64(p, nst2_d);
                else dl[d] = delta_f32(p, half_inv_nst_f);
                const auto gd = g + d * row;
                lo[d] = gd[p.bin];
                hi[d] = gd[p.bin + 1];
            }
        }
        J = (R)1;
        fn.begin();
#pragma unroll
        for (int d = 0; d < MAXD; ++d) {
            if (has(d)) {
                const R dx = hi[d] - lo[d];
                const R x = fma(dx, dl[d], lo[d]);
                J = J * (ngR * dx);
                fn.axis(d, x);
                if constexpr (PROBE) {
                    delta_out[d] = dl[d];
                    x_out[d] = x;
                }
            }
        }
        f = fn.finish();
        return J * f;
    }
};

}  // namespace vg
