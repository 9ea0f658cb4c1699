"""Auxiliary paths of the C ABI on the GPU against the oracle:

* checkpoint: 5 iterations + vegas_get_state / vegas_set_state into a new
  context + 5 iterations equal 10 iterations in one context, bit for bit
  (ORDERED accumulation), and both equal the oracle's run
* an integrand that overflows on part of the domain: the count of
  non-finite weights equals the oracle's, those weights count as 0, and
  vegas_result reports VEGAS_ENONFINITE
* Kahan accumulation (FP32 sample path) against the FP64 oracle, with its
  error stated
* the d=16, 1024-interval global-histogram path is in test_gpu_parity's
  iteration cases
"""
import math
import sys

import numpy as np
import pytest

import vegas_inputs as vi

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make(w, precision="f64", accum="fp64", max_iter=0):
    from paper_2408_09229_amd import Vegas, make_config
    cfg = make_config(w.dim, w.n_g, w.n_eval, n_strat=w.n_strat, n_min=w.n_min, alpha=w.alpha, beta=w.beta,
                      seed=w.seed, precision=precision, accum=accum, max_iter=max_iter)
    return Vegas(cfg, w.family, w.params, w.lo, w.hi)


PPEAK = vi.Workload("ppeak3_ckpt", 3, vi.GENZ_PPEAK, np.array([1.0, 6.0, 9.0, 12.0, 0.3, 0.6, 0.45]), n_g=32,
                    n_eval=50_003, n_iter=10)


def test_checkpoint_resume_bit_exact(orc):
    w = PPEAK
    say("[checkpoint]")
    a = make(w, accum="ordered", max_iter=16)
    a.adapt(2)
    a.integrate(8)
    Ia, sa = a.get_iterations()
    ra = a.result()
    b = make(w, accum="ordered", max_iter=16)
    b.adapt(2)
    b.integrate(3)
    state = b.get_state()
    b.close()
    c = make(w, accum="ordered", max_iter=16)
    c.set_state(state)
    c.integrate(5)
    Ic, sc = c.get_iterations()
    rc = c.result()
    assert np.array_equal(Ia, Ic) and np.array_equal(sa, sc)
    assert np.array_equal(a.get_map(), c.get_map()) and np.array_equal(a.get_nh(), c.get_nh())
    assert (ra.integral, ra.sigma2, ra.chi2_dof, ra.n_iter_combined) == \
        (rc.integral, rc.sigma2, rc.chi2_dof, rc.n_iter_combined)
    # the oracle's own run of 2 + 8 iterations
    o = orc.run(w.dim, w.n_g, w.n_eval, w.family, w.params, n_adapt=2, n_iter=8, seed=w.seed)
    assert np.array_equal(Ia, o.I_t) and np.array_equal(sa, o.s2_t)
    assert ra.integral == o.integral and ra.sigma2 == o.sigma2
    # a state image of another problem is refused
    d = make(w.with_(n_g=16), accum="ordered", max_iter=16)
    from paper_2408_09229_amd._binding import VegasError
    with pytest.raises(VegasError):
        d.set_state(state)
    for x in (a, c, d):
        x.close()


def test_nonfinite_weights_counted(orc):
    """A * (x_0 + x_1) with A = 1e308 overflows to +inf wherever
    x_0 + x_1 exceeds about 1.797: the GPU's count of such weights equals the
    oracle's exactly (the FP64 points are bit-exact), and vegas_result
    reports VEGAS_ENONFINITE with that count.  (The finite weights near
    1e308 overflow the sums too, on both sides alike.)"""
    from paper_2408_09229_amd._binding import VEGAS_ENONFINITE, VegasError
    w = vi.Workload("linear_overflow", 2, vi.LINEAR, np.array([1e308]), n_g=16, n_eval=40_001, n_iter=1)
    say("[nonfinite]")
    v = make(w, max_iter=4)
    v.integrate(1)
    I, s2 = v.get_iterations()
    ns, nc, _ = orc.strata(w.n_eval, w.dim, w.n_min, w.n_strat)
    nh = orc.alloc(np.zeros(nc), w.n_min, w.n_eval, w.beta, adapt=False)
    o = orc.iterate(w.dim, w.n_g, w.n_eval, ns, nc, w.seed, 0, 0, w.family, w.params,
                    orc.init_grid(w.dim, w.n_g), nh)
    say(f"  oracle non-finite weights {o.n_nonfinite}")
    assert o.n_nonfinite > 100
    with pytest.raises(VegasError) as e:
        v.result()
    assert e.value.status == VEGAS_ENONFINITE
    r = v.result(allow_nonfinite=True)
    assert r.n_nonfinite == o.n_nonfinite
    assert np.isfinite(I[0]) == np.isfinite(o.I) and np.isfinite(s2[0]) == np.isfinite(o.s2)
    if np.isfinite(o.I):
        assert abs(I[0] - o.I) <= 1e-12 * abs(o.I)
    v.close()


@pytest.mark.parametrize("accum", ["kahan", "fp64"])
def test_fp32_accumulation_against_oracle(orc, accum):
    """The FP32 sample path with Kahan (or FP64) accumulation, first iteration
    against the FP64 oracle on the same samples.  Roos-Arnold in d=5 is a
    product of |4x - 2| factors: the FP32 path rounds the offset, the map
    fma, each factor and product (about 3 roundings per axis plus the
    weight), so a weight is within (3D + 2) 2^-24 relative of the FP64 one;
    the estimate, a mean of such weights, within the same bound.  The cube
    variances are differences of close weights and are held to 1e-4."""
    w = vi.Workload("roos5_f32", 5, vi.ROOS, np.array([1.0]), n_g=8, n_eval=30_001, n_iter=1)
    say(f"[fp32 accumulation] {accum}")
    v = make(w, precision="f32", accum=accum, max_iter=4)
    v.integrate(1)
    I, s2 = v.get_iterations()
    ns, nc, _ = orc.strata(w.n_eval, w.dim, w.n_min, w.n_strat)
    nh = orc.alloc(np.zeros(nc), w.n_min, w.n_eval, w.beta, adapt=False)
    o = orc.iterate(w.dim, w.n_g, w.n_eval, ns, nc, w.seed, 0, 0, w.family, w.params,
                    orc.init_grid(w.dim, w.n_g), nh)
    eI = abs(I[0] - o.I) / abs(o.I)
    es = abs(s2[0] - o.s2) / o.s2
    say(f"  {accum}: I {I[0]:.10e} oracle {o.I:.10e}: relative error {eI:.2e}; sigma^2 relative error {es:.2e}")
    assert eI <= (3 * w.dim + 2) * 2.0 ** -24
    assert es <= 1e-4
    v.close()
