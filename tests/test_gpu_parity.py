"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

* per-sample path (cube, bins exact; delta, x, J exact in FP64; f to 1e-14)
* one iteration from the same map and allocation: I_t and sigma_t^2 within
  1e-12 relative (FP64), per-cube variance and histograms
* allocation and map refinement on injected accumulators: bit-exact
* whole runs: closed form within 3 sigma
All inputs come from vegas_inputs; every expected value from oracle/.
"""
import math
import sys

import numpy as np
import pytest

import vegas_inputs as vi
from tests import closed_forms as cf

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available()
    from paper_2408_09229_amd import Vegas, make_config

    def make(w: vi.Workload, **kw):
        cfg = make_config(w.dim, w.n_g, w.n_eval, n_strat=w.n_strat, n_min=w.n_min, alpha=w.alpha,
                          beta=w.beta, seed=w.seed, precision=kw.pop("precision", w.precision), **kw)
        return Vegas(cfg, w.family, w.params, w.lo, w.hi)
    return make


def _state(orc, w):
    ns, nc, _ = orc.strata(w.n_eval, w.dim, w.n_min, w.n_strat)
    return ns, nc


def _random_state(orc, w, seed):
    ns, nc = _state(orc, w)
    rng = np.random.default_rng(seed)
    grid = np.stack([np.sort(np.concatenate([[w.lo[d], w.hi[d]],
                                             w.lo[d] + (w.hi[d] - w.lo[d]) * rng.random(w.n_g - 1) ** 2]))
                     for d in range(w.dim)])
    nh = orc.alloc(rng.lognormal(0, 1.5, nc), w.n_min, w.n_eval, 0.75)
    return grid, nh


PROBE_CASES = [
    vi.Workload("tiny_3x8x2", 2, vi.GENZ_PPEAK, np.array([1.0, 6.0, 9.0, 0.3, 0.6]), n_g=8, n_eval=40,
                n_iter=1, n_strat=3),
    vi.Workload("probe_12x128x4", 4, vi.GAUSS_DIAG, vi.gauss_diag_params(1.0, 0.1, [0.5]), n_g=128,
                n_eval=12 ** 4 * 3, n_iter=1, n_strat=12),
    vi.gauss3_8d().with_(name="gauss3_8d_f64", n_eval=50_000, n_g=64, precision="f64"),
    vi.Workload("corr16", 16, vi.GAUSS_CORR, np.array([0.5, 0.03, 0.9]), n_g=32, n_eval=300_000, n_iter=1),
] + [w.with_(n_eval=min(w.n_eval, 60_000)) for w in vi.tab3_cases()]


@pytest.mark.parametrize("w", PROBE_CASES, ids=lambda w: w.name)
@pytest.mark.parametrize("t", [0, 5])
def test_probe_bitexact(orc, V, w, t):
    say(f"[probe] {w.name} t={t}")
    v = V(w)
    ns, nc = _state(orc, w)
    grid, nh = _random_state(orc, w, 7 + t)
    v.set_map(grid)
    v.set_nh(nh)
    n = min(w.n_eval, 4000)
    rng = np.random.default_rng(1)
    k0 = int(rng.integers(0, w.n_eval - n + 1))
    r = v.probe(t, k0, n)
    start = np.concatenate([[0], np.cumsum(nh.astype(np.int64))])
    for i in range(0, n, max(1, n // 400)):
        k = k0 + i
        h = int(np.searchsorted(start, k, side="right") - 1)
        bins, delta, x, J, f = orc.sample(w.dim, w.n_g, ns, w.seed, 0, t, k, h, grid, w.family, w.params)
        assert r["cube"][i] == h
        assert np.array_equal(r["bins"][i], bins)
        assert np.array_equal(r["delta"][i], delta)
        assert np.array_equal(r["x"][i], x)
        assert r["jac"][i] == J
        # the GPU evaluates the Gaussian exponent in an algebraically equal
        # form (mean and spread over the D axes); its rounding grows with D
        # and with the exponent, i.e. with |ln f|
        tol = 2e-15 * (w.dim + 1) * (5.0 + abs(math.log(abs(f)))) if f != 0 else 0.0
        assert abs(r["f"][i] - f) <= tol * abs(f) + 1e-300, (r["f"][i], f)
    v.close()


ITER_CASES = vi.small_cases() + [
    vi.Workload("ragged_one_tile", 3, vi.GENZ_GAUSS, np.array([1.0, 5.0, 7.0, 9.0, 0.2, 0.5, 0.8]),
                n_g=16, n_eval=1_537, n_iter=1),
    vi.Workload("corr16_small", 16, vi.GAUSS_CORR, np.array([0.5, 0.03, 0.9]), n_g=64, n_eval=200_003,
                n_iter=1),
    vi.Workload("cosine_big_cubes", 2, vi.COSINE, np.array([1.0]), n_g=32, n_eval=400_000, n_iter=1,
                n_strat=3),
    # 16 x 1024 intervals: the histograms do not fit in LDS beside the fill's
    # other tables, so they are global FP64 / u32 atomics (the path of the
    # d=16 benchmark workload)
    vi.Workload("corr16_ng1024", 16, vi.GAUSS_CORR, np.array([0.5, 0.2, 0.3]), n_g=1024, n_eval=200_003,
                n_iter=1),
] + vi.tab3_cases()


@pytest.mark.parametrize("w", ITER_CASES, ids=lambda w: w.name)
def test_iteration_fp64_parity(orc, V, w):
    """Iteration t of the GPU from the oracle's own state after t iterations
    (uniform start, then the adapted map and allocation of the oracle's
    trajectory): I_t and sigma_t^2 within 1e-12, counts exact."""
    say(f"[iteration] {w.name}")
    v = V(w, precision="f64")
    ns, nc = _state(orc, w)
    grid = orc.init_grid(w.dim, w.n_g, w.lo, w.hi)
    nh = orc.alloc(np.zeros(nc), w.n_min, w.n_eval, w.beta, adapt=False)
    for step in range(3):
        if step > 0:
            v.set_map(grid)
            v.set_nh(nh)
        v.integrate(1)
        I, s2 = v.get_iterations()
        H, Cn, vv = v.get_accumulators()
        o = orc.iterate(w.dim, w.n_g, w.n_eval, ns, nc, w.seed, 0, step, w.family, w.params, grid, nh)
        assert abs(I[step] - o.I) <= 1e-12 * abs(o.I), (step, I[step], o.I)
        assert abs(s2[step] - o.s2) <= 1e-12 * o.s2 + 1e-300, (step, s2[step], o.s2)
        assert np.array_equal(Cn, o.C)
        assert np.allclose(H, o.H, rtol=1e-12, atol=1e-300)
        scale = max(o.v.max(), 1e-300)
        assert np.allclose(vv, o.v, rtol=1e-10, atol=1e-12 * scale)
        # the GPU's own update of this iteration (for these sizes the fix-up,
        # estimate and map run in one launch), bit-exact against the oracle
        # applied to the GPU's accumulators
        assert np.array_equal(v.get_map(), orc.map_update(grid, H, Cn, w.alpha))
        assert np.array_equal(v.get_nh(), orc.alloc(vv, w.n_min, w.n_eval, w.beta))
        # the oracle's own next state
        nh = orc.alloc(o.v, w.n_min, w.n_eval, w.beta)
        grid = orc.map_update(grid, o.H, o.C, w.alpha)
    v.close()


@pytest.mark.parametrize("beta", [0.75, 1.0, 0.5, 0.3])
def test_alloc_bitexact(orc, V, beta):
    w = vi.Workload("alloc", 3, vi.CONST, np.array([1.0]), n_g=8, n_eval=2_000_003, n_iter=1, beta=beta)
    say(f"[alloc] beta={beta}")
    v = V(w)
    ns, nc = _state(orc, w)
    rng = np.random.default_rng(int(beta * 100))
    vh = rng.lognormal(0, 3, nc)
    vh[rng.random(nc) < 0.05] = 0.0
    H = rng.random((w.dim, w.n_g))
    Cn = np.ones((w.dim, w.n_g))
    v.set_accumulators(H, Cn, vh)
    v.update()
    got = v.get_nh()
    want = orc.alloc(vh, w.n_min, w.n_eval, beta)
    assert np.array_equal(got, want)
    assert int(got.sum()) == w.n_eval
    v.close()


@pytest.mark.parametrize("alpha", [0.5, 1.0, 1.5, 0.7])
@pytest.mark.parametrize("n_g", [1, 2, 7, 1024])
def test_map_update_bitexact(orc, V, alpha, n_g):
    w = vi.Workload("map", 3, vi.CONST, np.array([1.0]), n_g=n_g, n_eval=10_000, n_iter=1, alpha=alpha)
    say(f"[map] alpha={alpha} n_g={n_g}")
    v = V(w)
    ns, nc = _state(orc, w)
    rng = np.random.default_rng(n_g)
    grid, _ = _random_state(orc, w, 3)
    v.set_map(grid)
    Cn = rng.integers(0, 50, (w.dim, n_g)).astype(float)
    H = np.where(Cn > 0, rng.lognormal(0, 2, (w.dim, n_g)) * Cn, 0.0)
    H[:, 0] += 1.0
    Cn[:, 0] += 1.0
    v.set_accumulators(H, Cn, np.ones(nc))
    v.update()
    got = v.get_map()
    want = orc.map_update(grid, H, Cn, alpha)
    assert np.array_equal(got, want), np.max(np.abs(got - want))
    v.close()


@pytest.mark.parametrize("w", vi.closed_form_cases(), ids=lambda w: w.name)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_run_closed_form(V, w, prec):
    say(f"[run] {w.name} {prec}")
    v = V(w, precision=prec)
    v.integrate(w.n_iter)
    r = v.result()
    exact = cf.exact(w)
    assert abs(r.integral - exact) < 3.0 * math.sqrt(r.sigma2), (r.integral, exact, math.sqrt(r.sigma2))
    assert r.n_iter_combined == w.n_iter
    v.close()


def test_gauss_prod_4d_config(orc, V):
    w = vi.gauss_prod_4d()
    say(f"[cfg] {w.name}")
    v = V(w)
    v.integrate(w.n_iter)
    r = v.result()
    exact = cf.exact(w)
    assert abs(r.integral - exact) < 3.0 * math.sqrt(r.sigma2)
    # the first iteration starts from the same state as the oracle's run
    I, s2 = v.get_iterations()
    o = orc.run(w.dim, w.n_g, w.n_eval, w.family, w.params, n_iter=1, seed=w.seed)
    assert abs(I[0] - o.I_t[0]) <= 1e-12 * abs(o.I_t[0])
    v.close()


ORDERED_CASES = [
    vi.Workload("ppeak3_ord", 3, vi.GENZ_PPEAK, np.array([1.0, 6.0, 9.0, 12.0, 0.3, 0.6, 0.45]), n_g=16,
                n_eval=6_007, n_iter=5),
    vi.Workload("roos2_ord", 2, vi.ROOS, np.array([1.0]), n_g=8, n_eval=2_003, n_iter=5, alpha=0.7, beta=0.3),
    vi.Workload("linear4_ord", 4, vi.LINEAR, np.array([2.0]), n_g=32, n_eval=10_000, n_iter=5, alpha=1.5),
]


@pytest.mark.parametrize("w", ORDERED_CASES, ids=lambda w: w.name)
def test_ordered_trajectory_bitexact(orc, V, w):
    """ORDERED accumulation: a whole trajectory (estimates, map, allocation)
    equals the oracle's bit for bit, for integrands built from correctly
    rounded operations."""
    say(f"[ordered] {w.name}")
    v = V(w, accum="ordered")
    v.integrate(w.n_iter)
    I, s2 = v.get_iterations()
    g = v.get_map()
    nh = v.get_nh()
    o = orc.run(w.dim, w.n_g, w.n_eval, w.family, w.params, n_iter=w.n_iter, seed=w.seed, alpha=w.alpha,
                beta=w.beta)
    assert np.array_equal(I, o.I_t), (I - o.I_t)
    assert np.array_equal(s2, o.s2_t)
    assert np.array_equal(g, o.grid)
    assert np.array_equal(nh, o.nh)
    r = v.result()
    assert r.integral == o.integral and r.sigma2 == o.sigma2
    v.close()


def test_ordered_reproducible(V):
    w = vi.gauss_prod_4d().with_(n_eval=8_000, n_g=16)
    say("[ordered] reproducible")
    runs = []
    for _ in range(2):
        v = V(w, accum="ordered")
        v.integrate(4)
        runs.append((v.get_iterations(), v.get_map(), v.get_nh()))
        v.close()
    (Ia, sa), ga, na = runs[0]
    (Ib, sb), gb, nb = runs[1]
    assert np.array_equal(Ia, Ib) and np.array_equal(sa, sb)
    assert np.array_equal(ga, gb) and np.array_equal(na, nb)


@pytest.mark.parametrize("w", [vi.gauss3_8d().with_(name="gauss3_8d_kahan", n_eval=3_000_007, n_g=256, n_iter=5),
                               vi.closed_form_cases()[1]], ids=lambda w: w.name)
def test_kahan_accumulation(V, w):
    """Compensated FP32 accumulators: on the same samples the first
    iteration's estimate agrees with FP64 accumulation to FP32 resolution,
    and the run lands within 3 sigma of the closed form."""
    say(f"[kahan] {w.name}")
    a = V(w, precision="f32", accum="kahan")
    b = V(w, precision="f32")
    a.adapt(1)
    b.adapt(1)
    Ia, sa = a.get_iterations()
    Ib, sb = b.get_iterations()
    assert abs(Ia[0] - Ib[0]) <= 1e-6 * abs(Ib[0]), (Ia[0], Ib[0])
    assert abs(sa[0] - sb[0]) <= 1e-4 * sb[0], (sa[0], sb[0])
    # unadapted early iterations would bias the Eq. 8-9 average: adapt
    # first, then combine
    a.adapt(4)
    a.integrate(w.n_iter)
    r = a.result()
    exact = cf.exact(w)
    assert abs(r.integral - exact) < 3.0 * math.sqrt(r.sigma2), (r.integral, exact, math.sqrt(r.sigma2))
    a.close()
    b.close()


def test_kahan_overflow_reported(V):
    """Squared weights beyond FP32 range: the compensated FP32 variance
    overflows.  The result says so (VEGAS_ENONFINITE) and the allocation
    falls back to uniform instead of using the overflowed variances."""
    from paper_2408_09229_amd import VegasError
    D = 12
    # typical weights ~1e20 (squares past FP32), the largest well inside FP32
    prm = np.concatenate([[1e8], np.full(D, 20.0), np.full(D, 0.5)])
    w = vi.Workload("ppeak12_kahan", D, vi.GENZ_PPEAK, prm, n_g=64, n_eval=200_000, n_iter=1)
    say(f"[kahan overflow] {w.name}")
    v = V(w, precision="f32", accum="kahan")
    v.adapt(2)
    nh = v.get_nh()
    assert int(nh.sum()) == w.n_eval and int(nh.min()) >= w.n_min
    with pytest.raises(VegasError) as e:
        v.result()
    assert e.value.status == -5
    v.close()
