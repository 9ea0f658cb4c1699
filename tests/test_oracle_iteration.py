"""Oracle pins for one iteration and whole runs.

* D=1, one stratum, one interval reduces to textbook Monte Carlo: the mean and
  the unbiased variance / n of f at the drawn points (numpy).
* f = const with a power-of-two uniform map: sigma = 0 and I exact.
* Brute-force aggregation on a tiny problem: per-cube two-pass statistics and
  the per-axis histograms rebuilt sample by sample.
* Unbiasedness over seed ensembles on a non-uniform map.
* Closed forms within 3 sigma at a fixed seed; the converged map of a
  separable Gaussian approaches the inverse CDF of |f| (erfinv closed form).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import vegas_inputs as vi
from tests import closed_forms as cf


def test_textbook_mc(orc):
    n = 1001
    A = 3.0
    o = orc.iterate(1, 1, n, 1, 1, 42, 0, 5, vi.LINEAR, np.array([A]), orc.init_grid(1, 1), [n])
    r = np.array([orc.word(42, 0, 5, k, 0) for k in range(n)], dtype=np.float64)
    x = (2 * r + 1) / 2.0 ** 33          # exact in double
    f = A * x
    assert abs(o.I - f.mean()) <= 1e-14 * f.mean()
    assert abs(o.s2 - f.var(ddof=1) / n) <= 1e-12 * o.s2
    assert o.C[0, 0] == n and abs(o.H[0, 0] - (f * f).sum()) <= 1e-13 * o.H[0, 0]


def test_const_integrand_exact(orc):
    D, n_g = 3, 16
    ns, nc, _ = orc.strata(5000, D)
    nh = orc.alloc(np.zeros(nc), 2, 5000, 0.75, adapt=False)
    lo, hi = np.array([0.0, -1.0, 2.0]), np.array([1.0, 1.0, 2.5])
    o = orc.iterate(D, n_g, 5000, ns, nc, 0, 0, 0, vi.CONST, np.array([1.75]),
                    orc.init_grid(D, n_g, lo, hi), nh)
    assert o.s2 == 0.0                       # every w is the same number
    assert abs(o.I - 1.75 * 1.0 * 2.0 * 0.5) <= 1e-13   # a sum of N_c cube means


def test_bruteforce_aggregation(orc):
    D, n_g, n_eval, fam = 2, 4, 61, vi.GENZ_PPEAK
    p = np.array([1.0, 8.0, 5.0, 0.3, 0.7])
    ns, nc, _ = orc.strata(n_eval, D, n_strat=3)
    rng = np.random.default_rng(1)
    grid = np.stack([np.sort(np.concatenate([[0, 1], rng.random(n_g - 1)])) for _ in range(D)])
    v = rng.lognormal(0, 1, nc)
    nh = orc.alloc(v, 2, n_eval, 0.75)
    o = orc.iterate(D, n_g, n_eval, ns, nc, 9, 0, 2, fam, p, grid, nh)
    H = np.zeros((D, n_g)); Cn = np.zeros((D, n_g))
    k = 0
    I = 0.0; S2 = 0.0
    for h in range(nc):
        ws = []
        for _ in range(int(nh[h])):
            bins, delta, x, J, f = orc.sample(D, n_g, ns, 9, 0, 2, k, h, grid, fam, p)
            w = J * f
            ws.append(w)
            for d in range(D):
                H[d, bins[d]] += w * w
                Cn[d, bins[d]] += 1
            k += 1
        m = sum(ws) / len(ws)
        var = sum((wi - m) ** 2 for wi in ws) / (len(ws) - 1)
        assert o.m[h] == m and o.v[h] == var
        I += m / nc
        S2 += var / (float(nc) * float(nc) * len(ws))
    assert k == n_eval
    assert np.array_equal(H, o.H) and np.array_equal(Cn, o.C)
    assert o.I == I and o.s2 == S2


def test_histogram_totals(orc):
    w = vi.gauss_prod_4d().with_(n_eval=20_000, n_g=32)
    ns, nc, _ = orc.strata(w.n_eval, w.dim)
    nh = orc.alloc(np.zeros(nc), 2, w.n_eval, 0.75, adapt=False)
    o = orc.iterate(w.dim, w.n_g, w.n_eval, ns, nc, 0, 0, 0, w.family, w.params,
                    orc.init_grid(w.dim, w.n_g), nh)
    assert np.all(o.C.sum(1) == w.n_eval)
    tot = o.H.sum(1)
    assert np.allclose(tot, tot[0], rtol=1e-12)


@pytest.mark.parametrize("fam,params", [(vi.LINEAR, np.array([1.0])),
                                        (vi.GAUSS_DIAG, vi.gauss_diag_params(1.0, 0.2, [0.4]))])
def test_unbiased_on_nonuniform_map(orc, fam, params):
    # E[I_t] = I and E[sigma_t^2] = Var(I_t) for any fixed map and allocation
    D, n_g, n_eval = 2, 8, 400
    rng = np.random.default_rng(11)
    grid = np.stack([np.sort(np.concatenate([[0, 1], rng.random(n_g - 1) ** 2])) for _ in range(D)])
    ns, nc, _ = orc.strata(n_eval, D)
    nh = orc.alloc(rng.lognormal(0, 1, nc), 2, n_eval, 0.75)
    exact = cf.exact(vi.Workload("t", D, fam, params, n_g, n_eval, 1))
    I, S2 = [], []
    for seed in range(400):
        o = orc.iterate(D, n_g, n_eval, ns, nc, seed, 0, 0, fam, params, grid, nh)
        I.append(o.I)
        S2.append(o.s2)
    I, S2 = np.array(I), np.array(S2)
    se = I.std(ddof=1) / math.sqrt(I.size)
    assert abs(I.mean() - exact) < 4 * se, (I.mean(), exact, se)
    assert 0.8 < S2.mean() / I.var(ddof=1) < 1.25


def test_gauss_prod_4d_full_run_closed_form(orc):
    w = vi.gauss_prod_4d()
    r = orc.run(w.dim, w.n_g, w.n_eval, w.family, w.params, n_iter=w.n_iter, seed=w.seed)
    exact = cf.exact(w)
    assert abs(r.integral - exact) < 3.0 * math.sqrt(r.sigma2)
    assert math.sqrt(r.sigma2) / exact < 5e-4          # adaptation works
    assert r.s2_t[-1] < 0.05 * r.s2_t[0]


@pytest.mark.parametrize("w", vi.closed_form_cases(), ids=lambda w: w.name)
def test_small_cases_closed_form(orc, w):
    r = orc.run(w.dim, w.n_g, w.n_eval, w.family, w.params, n_iter=w.n_iter, seed=w.seed)
    exact = cf.exact(w)
    assert abs(r.integral - exact) < 3.0 * math.sqrt(r.sigma2), (r.integral, exact, r.sigma2)


def test_map_converges_to_fixed_point(orc):
    # With a uniform allocation the samples are uniform inside each interval,
    # so d_i estimates N_g^2 dx_i int_i f^2 dx.  The refinement stops moving
    # when all d_i agree: the converged grid makes dx_i * int_i f^2 equal,
    # which the erf closed form of int f^2 checks interval by interval.
    s = 0.1
    p = vi.gauss_diag_params(1.0, s, [0.5])
    n_g = 32

    def f2(a, b):
        return float(s * mp.sqrt(mp.pi) / 2 * (mp.erf((b - 0.5) / s) - mp.erf((a - 0.5) / s)))

    def spread(g):
        q = np.array([(g[i + 1] - g[i]) * f2(g[i], g[i + 1]) for i in range(n_g)])
        return q / q.mean()

    r = orc.run(1, n_g, 50_000, vi.GAUSS_DIAG, p, n_iter=25, seed=3, adapt_strat=False)
    q = spread(r.grid[0])
    assert q.max() / q.min() < 1.15, q
    assert np.all(np.abs(q[2:-2] - 1) < 0.01), q
    q0 = spread(np.linspace(0, 1, n_g + 1))
    assert q0.max() / q0.min() > 1e6                            # far from the start
