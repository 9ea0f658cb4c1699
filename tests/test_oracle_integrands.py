"""Oracle pins: each integrand family against library routines and
closed-form one-dimensional integrals (scipy quad, scipy.stats)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import vegas_inputs as vi
from tests import closed_forms as cf


def _quad1(orc, fam, params):
    return integrate.quad(lambda t: orc.integrand(fam, [t], params), 0.0, 1.0,
                          epsabs=1e-14, epsrel=1e-12, limit=400)[0]


@pytest.mark.parametrize("fam,params,exact", [
    (vi.GAUSS_DIAG, vi.gauss_diag_params(2.0, 0.1, [0.5]), None),
    (vi.GAUSS_DIAG, vi.gauss_diag_params(1.0, 0.05, [0.33, 0.5, 0.9]), None),
    (vi.GENZ_PPEAK, np.array([1.5, 7.0, 0.3]), None),
    (vi.GENZ_GAUSS, np.array([0.5, 9.0, 0.7]), None),
    (vi.LINEAR, np.array([3.0]), 1.5),
    (vi.ROOS, np.array([2.0]), 2.0),
    (vi.CONST, np.array([4.25]), 4.25),
    (vi.COSINE, np.array([1.0]), math.sin(1.0)),
    (vi.EXP_SQ, np.array([1.5]), None),
    (vi.MOROKOFF, np.array([0.75]), 0.75),
])
def test_family_1d_integral(orc, fam, params, exact):
    w = vi.Workload("t", 1, fam, params, n_g=1, n_eval=1, n_iter=1)
    want = cf.exact(w) if exact is None else exact
    assert abs(_quad1(orc, fam, params) - want) <= 1e-10 * abs(want)


@pytest.mark.parametrize("fam", [vi.GENZ_PPEAK, vi.GENZ_GAUSS])
def test_genz_separable(orc, fam):
    # the D-dim value is A times the product (PPEAK) / exp-sum (GAUSS) of the
    # one-dimensional factors: a misplaced parameter index breaks it.
    rng = np.random.default_rng(5)
    D = 5
    a = rng.uniform(5, 20, D); u = rng.uniform(0.1, 0.9, D)
    p = np.concatenate([[2.5], a, u])
    for _ in range(20):
        x = rng.random(D)
        one = [orc.integrand(fam, [x[d]], np.array([1.0, a[d], u[d]])) for d in range(D)]
        assert abs(orc.integrand(fam, x, p) - 2.5 * np.prod(one)) <= 1e-13 * abs(orc.integrand(fam, x, p))


@pytest.mark.parametrize("D,mu,s,rho", [(16, 0.5, 0.03, 0.9), (3, 0.4, 0.2, 0.3), (2, 0.5, 0.1, -0.5)])
def test_gauss_corr_vs_scipy(orc, D, mu, s, rho):
    cov = s * s * ((1 - rho) * np.eye(D) + rho * np.ones((D, D)))
    rv = stats.multivariate_normal(mean=np.full(D, mu), cov=cov)
    rng = np.random.default_rng(D)
    for _ in range(30):
        x = rv.rvs(random_state=rng) if rng.random() < 0.7 else rng.random(D)
        got = orc.integrand(vi.GAUSS_CORR, x, np.array([mu, s, rho]))
        want = rv.pdf(x)
        assert abs(got - want) <= 1e-11 * want + 1e-300


def test_gauss_diag_multi_d_is_product(orc):
    # exp of a sum equals the product of the axis factors (cfg gauss_prod_4d)
    w = vi.gauss_prod_4d()
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.random(4)
        want = np.prod(np.exp(-(x - 0.5) ** 2 / (2 * 0.01)))
        assert abs(orc.integrand(w.family, x, w.params) - want) <= 1e-14


def test_gauss_corr_closed_form_against_direct_sampling():
    """The box mass of the equicorrelated Gaussian (a 1-d quadrature) against
    direct sampling of the normal distribution, and at rho = 0 against the
    product of erfs."""
    from tests import closed_forms as cf
    rng = np.random.default_rng(0)
    for s, rho in [(0.2, 0.5), (0.15, 0.3)]:
        want = cf.gauss_corr(np.array([0.5, s, rho]), 16)
        n = 2_000_000
        z = rng.standard_normal((n, 17))
        x = 0.5 + s * (np.sqrt(1 - rho) * z[:, :16] + np.sqrt(rho) * z[:, 16:17])
        p = np.count_nonzero(np.all((x >= 0) & (x <= 1), axis=1)) / n
        assert abs(p - want) < 5 * np.sqrt(p * (1 - p) / n), (s, rho, p, want)
    s = 0.2
    prod = cf.gauss_diag(np.array([1.0, s, 1.0, 0.5]), 6) / (2 * np.pi * s * s) ** 3
    assert abs(cf.gauss_corr(np.array([0.5, s, 0.0]), 6) - prod) < 1e-12


def _quad2(orc, fam, params):
    return integrate.dblquad(lambda b, a: orc.integrand(fam, [a, b], params), 0.0, 1.0, 0.0, 1.0,
                             epsabs=1e-13, epsrel=1e-11)[0]


@pytest.mark.parametrize("fam,params", [
    (vi.SIN_EXP, np.array([1.25])),
    (vi.EXP_SQ, np.array([0.5])),
    (vi.MOROKOFF, np.array([2.0])),
])
def test_family_2d_integral(orc, fam, params):
    """Tab. 3 #1, #4, #6 in two dimensions against their closed forms
    (sin + exp: e - cos 1; exp of the squared norm: the erfi product;
    Morokoff-Caflisch: A, since (1 + 1/2)^2 (int_0^1 sqrt x dx)^2 = 1)."""
    w = vi.Workload("t", 2, fam, params, n_g=1, n_eval=1, n_iter=1)
    want = cf.exact(w)
    assert abs(_quad2(orc, fam, params) - want) <= 1e-9 * abs(want)


def test_sin_exp_uses_the_first_two_axes(orc):
    """sin + exp reads x_0 and x_1 only: in 3-d the third axis changes
    nothing, and the two terms swap roles with the axes."""
    p = np.array([1.0])
    for x in ([0.2, 0.7, 0.1], [0.9, 0.05, 0.6]):
        a = orc.integrand(vi.SIN_EXP, x, p)
        assert a == orc.integrand(vi.SIN_EXP, [x[0], x[1], 0.99], p)
        assert abs(a - (math.sin(x[0]) + math.exp(x[1]))) <= 1e-15 * a


def test_morokoff_3d_mean_is_one(orc):
    """Morokoff-Caflisch in 3-d by a tensor Gauss-Jacobi rule exact for the
    x^(1/3) weights: the integral is A = 1 (closed form)."""
    from scipy.special import roots_jacobi
    # int_0^1 x^(1/3) g(x) dx with weight x^(1/3): Jacobi on [-1,1] with
    # beta = 1/3 after x = (1 + t)/2
    t, wt = roots_jacobi(8, 0.0, 1.0 / 3.0)
    xs = (1 + t) / 2
    ws = wt / 2 ** (1 + 1 / 3)
    tot = 0.0
    for i, a in enumerate(xs):
        for j, b in enumerate(xs):
            for k, c in enumerate(xs):
                # the rule integrates the x^(1/3) factors; divide them out of f
                tot += ws[i] * ws[j] * ws[k] * orc.integrand(vi.MOROKOFF, [a, b, c], np.array([1.0])) / \
                    (a * b * c) ** (1 / 3)
    assert abs(tot - 1.0) < 1e-12
