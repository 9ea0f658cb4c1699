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
