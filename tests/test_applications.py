"""The paper's application integrands (Sec. 4.5-4.6), CPU only.

* the Asian call's closed form (Black-Scholes with the summed variance)
  against 1-d quadrature over the normal sum, and at n = 1 against the
  textbook Black-Scholes price 10.4506 (S = K = 100, r = 5 %, sigma = 20 %,
  T = 1);
* the lattice path integral's closed form (a Gaussian integral) against
  direct quadrature over one and two interior points, and near the
  continuum value |psi_0(x)|^2 e^{-T/2} at N = 8, T = 4;
* both device sources compile for gfx950 (hipRTC, no device needed).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from tests import closed_forms as cf


@pytest.mark.parametrize("n", [1, 3, 8])
def test_asian_closed_form_against_quadrature(n):
    s0, k, r, sig, t = 100.0, 100.0, 0.05, 0.2, 1.0

    def f(z):
        s = s0 * math.exp((r - sig * sig / 2) * t + sig * math.sqrt(t * n) * z)
        return math.exp(-r * t) * max(s - k, 0.0) * stats.norm.pdf(z)

    q = integrate.quad(f, -14, 14, points=[0.0], limit=400, epsabs=1e-12, epsrel=1e-12)[0]
    assert abs(cf.asian_call([s0, k, r, sig, t], n) - q) < 1e-9 * q


def test_asian_n1_is_black_scholes():
    assert abs(cf.asian_call([100.0, 100.0, 0.05, 0.2, 1.0], 1) - 10.450583572185565) < 1e-10


def _action(path, a, m):
    return sum(m / (2 * a) * (path[j + 1] - path[j]) ** 2 + a * path[j] ** 2 / 2 for j in range(len(path) - 1))


@pytest.mark.parametrize("xe", [0.0, 1.0])
def test_feynman_closed_form_against_quadrature(xe):
    a, m = 0.5, 1.0
    A2 = (m / (2 * math.pi * a)) ** 1.0
    q1 = integrate.quad(lambda y: A2 * math.exp(-_action([xe, y, xe], a, m)), -12, 12, epsabs=1e-13)[0]
    assert abs(cf.feynman_ho([xe, a, m], 1) - q1) < 1e-10
    A3 = (m / (2 * math.pi * a)) ** 1.5
    q2 = integrate.dblquad(lambda y2, y1: A3 * math.exp(-_action([xe, y1, y2, xe], a, m)), -12, 12, -12, 12,
                           epsabs=1e-12)[0]
    assert abs(cf.feynman_ho([xe, a, m], 2) - q2) < 1e-9


def test_feynman_near_continuum():
    # N = 8, T = 4: the lattice propagator at x = 0 within 4 % of the
    # continuum |psi_0(0)|^2 e^{-E_0 T} = e^{-2} / sqrt(pi) (discretisation)
    v = cf.feynman_ho([0.0, 0.5, 1.0], 7)
    assert abs(v / (math.exp(-2.0) / math.sqrt(math.pi)) - 1.0) < 0.04


@pytest.mark.parametrize("name,dim", [("ASIAN_CALL", 8), ("FEYNMAN_HO", 7)])
def test_sources_compile(name, dim):
    import paper_2408_09229_amd as pk
    from paper_2408_09229_amd import integrands
    pk.UserIntegrand.check(getattr(integrands, name), dim, "f64")
