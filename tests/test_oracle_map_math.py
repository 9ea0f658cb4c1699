"""Oracle pins: deterministic log/exp, map refinement, Eq. 8-9.

det_log/det_exp against mpmath (<= 2 ulp).  The map update against an
independent 50-digit mpmath evaluation of the same reading (smooth,
normalise, damp, rebin), plus identities: alpha = 0 and all-zero weights leave
the map alone, equal weights keep a uniform grid.  Eq. 8-9 on hand-computed
inputs.
"""
import math

import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 50


def _ulp_err(got, want):
    want = mp.mpf(want)
    if want == 0:
        return abs(got)
    return float(abs(mp.mpf(got) - want) / (abs(want) * mp.mpf(2) ** -52))


def test_det_log(orc):
    rng = np.random.default_rng(1)
    xs = list(10.0 ** rng.uniform(-300, 300, 2000)) + list(1 + rng.uniform(-0.3, 0.3, 500)) + \
        [1.0, 2.0, 0.5, math.sqrt(0.5), 5e-324, 2.2250738585072014e-308, 1.7976931348623157e308]
    worst = 0.0
    for x in xs:
        want = mp.log(mp.mpf(x))
        got = orc.det_log(x)
        if abs(want) < 1e-3:
            assert abs(mp.mpf(got) - want) <= 2 * 2.0 ** -52 * max(abs(want), mp.mpf(2) ** -60)
        else:
            worst = max(worst, _ulp_err(got, want))
    assert worst <= 2.0, worst
    assert orc.det_log(1.0) == 0.0
    assert orc.det_log(0.0) == -math.inf
    assert math.isnan(orc.det_log(-1.0))


def test_det_exp(orc):
    rng = np.random.default_rng(2)
    xs = list(rng.uniform(-700, 700, 3000)) + list(rng.uniform(-1, 1, 500)) + [0.0, 1.0, -1.0, 0.5 * math.log(2)]
    worst = max(_ulp_err(orc.det_exp(x), mp.exp(mp.mpf(x))) for x in xs)
    assert worst <= 2.0, worst
    assert orc.det_exp(0.0) == 1.0
    assert orc.det_exp(-800.0) == 0.0
    assert orc.det_exp(800.0) == math.inf


def _mp_update(x, H, Cn, alpha):
    """The refinement reading evaluated at 50 digits."""
    n = len(H)
    d = [mp.mpf(H[i]) / mp.mpf(Cn[i]) if Cn[i] > 0 else mp.mpf(0) for i in range(n)]
    if all(h == 0 for h in H) or alpha == 0:
        return [mp.mpf(v) for v in x]
    if n == 1:
        e = d[:]
    else:
        e = [(7 * d[0] + d[1]) / 8] + [(d[i - 1] + 6 * d[i] + d[i + 1]) / 8 for i in range(1, n - 1)] + \
            [(d[n - 2] + 7 * d[n - 1]) / 8]
    S = sum(e)
    e = [v / S for v in e]
    g = []
    for v in e:
        if v == 0:
            g.append(mp.mpf(0))
        elif v == 1:
            g.append(mp.mpf(1))
        else:
            g.append(((1 - v) / mp.log(1 / v)) ** alpha)
    c = [mp.mpf(0)]
    for v in g:
        c.append(c[-1] + v)
    G = c[-1]
    xn = [mp.mpf(x[0])]
    i = 0
    for j in range(1, n):
        tau = j * G / n
        while not (c[i] <= tau < c[i + 1]):
            i += 1
        xn.append(mp.mpf(x[i]) + (tau - c[i]) / g[i] * (mp.mpf(x[i + 1]) - mp.mpf(x[i])))
    xn.append(mp.mpf(x[n]))
    return xn


@pytest.mark.parametrize("n_g", [1, 2, 3, 5, 16, 64])
@pytest.mark.parametrize("alpha", [0.5, 1.0, 1.5, 0.7])
def test_map_update_vs_mpmath(orc, n_g, alpha):
    rng = np.random.default_rng(n_g * 10 + int(alpha * 10))
    x = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, n_g - 1)]))
    Cn = rng.integers(0, 40, n_g).astype(float)
    H = np.where(Cn > 0, rng.lognormal(0, 2, n_g) * Cn, 0.0)
    if not H.any():
        H[0], Cn[0] = 1.0, 1.0
    got = orc.map_update_axis(x, H, Cn, alpha)
    want = _mp_update(x, H, Cn, alpha)
    err = max(abs(float(got[i] - want[i])) for i in range(n_g + 1))
    assert err < 1e-12, err
    assert got[0] == x[0] and got[-1] == x[-1]
    assert np.all(np.diff(got) >= 0)


def test_map_update_smoothing_of_single_bin(orc):
    # all weight in one interior bin: smoothing spreads it 1:6:1 to the
    # neighbours; the rebinned grid must match the 50-digit evaluation.
    n_g = 8
    x = np.linspace(0, 1, n_g + 1)
    H = np.zeros(n_g); H[3] = 5.0
    Cn = np.ones(n_g)
    got = orc.map_update_axis(x, H, Cn, 1.0)
    want = _mp_update(x, H, Cn, 1.0)
    assert max(abs(float(got[i] - want[i])) for i in range(n_g + 1)) < 1e-14
    # the neighbours of bin 3 take weight: new points crowd into [2/8, 5/8]
    assert np.sum((got > 0.25) & (got < 0.625)) >= 3


def test_map_update_identities(orc):
    x = np.linspace(0.0, 1.0, 33) ** 2
    H = np.random.default_rng(0).random(32)
    Cn = np.ones(32)
    assert np.array_equal(orc.map_update_axis(x, H, Cn, 0.0), x)
    assert np.array_equal(orc.map_update_axis(x, np.zeros(32), Cn, 0.5), x)
    u = np.array([i / 32 for i in range(33)])
    eq = orc.map_update_axis(u, 3.0 * np.full(32, 7.0), np.full(32, 7.0), 0.5)
    assert np.max(np.abs(eq - u)) < 1e-14


def test_combine_by_hand(orc):
    I, s2, chi = orc.combine([1.0, 2.0], [1.0, 4.0])
    assert abs(I - 1.2) < 1e-15 and abs(s2 - 0.8) < 1e-15 and abs(chi - 0.2) < 1e-15
    I, s2, chi = orc.combine([3.0, 5.0, 4.0], [0.0, 1.0, 0.0])
    assert I == 3.5 and s2 == 0.0
    I, s2, chi = orc.combine([2.5], [0.25])
    assert I == 2.5 and s2 == 0.25 and chi == 0.0
    I, s2, chi = orc.combine([1.0, 1.0, 4.0], [1.0, 1.0, 1.0])
    assert I == 2.0 and abs(s2 - 1 / 3) < 1e-16 and chi == (1 + 1 + 4) / 2


def test_combine_empty_iterations(orc):
    """An iteration whose weights were all zero (I = 0 and sigma^2 = 0) is
    left out when another iteration saw a nonzero estimate; if every one is
    empty the result is 0 with sigma^2 0.  By hand: weights 100 and 25 give
    (100 * 1.0 + 25 * 1.2) / 125 = 1.04 and sigma^2 = 1/125; chi^2 over the
    two informative iterations is (100 * 0.04^2 + 25 * 0.16^2) / 1 = 0.8."""
    I, s2, chi = orc.combine([0.0, 1.0, 1.2], [0.0, 0.01, 0.04])
    assert abs(I - 1.04) < 1e-15 and abs(s2 - 0.008) < 1e-17 and abs(chi - 0.8) < 1e-14
    I, s2, chi = orc.combine([0.0, 0.0], [0.0, 0.0])
    assert I == 0.0 and s2 == 0.0 and chi == 0.0
    # an exact nonzero iteration still decides the result over an empty one
    I, s2, chi = orc.combine([0.0, 2.0, 1.9], [0.0, 0.0, 0.5])
    assert I == 2.0 and s2 == 0.0
