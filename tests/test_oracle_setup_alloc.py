"""Oracle pins: strata sizes and the integer allocation (Eq. 7 reading).

Strata: brute force over m.  Allocation: Python big integers redo the
quantise / scan / systematic rounding exactly, plus invariants the reading
fixes (sum = N_ev, n_h >= n_min, beta = 0 uniform, proportionality).
"""
import numpy as np
import pytest


@pytest.mark.parametrize("n_eval,dim", [(100_000, 4), (10 ** 8, 8), (2 * 10 ** 8, 4), (10 ** 6, 16),
                                        (4, 1), (7, 1), (1000, 1), (5, 3), (10 ** 4, 12), (123_457, 2)])
def test_strata_bruteforce(orc, n_eval, dim):
    got = orc.strata(n_eval, dim)
    m = 1
    while 4 * (m + 1) ** dim <= n_eval:
        m += 1
    while m > 1 and not (m ** dim < 2 ** 31 - 1 and 2 * m ** dim <= n_eval):
        m -= 1
    assert got == (m, m ** dim, n_eval - 2 * m ** dim)


def test_strata_budget_too_small(orc):
    assert orc.strata(1, 1) is None
    assert orc.strata(1, 5) is None
    assert orc.strata(3, 2) == (1, 1, 1)      # one cube, three samples


def test_strata_published_sizes(orc):
    # the workload sizes stated for the benchmark configurations
    assert orc.strata(100_000, 4)[0] == 12
    assert orc.strata(10 ** 8, 8)[0] == 8
    assert orc.strata(2 * 10 ** 8, 4)[0] == 84
    assert orc.strata(10 ** 6, 16)[0] == 2


def _bigint_alloc(q, n_min, n_eval):
    n = len(q)
    R = n_eval - n_min * n
    qmax = max(q)
    if qmax > 0:
        from fractions import Fraction
        # floor((q/qmax) 2^32) with the division rounded once to double
        Q = [int(np.floor((qi / qmax) * 4294967296.0)) for qi in q]
    else:
        Q = [1] * n
    T = sum(Q)
    out, C = [], 0
    for Qh in Q:
        Cn = C + Qh
        out.append(n_min + (R * Cn) // T - (R * C) // T)
        C = Cn
    return out


@pytest.mark.parametrize("beta", [0.75, 1.0, 0.5, 0.3, 2.0])
def test_alloc_bigint(orc, beta):
    rng = np.random.default_rng(7)
    for n in [1, 2, 17, 1000]:
        v = rng.lognormal(0, 3, size=n)
        v[rng.random(n) < 0.1] = 0.0
        n_eval = 5 * n + int(rng.integers(0, 10 * n + 1))
        nh = orc.alloc(v, 2, n_eval, beta)
        q = [orc.alloc_weight(x, beta) for x in v]
        assert list(map(int, nh)) == _bigint_alloc(q, 2, n_eval)
        assert int(nh.sum()) == n_eval
        assert nh.min() >= 2


def test_alloc_weight_powers(orc):
    import mpmath as mp
    mp.mp.dps = 30
    for v in [1e-300, 1e-20, 0.37, 1.0, 3.5, 1e10, 1e300]:
        for beta in [0.75, 1.0, 0.5, 0.3, 1.7]:
            got = orc.alloc_weight(v, beta)
            want = float(mp.mpf(v) ** (mp.mpf(beta) / 2))
            # exp(b ln v) inherits the rounding of its exponent: |ln q| eps
            tol = (4.0 + 2.0 * abs(float(mp.log(want)))) * 1.12e-16
            assert abs(got - want) <= tol * want, (v, beta)
    assert orc.alloc_weight(0.0, 0.75) == 0.0


def test_alloc_invariants(orc):
    rng = np.random.default_rng(3)
    n = 5000
    v = rng.lognormal(0, 2, size=n)
    n_eval = 6 * n + 13
    nh = orc.alloc(v, 2, n_eval, 0.75).astype(np.int64)
    assert nh.sum() == n_eval and nh.min() >= 2
    # proportional to q within one sample (systematic rounding), up to the
    # 2^-32 quantisation of q/q_max
    q = np.array([orc.alloc_weight(x, 0.75) for x in v])
    ideal = 2 + (n_eval - 2 * n) * q / q.sum()
    assert np.max(np.abs(nh - ideal)) < 1.0 + 1e-6
    # monotone in q up to the rounding
    order = np.argsort(q)
    assert np.all(np.diff(nh[order]) >= -1)
    # beta = 0, adapt off, or all-zero variance: uniform split
    for nh2 in (orc.alloc(v, 2, n_eval, 0.0), orc.alloc(v, 2, n_eval, 0.75, adapt=False),
                orc.alloc(np.zeros(n), 2, n_eval, 0.75)):
        assert nh2.sum() == n_eval and int(nh2.max()) - int(nh2.min()) <= 1
