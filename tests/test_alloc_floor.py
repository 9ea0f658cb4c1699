"""The allocation kernel's floor(R C / T) (Eq. 7's cumulative share, in
integers) takes the floor of a double estimate when the estimate's fraction
is at least 2^-16 from both integers, and checks with 128-bit products
otherwise.  This models that fast path in IEEE double (Python floats round
the same way: one rounding per conversion, division and product) and checks
it against exact integer division wherever it is taken, on random and on
adversarial operands (R C / T at or next to an integer)."""
import math
import random

import pytest

MARGIN = 2.0 ** -16


def fast_floor(R, C, T):
    """None where the kernel falls back to the exact check."""
    rT = float(R) / float(T)
    est = float(C) * rT
    fl = math.floor(est)
    fr = est - fl
    if MARGIN < fr < 1.0 - MARGIN:
        return fl
    return None


def _cases(rng, n):
    for _ in range(n):
        R = rng.randrange(0, 1 << 32)
        T = rng.randrange(1, 1 << rng.choice([20, 40, 58]))
        C = rng.randrange(0, T + 1)
        yield R, C, T
    # at and next to integers: C near k T / R
    for _ in range(n):
        R = rng.randrange(1, 1 << 32)
        T = rng.randrange(R, 1 << 58)
        k = rng.randrange(0, R + 1)
        c0 = (k * T) // R
        for C in (c0 - 1, c0, c0 + 1):
            if 0 <= C <= T:
                yield R, C, T


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fast_floor_is_exact_where_taken(seed):
    rng = random.Random(seed)
    taken = 0
    for R, C, T in _cases(rng, 20000):
        f = fast_floor(R, C, T)
        if f is not None:
            taken += 1
            assert f == (R * C) // T, (R, C, T)
    assert taken > 20000  # the fast path covers most operands


def test_exact_integers_fall_back():
    # R C / T an integer: the estimate sits on (or within rounding of) it
    for R, C, T in [(12, 6, 12), (1 << 31, 1 << 40, 1 << 41), (1000, 0, 7), (5, 7, 7)]:
        assert fast_floor(R, C, T) is None
