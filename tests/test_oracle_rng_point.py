"""Oracle pins: Philox4x32-10, the sample counter layout, fixed-point y/bins.

Philox is pinned to the published known-answer vectors (tests/golden); the
bin/offset arithmetic to exact rational brute force with fractions.Fraction.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(orc.philox4x32_10(ctr, key)) == want


def test_word_counter_layout(orc):
    # counter = (k lo, k hi, t, inst<<8 | d/4), key = (seed lo, seed hi), word d%4
    seed = 0x0123456789ABCDEF
    for (inst, t, k, d) in [(0, 0, 0, 0), (0, 3, 12345, 5), (7, 1, (1 << 32) + 9, 15), (2, 9, 77, 2)]:
        out = orc.philox4x32_10([k & 0xFFFFFFFF, k >> 32, t, (inst << 8) | (d // 4)],
                                [seed & 0xFFFFFFFF, seed >> 32])
        assert orc.word(seed, inst, t, k, d) == int(out[d % 4])


def test_philox_uniformity(orc):
    # chi^2 over 256 bins of the top byte of 65536 words: a gross defect fails.
    words = np.array([orc.word(0, 0, 0, k, d) for k in range(16384) for d in range(4)],
                     dtype=np.uint64)
    counts = np.bincount((words >> 24).astype(np.int64), minlength=256)
    e = words.size / 256
    chi2 = ((counts - e) ** 2 / e).sum()
    assert 170 < chi2 < 350     # 255 dof; ~5 sigma window


def _exact_point(s, r, n_st, n_g):
    y = (Fraction(s) + Fraction(2 * r + 1, 2 ** 33)) / n_st
    yg = y * n_g
    i = yg.numerator // yg.denominator
    return i, float(yg - i)          # float(Fraction) rounds correctly


@pytest.mark.parametrize("n_st,n_g", [(1, 1), (3, 8), (12, 128), (7, 5), (84, 1024), (2, 1024), (1, 3)])
def test_point_matches_rational(orc, n_st, n_g):
    rng = np.random.default_rng(n_st * 1000 + n_g)
    rs = list(rng.integers(0, 2 ** 32, size=200)) + [0, 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32 - 2]
    for s in sorted({0, n_st - 1, n_st // 2}):
        for r in rs:
            want = _exact_point(s, int(r), n_st, n_g)
            got = orc.point(s, int(r), n_st, n_g)
            assert got[0] == want[0] and got[1] == want[1], (s, r, got, want)


def test_point_exhaustive_small_word(orc):
    # Every (s, r) for r in a dense range on a tiny grid: bins cover each
    # interval exactly in proportion (s, r) -> y is uniform on the strata.
    n_st, n_g = 3, 8
    for s in range(n_st):
        for r in range(0, 2 ** 32, 2 ** 22):
            want = _exact_point(s, r, n_st, n_g)
            assert orc.point(s, r, n_st, n_g) == want
