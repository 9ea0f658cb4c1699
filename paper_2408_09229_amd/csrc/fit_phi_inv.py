"""Coefficients of the warp's inverse normal distribution function (flow_dev.hpp:
phi_inv_lower), fitted here; run with python3 to print them and their error.

Phi^-1(m) = -sqrt(2) erfinv(1 - 2m) for 0 < m <= 1/2, and erfinv(x) = x p(w)
with w = -ln((1 - x)(1 + x)) = -ln(4 m (1 - m)), which is formed from m without
cancellation.  p is a degree-8 polynomial in w - 2.5 for w < 5 and in
sqrt(w) - 3 for 5 <= w <= 16.2 (m >= 1e-7), the two-piece form of M. Giles,
"Approximating the erfinv function" (GPU Computing Gems, Jade edition, 2011).
Each piece is a least-squares fit to erfinv(x)/x on 40 001 points, reweighted
toward the largest relative errors (30 rounds), rounded to FP32; the check
evaluates both pieces by FP32 Horner steps against scipy's ndtri.
"""
import numpy as np
from scipy.special import erfinv, ndtri


def fit(wlo, whi, var, deg=8, rounds=30):
    w = np.linspace(wlo, whi, 40001)
    x = np.sqrt(1 - np.exp(-w))
    f = np.where(x > 0, erfinv(x) / np.where(x > 0, x, 1.0), np.sqrt(np.pi) / 2)
    t = var(w)
    wt = 1 / f
    for _ in range(rounds):
        A = np.vander(t, deg + 1) * wt[:, None]
        c, *_ = np.linalg.lstsq(A, f * wt, rcond=None)
        err = np.abs(np.polyval(c, t) / f - 1)
        wt = wt * (1 + 50 * err / err.max())
    return c.astype(np.float32)


def horner32(c, t):
    p = np.full_like(t, c[0])
    for a in c[1:]:
        p = (p.astype(np.float64) * t + a).astype(np.float32)
    return p


def main():
    c1 = fit(0.0, 5.0, lambda w: w - 2.5)
    c2 = fit(5.0, 16.2, lambda w: np.sqrt(w) - 3.0)
    m = np.logspace(-7, np.log10(0.4999), 400000)
    w = -np.log(4 * m * (1 - m))
    p = np.where(w < 5.0, horner32(c1, (w - 2.5).astype(np.float32)),
                 horner32(c2, (np.sqrt(w) - 3).astype(np.float32)))
    r = np.abs(-np.sqrt(2) * p.astype(np.float64) * (1 - 2 * m) / ndtri(m) - 1)
    print("max relative error %.3e (%.1f FP32 ulps)" % (r.max(), r.max() / 2.0 ** -24))
    print("central:", ", ".join("%.9ef" % v for v in c1))
    print("tail:   ", ", ".join("%.9ef" % v for v in c2))


if __name__ == "__main__":
    main()
