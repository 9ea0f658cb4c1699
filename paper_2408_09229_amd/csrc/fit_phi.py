"""Coefficients of the warp's Gaussian distribution function and its inverse
(flow_dev.hpp: phi_lower, phi_inv_lower), fitted here; run with python3 to
print them with their errors, measured by emulating the device's FP32
operation sequence (fma and roundings) against scipy in FP64.

Inverse, Phi^-1(m) = -sqrt(2) erfinv(1 - 2m) for 0 < m <= 1/2: erfinv(x) =
x p(w) with w = -ln((1 - x)(1 + x)) = -ln(4 m (1 - m)), which is formed
from m without cancellation.  p is a degree-8 polynomial in w - 2.5 for
w < 5 and in sqrt(w) - 3 for 5 <= w <= 16.2 (m >= 1e-7), the two-piece form
of M. Giles, "Approximating the erfinv function" (GPU Computing Gems, Jade
edition, 2011).  Each piece is a least-squares fit to erfinv(x)/x,
reweighted toward the largest relative errors.

Lower tail, h(a) = Phi(-a) for a >= 0: h = t 2^(Q(s) - a^2 log2(e) / 2)
with t = 1 / (1 + c a) and s = 2t - 1 in [-1, 1] (the form of the
rational-exponent erfc approximations, e.g. Numerical Recipes' erfcc, with
a polynomial of our own fit).  Q(s) = log2(h) + a^2 log2(e) / 2 - log2(t)
is smooth on the whole of t in (0, 1] (h ~ phi(a) / a as a grows), here of
degree 10 with c = 0.4.  On the device the exponent's roundings (a^2,
its product by log2(e)/2, and the difference with Q) are carried as a
first-order correction 1 + ln2 (dy), so that the error stays a few ulps
where the exponent is large.
"""
import numpy as np
from scipy.special import erfinv, log_ndtr, ndtr, ndtri

LOG2E = 1.4426950408889634
K = 0.5 * LOG2E
PHI_C = 0.4


def _reweighted_fit(t, f, deg, rounds, weight, relative=True):
    wt = 1 / np.abs(f) if relative else np.ones_like(f)
    for _ in range(rounds):
        A = np.vander(t, deg + 1) * wt[:, None]
        c, *_ = np.linalg.lstsq(A, f * wt, rcond=None)
        err = np.abs(np.polyval(c, t) - f) * (1 / np.abs(f) if relative else 1)
        wt = wt * (1 + weight * err / err.max())
    return c.astype(np.float32)


def fit_inverse():
    out = []
    for wlo, whi, var in ((0.0, 5.0, lambda w: w - 2.5), (5.0, 16.2, lambda w: np.sqrt(w) - 3.0)):
        w = np.linspace(wlo, whi, 40001)
        x = np.sqrt(1 - np.exp(-w))
        f = np.where(x > 0, erfinv(x) / np.where(x > 0, x, 1.0), np.sqrt(np.pi) / 2)
        out.append(_reweighted_fit(var(w), f, 8, 30, 50))
    return out


def fit_lower(deg=10, amax=13.5):
    a = np.linspace(0, amax, 80001)
    t = 1 / (1 + PHI_C * a)
    q = log_ndtr(-a) * LOG2E + K * a * a - np.log2(t)
    return _reweighted_fit(2 * t - 1, q, deg, 40, 20, relative=False)


def r32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fma32(a, b, c):
    return r32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def horner32(c, t):
    p = np.full(t.shape, c[0], np.float32)
    for v in c[1:]:
        p = fma32(p, t, v)
    return p


def phi_lower32(co, a):
    """h(a) by the device's FP32 sequence (exact exp2 and reciprocal,
    rounded to FP32)."""
    kf = np.float32(K)
    kl = np.float32(K - float(kf))
    a = r32(a)
    t = r32(1 / fma32(np.float32(PHI_C), a, 1.0).astype(np.float64))
    p = horner32(co, fma32(2.0, t, -1.0))
    sq = r32(a.astype(np.float64) * a)
    sqlo = fma32(a, a, -sq.astype(np.float64))
    u = r32(np.float64(kf) * sq)
    corr = fma32(kf, sq, -u.astype(np.float64))
    corr = fma32(kf, sqlo, corr)
    corr = fma32(kl, sq, corr)
    y = r32(p.astype(np.float64) - u)
    ylo = r32(p.astype(np.float64) - r32(y.astype(np.float64) + u))
    f = fma32(r32(ylo.astype(np.float64) - corr), np.float32(np.log(2)), 1.0)
    e = r32(np.exp2(y.astype(np.float64)))
    return r32(r32(t.astype(np.float64) * e).astype(np.float64) * f)


def main():
    c1, c2 = fit_inverse()
    m = np.logspace(-7, np.log10(0.4999), 400000)
    w = -np.log(4 * m * (1 - m))
    p = np.where(w < 5.0, horner32(c1, r32(w - 2.5)), horner32(c2, r32(np.sqrt(w) - 3)))
    r = np.abs(-np.sqrt(2) * p.astype(np.float64) * (1 - 2 * m) / ndtri(m) - 1)
    print("Phi^-1: max relative error %.3e (%.1f FP32 ulps) for m in [1e-7, 0.4999]" % (r.max(), r.max() / 2.0 ** -24))
    print("  central:", ", ".join("%.9ef" % v for v in c1))
    print("  tail:   ", ", ".join("%.9ef" % v for v in c2))
    co = fit_lower()
    a = r32(np.linspace(0, 12, 400001))
    r = np.abs(phi_lower32(co, a) / ndtr(-a.astype(np.float64)) - 1) / 2.0 ** -24
    print("Phi(-a): max relative error %.1f FP32 ulps for a in [0, 12] (before the hardware exp2 and"
          " reciprocal's own ulp)" % r.max())
    print("  Q:      ", ", ".join("%.9ef" % v for v in co))


if __name__ == "__main__":
    main()
