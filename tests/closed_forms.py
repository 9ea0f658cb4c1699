"""Closed-form integrals of the integrand families over boxes (mpmath).

Used to pin both the oracle and the HIP path: an estimate must land within a
few standard deviations of these values.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

import vegas_inputs as vi

mp.mp.dps = 40


def gauss_diag(params, dim, lo=None, hi=None) -> float:
    """A sum_j prod_d int_lo^hi exp(-(x-c_j)^2/(2s^2)) dx (each axis by erf)."""
    A, s = mp.mpf(params[0]), mp.mpf(params[1])
    M = int(params[2])
    lo = np.zeros(dim) if lo is None else lo
    hi = np.ones(dim) if hi is None else hi
    tot = mp.mpf(0)
    r2 = mp.sqrt(2) * s
    for j in range(M):
        c = mp.mpf(params[3 + j])
        p = mp.mpf(1)
        for d in range(dim):
            p *= s * mp.sqrt(mp.pi / 2) * (mp.erf((mp.mpf(hi[d]) - c) / r2) - mp.erf((mp.mpf(lo[d]) - c) / r2))
        tot += p
    return float(A * tot)


def genz_ppeak(params, dim) -> float:
    """A prod_d a_d [atan(a_d (1-u_d)) + atan(a_d u_d)] on [0,1]^D."""
    A = mp.mpf(params[0])
    p = mp.mpf(1)
    for d in range(dim):
        a, u = mp.mpf(params[1 + d]), mp.mpf(params[1 + dim + d])
        p *= a * (mp.atan(a * (1 - u)) + mp.atan(a * u))
    return float(A * p)


def genz_gauss(params, dim) -> float:
    """A prod_d sqrt(pi)/(2 a_d) [erf(a_d (1-u_d)) + erf(a_d u_d)] on [0,1]^D."""
    A = mp.mpf(params[0])
    p = mp.mpf(1)
    for d in range(dim):
        a, u = mp.mpf(params[1 + d]), mp.mpf(params[1 + dim + d])
        p *= mp.sqrt(mp.pi) / (2 * a) * (mp.erf(a * (1 - u)) + mp.erf(a * u))
    return float(A * p)


def gauss_corr(params, dim) -> float:
    """Mass of N(mu 1, s^2 ((1-rho) I + rho 1 1^T)) in [0,1]^D.  With
    x_i = mu + s (sqrt(1-rho) z_i + sqrt(rho) t), t and z_i standard normal,
    the box probability is int phi(t) [Phi(b(t)) - Phi(a(t))]^D dt,
    a(t) = (-mu/s - sqrt(rho) t)/sqrt(1-rho), b(t) = ((1-mu)/s - sqrt(rho) t)/sqrt(1-rho)."""
    mu, s, rho = (mp.mpf(v) for v in params[:3])
    r1, rr = mp.sqrt(1 - rho), mp.sqrt(rho)
    Phi = lambda v: (1 + mp.erf(v / mp.sqrt(2))) / 2

    def g(t):
        a = (-mu / s - rr * t) / r1
        b = ((1 - mu) / s - rr * t) / r1
        return mp.npdf(t) * (Phi(b) - Phi(a)) ** dim

    return float(mp.quad(g, [-mp.inf, -8, -4, 0, 4, 8, mp.inf]))


def linear(params, dim) -> float:
    return float(params[0]) * dim / 2.0


def roos(params, dim) -> float:
    return float(params[0])      # int_0^1 |4x-2| dx = 1


def const(params, dim, lo=None, hi=None) -> float:
    lo = np.zeros(dim) if lo is None else lo
    hi = np.ones(dim) if hi is None else hi
    return float(params[0] * np.prod(np.asarray(hi) - np.asarray(lo)))


def cosine(params, dim) -> float:
    return float(params[0] * mp.sin(1) ** dim)


def sin_exp(params, dim) -> float:
    """A (sin x_0 + exp x_1) on [0,1]^D: A ((1 - cos 1) + (e - 1))."""
    return float(params[0] * ((1 - mp.cos(1)) + (mp.e - 1)))


def exp_sq(params, dim) -> float:
    """A prod_d int_0^1 exp(x^2) dx = A (sqrt(pi)/2 erfi(1))^D."""
    return float(params[0] * (mp.sqrt(mp.pi) / 2 * mp.erfi(1)) ** dim)


def morokoff(params, dim) -> float:
    """A (1 + 1/D)^D prod_d int_0^1 x^(1/D) dx = A (1 + 1/D)^D (1/(1 + 1/D))^D = A."""
    return float(params[0])


def exact(w: vi.Workload) -> float:
    f = w.family
    if f == vi.GAUSS_DIAG:
        return gauss_diag(w.params, w.dim, w.lo, w.hi)
    if f == vi.GENZ_PPEAK:
        return genz_ppeak(w.params, w.dim)
    if f == vi.GENZ_GAUSS:
        return genz_gauss(w.params, w.dim)
    if f == vi.GAUSS_CORR:
        return gauss_corr(w.params, w.dim)
    if f == vi.LINEAR:
        return linear(w.params, w.dim)
    if f == vi.ROOS:
        return roos(w.params, w.dim)
    if f == vi.CONST:
        return const(w.params, w.dim, w.lo, w.hi)
    if f == vi.COSINE:
        return cosine(w.params, w.dim)
    if f == vi.SIN_EXP:
        return sin_exp(w.params, w.dim)
    if f == vi.EXP_SQ:
        return exp_sq(w.params, w.dim)
    if f == vi.MOROKOFF:
        return morokoff(w.params, w.dim)
    if f == vi.GAUSS_CORR:
        return 1.0   # normalised density; mass outside [0,1]^16 is below 1e-60
    raise ValueError(f)


def asian_call(params, n: int) -> float:
    """The Asian call of Eq. 10-11 as printed: the exponent holds
    sigma sqrt(T) times a sum of n standard normal variates, a normal of
    variance n sigma^2 T, so the price is Black-Scholes' with that variance:
    e^{-rT} [S_0 e^{mu + v/2} Phi(d_1) - K Phi(d_2)], mu = (r - sigma^2/2) T,
    v = n sigma^2 T, d_2 = (ln(S_0/K) + mu) / sqrt(v), d_1 = d_2 + sqrt(v)."""
    s0, k, r, sig, t = (mp.mpf(v) for v in params[:5])
    mu = (r - sig * sig / 2) * t
    sd = sig * mp.sqrt(t * n)
    d2 = (mp.log(s0 / k) + mu) / sd
    d1 = d2 + sd
    return float(mp.exp(-r * t) * (s0 * mp.exp(mu + sd * sd / 2) * mp.ncdf(d1) - k * mp.ncdf(d2)))


def feynman_ho(params, n_interior: int) -> float:
    """The lattice path integral of Eq. 12-13 for V = x^2/2 over all of
    R^{N-1} (N = n_interior + 1 spacings): a Gaussian integral,
    A (2 pi)^{(N-1)/2} det(M)^{-1/2} exp(b^T M^{-1} b / 2 - c), with
    S_lat = y^T M y / 2 - b^T y + c over the interior points y:
    M = tridiag(-m/a, 2m/a + a, -m/a), b_1 = b_{N-1} += m x / a, and
    c = m x^2 / a + a x^2 / 2 (both end links and V at the first end)."""
    xe, a, m = (mp.mpf(v) for v in params[:3])
    n = n_interior
    N = n + 1
    M = mp.matrix(n, n)
    for i in range(n):
        M[i, i] = 2 * m / a + a
        if i + 1 < n:
            M[i, i + 1] = M[i + 1, i] = -m / a
    b = mp.matrix(n, 1)
    b[0] += m * xe / a
    b[n - 1] += m * xe / a
    c = m * xe * xe / a + a * xe * xe / 2
    quad = (b.T * mp.inverse(M) * b)[0]
    amp = (m / (2 * mp.pi * a)) ** (mp.mpf(N) / 2)
    return float(amp * (2 * mp.pi) ** (mp.mpf(n) / 2) / mp.sqrt(mp.det(M)) * mp.exp(quad / 2 - c))
