"""The paper's two application integrands (Sec. 4.5-4.6) as device sources
for run-time compilation (UserIntegrand), with their parameter layouts.

Both are written in FP64 (``vegas_real`` is double when compiled with
precision "f64").

* Asian call option (Sec. 4.5.1, Eq. 10-11), ``dim`` = the number of
  normal variates n:
  f(x) = e^{-rT} max(S_avg(x) - K, 0),
  S_avg(x) = S_0 exp((r - sigma^2/2) T + sigma sqrt(T) sum_i sqrt(2) erfinv(2 x_i - 1)),
  x in (0,1)^n, params [S_0, K, r, sigma, T].  Each sqrt(2) erfinv(2 x_i - 1)
  is a standard normal variate of x_i, so the sum is normal with variance n
  and the integral has a Black-Scholes form (its closed form is in the
  tests).  The formula is taken as printed: the exponent sums n variates
  with weight sigma sqrt(T) each.
* Feynman path integral of the harmonic oscillator (Sec. 4.6, Eq. 12-13),
  ``dim`` = N - 1 interior lattice points x_1 .. x_{N-1} of a path with
  both ends at x:
  f(x_1..x_{N-1}) = A exp(-S_lat),
  S_lat = sum_{j=0}^{N-1} (m/(2a) (x_{j+1} - x_j)^2 + a x_j^2 / 2),
  x_0 = x_N = x, a = T/N, A = (m / (2 pi a))^{N/2},
  params [x, a, m], over the box [-L, L]^{N-1} (the infinite domain cut
  where the integrand is negligible: L = 5 by default).
"""
from __future__ import annotations

import numpy as np

ASIAN_CALL = r"""
// Asian call option: params [S0, K, r, sigma, T]
__device__ vegas_real vegas_user_f(const vegas_real* x, int dim, const double* p)
{
    const double s0 = p[0], strike = p[1], r = p[2], sigma = p[3], t = p[4];
    double z = 0.0;
    for (int i = 0; i < dim; ++i) z += 1.4142135623730951 * erfinv(2.0 * (double)x[i] - 1.0);
    const double s_avg = s0 * exp((r - 0.5 * sigma * sigma) * t + sigma * sqrt(t) * z);
    const double pay = s_avg > strike ? s_avg - strike : 0.0;
    return (vegas_real)(exp(-r * t) * pay);
}
"""

FEYNMAN_HO = r"""
// harmonic-oscillator path integral on a lattice: params [x_end, a, m]
__device__ vegas_real vegas_user_f(const vegas_real* x, int dim, const double* p)
{
    const double xe = p[0], a = p[1], m = p[2];
    const int n = dim + 1;                       // lattice spacings
    double s = 0.0, prev = xe;
    for (int j = 0; j < n; ++j) {
        const double cur = j + 1 < n ? (double)x[j] : xe;
        const double d = cur - prev;
        s += 0.5 * m / a * d * d + 0.5 * a * prev * prev;
        prev = cur;
    }
    const double amp = pow(m / (6.283185307179586 * a), 0.5 * (double)n);
    return (vegas_real)(amp * exp(-s));
}
"""


def asian_params(s0: float = 100.0, strike: float = 100.0, r: float = 0.05, sigma: float = 0.2,
                 t: float = 1.0) -> np.ndarray:
    return np.array([s0, strike, r, sigma, t], dtype=np.float64)


def feynman_params(x_end: float = 0.0, t: float = 4.0, n: int = 8, m: float = 1.0) -> np.ndarray:
    """[x, a, m] for a path of n lattice spacings over Euclidean time t."""
    return np.array([x_end, t / n, m], dtype=np.float64)


def feynman_box(n: int = 8, half_width: float = 5.0):
    """(lo, hi) of the integration box of the n - 1 interior points."""
    return np.full(n - 1, -half_width), np.full(n - 1, half_width)
