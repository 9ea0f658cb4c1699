"""CPU FP64 oracle for the VEGAS+ iteration -- TEST INFRASTRUCTURE ONLY.

A ctypes view of ``oracle/vegas_oracle.c``.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import this module; the HIP library
and its Python binding never do.  Each function documents the passage of the
paper it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("VEGAS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_u32p = C.POINTER(C.c_uint32)
_i64p = C.POINTER(C.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: F401  (oracle/build.py)
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.orc_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_int]
    lib.orc_word.restype = C.c_uint32
    lib.orc_det_log.argtypes = [C.c_double]
    lib.orc_det_log.restype = C.c_double
    lib.orc_det_exp.argtypes = [C.c_double]
    lib.orc_det_exp.restype = C.c_double
    lib.orc_strata.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_int, _i64p, _i64p, _i64p]
    lib.orc_strata.restype = C.c_int
    lib.orc_point.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _u32p, _dp]
    lib.orc_integrand.argtypes = [C.c_int, C.c_int, _dp, _dp]
    lib.orc_integrand.restype = C.c_double
    lib.orc_alloc_weight.argtypes = [C.c_double, C.c_double]
    lib.orc_alloc_weight.restype = C.c_double
    lib.orc_alloc.argtypes = [_dp, C.c_int64, C.c_int, C.c_int64, C.c_double, C.c_int, _u32p]
    lib.orc_map_update_axis.argtypes = [_dp, C.c_int, _dp, _dp, C.c_double]
    lib.orc_combine.argtypes = [_dp, _dp, C.c_int, _dp, _dp, _dp]
    lib.orc_iterate.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_int64,
                                C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, _dp,
                                _dp, _u32p, _dp, _dp, _dp, _dp, _dp, _dp, _i64p]
    lib.orc_iterate.restype = C.c_int
    lib.orc_sample.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_uint64, C.c_uint32,
                               C.c_uint32, C.c_uint64, C.c_int64, _dp, C.c_int, _dp,
                               _u32p, _dp, _dp, _dp, _dp]
    lib.orc_init_grid.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
    lib.orc_run.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_double,
                            C.c_double, C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int,
                            _dp, _dp, _dp, C.c_int, C.c_int, _dp, _u32p, C.c_uint32,
                            _dp, _dp, _dp, _i64p]
    lib.orc_run.restype = C.c_int
    _lib = lib
    return lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(t))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


# --------------------------------------------------------------------------
# step functions
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    lib = _load()
    c = _u32(ctr)
    k = _u32(key)
    out = np.zeros(4, np.uint32)
    lib.orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def word(seed, inst, t, k, d) -> int:
    return int(_load().orc_word(seed, inst, t, k, d))


def det_log(x: float) -> float:
    return _load().orc_det_log(float(x))


def det_exp(x: float) -> float:
    return _load().orc_det_exp(float(x))


def strata(n_eval: int, dim: int, n_min: int = 2, n_strat: int = 0):
    """(N_st, N_c, R) or None when the budget cannot cover n_min per cube."""
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    rc = _load().orc_strata(n_eval, dim, n_min, n_strat, C.byref(a), C.byref(b), C.byref(c))
    if rc != 0:
        return None
    return a.value, b.value, c.value


def point(s: int, r: int, n_strat: int, n_g: int):
    b = C.c_uint32()
    dl = C.c_double()
    _load().orc_point(s, r, n_strat, n_g, C.byref(b), C.byref(dl))
    return b.value, dl.value


def integrand(family: int, x, params) -> float:
    x = _f64(x)
    p = _f64(params)
    return _load().orc_integrand(family, x.size, _p(p, C.c_double), _p(x, C.c_double))


def alloc_weight(v: float, beta: float) -> float:
    return _load().orc_alloc_weight(float(v), float(beta))


def alloc(v, n_min: int, n_eval: int, beta: float, adapt: bool = True):
    v = _f64(v)
    nh = np.zeros(v.size, np.uint32)
    _load().orc_alloc(_p(v, C.c_double), v.size, n_min, n_eval, beta, int(adapt),
                      _p(nh, C.c_uint32))
    return nh


def map_update_axis(x, H, Cn, alpha: float):
    x = _f64(x).copy()
    H = _f64(H)
    Cn = _f64(Cn)
    _load().orc_map_update_axis(_p(x, C.c_double), H.size, _p(H, C.c_double),
                                _p(Cn, C.c_double), alpha)
    return x


def map_update(grid, H, Cn, alpha: float):
    grid = _f64(grid)
    out = np.empty_like(grid)
    for d in range(grid.shape[0]):
        out[d] = map_update_axis(grid[d], H[d], Cn[d], alpha)
    return out


def combine(I, s2):
    I = _f64(I)
    s2 = _f64(s2)
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _load().orc_combine(_p(I, C.c_double), _p(s2, C.c_double), I.size,
                        C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def init_grid(dim: int, n_g: int, lo=None, hi=None):
    lo = _f64(np.zeros(dim) if lo is None else lo)
    hi = _f64(np.ones(dim) if hi is None else hi)
    g = np.zeros((dim, n_g + 1), np.float64)
    _load().orc_init_grid(dim, n_g, _p(lo, C.c_double), _p(hi, C.c_double), _p(g, C.c_double))
    return g


@dataclass
class IterOut:
    I: float
    s2: float
    m: np.ndarray
    v: np.ndarray
    H: np.ndarray
    C: np.ndarray
    n_nonfinite: int


def iterate(dim, n_g, n_eval, n_strat, n_cubes, seed, inst, t, family, params,
            grid, nh) -> IterOut:
    """One iteration over a given map and allocation (Alg. 1 body, Alg. 2)."""
    p = _f64(params)
    g = _f64(grid)
    nh = _u32(nh)
    m = np.zeros(n_cubes)
    v = np.zeros(n_cubes)
    H = np.zeros((dim, n_g))
    Cn = np.zeros((dim, n_g))
    I, s2 = C.c_double(), C.c_double()
    bad = C.c_int64()
    rc = _load().orc_iterate(dim, n_g, n_eval, n_strat, n_cubes, seed, inst, t, family,
                             _p(p, C.c_double), _p(g, C.c_double), _p(nh, C.c_uint32),
                             _p(m, C.c_double), _p(v, C.c_double), _p(H, C.c_double),
                             _p(Cn, C.c_double), C.byref(I), C.byref(s2), C.byref(bad))
    if rc != 0:
        raise ValueError(f"oracle iterate rejected its inputs (rc={rc})")
    return IterOut(I.value, s2.value, m, v, H, Cn, bad.value)


def sample(dim, n_g, n_strat, seed, inst, t, k, h, grid, family, params):
    g = _f64(grid)
    p = _f64(params)
    bins = np.zeros(dim, np.uint32)
    delta = np.zeros(dim)
    x = np.zeros(dim)
    J, f = C.c_double(), C.c_double()
    _load().orc_sample(dim, n_g, n_strat, seed, inst, t, k, h, _p(g, C.c_double), family,
                       _p(p, C.c_double), _p(bins, C.c_uint32), _p(delta, C.c_double),
                       _p(x, C.c_double), C.byref(J), C.byref(f))
    return bins, delta, x, J.value, f.value


@dataclass
class RunOut:
    I_t: np.ndarray
    s2_t: np.ndarray
    integral: float
    sigma2: float
    chi2_dof: float
    grid: np.ndarray
    nh: np.ndarray
    n_nonfinite: int


def run(dim, n_g, n_eval, family, params, *, n_adapt=0, n_iter=1, alpha=0.5, beta=0.75,
        seed=0, inst=0, n_min=2, n_strat=0, adapt_map=True, adapt_strat=True,
        lo=None, hi=None, grid=None, nh=None, t0=0) -> RunOut:
    """Alg. 1: n_adapt discarded iterations, then n_iter combined by Eq. 8-9."""
    st = strata(n_eval, dim, n_min, n_strat)
    if st is None:
        raise ValueError("budget too small for the strata")
    _, nc, _ = st
    lo = _f64(np.zeros(dim) if lo is None else lo)
    hi = _f64(np.ones(dim) if hi is None else hi)
    g = _f64(init_grid(dim, n_g, lo, hi) if grid is None else grid).copy()
    if nh is None:
        nh = alloc(np.zeros(nc), n_min, n_eval, beta, adapt=False)
    nh = _u32(nh).copy()
    p = _f64(params)
    tot = n_adapt + n_iter
    I_t = np.zeros(tot)
    s2_t = np.zeros(tot)
    res = np.zeros(3)
    bad = C.c_int64()
    rc = _load().orc_run(dim, n_g, n_eval, n_min, n_strat, alpha, beta, seed, inst,
                         int(adapt_map), int(adapt_strat), family, _p(p, C.c_double),
                         _p(lo, C.c_double), _p(hi, C.c_double), n_adapt, n_iter,
                         _p(g, C.c_double), _p(nh, C.c_uint32), t0,
                         _p(I_t, C.c_double), _p(s2_t, C.c_double), _p(res, C.c_double),
                         C.byref(bad))
    if rc != 0:
        raise ValueError(f"oracle run rejected its inputs (rc={rc})")
    return RunOut(I_t, s2_t, res[0], res[1], res[2], g, nh, bad.value)
