"""The C-ABI library loads and exports every entry point of include/vegas.h,
and its host-side validation (vegas_workspace_size makes no HIP call)
accepts the workloads and rejects bad configurations.  CPU only."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import vegas_inputs as vi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vegas.h")).read()
    return sorted(set(re.findall(r"\b(vegas_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def abi():
    from paper_2408_09229_amd import abi
    return abi


def test_exports_every_declared_symbol(abi):
    names = _declared()
    assert len(names) >= 20
    lib = C.CDLL(abi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(abi.EXPORTED)


def _size(abi, w, **kw):
    cfg = abi.make_config(w.dim, w.n_g, w.n_eval, alpha=w.alpha, beta=w.beta, seed=w.seed,
                          precision=w.precision, **kw)
    return abi.workspace_size(cfg, w.family, w.params, w.lo, w.hi)


@pytest.mark.parametrize("w", [vi.gauss_prod_4d(), vi.gauss3_8d(), vi.ridge_4d(), vi.corr_gauss_16d()],
                         ids=lambda w: w.name)
def test_workloads_validate(abi, w):
    n = _size(abi, w)
    assert n > 0
    # per-cube arrays dominate: at least start x2 + v
    st = __import__("oracle").strata(w.n_eval, w.dim)
    assert n >= st[1] * (4 + 4 + 8)


@pytest.mark.parametrize("change,status", [
    (dict(dim=0), -1), (dict(dim=17), -1), (dict(n_intervals=0), -1), (dict(n_eval=1), -1),
    (dict(n_min=1), -1), (dict(alpha=-0.1), -1), (dict(beta=float("nan")), -1),
    (dict(accum=1), -1), (dict(accum=7), -1), (dict(n_intervals=8192), -1), (dict(instance=1 << 24), -1),
])
def test_config_rejected(abi, change, status):
    w = vi.gauss_prod_4d()
    base = dict(dim=w.dim, n_intervals=w.n_g, n_eval=w.n_eval, n_strat=0, n_min=2, alpha=0.5, beta=0.75,
                seed=0, instance=0, precision=0, accum=0, adapt_map=1, adapt_strat=1, max_iter=0)
    base.update(change)
    cfg = abi.vegas_config(**base)
    it = abi._Integrand(w.family, w.params)
    n = C.c_size_t()
    st = abi.vegas_workspace_size(C.byref(cfg), C.byref(it.s), C.byref(n))
    assert st == status, abi.vegas_last_error()


def test_integrand_rejected(abi):
    cfg = abi.make_config(3, 8, 1000)
    n = C.c_size_t()
    for fam, p in [(99, [1.0]), (vi.GENZ_PPEAK, [1.0, 2.0]), (vi.GAUSS_DIAG, [1.0, -0.1, 1.0, 0.5]),
                   (vi.GAUSS_CORR, [0.5, 0.1, 1.0]), (vi.LINEAR, [float("inf")])]:
        it = abi._Integrand(fam, np.array(p))
        assert abi.vegas_workspace_size(C.byref(cfg), C.byref(it.s), C.byref(n)) == -1
    it = abi._Integrand(vi.CONST, np.array([1.0]), lo=np.array([0.0, 1.0, 0.0]), hi=np.array([1.0, 1.0, 1.0]))
    assert abi.vegas_workspace_size(C.byref(cfg), C.byref(it.s), C.byref(n)) == -1
    assert b"box" in abi.vegas_last_error()


def test_budget_too_small_for_strata(abi):
    cfg = abi.make_config(2, 4, 3, n_strat=2)      # 4 cubes x 2 samples > 3
    it = abi._Integrand(vi.CONST, np.array([1.0]))
    n = C.c_size_t()
    assert abi.vegas_workspace_size(C.byref(cfg), C.byref(it.s), C.byref(n)) == -1


def test_status_strings(abi):
    for s in range(-6, 1):
        assert abi.vegas_status_string(s)


def test_ordered_limits(abi):
    it = abi._Integrand(vi.CONST, np.array([1.0]))
    n = C.c_size_t()
    ok = abi.make_config(2, 8, 2000, accum="ordered")
    assert abi.vegas_workspace_size(C.byref(ok), C.byref(it.s), C.byref(n)) == 0
    f32 = abi.make_config(2, 8, 2000, accum="ordered", precision="f32")
    assert abi.vegas_workspace_size(C.byref(f32), C.byref(it.s), C.byref(n)) == -1
    big = abi.make_config(2, 1024, 10 ** 7, accum="ordered")
    assert abi.vegas_workspace_size(C.byref(big), C.byref(it.s), C.byref(n)) == -6


def test_kahan_needs_fp32(abi):
    it = abi._Integrand(vi.CONST, np.array([1.0]))
    n = C.c_size_t()
    ok = abi.make_config(3, 16, 5000, accum="kahan", precision="f32")
    assert abi.vegas_workspace_size(C.byref(ok), C.byref(it.s), C.byref(n)) == 0
    bad = abi.make_config(3, 16, 5000, accum="kahan", precision="f64")
    assert abi.vegas_workspace_size(C.byref(bad), C.byref(it.s), C.byref(n)) == -1
