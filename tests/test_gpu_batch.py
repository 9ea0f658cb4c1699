"""The persistent batch schedule on the GPU against the CPU oracle, through
the C ABI (the streams schedule has tests of its own).

* first iteration of every problem of a batch: I_0 and sigma_0^2 within
  1e-12 relative of the oracle (FP64), the refined map within 1e-12, the
  new allocation equal up to the rounding of per-cube variances
* the first iteration is the same bit for bit on every run
* whole runs: per-problem z-scores against the closed forms (no |z| > 5, the
  rate of |z| > 3 consistent with a normal tail)
* compensated FP32 accumulation against FP64 accumulation
* the autotuner's cache
* the batched workload at its full size (4096 problems, budgets 1e4..1e7):
  sampled problems against the oracle, z-scores of all of them
All inputs come from vegas_inputs; every expected value from oracle/ or the
closed forms.
"""
import math
import sys

import numpy as np
import pytest

import vegas_inputs as vi
from tests import closed_forms as cf

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the persistent batch schedule is switched off: its first device run ended "
                                      "in a memory fault whose cause is not yet found (vegas_batch_create returns "
                                      "VEGAS_EUNSUPPORTED for it)")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def exact(x: vi.BatchInstance) -> float:
    if x.family == vi.GENZ_PPEAK:
        return cf.genz_ppeak(x.params, x.dim)
    if x.family == vi.GENZ_GAUSS:
        return cf.genz_gauss(x.params, x.dim)
    return cf.gauss_diag(x.params, x.dim)


def configs(insts, *, n_g=vi.BATCH_N_G, precision="f64", accum="fp64", max_iter=16):
    from paper_2408_09229_amd import make_config
    return [make_config(x.dim, n_g, x.n_eval, seed=0, instance=i, precision=precision, accum=accum,
                        max_iter=max_iter) for i, x in enumerate(insts)]


def make_batch(insts, **kw):
    from paper_2408_09229_amd import VegasBatch
    tune = kw.pop("tune_cache", None)
    return VegasBatch(configs(insts, **kw), [(x.family, x.params) for x in insts], schedule="persistent",
                      tune_cache=tune)


def small_batch(n=24, seed=1, hi=2e5):
    insts = vi.genz_batch(n, seed=seed, budget_lo=1e4, budget_hi=hi)
    # one GAUSS_DIAG problem as well (the third batched family)
    insts.append(vi.BatchInstance(vi.GAUSS_DIAG, 4, vi.gauss_diag_params(1.0, 0.1, [0.4, 0.6]), 60_013))
    return insts


def binom_sf(k, n, p):
    """P(X >= k), X ~ Binomial(n, p)."""
    return 1.0 - sum(math.comb(n, j) * p ** j * (1 - p) ** (n - j) for j in range(k))


def z_stats(res, insts):
    z = np.array([(r["integral"] - exact(x)) / math.sqrt(r["sigma2"]) for r, x in zip(res, insts)])
    return z


@pytest.mark.parametrize("layout", [(8, 1 << 18), (2, 1 << 16)], ids=["pl8_item256k", "pl2_item64k"])
def test_batch_first_iteration_parity(orc, layout):
    insts = small_batch()
    say(f"[batch parity] n={len(insts)} layout={layout}")
    b = make_batch(insts)
    b.set_layout(*layout)
    b.adapt(1)
    for i, x in enumerate(insts):
        o = orc.run(x.dim, vi.BATCH_N_G, x.n_eval, x.family, x.params, n_adapt=0, n_iter=1, seed=0, inst=i)
        I, s2 = b.get_iterations(i)
        assert I.size == 1
        assert abs(I[0] - o.I_t[0]) <= 1e-12 * abs(o.I_t[0]), (i, I[0], o.I_t[0])
        assert abs(s2[0] - o.s2_t[0]) <= 1e-12 * abs(o.s2_t[0]), (i, s2[0], o.s2_t[0])
        g = b.get_map(i)
        assert np.max(np.abs(g - o.grid)) <= 1e-12, (i, np.max(np.abs(g - o.grid)))
        nh = b.get_nh(i, o.nh.size)
        assert int(nh.sum()) == x.n_eval and nh.min() >= 2
        # v_h are sums in another order: n_h may move by one where Q_h rounds
        d = np.abs(nh.astype(np.int64) - o.nh.astype(np.int64))
        assert d.max() <= 2 and np.mean(d != 0) <= 1e-2, (i, d.max(), np.mean(d != 0))


def test_batch_reproducible():
    """The first iteration's estimates do not depend on which workgroup took
    which item (later iterations follow maps refined from LDS atomic sums,
    whose last bits follow the order of the adds)."""
    insts = small_batch(12, seed=2)
    say("[batch reproducible]")
    runs = []
    for _ in range(2):
        b = make_batch(insts, precision="f32")
        b.set_layout(4, 1 << 16)
        b.adapt(1)
        runs.append([np.concatenate(b.get_iterations(i)) for i in range(len(insts))])
        b.close()
    for a, c in zip(*runs):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_closed_form(precision):
    insts = vi.genz_batch(256, seed=3, budget_lo=1e4, budget_hi=1e5)
    say(f"[batch closed form] {precision} n={len(insts)}")
    b = make_batch(insts, precision=precision)
    b.adapt(vi.BATCH_ADAPT)
    b.integrate(vi.BATCH_ITER)
    res = b.results()
    z = z_stats(res, insts)
    assert np.all(np.isfinite(z))
    k = int(np.sum(np.abs(z) > 3))
    say(f"  max|z| {np.abs(z).max():.2f}, |z|>3: {k}/{z.size}")
    assert np.abs(z).max() < 5
    assert binom_sf(k, z.size, 0.0027) > 1e-3


def test_batch_kahan():
    insts = small_batch(16, seed=4)[:-1]
    say("[batch kahan]")
    out = {}
    for acc in ("fp64", "kahan"):
        b = make_batch(insts, precision="f32", accum=acc)
        b.adapt(1)
        out[acc] = [b.get_iterations(i) for i in range(len(insts))]
        b.close()
    for (I64, s64), (Ik, sk) in zip(out["fp64"], out["kahan"]):
        assert abs(Ik[0] - I64[0]) <= 1e-6 * abs(I64[0])
        assert abs(sk[0] - s64[0]) <= 1e-4 * abs(s64[0])


def test_batch_autotune_cache(tmp_path):
    insts = small_batch(8, seed=5)
    path = tmp_path / "tune.txt"
    say("[batch autotune]")
    b = make_batch(insts, precision="f32", tune_cache=str(path))
    inf = b.info()
    assert inf.tuned == 1 and inf.tune_ms > 0
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    b.adapt(2)
    assert all(np.all(np.isfinite(b.get_iterations(i)[0])) for i in range(len(insts)))
    b.close()
    b2 = make_batch(insts, precision="f32", tune_cache=str(path))
    inf2 = b2.info()
    assert inf2.tuned == 2
    assert (inf2.per_lane, inf2.item_samples) == (inf.per_lane, inf.item_samples)
    assert len(path.read_text().splitlines()) == 1


def test_batch_rejects():
    from paper_2408_09229_amd import VegasError
    insts = small_batch(2)
    cfgs = configs(insts)
    cfgs[1].precision = 1                  # mixed precision
    from paper_2408_09229_amd import VegasBatch
    with pytest.raises(VegasError):
        VegasBatch(cfgs, [(x.family, x.params) for x in insts], schedule="persistent")
    b = make_batch(insts)
    b.adapt(1)
    with pytest.raises(VegasError):
        b.set_layout(4, 1 << 16)           # layout fixed after the first iteration
    with pytest.raises(VegasError):
        make_batch(insts).set_layout(3, 1000)


def test_batch_full_size(orc):
    """The batched workload at its full size, as the benchmark runs it."""
    insts = vi.genz_batch(4096, seed=0)
    say(f"[batch full] n={len(insts)} evals/iter={sum(x.n_eval for x in insts):.3e}")
    b = make_batch(insts, precision=vi.BATCH_PRECISION)
    b.adapt(vi.BATCH_ADAPT)
    b.integrate(vi.BATCH_ITER)
    res = b.results()
    # sampled problems: first iteration against the oracle (FP32 sample path:
    # the same samples and bins, f and J to FP32 rounding)
    # (product-peak values and low-dimensional Gaussians stay far from the
    # FP32 underflow that the oracle's FP64 would resolve)
    small = sorted(range(len(insts)), key=lambda i: insts[i].n_eval)
    pp = [i for i in small if insts[i].family == vi.GENZ_PPEAK]
    gg = [i for i in small if insts[i].family == vi.GENZ_GAUSS and insts[i].dim <= 4]
    picks = pp[:3] + gg[:2] + [pp[len(pp) // 2]]
    for i in picks:
        x = insts[i]
        o = orc.run(x.dim, vi.BATCH_N_G, x.n_eval, x.family, x.params, n_adapt=0, n_iter=1, seed=0, inst=i)
        I, s2 = b.get_iterations(i)
        say(f"  inst {i} d={x.dim} n={x.n_eval}: I0 {I[0]:.10e} oracle {o.I_t[0]:.10e}")
        assert abs(I[0] - o.I_t[0]) <= 1e-4 * abs(o.I_t[0])
        assert abs(s2[0] - o.s2_t[0]) <= 1e-3 * abs(o.s2_t[0])
    z = z_stats(res, insts)
    k = int(np.sum(np.abs(z) > 3))
    say(f"  max|z| {np.abs(z).max():.2f}, |z|>3: {k}/{z.size}")
    assert np.all(np.isfinite(z))
    assert np.abs(z).max() < 5
    assert binom_sf(k, z.size, 0.0027) > 1e-3
