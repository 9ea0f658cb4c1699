"""The learned warp on the GPU against the CPU flow oracle, through the C ABI.

* the BF16 MFMA lane layout the kernels assume (one product against numpy)
* sampling pass: w = F(y) and log J_F of every sample against the oracle's
  forward pass with BF16 emulation, y rebuilt from the oracle's Philox words
* the identity warp gives the plain iteration's estimate
* a fixed, non-trivial warp keeps the estimate unbiased (closed form)
All inputs are seeded; expected values come from oracle/ or closed forms.
"""
import math
import sys

import numpy as np
import pytest

import vegas_inputs as vi
from oracle import flow as fl
from tests import closed_forms as cf

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def random_theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    th = fl.init_params(16, seed)
    for L in fl.unpack(th, 16):
        L["W3"][...] = rng.normal(0, scale, L["W3"].shape)
        L["b3"][...] = rng.normal(0, 0.3, L["b3"].shape)
        L["b1"][...] = rng.normal(0, 0.1, L["b1"].shape)
    return th


def make(w, **kw):
    from paper_2408_09229_amd import Vegas, make_config
    cfg = make_config(w.dim, w.n_g, w.n_eval, n_strat=w.n_strat, n_min=w.n_min, alpha=w.alpha, beta=w.beta,
                      seed=w.seed, precision="f32", **kw)
    return Vegas(cfg, w.family, w.params, w.lo, w.hi)


def corr16(n_eval=20_011, n_g=32):
    return vi.Workload("corr16_flow", 16, vi.GAUSS_CORR, np.array([0.5, 0.2, 0.5]), n_g=n_g, n_eval=n_eval,
                       n_iter=1, precision="f32")


def test_mfma_layout():
    from paper_2408_09229_amd._binding import mfma_probe
    rng = np.random.default_rng(0)
    A = rng.normal(size=(32, 16))
    B = rng.normal(size=(16, 32))
    D = mfma_probe(A, B)
    want = fl.bf16(A) @ fl.bf16(B)
    assert np.max(np.abs(D - want)) < 1e-4 * max(1.0, np.abs(want).max())


def oracle_y(orc, w, nh, t, ks):
    """Stratified points of samples ks (FP64, by definition)."""
    ns, nc, _ = orc.strata(w.n_eval, w.dim, w.n_min, w.n_strat)
    start = np.concatenate([[0], np.cumsum(nh.astype(np.int64))])
    ys = np.zeros((len(ks), w.dim))
    for i, k in enumerate(ks):
        h = int(np.searchsorted(start, k, side="right") - 1)
        for d in range(w.dim):
            s = h % ns
            h //= ns
            r = orc.word(w.seed, 0, t, int(k), d)
            ys[i, d] = (s + (2.0 * r + 1.0) / 2.0 ** 33) / ns
    return ys


def test_flow_sample_parity(orc):
    w = corr16()
    say("[flow sample]")
    v = make(w)
    th = random_theta(1)
    v.attach_flow(th.astype(np.float32))
    v.enable_flow(True)
    nh = v.get_nh()
    v.adapt(1)
    W, LJ, OM = v.flow_samples()
    ks = np.random.default_rng(2).choice(w.n_eval, 1500, replace=False)
    ys = oracle_y(orc, w, nh, 0, ks)
    # the oracle in FP64 with the GPU's BF16 roundings, from the FP32 params
    wo, ljo = fl.forward(th.astype(np.float32).astype(np.float64), ys, emu=True)
    dw = np.abs(W[ks] - wo).max(axis=1)
    dl = np.abs(LJ[ks] - ljo)
    say(f"  |dw| median {np.median(dw):.2e} p95 {np.percentile(dw, 95):.2e} max {dw.max():.2e}; "
        f"|dlj| median {np.median(dl):.2e} max {dl.max():.2e}")
    assert np.median(dw) < 1e-6 and np.percentile(dw, 95) < 2e-5 and dw.max() < 1e-2
    assert np.median(dl) < 1e-5 and np.percentile(dl, 95) < 1e-4 and dl.max() < 0.1
    assert np.all(np.isfinite(OM))
    v.close()


def test_identity_warp_equals_plain():
    w = corr16()
    say("[flow identity]")
    a = make(w)
    b = make(w)
    b.attach_flow(fl.init_params(16, 0).astype(np.float32))
    b.enable_flow(True)
    a.adapt(1)
    b.adapt(1)
    Ia, sa = a.get_iterations()
    Ib, sb = b.get_iterations()
    assert abs(Ia[0] - Ib[0]) <= 1e-4 * abs(Ia[0]), (Ia[0], Ib[0])
    assert abs(sa[0] - sb[0]) <= 1e-3 * sa[0], (sa[0], sb[0])
    a.close()
    b.close()


def test_fixed_warp_unbiased():
    """A fixed non-trivial warp, a product Gaussian in 16-d (closed form)."""
    s = 0.2
    w = vi.Workload("gauss16_flow", 16, vi.GAUSS_DIAG, vi.gauss_diag_params(vi.normal_peak(s, 16), s, [0.5]),
                    n_g=64, n_eval=400_000, n_iter=5, precision="f32")
    say("[flow unbiased]")
    v = make(w)
    v.attach_flow(random_theta(5, scale=0.2).astype(np.float32))
    v.enable_flow(True)
    v.adapt(4)
    v.integrate(w.n_iter)
    r = v.result()
    exact = cf.exact(w)
    say(f"  {r.integral:.6f} +- {math.sqrt(r.sigma2):.2e} (exact {exact:.6f})")
    assert abs(r.integral - exact) < 3.0 * math.sqrt(r.sigma2)
    v.close()


def test_flow_grad_parity():
    """GPU gradient of the warp's loss against the oracle with BF16
    emulation, per layer (relative L2)."""
    w = corr16()
    say("[flow grad]")
    v = make(w)
    th = random_theta(3).astype(np.float32)
    v.attach_flow(th)
    v.enable_flow(True)
    v.adapt(1)
    W, LJ, OM = v.flow_samples()
    g_gpu = v.flow_grad().astype(np.float64)
    om = OM.astype(np.float64)
    coef = om * om / np.sum(om * om)
    _, g_orc = fl.loss_grad(th.astype(np.float64), W.astype(np.float64), coef, emu=True)
    n = fl.n_params(16) // 4
    for l in range(4):
        a, b = g_gpu[l * n:(l + 1) * n], g_orc[l * n:(l + 1) * n]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(f"  layer {l}: |g| {np.linalg.norm(b):.3e} rel L2 {rel:.2e}")
        assert rel < 2e-2
    v.close()


def test_flow_training_gain():
    """Trained warp against plain VEGAS+ on a correlated 16-d Gaussian
    (s 0.2, rho 0.5): after 100 training steps the median iteration variance
    at equal evaluations is below 0.6 of plain VEGAS+, the judge keeps the
    warp, and the combined
    warped and plain estimates agree."""
    w = vi.Workload("corr16_train", 16, vi.GAUSS_CORR, np.array([0.5, 0.2, 0.5]), n_g=64, n_eval=200_003,
                    n_iter=1, precision="f32")
    say("[flow train]")
    v = make(w)
    v.adapt(6)
    v.integrate(10)
    plain = v.result()
    v.attach_flow(fl.init_params(16, 0).astype(np.float32), lr=3e-4, train=True, judge=True)
    v.enable_flow(True)
    v.adapt(100)
    I, s2 = v.get_iterations()
    on, kept, rejected = v.flow_status()
    plain_s2 = np.median(s2[6:16])
    warped_s2 = np.median(s2[-10:])
    say(f"  plain median sigma^2 {plain_s2:.3e}, warped (last 10) {warped_s2:.3e}, ratio "
        f"{warped_s2 / plain_s2:.3f}; judge kept {kept} rejected {rejected}, on={on}")
    assert on and kept >= 80
    assert warped_s2 < 0.6 * plain_s2
    Iw = np.sum(I[-10:] / s2[-10:]) / np.sum(1 / s2[-10:])
    sw = 1.0 / np.sum(1 / s2[-10:])
    assert abs(Iw - plain.integral) < 4.0 * math.sqrt(sw + plain.sigma2), (Iw, plain.integral)
    v.close()


def test_flow_judge_falls_back():
    """A badly scaled fixed warp: the judge rejects it three times, switches
    it off, and plain VEGAS+ carries on."""
    w = vi.Workload("corr16_judge", 16, vi.GAUSS_CORR, np.array([0.5, 0.2, 0.5]), n_g=64, n_eval=100_003,
                    n_iter=1, precision="f32")
    say("[flow judge]")
    v = make(w)
    v.adapt(6)
    v.attach_flow(random_theta(9, scale=30.0).astype(np.float32), judge=True)
    v.enable_flow(True)
    v.adapt(6)
    on, kept, rejected = v.flow_status()
    say(f"  kept {kept} rejected {rejected} on={on}")
    assert not on and rejected >= 3
    v.integrate(3)
    r = v.result()
    assert math.isfinite(r.integral) and r.sigma2 > 0
    v.close()
