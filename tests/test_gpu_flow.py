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


def random_theta(seed, scale=0.3, bscale=0.3):
    rng = np.random.default_rng(seed)
    th = fl.init_params(16, seed)
    for L in fl.unpack(th, 16):
        L["W3"][...] = rng.normal(0, scale, L["W3"].shape)
        L["b3"][...] = rng.normal(0, bscale, L["b3"].shape)
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
    """Stratified points of samples ks as the warp's sampling pass defines
    them: y = (s 2^33 + 2r + 1) / (N_st 2^33) in FP64 (the numerator is
    exact); s from the cube's digits, r the oracle's Philox word."""
    ns, nc, _ = orc.strata(w.n_eval, w.dim, w.n_min, w.n_strat)
    start = np.concatenate([[0], np.cumsum(nh.astype(np.int64))])
    ys = np.zeros((len(ks), w.dim))
    for i, k in enumerate(ks):
        h = int(np.searchsorted(start, k, side="right") - 1)
        for d in range(w.dim):
            s = h % ns
            h //= ns
            r = orc.word(w.seed, 0, t, int(k), d)
            ys[i, d] = (s * 2.0 ** 33 + (2.0 * r + 1.0)) / (ns * 2.0 ** 33)
    return ys


def roundtrip_bound(y):
    """|Phi(Phi^-1(y)) - y| in FP32 for the warp's sampling pass: min(y,
    1 - y) rounded to FP32 (2^-24 relative), the device's fitted Phi^-1 and
    Phi to 3.5 and about 6 ulps plus the hardware exp2's and reciprocal's
    (16 allowed in all), each relative error of z = Phi^-1(y) moving the tail
    probability m = min(y, 1 - y) by z^2 + 1 times itself at most (the
    tail's log-derivative d ln m / d ln z is about z^2), and the rounding of
    w itself (2^-25 absolute at most)."""
    from scipy.special import ndtri
    m = np.minimum(y, 1.0 - y)
    z = ndtri(m)
    return 16 * 2.0 ** -24 * (z * z + 1.0) * m + 2.0 ** -25


# N_st = 1 (every cube digit 0) and N_st = 2 (2^16 cubes: digits by shifts)
STRATA_CASES = [(20_011, 1), (270_001, 2)]


@pytest.mark.parametrize("n_eval,n_st", STRATA_CASES)
def test_flow_sample_parity(orc, n_eval, n_st):
    w = corr16(n_eval)
    assert orc.strata(w.n_eval, w.dim, w.n_min, w.n_strat)[0] == n_st
    say(f"[flow sample] n_eval {n_eval}, N_st {n_st}")
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


@pytest.mark.parametrize("n_eval,n_st", STRATA_CASES)
def test_library_init_is_identity(orc, n_eval, n_st):
    """The library's own starting weights (no parameters passed): W1 and W2
    inside +-1/sqrt(fan_in) and spread over it, the last layer zero; the warp
    is then the identity: log J_F = 0 exactly, and w = Phi(Phi^-1(y)) in
    FP32 equals y up to the roundings of the two FP32 functions."""
    w = corr16(n_eval)
    assert orc.strata(w.n_eval, w.dim, w.n_min, w.n_strat)[0] == n_st
    say(f"[flow init] n_eval {n_eval}, N_st {n_st}")
    v = make(w)
    v.attach_flow(None, init_seed=7)
    th = v.flow_params().astype(np.float64)
    for L in fl.unpack(th, 16):
        assert np.all(np.abs(L["W1"]) <= 1 / np.sqrt(8)) and np.std(L["W1"]) > 0.5 / np.sqrt(3 * 8)
        assert np.all(np.abs(L["W2"]) <= 1 / 8) and np.std(L["W2"]) > 0.5 / np.sqrt(3 * 64)
        assert np.all(L["W3"] == 0) and np.all(L["b3"] == 0) and np.all(L["b1"] == 0) and np.all(L["b2"] == 0)
    # another seed gives other weights, the same seed the same
    v2 = make(w)
    v2.attach_flow(None, init_seed=8)
    v3 = make(w)
    v3.attach_flow(None, init_seed=7)
    assert not np.array_equal(v2.flow_params(), v.flow_params())
    assert np.array_equal(v3.flow_params(), v.flow_params())
    v.enable_flow(True)
    nh = v.get_nh()
    v.adapt(1)
    W, LJ, _ = v.flow_samples()
    ks = np.random.default_rng(3).choice(w.n_eval, 400, replace=False)
    ys = oracle_y(orc, w, nh, 0, ks)
    dw = np.abs(W[ks].astype(np.float64) - ys)
    say(f"  |w - y| / roundtrip bound: max {np.max(dw / roundtrip_bound(ys)):.3f}")
    assert np.all(dw <= roundtrip_bound(ys))
    assert np.all(LJ == 0.0)
    for x in (v, v2, v3):
        x.close()


def test_identity_warp_equals_plain():
    """The identity warp against the plain iteration on the same samples.
    The warped path's w = Phi(Phi^-1(y)) differs from the plain path's
    exact y by the FP32 round trip (roundtrip_bound), and it splits w N_g
    exactly: per-sample weights agree within the bound that this moves ln f
    by (stated below) wherever the bins agree (bins may differ only where y
    lies within the round trip of an interval end), and the iteration's
    estimate and variance to 1e-5."""
    w = corr16()
    say("[flow identity]")
    a = make(w)
    b = make(w)
    b.attach_flow(None)
    b.enable_flow(True)
    # the plain path's samples of iteration 0, probed before the iteration
    # refines the map and the allocation
    pr = a.probe(0, 0, w.n_eval)
    a.adapt(1)
    b.adapt(1)
    Ia, sa = a.get_iterations()
    Ib, sb = b.get_iterations()
    say(f"  I rel {abs(Ia[0] - Ib[0]) / abs(Ia[0]):.2e}, s2 rel {abs(sa[0] - sb[0]) / sa[0]:.2e}")
    assert abs(Ia[0] - Ib[0]) <= 1e-5 * abs(Ia[0]), (Ia[0], Ib[0])
    assert abs(sa[0] - sb[0]) <= 1e-5 * sa[0], (sa[0], sb[0])
    # the warped iteration's importance-weighted map histograms (weights
    # 1/J_F = 1) refine the map as the plain iteration's counts do
    ga, gb = a.get_map(), b.get_map()
    say(f"  map max |diff| {np.max(np.abs(ga - gb)):.2e}")
    assert np.max(np.abs(ga - gb)) < 1e-5
    W, LJ, OM = b.flow_samples()
    bins_w = np.minimum(np.floor(W.astype(np.float64) * w.n_g), w.n_g - 1).astype(np.int64)
    same = np.all(bins_w == pr["bins"].astype(np.int64), axis=1)
    wp = pr["jac"] * pr["f"]
    rel = np.abs(OM - wp) / np.maximum(np.abs(wp), 1e-300)
    say(f"  bins differ for {np.sum(~same)} of {w.n_eval} samples; weight rel diff max {rel[same].max():.2e}")
    # Bound per sample.  (a) w differs from y by the round trip (|dw| <=
    # roundtrip_bound(y)), which moves x_d by N_g dx_d |dw| (the uniform map
    # of iteration 0 has N_g dx_d = 1 and x = y); each path also rounds its
    # offset and its point x_d < 1 (2^-25 each, the offset's scaled by
    # dx_d < 1), so x_d differs by at most roundtrip_bound + 3 2^-25 and ln f
    # by that times |d ln f / dx_d|, d ln f / dx = -Sigma^-1 (x - mu).  (b) Each path rounds its own FP32
    # evaluation of the exponent e = c1 S + c2 vbar^2 + z (log2 units; S the
    # spread sum_d u_d^2 - (sum_d u_d)^2 / D of u_d = x_d - x_0, vbar the mean
    # offset): S to (D + 2) ulps of its two terms, c2 vbar^2 to 8 ulps,
    # e to 3 ulps, the point and exp2 to 4 more; twice that for two paths.
    mu, s_, rho = w.params
    D = w.dim
    Sig = s_ * s_ * ((1 - rho) * np.eye(D) + rho * np.ones((D, D)))
    x = pr["x"]
    dlnf = (np.abs((x - mu) @ np.linalg.inv(Sig)) * (roundtrip_bound(x) + 3 * 2.0 ** -25)).sum(axis=1)
    c1 = 0.5 / (s_ * s_ * (1 - rho)) / math.log(2)
    c2 = 0.5 * D / (s_ * s_ * (1 + (D - 1) * rho)) / math.log(2)
    u = x[:, 1:] - x[:, :1]
    a1, a2 = u.sum(axis=1), (u * u).sum(axis=1)
    vbar = (x[:, 0] - mu) + a1 / D
    e = c1 * (a2 - a1 * a1 / D) + c2 * vbar * vbar
    ulps = c1 * (D + 2) * (a2 + a1 * a1 / D) + 8 * c2 * vbar * vbar + 3 * np.abs(e) + 4
    tol = dlnf * 1.01 + 2 * 2.0 ** -24 * math.log(2) * ulps
    say(f"  worst weight rel diff / bound {np.max(rel[same] / tol[same]):.2f}")
    assert np.sum(~same) <= 1e-3 * w.n_eval
    assert np.all(rel[same] <= tol[same])
    a.close()
    b.close()


def test_flow_adam_against_oracle():
    """Three Adam steps of the GPU on fixed gradients against the oracle's
    Adam in FP64: every parameter within 4 FP32 ulps of the oracle plus
    1e-5 of the step size."""
    w = corr16()
    say("[flow adam]")
    v = make(w)
    th0 = random_theta(11).astype(np.float32)
    lr = 1e-2
    v.attach_flow(th0, lr=lr)
    rng = np.random.default_rng(12)
    th = th0.astype(np.float64)
    m = np.zeros_like(th)
    vv = np.zeros_like(th)
    for step in range(1, 4):
        g = (rng.normal(size=th.size) * 10.0 ** rng.uniform(-6, 1, size=th.size)).astype(np.float32)
        v.flow_adam_step(g)
        th, m, vv = fl.adam(th, g.astype(np.float64), m, vv, step, lr)
    got = v.flow_params().astype(np.float64)
    tol = 4 * np.spacing(np.abs(th).astype(np.float32)).astype(np.float64) + 1e-5 * lr
    err = np.abs(got - th)
    say(f"  max |err| {err.max():.2e}, worst err/tol {np.max(err / tol):.2f}")
    assert np.all(err <= tol)
    v.close()


def test_fixed_warp_unbiased():
    """A fixed non-trivial warp, a product Gaussian in 16-d (closed form).
    The warp is mild (log-scales and shifts of a few hundredths): a strong
    random warp makes the weights heavy-tailed, and then the iterations'
    own variance estimates, which Eq. 8-9 weighs by, are not reliable."""
    s = 0.2
    w = vi.Workload("gauss16_flow", 16, vi.GAUSS_DIAG, vi.gauss_diag_params(vi.normal_peak(s, 16), s, [0.5]),
                    n_g=64, n_eval=400_000, n_iter=5, precision="f32")
    say("[flow unbiased]")
    v = make(w)
    v.attach_flow(random_theta(5, scale=0.02, bscale=0.05).astype(np.float32))
    v.enable_flow(True)
    v.adapt(4)
    v.integrate(w.n_iter)
    r = v.result()
    exact = cf.exact(w)
    say(f"  {r.integral:.6f} +- {math.sqrt(r.sigma2):.2e} (exact {exact:.6f})")
    assert abs(r.integral - exact) < 3.0 * math.sqrt(r.sigma2)
    v.close()


# 20 011 samples: one chunk of 32 per wave of the gradient kernel (its
# single-chunk variant); 40 009: more chunks than waves (the variant that
# sums several chunks per wave)
@pytest.mark.parametrize("n_eval", [20_011, 40_009])
def test_flow_grad_parity(n_eval):
    """GPU gradient of the warp's loss against the oracle with BF16
    emulation, per layer: relative L2 below 1e-4 (measured 3e-7 to 9e-7;
    FP32 arithmetic against FP64, with the same BF16 operands)."""
    w = corr16(n_eval)
    say(f"[flow grad] n_eval {n_eval}")
    v = make(w)
    th = random_theta(3).astype(np.float32)
    v.attach_flow(th)
    v.enable_flow(True)
    v.adapt(1)
    W, LJ, OM, Z = v.flow_samples(with_z=True)
    g_gpu = v.flow_grad().astype(np.float64)
    om = OM.astype(np.float64)
    coef = om * om / np.sum(om * om)
    _, g_orc = fl.loss_grad(th.astype(np.float64), Z.astype(np.float64), coef, emu=True)
    n = fl.n_params(16) // 4
    for l in range(4):
        a, b = g_gpu[l * n:(l + 1) * n], g_orc[l * n:(l + 1) * n]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(f"  layer {l}: |g| {np.linalg.norm(b):.3e} rel L2 {rel:.2e}")
        assert rel < 1e-4
    v.close()


def test_inplace_copies_equal_full_repack():
    """Training steps write each updated weight's two BF16 copies into the
    packed operands in place; those operands must equal a full repack of
    the same parameters: the loss gradient (which runs on them) is the same
    bit for bit before and after the parameters are loaded again."""
    w = corr16()
    say("[flow in-place repack]")
    v = make(w)
    v.attach_flow(None, lr=1e-2, train=True, steps_per_iter=4, init_seed=5)
    v.enable_flow(True)
    v.adapt(3)
    g1 = v.flow_grad()
    th = v.flow_params()
    v.set_flow_params(th)
    g2 = v.flow_grad()
    assert np.all(np.isfinite(g1)) and np.any(g1 != 0)
    assert np.array_equal(g1, g2)
    v.close()


def test_flow_training_gain():
    """Trained warp against plain VEGAS+ on a correlated 16-d Gaussian
    (s 0.2, rho 0.5), from the library's own starting weights: after 100
    iterations with the guard judge the median variance of the last ten
    warped iterations at equal evaluations is below 0.6 of plain VEGAS+'s,
    the judge keeps the warp, every 16th iteration is a plain control that
    is not combined, and the warped and plain estimates agree."""
    w = vi.Workload("corr16_train", 16, vi.GAUSS_CORR, np.array([0.5, 0.2, 0.5]), n_g=64, n_eval=200_003,
                    n_iter=1, precision="f32")
    say("[flow train]")
    v = make(w)
    v.adapt(6)
    v.integrate(10)
    plain = v.result()
    v.attach_flow(None, lr=3e-4, train=True, judge=1)
    v.enable_flow(True)
    v.adapt(100)
    I, s2 = v.get_iterations()
    kinds = v.flow_kinds()
    on, kept, rejected = v.flow_status()
    assert np.all(kinds[:16] == 0)
    ctrl = np.nonzero(kinds == 2)[0]
    assert np.array_equal(ctrl, 16 + np.arange(15, 100, 16)), ctrl
    warped = np.nonzero(kinds == 1)[0]
    plain_s2 = np.median(s2[6:16])
    warped_s2 = np.median(s2[warped[-10:]])
    say(f"  plain median sigma^2 {plain_s2:.3e}, warped (last 10) {warped_s2:.3e}, ratio "
        f"{warped_s2 / plain_s2:.3f}; judge kept {kept} rejected {rejected}, on={on}")
    assert on and kept >= 80
    assert warped_s2 < 0.6 * plain_s2
    sel = warped[-10:]
    Iw = np.sum(I[sel] / s2[sel]) / np.sum(1 / s2[sel])
    sw = 1.0 / np.sum(1 / s2[sel])
    assert abs(Iw - plain.integral) < 4.0 * math.sqrt(sw + plain.sigma2), (Iw, plain.integral)
    v.close()


def test_flow_judge_falls_back():
    """A badly scaled fixed warp: the guard rejects it three times, switches
    it off, and plain VEGAS+ carries on."""
    w = vi.Workload("corr16_judge", 16, vi.GAUSS_CORR, np.array([0.5, 0.2, 0.5]), n_g=64, n_eval=100_003,
                    n_iter=1, precision="f32")
    say("[flow judge]")
    v = make(w)
    v.adapt(6)
    v.attach_flow(random_theta(9, scale=30.0).astype(np.float32), judge=1)
    v.enable_flow(True)
    v.adapt(6)
    on, kept, rejected = v.flow_status()
    say(f"  kept {kept} rejected {rejected} on={on}")
    assert not on and rejected >= 3
    v.integrate(3)
    r = v.result()
    assert math.isfinite(r.integral) and r.sigma2 > 0
    v.close()


def test_flow_cost_judge_switches_off():
    """The cost judge on a product Gaussian, where the separable VEGAS+ map
    is already the best importance density: an untrained identity warp has
    the plain variance at a higher cost per iteration, so it loses the
    comparison with the plain controls (every 4th iteration) twice and is
    switched off; plain iterations follow."""
    s = 0.2
    w = vi.Workload("gauss16_cost", 16, vi.GAUSS_DIAG, vi.gauss_diag_params(vi.normal_peak(s, 16), s, [0.5]),
                    n_g=64, n_eval=100_003, n_iter=1, precision="f32")
    say("[flow cost judge]")
    v = make(w)
    v.adapt(4)
    v.attach_flow(None, judge=2, control_period=4)
    v.enable_flow(True)
    v.integrate(16)
    on, kept, rejected = v.flow_status()
    kinds = v.flow_kinds()
    say(f"  kinds {kinds.tolist()} kept {kept} rejected {rejected} on={on}")
    assert not on
    assert kinds[7] == 2 and kinds[-1] == 0
    r = v.result()
    assert r.n_iter_combined == 16 - int(np.sum(kinds == 2))
    v.close()


def test_flow_judge_on_side_stream():
    """The judge reads each iteration's estimate on the host: on a side stream
    (torch.cuda.Stream, which does not wait for the default stream) it must
    read the finished values.  The same guarded, training run on the default
    stream and on a side stream, the default stream busy with other work
    meanwhile, keeps the same record and gives the same estimate up to the
    histogram sums' rounding order.  Every tensor of the side-stream run is
    allocated under that stream, and the busy work allocates nothing, so no
    memory changes hands between the streams."""
    import torch
    from paper_2408_09229_amd import Vegas, make_config
    w = corr16(n_eval=100_003, n_g=64)
    say("[flow judge, side stream]")
    busy_a = torch.randn(4096, 4096, device="cuda")
    busy_b = torch.empty_like(busy_a)
    torch.cuda.synchronize()
    out = []
    for side in (False, True):
        st = torch.cuda.Stream() if side else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            cfg = make_config(w.dim, w.n_g, w.n_eval, seed=w.seed, precision="f32")
            v = Vegas(cfg, w.family, w.params, stream=st)
            v.adapt(4)
            v.attach_flow(None, lr=1e-3, train=True, loss="kl", judge="guard", steps_per_iter=4, train_stride=4)
            v.enable_flow(True)
            if side:
                with torch.cuda.stream(torch.cuda.default_stream()):
                    for _ in range(8):
                        torch.matmul(busy_a, busy_a, out=busy_b)
                        torch.matmul(busy_b, busy_b, out=busy_a)
            v.integrate(10)
            r = v.result()
            out.append((v.flow_status(), r.integral, math.sqrt(r.sigma2)))
            say(f"  side={side}: status {out[-1][0]} I {r.integral:.8f} +- {math.sqrt(r.sigma2):.2e}")
            v.close()
        torch.cuda.synchronize()
    (s0, I0, e0), (s1, I1, e1) = out
    assert s0 == s1 and s0[0]
    assert abs(I0 - I1) <= 1e-6 * abs(I0) + 1e-3 * e0
