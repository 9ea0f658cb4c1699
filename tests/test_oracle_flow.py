"""Pins of the coupling-flow warp oracle (oracle/flow.py), CPU only.

* identity at initialisation (zero last layer -> s = t = 0)
* F^-1(F(y)) = y and both passes give the same log J_F
* log J_F equals log|det| of a central-difference Jacobian of F
* one affine layer against the closed-form density of Phi(e^s Phi^-1(y) + t)
* a 2-d warp set by hand to the Cholesky factor of a correlated Gaussian
  turns uniform points into that Gaussian's copula exactly (weights all 1)
* the analytic loss gradient equals central differences of the loss
* BF16 rounding equals torch's float32 -> bfloat16 conversion
* a few Adam steps on the variance loss lower the variance of the weights of
  a correlated target (the gradient points the right way)
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import flow as fl

D = 16


def random_theta(dim, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    th = fl.init_params(dim, seed)
    for L in fl.unpack(th, dim):
        L["W3"][...] = rng.normal(0, scale, L["W3"].shape)
        L["b1"][...] = rng.normal(0, 0.1, L["b1"].shape)
        L["b2"][...] = rng.normal(0, 0.1, L["b2"].shape)
        L["b3"][...] = rng.normal(0, 0.5, L["b3"].shape)
    return th


def test_shapes_and_count():
    assert fl.n_params(16) == 4 * (64 * 8 + 64 + 64 * 64 + 64 + 16 * 64 + 16)
    for A, B in fl.masks(16):
        assert len(A) == len(B) == 8 and len(np.intersect1d(A, B)) == 0


def test_identity_at_init():
    th = fl.init_params(D, 3)
    y = np.random.default_rng(0).random((200, D))
    w, lj = fl.forward(th, y)
    assert np.max(np.abs(w - y)) < 1e-14
    assert np.all(lj == 0.0)


def test_round_trip():
    th = random_theta(D, 1, scale=0.1)
    # (away from the cube's faces, where Phi(z) rounds to 1 in FP64 for z > 8.3)
    y = 0.02 + 0.96 * np.random.default_rng(2).random((500, D))
    w, lj, zf = fl.forward(th, y, return_z=True)
    assert np.all((w > 0) & (w < 1))
    # through w itself only where Phi^-1(w) is well conditioned in FP64
    ok = np.all((w > 1e-6) & (w < 1 - 1e-6), axis=1)
    assert ok.sum() > 300
    y2, lj2 = fl.inverse(th, w[ok])
    assert np.max(np.abs(y2 - y[ok])) < 1e-10
    assert np.max(np.abs(lj2 - lj[ok])) < 1e-9
    z0, lj3 = fl.inverse_z(th, zf)
    assert np.max(np.abs(stats.norm.cdf(z0) - y)) < 1e-12
    assert np.max(np.abs(lj3 - lj)) < 1e-10


def test_logdet_against_finite_differences():
    dim = 6
    th = random_theta(dim, 4, scale=0.2)
    rng = np.random.default_rng(5)
    y = 0.05 + 0.9 * rng.random((20, dim))
    w, lj = fl.forward(th, y)
    h = 1e-6
    for i in range(len(y)):
        J = np.zeros((dim, dim))
        for j in range(dim):
            e = np.zeros(dim)
            e[j] = h
            J[:, j] = (fl.forward(th, (y[i] + e)[None])[0][0] - fl.forward(th, (y[i] - e)[None])[0][0]) / (2 * h)
        sign, ld = np.linalg.slogdet(J)
        assert sign > 0
        assert abs(ld - lj[i]) < 1e-6 * max(1.0, abs(lj[i])), (ld, lj[i])


def test_one_layer_closed_form():
    """Layer 1 alone with constant outputs (W3 = 0, b3 = (a, t)): each moved
    axis becomes w = Phi(e^s Phi^-1(y) + t) with s = 3 tanh(a/3), whose
    density is that of N(t, e^2s) seen through Phi: q(w) = phi((Phi^-1(w) -
    t) e^-s) e^-s / phi(Phi^-1(w)); log J_F = -sum log q(w_B)."""
    dim = 4
    th = fl.init_params(dim, 0)
    L0 = fl.unpack(th, dim)[0]
    a = np.array([0.7, -1.9])
    t = np.array([0.4, -1.1])
    L0["b3"][...] = np.concatenate([a, t])
    s = 3.0 * np.tanh(a / 3.0)
    y = np.random.default_rng(9).random((300, dim))
    w, lj = fl.forward(th, y)
    A, B = fl.masks(dim)[0]
    assert np.array_equal(w[:, A], y[:, A]) or np.max(np.abs(w[:, A] - y[:, A])) < 1e-14
    # y is the distribution function of N(t, e^2s) at Phi^-1(w)
    back = stats.norm(loc=t, scale=np.exp(s)).cdf(stats.norm.ppf(w[:, B]))
    assert np.max(np.abs(back - y[:, B])) < 1e-10
    ok = np.all((w[:, B] > 1e-6) & (w[:, B] < 1 - 1e-6), axis=1)
    assert ok.sum() > 200
    zb = stats.norm.ppf(w[ok][:, B])
    logq = stats.norm(loc=t, scale=np.exp(s)).logpdf(zb) - stats.norm.logpdf(zb)
    assert np.max(np.abs(lj[ok] + logq.sum(axis=1))) < 1e-10


def test_cholesky_warp_is_exact_for_a_correlated_gaussian():
    """dim 2, rho = 0.8: layer 1 moves axis 1 by z_1 -> sqrt(1 - rho^2) z_1 +
    rho z_0 (the MLP computes rho z_0 = 2 rho (relu(z_0/2) - relu(-z_0/2))),
    the other layers stay the identity.  Then w has the Gaussian copula of
    correlation rho, so omega = c_rho(w) J_F(y) is 1 for every y."""
    dim, rho = 2, 0.8
    th = fl.init_params(dim, 0)
    for L in fl.unpack(th, dim):
        L["W1"][...] = 0.0
        L["W2"][...] = 0.0
    L0 = fl.unpack(th, dim)[0]
    L0["W1"][0, 0], L0["W1"][1, 0] = 1.0, -1.0
    L0["W2"][0, 0], L0["W2"][1, 1] = 1.0, 1.0
    s = 0.5 * math.log(1.0 - rho * rho)
    L0["b3"][0] = 3.0 * math.atanh(s / 3.0)
    L0["W3"][1, 0], L0["W3"][1, 1] = 2.0 * rho, -2.0 * rho
    y = np.random.default_rng(4).random((2000, dim))
    w, lj = fl.forward(th, y)
    z = stats.norm.ppf(w)
    cop = stats.multivariate_normal(mean=[0, 0], cov=[[1, rho], [rho, 1]]).logpdf(z) - stats.norm.logpdf(z).sum(1)
    om = np.exp(cop + lj)
    assert np.max(np.abs(om - 1.0)) < 1e-9


def test_gradient_against_finite_differences():
    dim = 4
    th = random_theta(dim, 7, scale=0.2)
    rng = np.random.default_rng(8)
    zf = rng.normal(0, 1.0, (30, dim))
    coef = rng.random(30)
    total, g = fl.loss_grad(th, zf, coef)
    h = 1e-5
    idx = rng.choice(th.size, 60, replace=False)
    n_ok = 0
    for i in idx:
        tp = th.copy()
        tm = th.copy()
        tp[i] += h
        tm[i] -= h
        # the loss from the plain inverse pass, not from loss_grad's chain
        Lp = float((coef * fl.inverse_z(tp, zf)[1]).sum())
        Lm = float((coef * fl.inverse_z(tm, zf)[1]).sum())
        fd = (Lp - Lm) / (2 * h)
        # truncation O(h^2) plus the loss's own rounding over 2h
        if abs(fd - g[i]) > 1e-5 * max(1.0, abs(g[i])) + 1e-14 * abs(total) / h:
            pytest.fail(f"param {i}: analytic {g[i]} vs central difference {fd}")
        n_ok += 1
    assert n_ok == len(idx)
    assert np.linalg.norm(g) > 0


def test_bf16_matches_torch():
    import torch
    x = np.concatenate([[1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 1e-30, 3.3e38, 0.0],
                        np.random.default_rng(3).normal(0, 10, 1000)])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(fl.bf16(x), want)


def test_training_lowers_variance():
    """Target: a correlated Gaussian on [0,1]^4 (rho 0.8, s 0.12).  With
    x = w, omega = g(F(y)) J_F(y); Adam on the variance loss lowers the
    variance of omega below the identity warp's."""
    dim = 4
    rng = np.random.default_rng(11)
    s, rho = 0.12, 0.8
    cov = s * s * ((1 - rho) * np.eye(dim) + rho * np.ones((dim, dim)))
    ic = np.linalg.inv(cov)
    norm = 1.0 / np.sqrt((2 * np.pi) ** dim * np.linalg.det(cov))

    def g(x):
        u = x - 0.5
        return norm * np.exp(-0.5 * np.einsum("ni,ij,nj->n", u, ic, u))

    def var_of(th, n=200000, seed=0):
        y = np.random.default_rng(seed).random((n, dim))
        w, lj = fl.forward(th, y)
        om = g(w) * np.exp(lj)
        return om.var(), om.mean()

    th = fl.init_params(dim, 0)
    v0, m0 = var_of(th)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in range(1, 101):
        y = rng.random((10000, dim))
        w, lj, zf = fl.forward(th, y, return_z=True)
        om = g(w) * np.exp(lj)
        c = om ** 2 / np.sum(om ** 2)
        _, gr = fl.loss_grad(th, zf, c)
        th, m, v = fl.adam(th, gr, m, v, step, 1e-3)
    v1, m1 = var_of(th)
    assert abs(m0 - 1) < 0.1 and abs(m1 - 1) < 0.1      # unbiased both ways
    assert v1 < 0.8 * v0, (v0, v1)


def test_adam_two_steps_by_hand():
    """Adam (Kingma & Ba) worked by hand for one coordinate, lr 0.1.

    A constant gradient g: after the bias correction the first moment is g
    and the second g^2 at every step, so each step moves by lr g/(|g| + eps).
    A gradient that flips sign, g then -g: m_2 = 0.9 (0.1 g) - 0.1 g = -0.01 g,
    corrected by 1 - 0.9^2 = 0.19 to -g/19; v_2 = 0.999 (0.001 g^2) + 0.001 g^2
    = 0.001999 g^2, corrected by 1 - 0.999^2 = 0.001999 to g^2; so the second
    step moves by +lr/19 (for g > 0).  Without the bias correction the first
    step would be lr 0.1 g / sqrt(0.001) g = 3.16 lr."""
    lr, g = 0.1, 0.5
    th = np.array([1.0])
    m = np.zeros(1)
    v = np.zeros(1)
    th1, m, v = fl.adam(th, np.array([g]), m, v, 1, lr)
    assert abs(th1[0] - (1.0 - lr * g / (g + 1e-8))) < 1e-15
    th2, m2, v2 = fl.adam(th1, np.array([g]), m, v, 2, lr)
    assert abs(th2[0] - (th1[0] - lr * g / (g + 1e-8))) < 1e-15
    th2f, m2f, v2f = fl.adam(th1, np.array([-g]), m, v, 2, lr)
    assert abs(m2f[0] - (-0.01 * g)) < 1e-15 and abs(v2f[0] - 0.001999 * g * g) < 1e-17
    assert abs(th2f[0] - (th1[0] + lr * (g / 19.0) / (g + 1e-8))) < 1e-12
