"""Coupling-flow warp oracle -- TEST INFRASTRUCTURE ONLY (plain FP64 numpy).

The learned warp stacks a normalising flow F on the VEGAS map: a stratified
point y in [0,1]^D goes to w = F(y), and w goes through the separable map to
x.  The weight of the sample is f(x) J_map(w) J_F(y), so the estimate stays
unbiased for any F, because J_F is the exact Jacobian determinant.  The paper
has no such warp: this follows the problem statement's description of it
(four monotone coupling layers, 2x64 MLP conditioners, BF16 matrix products
with FP32 accumulation) with the readings listed here.

Readings (all fixed here, shared by the GPU path through its tests):
  * Gaussian coordinates: the flow acts on z = Phi^-1(y) (Phi the standard
    normal distribution function) and returns w = Phi(z_4).  The separable
    VEGAS map leaves the integrand's dependence between axes to the warp,
    and for an integrand that is a correlated Gaussian (or close to one) that
    dependence is an affine map of z, which affine coupling layers express.
  * Masks: layer 1 conditions on the first half of the axes and transforms
    the second, layer 2 the reverse, layer 3 conditions on the even axes,
    layer 4 on the odd ones.
  * Conditioner: x = z_A / 2; h1 = relu(W1 x + b1); h2 = relu(W2 h1 + b2);
    o = W3 h2 + b3 with 2 |B| outputs: raw log-scales a (first |B|) and
    shifts t (last |B|) of the transformed axes, in axis order.
  * Transform of a moved axis: s = S tanh(a / S) with S = 3 (log-scale kept
    in [-3, 3]), z_B -> z_B e^s + t.  Monotone in z_B; the inverse is
    (z_B - t) e^-s.
  * log J_F(y) = sum over layers and moved axes of s + sum_d (z_0d^2 - z_4d^2)/2
    (the log-densities of the two changes of variable y <-> z and z <-> w).
  * Initialisation: W1, W2 uniform in +-1/sqrt(fan_in), everything else 0, so
    s = t = 0 and F is the identity.
  * Training data of one iteration: the final Gaussian coordinates z_4 of its
    samples (w = Phi(z_4)) and their weights omega.  Loss
    L = sum_k c_k log J_F(F^-1(w_k)) with c_k = omega_k^2 / sum omega^2
    (variance) or |omega_k| / sum |omega| (KL).  Since the warp's density at
    w is 1 / J_F(F^-1(w)), the variance loss's gradient is a positive multiple
    of the gradient of the estimator's variance, sum g^2/q, and the KL loss's
    that of the KL divergence from |g| / int |g| to q.  The gradient is taken
    through the inverse chain from z_4 (fixed) down to z_0.
  * Adam with beta1 0.9, beta2 0.999, eps 1e-8.

``emu=True`` rounds, to BF16 with round-to-nearest-even, exactly the values
the GPU feeds to its BF16 matrix instructions: the conditioner inputs, the
weights, the hidden activations, and in the backward pass the gradients of
the layer outputs that enter products.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
from scipy.special import ndtr, ndtri

HIDDEN = 64
N_LAYERS = 4
S_MAX = 3.0          # log-scale bound S
X_SCALE = 0.5        # conditioner input x = X_SCALE z_A


# --------------------------------------------------------------------------
# layout
# --------------------------------------------------------------------------
def masks(dim: int):
    """(A, B) index arrays of the four layers."""
    ax = np.arange(dim)
    h = dim // 2
    conds = [ax[:h], ax[h:], ax[0::2], ax[1::2]]
    return [(a, np.setdiff1d(ax, a)) for a in conds]


def layer_shapes(dim: int):
    out = []
    for a, b in masks(dim):
        na, nb = len(a), len(b)
        out.append([("W1", (HIDDEN, na)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
                    ("W3", (2 * nb, HIDDEN)), ("b3", (2 * nb,))])
    return out


def n_params(dim: int) -> int:
    return int(sum(np.prod(s) for lay in layer_shapes(dim) for _, s in lay))


def unpack(theta: np.ndarray, dim: int) -> List[dict]:
    """Flat parameter vector -> per-layer dicts of views (layer by layer,
    W1, b1, W2, b2, W3, b3, row-major)."""
    out, o = [], 0
    for lay in layer_shapes(dim):
        d = {}
        for name, shape in lay:
            n = int(np.prod(shape))
            d[name] = theta[o:o + n].reshape(shape)
            o += n
        out.append(d)
    return out


def init_params(dim: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    theta = np.zeros(n_params(dim))
    for L, (a, _) in zip(unpack(theta, dim), masks(dim)):
        L["W1"][...] = rng.uniform(-1, 1, L["W1"].shape) / np.sqrt(len(a))
        L["W2"][...] = rng.uniform(-1, 1, L["W2"].shape) / np.sqrt(HIDDEN)
    return theta


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# one coupling layer
# --------------------------------------------------------------------------
@dataclass
class Cache:
    x: np.ndarray      # (N, nA) conditioner input (as fed to the product)
    h1: np.ndarray     # (N, H)
    h2: np.ndarray
    s: np.ndarray      # (N, nB) log-scales
    zb: np.ndarray     # (N, nB) the moved axes on the y side of the layer


def _mlp(L, zA, emu):
    r = bf16 if emu else (lambda v: v)
    x = r(X_SCALE * zA)
    h1 = np.maximum(x @ r(L["W1"]).T + L["b1"], 0.0)
    h1 = r(h1)
    h2 = np.maximum(h1 @ r(L["W2"]).T + L["b2"], 0.0)
    h2 = r(h2)
    o = h2 @ r(L["W3"]).T + L["b3"]
    return x, h1, h2, o


def _scale_shift(o, nb):
    s = S_MAX * np.tanh(o[:, :nb] / S_MAX)
    return s, o[:, nb:]


def layer_forward(L, z, A, B, emu=False):
    """Forward layer in Gaussian coordinates: z_B -> z_B e^s + t."""
    x, h1, h2, o = _mlp(L, z[:, A], emu)
    s, t = _scale_shift(o, len(B))
    out = z.copy()
    out[:, B] = z[:, B] * np.exp(s) + t
    return out, Cache(x, h1, h2, s, z[:, B].copy())


def layer_inverse(L, u, A, B, emu=False):
    """Inverse layer: u_B -> (u_B - t) e^-s."""
    x, h1, h2, o = _mlp(L, u[:, A], emu)
    s, t = _scale_shift(o, len(B))
    out = u.copy()
    out[:, B] = (u[:, B] - t) * np.exp(-s)
    return out, Cache(x, h1, h2, s, out[:, B].copy())


# --------------------------------------------------------------------------
# the flow
# --------------------------------------------------------------------------
def forward(theta, y, emu=False, return_z=False):
    """w = F(y) and log J_F(y) for rows y of an (N, D) array (and the final
    Gaussian coordinates z_4 with return_z)."""
    y = np.asarray(y, dtype=np.float64)
    dim = y.shape[1]
    z0 = ndtri(y)
    z = z0
    lj = np.zeros(y.shape[0])
    for L, (A, B) in zip(unpack(theta, dim), masks(dim)):
        z, c = layer_forward(L, z, A, B, emu)
        lj += c.s.sum(axis=1)
    lj += 0.5 * (z0 * z0 - z * z).sum(axis=1)
    w = ndtr(z)
    return (w, lj, z) if return_z else (w, lj)


def inverse_z(theta, zf, emu=False):
    """z_0 = F^-1 in Gaussian coordinates from the final coordinates z_4, and
    log J_F at y = Phi(z_0)."""
    zf = np.asarray(zf, dtype=np.float64)
    dim = zf.shape[1]
    u = zf
    lj = np.zeros(zf.shape[0])
    for L, (A, B) in reversed(list(zip(unpack(theta, dim), masks(dim)))):
        u, c = layer_inverse(L, u, A, B, emu)
        lj += c.s.sum(axis=1)
    lj += 0.5 * (u * u - zf * zf).sum(axis=1)
    return u, lj


def inverse(theta, w, emu=False):
    """y = F^-1(w) and log J_F(y)."""
    z0, lj = inverse_z(theta, ndtri(np.asarray(w, dtype=np.float64)), emu)
    return ndtr(z0), lj


def loss_grad(theta, zf, coef, emu=False):
    """L = sum_k coef_k log J_F(F^-1(w_k)), w_k = Phi(zf_k), and dL/dtheta
    (same layout as theta).

    Backward through the inverse chain u_4 = zf -> u_3 -> .. -> u_0: the
    loss's dependence on theta is through each layer's log-scales and through
    z_0 = u_0 (the term z_0^2 / 2); for layer l the upstream gradient
    g = dL/du_l of the layers already passed gives dL/dtheta_l and
    dL/du_{l+1}."""
    zf = np.asarray(zf, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.float64)
    N, dim = zf.shape
    layers = list(zip(unpack(theta, dim), masks(dim)))
    grad = np.zeros_like(theta)
    gl = unpack(grad, dim)
    # inverse pass, keeping every layer's input u_{l+1} and cache
    u = zf
    caches = [None] * N_LAYERS
    for l in reversed(range(N_LAYERS)):
        L, (A, B) = layers[l]
        u, caches[l] = layer_inverse(L, u, A, B, emu)
    z0 = u
    total = float((coef * (sum(c.s.sum(axis=1) for c in caches) + 0.5 * (z0 * z0 - zf * zf).sum(axis=1))).sum())
    r = bf16 if emu else (lambda v: v)
    g = coef[:, None] * z0                  # dL/du_0
    for l in range(N_LAYERS):
        L, (A, B) = layers[l]
        c = caches[l]
        nb = len(B)
        es = np.exp(-c.s)
        gb = g[:, B]
        # u_l,B = (u_{l+1},B - t) e^-s
        ds = coef[:, None] - gb * c.zb
        dt = -gb * es
        da = ds * (1.0 - (c.s / S_MAX) ** 2)
        do = np.concatenate([da, dt], axis=1)
        G = gl[l]
        G["W3"] += r(do).T @ c.h2
        G["b3"] += do.sum(axis=0)
        dh2 = (r(do) @ r(L["W3"])) * (c.h2 > 0)
        G["W2"] += r(dh2).T @ c.h1
        G["b2"] += dh2.sum(axis=0)
        dh1 = (r(dh2) @ r(L["W2"])) * (c.h1 > 0)
        G["W1"] += r(dh1).T @ c.x
        G["b1"] += dh1.sum(axis=0)
        dx = r(dh1) @ r(L["W1"])
        gnew = g.copy()
        gnew[:, A] = g[:, A] + X_SCALE * dx
        gnew[:, B] = gb * es
        g = gnew
    return total, grad


def adam(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
