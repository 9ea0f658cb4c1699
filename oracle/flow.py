"""Coupling-flow warp oracle -- TEST INFRASTRUCTURE ONLY (plain FP64 numpy).

The learned warp stacks a normalising flow F on the VEGAS map: a stratified
point y in [0,1]^D goes to w = F(y), and w goes through the separable map to
x.  The weight of the sample is f(x) J_map(w) J_F(y), so the estimate stays
unbiased for any F, because J_F is the exact Jacobian determinant.  The paper
has no such warp: this follows the problem statement's description of it
(four coupling layers, 2x64 MLP conditioners, BF16 matrix products with FP32
accumulation) with the readings listed here.

Readings (all fixed here, shared by the GPU path through its tests):
  * Masks: layer 1 conditions on the first half of the axes and transforms
    the second, layer 2 the reverse, layer 3 conditions on the even axes,
    layer 4 on the odd ones.
  * Conditioner: x = 2 z_A - 1; h1 = relu(W1 x + b1); h2 = relu(W2 h1 + b2);
    o = W3 h2 + b3, o = (logits of K bins) for each transformed axis.
  * Bin probabilities p = (1 - eps) softmax(o) + eps/K, eps = 1e-3, K = 16.
  * Transform of a coordinate z in bin b = min(floor(K z), K-1):
    C(z) = sum_{k<b} p_k + (K z - b) p_b, with derivative K p_b.  The inverse
    finds the bin of v among the cumulative sums and inverts the linear piece.
  * Initialisation: W1, W2 uniform in +-1/sqrt(fan_in), everything else 0, so
    p = 1/K and F is the identity.
  * Training loss of one iteration: L = sum_k c_k log J_F(F^-1(w_k)) with
    c_k = omega_k^2 / sum omega^2 on the stored samples (w_k, omega_k).  Its
    gradient is the gradient of the estimator's variance, sum g^2/q, in the
    direction that matters (log q(w) = -log J_F(F^-1(w))), up to a positive
    factor; the inverse pass is differentiated.
  * Adam with beta1 0.9, beta2 0.999, eps 1e-8.

``bf16=True`` rounds, to BF16 with round-to-nearest-even, exactly the values
the GPU feeds to its BF16 matrix instructions: the conditioner inputs, the
weights, the hidden activations, and in the backward pass the gradients of
the layer outputs that enter products.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

K_BINS = 16
HIDDEN = 64
EPS = 1e-3
N_LAYERS = 4


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
                    ("W3", (nb * K_BINS, HIDDEN)), ("b3", (nb * K_BINS,))])
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
    s: np.ndarray      # (N, nB, K) softmax
    p: np.ndarray      # (N, nB, K) bin probabilities
    cum: np.ndarray    # (N, nB, K+1) exclusive cumulative sums, cum[..., K] = total
    b: np.ndarray      # (N, nB) bin of each transformed coordinate
    logj: np.ndarray   # (N,)


def _mlp(L, zA, emu):
    r = bf16 if emu else (lambda v: v)
    x = r(2.0 * zA - 1.0)
    h1 = np.maximum(x @ r(L["W1"]).T + L["b1"], 0.0)
    h1 = r(h1)
    h2 = np.maximum(h1 @ r(L["W2"]).T + L["b2"], 0.0)
    h2 = r(h2)
    o = h2 @ r(L["W3"]).T + L["b3"]
    return x, h1, h2, o


def _probs(o, nb):
    o = o.reshape(o.shape[0], nb, K_BINS)
    e = np.exp(o - o.max(axis=2, keepdims=True))
    s = e / e.sum(axis=2, keepdims=True)
    return s, (1.0 - EPS) * s + EPS / K_BINS


def _cums(p):
    c = np.zeros(p.shape[:2] + (K_BINS + 1,))
    c[..., 1:] = np.cumsum(p, axis=2)
    return c


def layer_forward(L, z, A, B, emu=False):
    x, h1, h2, o = _mlp(L, z[:, A], emu)
    s, p = _probs(o, len(B))
    cum = _cums(p)
    zb = z[:, B]
    b = np.clip(np.floor(K_BINS * zb).astype(np.int64), 0, K_BINS - 1)
    pb = np.take_along_axis(p, b[..., None], 2)[..., 0]
    cb = np.take_along_axis(cum, b[..., None], 2)[..., 0]
    out = z.copy()
    out[:, B] = cb + (K_BINS * zb - b) * pb
    logj = np.log(K_BINS * pb).sum(axis=1)
    return out, Cache(x, h1, h2, s, p, cum, b, logj)


def layer_inverse(L, u, A, B, emu=False):
    x, h1, h2, o = _mlp(L, u[:, A], emu)
    s, p = _probs(o, len(B))
    cum = _cums(p)
    v = u[:, B]
    # bin: the last k with cum_k <= v (k < K)
    b = np.clip((cum[..., :K_BINS] <= v[..., None]).sum(axis=2) - 1, 0, K_BINS - 1)
    pb = np.take_along_axis(p, b[..., None], 2)[..., 0]
    cb = np.take_along_axis(cum, b[..., None], 2)[..., 0]
    out = u.copy()
    out[:, B] = np.clip((b + (v - cb) / pb) / K_BINS, 0.0, 1.0)
    logj = np.log(K_BINS * pb).sum(axis=1)
    return out, Cache(x, h1, h2, s, p, cum, b, logj)


# --------------------------------------------------------------------------
# the flow
# --------------------------------------------------------------------------
def forward(theta, y, emu=False):
    """w = F(y) and log J_F(y), for rows y of an (N, D) array."""
    y = np.asarray(y, dtype=np.float64)
    dim = y.shape[1]
    z = y
    lj = np.zeros(y.shape[0])
    for L, (A, B) in zip(unpack(theta, dim), masks(dim)):
        z, c = layer_forward(L, z, A, B, emu)
        lj += c.logj
    return z, lj


def inverse(theta, w, emu=False):
    """y = F^-1(w) and log J_F(y)."""
    w = np.asarray(w, dtype=np.float64)
    dim = w.shape[1]
    u = w
    lj = np.zeros(w.shape[0])
    layers = list(zip(unpack(theta, dim), masks(dim)))
    for L, (A, B) in reversed(layers):
        u, c = layer_inverse(L, u, A, B, emu)
        lj += c.logj
    return u, lj


def loss_grad(theta, w, coef, emu=False):
    """L = sum_k coef_k log J_F(F^-1(w_k)) and dL/dtheta (same layout as theta).

    Backward through the inverse chain u_4 = w -> u_3 -> .. -> u_0 = y: for
    layer l the upstream gradient g = dL/du_{l-1} of the layers already
    passed, and the layer's own log-Jacobian, give dL/dtheta_l and
    dL/du_l."""
    w = np.asarray(w, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.float64)
    N, dim = w.shape
    layers = list(zip(unpack(theta, dim), masks(dim)))
    grad = np.zeros_like(theta)
    gl = unpack(grad, dim)
    # inverse pass, keeping every layer's input u_l and cache
    u = w
    ins, caches = [None] * N_LAYERS, [None] * N_LAYERS
    for l in reversed(range(N_LAYERS)):
        L, (A, B) = layers[l]
        ins[l] = u
        u, caches[l] = layer_inverse(L, u, A, B, emu)
    total = float((coef * sum(c.logj for c in caches)).sum())
    r = bf16 if emu else (lambda v: v)
    g = np.zeros((N, dim))                  # dL/du_0: y enters no log-Jacobian
    for l in range(N_LAYERS):
        L, (A, B) = layers[l]
        c = caches[l]
        v = ins[l][:, B]
        b = c.b
        pb = np.take_along_axis(c.p, b[..., None], 2)[..., 0]
        cb = np.take_along_axis(c.cum, b[..., None], 2)[..., 0]
        gz = g[:, B]
        # z = (b + (v - cum_b)/p_b)/K
        dp = np.zeros_like(c.p)
        kk = np.arange(K_BINS)[None, None, :]
        below = kk < b[..., None]
        at = kk == b[..., None]
        dp += below * (gz * (-1.0 / (K_BINS * pb)))[..., None]
        dp += at * (gz * (-(v - cb) / (K_BINS * pb * pb)) + coef[:, None] / pb)[..., None]
        gv = gz / (K_BINS * pb)
        # p = (1 - eps) s + eps/K; s = softmax(o)
        ds = (1.0 - EPS) * dp
        do = c.s * (ds - (c.s * ds).sum(axis=2, keepdims=True))
        do = do.reshape(N, -1)
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
        gnew[:, A] = g[:, A] + 2.0 * dx
        gnew[:, B] = gv
        g = gnew
    return total, grad


def adam(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
