"""FP64 CPU reference of the learned warm start (test infrastructure only).

The warm start is not part of the paper; it is this library's extension of the
inner sweep (Section IV, eq. ADMoM_NTF): a small MLP maps one row's NNLS
problem  min_{h >= 0} 1/2 h^T G h - w^T h  (G = G_n + rho I minus rho I, i.e.
the Gram Hadamard product, and w a row of the MTTKRP) to an approximate
solution, and a KKT judge decides, row by row, whether the inner ADMoM
iterations start from it or from the previous iterate.

Parameter layout (one flat vector, row-major blocks):
  W1 [H, D], b1 [H], W2 [H, H], b2 [H], W3 [F, H], b3 [F]
with D = F(F+1)/2 + F inputs and H hidden units; ReLU after the two hidden
layers, linear output (a ReLU there can leave every output at zero for good:
a row whose output pre-activations are all negative gets no gradient); the
candidate is the output projected onto h >= 0.

Inputs of a row: the upper triangle of G / rho (row by row, j >= i) followed
by w / ||w||; the network predicts h * rho / ||w||.  NNLS is scale
equivariant (h*(aG, bw) = (b/a) h*(G, w)), so this normalisation loses nothing.

Only tests, the smoke check and the benchmark's CPU leg may import this file.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

__all__ = ["layout", "init_params", "unpack", "features", "forward", "backward", "mse_loss",
           "adam_step", "predict_rows", "kkt_violation", "warm_start"]


def layout(F: int, H: int = 256) -> Dict[str, Tuple[int, Tuple[int, ...]]]:
    """Offsets and shapes of the parameter blocks in the flat vector."""
    D = F * (F + 1) // 2 + F
    blocks = [("W1", (H, D)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (F, H)),
              ("b3", (F,))]
    out, off = {}, 0
    for name, shape in blocks:
        out[name] = (off, shape)
        off += int(np.prod(shape))
    out["_total"] = (off, ())
    return out


def init_params(F: int, H: int = 256, seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (float64)."""
    lay = layout(F, H)
    rng = np.random.default_rng(seed)
    p = np.zeros(lay["_total"][0])
    for name in ("W1", "W2", "W3"):
        off, shape = lay[name]
        fan_in = shape[1]
        lim = math.sqrt(6.0 / fan_in)
        p[off:off + shape[0] * shape[1]] = rng.uniform(-lim, lim, shape[0] * shape[1])
    return p


def unpack(p: np.ndarray, F: int, H: int = 256) -> Dict[str, np.ndarray]:
    lay = layout(F, H)
    return {k: p[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in lay.items() if k != "_total"}


def features(G: np.ndarray, W: np.ndarray, rho: float):
    """Row inputs [rows, D] and the per-row output scale ||w|| / rho."""
    G = np.asarray(G, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    F = G.shape[0]
    iu = np.triu_indices(F)
    g = (G / rho)[iu]
    nw = np.linalg.norm(W, axis=1)
    safe = np.where(nw > 0, nw, 1.0)
    X = np.concatenate([np.broadcast_to(g, (W.shape[0], g.size)), W / safe[:, None]], axis=1)
    return X, nw / rho


def forward(p: np.ndarray, X: np.ndarray, F: int, H: int = 256):
    P = unpack(p, F, H)
    z1 = X @ P["W1"].T + P["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ P["W2"].T + P["b2"]
    a2 = np.maximum(z2, 0.0)
    y = a2 @ P["W3"].T + P["b3"]          # linear output layer
    return y, (X, a1, a2, y)


def mse_loss(y: np.ndarray, t: np.ndarray) -> float:
    """1/(2B) sum ||y - t||^2 over the batch."""
    return 0.5 * float(np.sum((y - t) ** 2)) / y.shape[0]


def backward(p: np.ndarray, cache, dy: np.ndarray, F: int, H: int = 256) -> np.ndarray:
    """Gradient of sum(dy * y) w.r.t. the flat parameters (ReLU derivative 0 at 0;
    the output layer is linear)."""
    P = unpack(p, F, H)
    X, a1, a2, y = cache
    g = {}
    d3 = dy                                # (linear output layer)
    g["W3"] = d3.T @ a2
    g["b3"] = d3.sum(axis=0)
    da2 = d3 @ P["W3"]
    d2 = da2 * (a2 > 0)
    g["W2"] = d2.T @ a1
    g["b2"] = d2.sum(axis=0)
    da1 = d2 @ P["W2"]
    d1 = da1 * (a1 > 0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    lay = layout(F, H)
    out = np.zeros_like(p)
    for k, (o, s) in lay.items():
        if k != "_total":
            out[o:o + int(np.prod(s))] = g[k].ravel()
    return out


def adam_step(p, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction; returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def predict_rows(p, G, W, rho, H: int = 256):
    F = G.shape[0]
    X, sc = features(G, W, rho)
    y, _ = forward(p, X, F, H)
    return y * sc[:, None]


def kkt_violation(G, W, Hr):
    """||min(h, h G - w)|| per row (eq. KKT_NTF for one row's NNLS)."""
    return np.linalg.norm(np.minimum(Hr, Hr @ G - W), axis=1)


def natural_residual(G, W, Hr, rho):
    """||min(h, (h G - w) / rho)|| per row: the KKT violation of one row's
    NNLS (eq. KKT_NTF with Y = -rho U, so rho u = h G - w) in the units of h.
    It is h - max(0, h - (h G - w)/rho), the change one projected-gradient
    step of length 1/rho would make, zero exactly at the row's solution."""
    return np.linalg.norm(np.minimum(Hr, (Hr @ G - W) / rho), axis=1)


def warm_start(p, G, W, rho, H_prev, U_prev, Hid: int = 256):
    """Per row: the MLP candidate (h, u with u = max(0, (hG - w)/rho) on the
    zero set of h) or the previous iterate, whichever has the smaller KKT
    violation in the units of h (natural_residual; ties keep the previous
    iterate)."""
    h = np.maximum(predict_rows(p, G, W, rho, Hid), 0.0)   # the candidate, projected onto h >= 0
    g = h @ G - W
    u = np.where(h > 0, 0.0, np.maximum(g / rho, 0.0))
    k_new = natural_residual(G, W, h, rho)
    k_old = natural_residual(G, W, H_prev, rho)
    take = k_new < k_old
    Hs = np.where(take[:, None], h, H_prev)
    Us = np.where(take[:, None], u, U_prev)
    return Hs, Us, take
