"""CPU reference of the learned smooth-zone gate (test infrastructure only).

Definitions (the paper has no learned component; these are the readings the
GPU gate is built to):
  features  per zone, per variable v, the 13-zone cross (centre, then x-2,
            x-1, x+1, x+2, y-2, ..., z+2; 9 zones in 2D) of zone averages,
            centred on the zone value and scaled by
            (max - min + 1e-12 * max(1, |centre|)) over the cross; ordered
            [v][cross] -> 65 features in 3D, 36 in 2D.  Ghost zones as in the
            step (periodic wrap / zero-gradient clamp).
  label     smooth  <=>  max over variables and over the 1D WENO applications
            centred at the zone of max_k |omega_k / gamma_k - 1|  <= 0.25
            (the oracle's zone_maxdev).
  network   x (rounded to BF16) -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1' + b2)
            (64) -> logit = w3 . h2' + b3, where h' is h rounded to BF16 and
            W1, W2, w3 are BF16; biases FP32; p = sigmoid(logit).
  loss      class-weighted binary cross entropy, mean over the batch:
            L = -(1/B) sum_i c_i [y_i log p_i + (1 - y_i) log(1 - p_i)].
  training  Adam on FP32 master weights; BF16 copies used in the forward.
Everything here is FP64 numpy apart from the BF16 roundings, which are the
definition of the network's inputs and weights.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def cross_offsets(ndim):
    offs = [(0, 0, 0)]
    for ax in range(ndim):
        for o in (-2, -1, 1, 2):
            d = [0, 0, 0]
            d[ax] = o
            offs.append(tuple(d))
    return offs


def _pad(U, ndim, bc):
    """Ghost zones (2 per side) by periodic wrap or zero-gradient clamp."""
    out = U
    for ax in range(ndim):
        arr_ax = U.ndim - 1 - ax                  # x is the last array axis
        pw = [(0, 0)] * U.ndim
        pw[arr_ax] = (2, 2)
        out = np.pad(out, pw, mode="wrap" if bc[ax] in ("periodic", 0) else "edge")
    return out


def features(U, ndim, bc):
    """(N, nv * (4 ndim + 1)) features of every interior zone, x fastest."""
    nv = ndim + 2
    P = _pad(np.asarray(U, np.float64), ndim, bc)
    shp = U.shape[1:]
    vals = []
    for (dx, dy, dz) in cross_offsets(ndim):
        if ndim == 3:
            sl = P[:, 2 + dz:2 + dz + shp[0], 2 + dy:2 + dy + shp[1], 2 + dx:2 + dx + shp[2]]
        else:
            sl = P[:, 2 + dy:2 + dy + shp[0], 2 + dx:2 + dx + shp[1]]
        vals.append(sl.reshape(nv, -1))
    V = np.stack(vals, axis=1)                    # (nv, ncross, N)
    c = V[:, :1, :]
    scale = V.max(axis=1, keepdims=True) - V.min(axis=1, keepdims=True) + 1e-12 * np.maximum(1.0, np.abs(c))
    F = (V - c) / scale
    return F.reshape(nv * len(vals), -1).T.copy()


def init_params(nfeat, seed=0):
    """Seeded He-normal weights (FP32 masters), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = (rng.standard_normal((HIDDEN, nfeat)) * np.sqrt(2.0 / nfeat)).astype(np.float32)
    W2 = (rng.standard_normal((HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN)).astype(np.float32)
    w3 = (rng.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN)).astype(np.float32)
    return {"W1": W1, "b1": np.zeros(HIDDEN, np.float32), "W2": W2, "b2": np.zeros(HIDDEN, np.float32),
            "w3": w3, "b3": np.zeros(1, np.float32)}


def forward(params, X, rounding=True):
    """Logits and the intermediate values the backward pass needs.
    rounding=False gives the same network without the BF16 roundings (used
    to check the analytic gradients by finite differences)."""
    r = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    x = r(X)
    W1, W2, w3 = r(params["W1"]), r(params["W2"]), r(params["w3"])
    z1 = x @ W1.T + np.asarray(params["b1"], np.float64)
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + np.asarray(params["b2"], np.float64)
    h2 = r(np.maximum(z2, 0.0))
    logit = h2 @ w3 + float(params["b3"][0])
    return logit, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, W1=W1, W2=W2, w3=w3)


def loss_and_grads(params, X, y, cw, rounding=True):
    """Weighted BCE and its gradients with respect to the master parameters
    (the BF16 roundings are treated as identity in the backward pass)."""
    logit, c = forward(params, X, rounding)
    B = X.shape[0]
    y = np.asarray(y, np.float64)
    cw = np.asarray(cw, np.float64)
    # log(1 + exp(-|z|)) form of the BCE
    loss = np.mean(cw * (np.maximum(logit, 0) - logit * y + np.log1p(np.exp(-np.abs(logit)))))
    p = 1.0 / (1.0 + np.exp(-logit))
    dz = cw * (p - y) / B
    g = {}
    g["w3"] = c["h2"].T @ dz
    g["b3"] = np.array([dz.sum()])
    dh2 = np.outer(dz, c["w3"]) * (c["z2"] > 0)
    g["W2"] = dh2.T @ c["h1"]
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ c["W2"]) * (c["z1"] > 0)
    g["W1"] = dh1.T @ c["x"]
    g["b1"] = dh1.sum(axis=0)
    return loss, g


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on FP32 masters (state: dict with m, v, t)."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k], dtype=np.float64))
        v = state.setdefault("v_" + k, np.zeros_like(params[k], dtype=np.float64))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = (params[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return params


def logit_threshold(theta):
    return float(np.log(theta / (1.0 - theta)))
