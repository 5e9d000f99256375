"""FP64 reference of the calibration network (parity of the BF16 matrix-core kernels).

The paper names calibrating the simulator's parameters from aggregate data as its
goal beyond grid search (section 1; section 6).  The network maps a daily incidence
curve to the parameters (R, S_0..S_8): fully connected 192 -> 256 -> 256 -> 16 with
ReLU after the hidden layers, trained on mean squared error of the normalised
parameters with Adam.

Quantisation points mirror the GPU's storage (BF16 weights, inputs and hidden
activations; FP32 output and gradients); every product and sum here is FP64.
Parameter blob layout: W1 [256,192], b1 [256], W2 [256,256], b2 [256], W3 [16,256], b3 [16].
"""
from __future__ import annotations

import numpy as np

IN, H, OUT = 192, 256, 16
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)), ("b3", (OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16_round(x):
    """Round to the nearest BF16 value, ties to even (from the FP32 value of x)."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def unpack(blob):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(blob[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[n], np.float64).ravel() for n, _ in SHAPES])


def init_params(seed=0):
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def forward(blob, x, quantize=True):
    """y [B,16] and the cache for backward.  With quantize, x, the weights and the
    hidden activations are taken at their BF16 values."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, np.float64))
    P = unpack(blob)
    W = {k: q(v) for k, v in P.items()}
    x = q(x)
    h1 = q(np.maximum(x @ W["W1"].T + W["b1"], 0.0))
    h2 = q(np.maximum(h1 @ W["W2"].T + W["b2"], 0.0))
    y = h2 @ W["W3"].T + W["b3"]
    return y, dict(x=x, h1=h1, h2=h2, W=W, q=q)


def loss_and_backward(blob, x, target, n_out, quantize=True):
    """MSE over the first n_out outputs (mean over B * n_out) and its gradient with
    respect to the parameter blob.  Upstream gradients are taken at BF16 where the
    GPU feeds them to the matrix cores."""
    y, c = forward(blob, x, quantize)
    q, W = c["q"], c["W"]
    B = y.shape[0]
    diff = np.zeros_like(y)
    diff[:, :n_out] = y[:, :n_out] - np.asarray(target, np.float64)[:, :n_out]
    loss = float((diff ** 2).sum() / (B * n_out))
    dy = 2.0 * diff / (B * n_out)
    g = {}
    g["W3"] = q(dy).T @ c["h2"]
    g["b3"] = dy.sum(0)
    dh2 = (q(dy) @ W["W3"]) * (c["h2"] > 0)
    g["W2"] = q(dh2).T @ c["h1"]
    g["b2"] = dh2.sum(0)
    dh1 = (q(dh2) @ W["W2"]) * (c["h1"] > 0)
    g["W1"] = q(dh1).T @ c["x"]
    g["b1"] = dh1.sum(0)
    return loss, pack(g), y


def adam(master, m, v, g, lr, b1, b2, eps, step):
    """One Adam step (Kingma & Ba 2015) with bias correction; returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v
