"""CPU FP64 reference for the learned warm start (test infrastructure only).

A small fully convolutional network maps the filtered density (one channel,
element grid) to the three fluctuation fields chi^i (node grid, index
identity between element (i,j,k) and node (i,j,k)):

  5 layers of 3x3x3 periodic convolution, channels 1 -> 16 -> 16 -> 16 -> 16 -> 3,
  ReLU after layers 1-4, output mean removed per channel.

Convolution convention (a correlation, periodic):
  y[co, z, y, x] = b[co] + sum_ci sum_t W[co, ci, t] x[ci, z+dz_t, y+dy_t, x+dx_t]
with tap t = 9 (dz+1) + 3 (dy+1) + (dx+1).  Loss: mean over every value of
(out - chi)^2 with both sides mean-removed per channel.

Nothing here is shared with the HIP path; arrays are float64 numpy.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = [1, 16, 16, 16, 16, 3]


def shift(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """s[..., z, y, x] = x[..., z+dz, y+dy, x+dx] (periodic)."""
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3_fwd(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x: (Cin, N, N, N); W: (Cout, Cin, 27); b: (Cout,) -> (Cout, N, N, N)."""
    y = np.zeros((W.shape[0],) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += np.einsum("oc,czyx->ozyx", W[:, :, t], shift(x, dz, dy, dx))
    return y + b[:, None, None, None]


def conv3_bwd(x: np.ndarray, W: np.ndarray, dy: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Gradients of sum(dy * conv3_fwd(x, W, b)) w.r.t. x, W and b."""
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, (dz, dyy, dxx) in enumerate(TAPS):
        xs = shift(x, dz, dyy, dxx)
        dW[:, :, t] = np.einsum("ozyx,czyx->oc", dy, xs)
        # x[c, v + d] receives W[o, c, t] dy[o, v]  ->  dx[c, u] += W dy[o, u - d]
        dx += np.einsum("oc,ozyx->czyx", W[:, :, t], shift(dy, -dz, -dyy, -dxx))
    db = dy.sum(axis=(1, 2, 3))
    return dx, dW, db


def init_params(seed: int, channels: List[int] = CHANNELS) -> List[Dict[str, np.ndarray]]:
    """He-style uniform initialization (fan-in 27 Cin), zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        lim = np.sqrt(6.0 / (27 * cin))
        params.append({"W": g.uniform(-lim, lim, size=(cout, cin, 27)), "b": np.zeros(cout)})
    return params


def net_forward(params, x: np.ndarray):
    """Returns (out, cache); out is mean-removed per channel."""
    acts = [x]
    h = x
    for li, p in enumerate(params):
        h = conv3_fwd(h, p["W"], p["b"])
        if li < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    out = h - h.mean(axis=(1, 2, 3), keepdims=True)
    return out, acts


def net_backward(params, acts, dout: np.ndarray):
    """Gradients of sum(dout * out) for every layer's W and b."""
    # through the mean removal
    g = dout - dout.mean(axis=(1, 2, 3), keepdims=True)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        if li < len(params) - 1:
            g = g * (acts[li + 1] > 0.0)
        dx, dW, db = conv3_bwd(acts[li], params[li]["W"], g)
        grads[li] = {"W": dW, "b": db}
        g = dx
    return grads


def loss(out: np.ndarray, chi: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean squared error against the mean-removed target; returns (L, dL/dout)."""
    tgt = chi - chi.mean(axis=(1, 2, 3), keepdims=True)
    d = out - tgt
    return float(np.mean(d * d)), 2.0 * d / d.size
