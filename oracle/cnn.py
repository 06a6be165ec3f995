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

Two modes.  The exact mode (net_forward / net_backward) is the network in
float64.  The bf16 mode (net_forward_bf16 / net_backward_bf16) applies the
rounding a bf16 implementation with float32 parameters must apply, at the
points where such an implementation stores bf16 values: the input density
(via float32), the weights, each ReLU activation, the loss gradient and
each masked input gradient, every rounding to nearest-even in bf16 (the top
16 bits of a float32); products and sums stay exact (float64), biases and
the last layer's output are not rounded.  It is the reference for comparing
a bf16 implementation element by element: only its accumulation order and
width differ from this.
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
    """x: (Cin, N, N, N); W: (Cout, Cin, 27); b: (Cout,) -> (Cout, N, N, N).
    Per tap, the channel mixing is a (Cout x Cin) by (Cin x N^3) matrix product."""
    cin = x.shape[0]
    y = np.zeros((W.shape[0], x[0].size))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += W[:, :, t] @ shift(x, dz, dy, dx).reshape(cin, -1)
    return y.reshape((W.shape[0],) + x.shape[1:]) + b[:, None, None, None]


def conv3_bwd(x: np.ndarray, W: np.ndarray, dy: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Gradients of sum(dy * conv3_fwd(x, W, b)) w.r.t. x, W and b."""
    cin, cout = x.shape[0], dy.shape[0]
    dx = np.zeros((cin, x[0].size))
    dW = np.zeros_like(W)
    dyf = dy.reshape(cout, -1)
    for t, (dz, dyy, dxx) in enumerate(TAPS):
        dW[:, :, t] = dyf @ shift(x, dz, dyy, dxx).reshape(cin, -1).T
        # x[c, v + d] receives W[o, c, t] dy[o, v]  ->  dx[c, u] += W dy[o, u - d]
        dx += W[:, :, t].T @ shift(dy, -dz, -dyy, -dxx).reshape(cout, -1)
    db = dyf.sum(axis=1)
    return dx.reshape(x.shape), dW, db


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


# ----------------------------------------------------------------- bf16 mode

def bf16(a) -> np.ndarray:
    """Round to bf16 through float32: the float32 value's upper 16 bits,
    rounded to nearest with ties to even (IEEE rounding of the 24-bit
    significand to 8 bits); returned as float64 (exact)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    keep = (u >> 16) & 1
    u = (u + 0x7FFF + keep) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def net_forward_bf16(params, rhof: np.ndarray):
    """The network with a bf16 implementation's rounding (module docstring):
    rhof (N, N, N) -> (out mean-removed (3, N, N, N), acts).  acts[l] is the
    bf16 input of layer l; acts[-1] the last layer's unrounded output."""
    acts = [bf16(rhof)[None]]
    h = acts[0]
    for li, p in enumerate(params):
        h = conv3_fwd(h, bf16(p["W"]), np.asarray(p["b"], dtype=np.float32).astype(np.float64))
        if li < len(params) - 1:
            h = bf16(np.maximum(h, 0.0))
        acts.append(h)
    out = h - h.mean(axis=(1, 2, 3), keepdims=True)
    return out, acts


def loss_bf16(out: np.ndarray, chi: np.ndarray) -> Tuple[float, np.ndarray]:
    """As loss(), with dL/dout rounded to bf16."""
    L, d = loss(out, chi)
    return L, bf16(d)


def net_backward_bf16(params, acts, dout: np.ndarray):
    """Gradients of sum(dout * out) with the bf16 weights; each layer's
    masked input gradient is rounded to bf16 before it feeds the layer
    below.  dout is taken as given (zero mean per channel is assumed, as
    loss() returns)."""
    g = dout
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        dx, dW, db = conv3_bwd(acts[li], bf16(params[li]["W"]), g)
        grads[li] = {"W": dW, "b": db}
        if li > 0:
            g = bf16(dx * (acts[li] > 0.0))
    return grads


def net_forward_bf16_at(params, rhof: np.ndarray, voxels) -> np.ndarray:
    """The bf16-mode network's last-layer output before the mean removal at
    the given voxels (list of (z, y, x)), each from its own receptive field:
    the periodic (2L+1)^3 window of the input around the voxel (L layers),
    then L unpadded 3x3x3 correlations, each shrinking the window by one
    voxel per side, with the same rounding as net_forward_bf16.  -> (K, 3)."""
    L = len(params)
    n = rhof.shape[0]
    r = np.arange(-L, L + 1)
    out = []
    for (z, y, x) in voxels:
        idx = np.ix_((z + r) % n, (y + r) % n, (x + r) % n)
        h = bf16(rhof[idx])[None]
        for li, p in enumerate(params):
            w = h.shape[1] - 2
            acc = np.zeros((p["W"].shape[0], w ** 3))
            Wb = bf16(p["W"])
            for t, (dz, dy, dx) in enumerate(TAPS):
                xs = h[:, 1 + dz:1 + dz + w, 1 + dy:1 + dy + w, 1 + dx:1 + dx + w].reshape(h.shape[0], -1)
                acc += Wb[:, :, t] @ xs
            h = acc.reshape((-1, w, w, w)) + np.asarray(p["b"], dtype=np.float32).astype(np.float64)[:, None, None, None]
            if li < L - 1:
                h = bf16(np.maximum(h, 0.0))
        out.append(h[:, 0, 0, 0])
    return np.array(out)
