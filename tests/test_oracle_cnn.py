"""Pins of the CNN reference (oracle/cnn.py): closed forms, the adjoint
identity, finite differences and PyTorch's circular conv3d (CPU, float64)."""
import numpy as np
import pytest

from oracle import cnn as C
import synth


def rnd(shape, seed):
    return synth.rng(seed).standard_normal(shape)


def test_conv_delta_and_constant():
    n = 5
    W = rnd((3, 2, 27), 1)
    b = rnd(3, 2)
    x = np.zeros((2, n, n, n))
    x[1, 0, 0, 0] = 1.0
    y = C.conv3_fwd(x, W, b)
    # y[o, v] = b + W[o,1,t] where v + d_t = 0 (mod n)
    for t, (dz, dy, dx) in enumerate(C.TAPS):
        np.testing.assert_allclose(y[:, (-dz) % n, (-dy) % n, (-dx) % n], b + W[:, 1, t], atol=1e-14)
    c = np.full((2, n, n, n), 0.7)
    yc = C.conv3_fwd(c, W, b)
    np.testing.assert_allclose(yc, np.broadcast_to((0.7 * W.sum(axis=(1, 2)) + b)[:, None, None, None], yc.shape), atol=1e-13)


def test_conv_matches_torch_circular():
    torch = pytest.importorskip("torch")
    n = 6
    x = rnd((4, n, n, n), 3)
    W = rnd((5, 4, 27), 4)
    b = rnd(5, 5)
    xt = torch.from_numpy(x)[None]
    Wt = torch.from_numpy(W.reshape(5, 4, 3, 3, 3))
    yt = torch.nn.functional.conv3d(torch.nn.functional.pad(xt, (1, 1, 1, 1, 1, 1), mode="circular"), Wt,
                                    torch.from_numpy(b))
    np.testing.assert_allclose(C.conv3_fwd(x, W, b), yt[0].numpy(), atol=1e-12)


def test_conv_adjoint_identity():
    n = 5
    x = rnd((3, n, n, n), 6)
    W = rnd((4, 3, 27), 7)
    dy = rnd((4, n, n, n), 8)
    y = C.conv3_fwd(x, W, np.zeros(4))
    dx, dW, db = C.conv3_bwd(x, W, dy)
    assert np.sum(y * dy) == pytest.approx(np.sum(x * dx), rel=1e-12)
    assert np.sum(y * dy) == pytest.approx(np.sum(W * dW), rel=1e-12)
    np.testing.assert_allclose(db, dy.sum(axis=(1, 2, 3)), atol=1e-12)


def test_network_gradient_finite_differences():
    n = 4
    chans = [1, 3, 3, 2]
    params = C.init_params(9, chans)
    for p in params:
        p["b"] = synth.rng(10).uniform(-0.1, 0.1, size=p["b"].shape)
    x = synth.rng(11).uniform(0, 1, size=(1, n, n, n))
    chi = rnd((2, n, n, n), 12)
    out, acts = C.net_forward(params, x)
    L, dout = C.loss(out, chi)
    grads = C.net_backward(params, acts, dout)
    h = 1e-6
    g = synth.rng(13)
    for li in range(len(params)):
        for key in ("W", "b"):
            arr = params[li][key]
            for _ in range(3):
                idx = tuple(g.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                Lp = C.loss(C.net_forward(params, x)[0], chi)[0]
                arr[idx] = old - h
                Lm = C.loss(C.net_forward(params, x)[0], chi)[0]
                arr[idx] = old
                fd = (Lp - Lm) / (2 * h)
                assert abs(fd - grads[li][key][idx]) <= 1e-7 * max(1.0, abs(fd)), (li, key, idx)


def test_output_mean_removed():
    n = 4
    params = C.init_params(1)
    out, _ = C.net_forward(params, synth.rng(2).uniform(0, 1, size=(1, n, n, n)))
    assert out.shape == (3, n, n, n)
    np.testing.assert_allclose(out.mean(axis=(1, 2, 3)), 0.0, atol=1e-14)
