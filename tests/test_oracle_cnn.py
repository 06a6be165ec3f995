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


# ------------------------------------------------------------- bf16 mode pins

def test_bf16_rounding_matches_torch_and_ties():
    """bf16() is round-to-nearest-even of float32 to 8 significand bits:
    against PyTorch's own float32 -> bfloat16 conversion on random values of
    every magnitude and sign, and on the tie cases by hand."""
    torch = pytest.importorskip("torch")
    g = synth.rng(21)
    v = (g.standard_normal(20000) * np.exp(g.uniform(-30, 30, 20000))).astype(np.float32)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 2.0 ** -130 * 1.5, 0.0, -0.0],
                    dtype=np.float32)
    v = np.concatenate([v, ties])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16(v), ref)
    assert C.bf16(1 + 2.0 ** -8) == 1.0                 # tie, even neighbour below
    assert C.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6   # tie, even neighbour above
    assert C.bf16(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7  # above the tie


def _f32_params(seed, chans):
    params = C.init_params(seed, chans)
    g = synth.rng(seed + 1)
    for p in params:
        p["W"] = p["W"].astype(np.float32).astype(np.float64)
        p["b"] = g.uniform(-0.1, 0.1, size=p["b"].shape).astype(np.float32).astype(np.float64)
    return params


def test_bf16_mode_without_rounding_is_the_exact_network(monkeypatch):
    """With the rounding replaced by the identity, the bf16 mode's forward and
    backward are the exact mode's (float32-representable parameters)."""
    n, chans = 5, [1, 4, 4, 3]
    params = _f32_params(30, chans)
    rhof = synth.rng(31).uniform(0, 1, size=(n, n, n))
    chi = synth.rng(32).standard_normal((3, n, n, n))
    out, acts = C.net_forward(params, rhof[None])
    _, dout = C.loss(out, chi)
    grads = C.net_backward(params, acts, dout)
    monkeypatch.setattr(C, "bf16", lambda a: np.asarray(a, dtype=np.float64))
    out_b, acts_b = C.net_forward_bf16(params, rhof)
    _, dout_b = C.loss_bf16(out_b, chi)
    grads_b = C.net_backward_bf16(params, acts_b, dout_b)
    np.testing.assert_allclose(out_b, out, rtol=0, atol=1e-14)
    for a, b in zip(grads_b, grads):
        np.testing.assert_allclose(a["W"], b["W"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(a["b"], b["b"], rtol=0, atol=1e-14)


def test_bf16_mode_rounds_where_stated():
    """Every stored activation of the bf16 forward is a bf16 value, the last
    layer's output is not rounded, and the forward differs from the exact
    network by bf16-sized amounts only."""
    n, chans = 6, [1, 4, 4, 3]
    params = _f32_params(40, chans)
    rhof = synth.rng(41).uniform(0, 1, size=(n, n, n))
    out_b, acts = C.net_forward_bf16(params, rhof)
    for a in acts[:-1]:
        np.testing.assert_array_equal(a, C.bf16(a))
    assert np.any(acts[-1] != C.bf16(acts[-1]))
    out, _ = C.net_forward(params, rhof[None])
    err = np.linalg.norm(out_b - out) / np.linalg.norm(out)
    assert 1e-5 < err < 3e-2


def test_receptive_field_forward_equals_full_forward():
    """net_forward_bf16_at (one voxel from its periodic 11^3 window) gives the
    full bf16 forward's pre-mean output, including voxels whose window wraps."""
    n = 12
    params = _f32_params(50, C.CHANNELS)
    rhof = synth.rng(51).uniform(0, 1, size=(n, n, n))
    _, acts = C.net_forward_bf16(params, rhof)
    vox = [(0, 0, 0), (11, 11, 11), (5, 0, 9), (3, 7, 11)]
    got = C.net_forward_bf16_at(params, rhof, vox)
    ref = np.array([acts[-1][:, z, y, x] for z, y, x in vox])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
