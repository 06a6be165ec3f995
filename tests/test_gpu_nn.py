"""Learned warm start on the GPU: bf16 MFMA forward/backward against the FP64
CNN reference (on the same bf16-rounded parameters and input), training
progress, and the warm-start path of the solver."""
import numpy as np
import pytest

import oracle as O
from oracle import cnn as C
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)


def bf16(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def setup(n, seed):
    import torch
    from paper_2405_19991_amd import Network
    from paper_2405_19991_amd.api import compact_to_layers
    net = Network(n_max=32, seed=seed)
    p = net.params()
    # non-zero biases so every path is exercised
    layers = compact_to_layers(p)
    g = synth.rng(seed + 1)
    q = 0
    for L in layers:
        q += L["W"].size
        p[q:q + L["b"].size] = g.uniform(-0.05, 0.05, size=L["b"].size)
        q += L["b"].size
    net.set_params(p)
    layers = compact_to_layers(p)
    for L in layers:
        L["W"] = bf16(L["W"])
    rhof = synth.smoothed_noise(n, 0.1, 0.9, seed + 2)
    x = bf16(rhof)[None]
    return net, layers, rhof, x, torch


def test_forward_matches_reference():
    n = 16
    net, layers, rhof, x, torch = setup(n, 3)
    out_ref, _ = C.net_forward(layers, x)
    rd = torch.from_numpy(rhof.reshape(-1)).cuda()
    chi0 = torch.empty(3 * n ** 3, dtype=torch.float64, device="cuda")
    net.forward(rd, chi0)
    torch.cuda.synchronize()
    out = chi0.cpu().numpy().reshape(3, n, n, n)
    assert rel(out, out_ref) < 3e-2
    np.testing.assert_allclose(out.mean(axis=(1, 2, 3)), 0.0, atol=1e-12)


def test_gradients_match_reference():
    n = 16
    net, layers, rhof, x, torch = setup(n, 5)
    chi = synth.random_vectors(n, 3, 6) * 0.1
    out_ref, acts = C.net_forward(layers, x)
    L_ref, dout = C.loss(out_ref, chi)
    g_ref = C.net_backward(layers, acts, dout)
    rd = torch.from_numpy(rhof.reshape(-1)).cuda()
    cd = torch.from_numpy(chi.reshape(-1)).cuda()
    net.zero_grads()
    L = net.accumulate(rd, cd)
    assert L == pytest.approx(L_ref, rel=3e-2)
    from paper_2405_19991_amd.api import compact_to_layers
    g = compact_to_layers(net.grads())
    for li in range(len(layers)):
        assert rel(g[li]["W"], g_ref[li]["W"]) < 6e-2, li
        if li < len(layers) - 1:
            assert rel(g[li]["b"], g_ref[li]["b"]) < 6e-2, li
        else:
            # the output mean removal makes the loss invariant to the last bias:
            # its exact gradient is zero; bf16 rounding of dL/dout leaves a residue
            assert np.abs(g[li]["b"]).max() < 1e-2 * np.abs(g_ref[li]["W"]).max(), li


def test_training_reduces_loss_and_warm_start_path():
    import torch
    from paper_2405_19991_amd import Homogenization, Network
    n = 16
    data = []
    prm = O.Params(tol=1e-10)
    for s in range(4):
        rho = synth.smoothed_noise(n, 0.1, 0.9, 40 + s)
        h = O.homogenize(rho, prm, with_energies=False)
        data.append((torch.from_numpy(h["rhof"].reshape(-1)).cuda(), torch.from_numpy(h["chi"].reshape(-1)).cuda()))
    net = Network(n_max=16, seed=1)
    losses = []
    for epoch in range(40):
        tot = 0.0
        net.zero_grads()
        for rd, cd in data:
            tot += net.accumulate(rd, cd)
        net.adam(3e-3, len(data))
        losses.append(tot / len(data))
    assert losses[-1] < 0.5 * losses[0]
    # the solver with a learned start still reaches the oracle's tensor
    rho = synth.smoothed_noise(n, 0.1, 0.9, 40)
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    with Homogenization(n, (1.0, 1e-3), (0.2, 0.2, 0.1, 0, 0, 0), vf=0.5, tol=1e-11, guess="learned") as h:
        h.set_network(net)
        h.set_density(rho)
        kappa, st = h.homogenize()
        used = h.timings()[6]
    assert st["converged"]
    assert np.linalg.norm(kappa - ref["kappa"]) / np.linalg.norm(ref["kappa"]) < 1e-9
    assert used in (0.0, 1.0)
