"""Learned warm start on the GPU: the bf16 MFMA network's forward pass,
input gradients and weight gradients element by element against the
oracle's bf16 mode (the same roundings, exact sums; oracle/cnn.py), at 16^3,
32^3 and 80^3 (80^3: 2000 bricks on the 1024-block grid, so blocks walk
several bricks; from 32^3 on each wgrad wave accumulates several voxel
groups), the forward pass at 128^3 on sampled voxels (each from its
receptive field), the size of the bf16 error against the exact float64
network, training progress, and the warm-start path of the solver.

Two kinds of comparison against the bf16 mode.
* Exact: weights and biases on a 2^-7 grid, densities on a 2^-4 grid, two
  layers with such random weights and identity pass-through layers around
  them, so that every float32 sum of the kernels is exact and the roundings
  meet identical values: the GPU output equals the oracle's bit for bit
  (up to the float64 mean removal), for a 16->16 layer and for the 16->3
  last layer.
* Random float32 weights: relative Frobenius error <= 1.5e-3 (forward) and
  <= 3e-3 (gradients), every element within 1e-2 (forward) / 5e-3
  (gradients) of the field's largest magnitude.  What is left is the float32
  accumulation order of the MFMA sums, which moves a few pre-activations
  across a bf16 rounding boundary (one unit, 2^-8 relative) and carries that
  through the later layers; measured: forward 7e-4 to 1.0e-3 (worst element
  3.7e-3 to 7.3e-3), gradients 8e-6 to 2.6e-3, falling with the grid size as
  the flips average out (about 2e-3 at 16^3, 5e-4 at 32^3, 1e-4 at 80^3)."""
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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def close(got, ref, what, fro=1.5e-3, elem=1e-2):
    e_f = rel(got, ref)
    e_m = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{what}: rel fro {e_f:.2e}, max elem {e_m:.2e}", flush=True)
    assert e_f <= fro and e_m <= elem, what


def setup(n_max, seed):
    """A network with He-initialised weights and nonzero biases (every path
    exercised); returns it and its parameters as float64 layers."""
    from paper_2405_19991_amd import Network
    from paper_2405_19991_amd.api import compact_to_layers
    net = Network(n_max=n_max, seed=seed)
    p = net.params()
    g = synth.rng(seed + 1)
    q = 0
    for L in compact_to_layers(p):
        q += L["W"].size
        p[q:q + L["b"].size] = g.uniform(-0.05, 0.05, size=L["b"].size)
        q += L["b"].size
    net.set_params(p)
    return net, compact_to_layers(net.params())


def gpu_forward(net, rhof):
    import torch
    n = rhof.shape[0]
    rd = torch.from_numpy(rhof.reshape(-1).copy()).cuda()
    chi0 = torch.empty(3 * n ** 3, dtype=torch.float64, device="cuda")
    net.forward(rd, chi0)
    torch.cuda.synchronize()
    return chi0.cpu().numpy().reshape(3, n, n, n)


def exact_params(active, seed):
    """Compact parameters: the layers in `active` get weights and biases that
    are small integers times 2^-7 (bf16-exact); every other layer passes its
    input through (centre tap 1 from channel c to channel c, and for the
    16 -> 3 last layer from every channel c to output c mod 3, so that all
    sixteen channels reach the output)."""
    from paper_2405_19991_amd.api import compact_to_layers
    chans = C.CHANNELS
    g = synth.rng(seed)
    parts = []
    for li, (cin, cout) in enumerate(zip(chans[:-1], chans[1:])):
        if li in active:
            W = g.integers(-3, 4, size=(cout, cin, 27)) * 2.0 ** -7
            b = g.integers(-4, 5, size=cout) * 2.0 ** -7
        else:
            W = np.zeros((cout, cin, 27))
            for c in range(cin):
                if c < cout or cout == 3:
                    W[c % cout, c, 13] = 1.0
            b = np.zeros(cout)
        parts += [W.reshape(-1), b]
    p = np.concatenate(parts).astype(np.float32)
    return p, compact_to_layers(p)


@pytest.mark.parametrize("active", [(0, 1), (0, 4)], ids=["layer16to16", "last_layer"])
@pytest.mark.parametrize("n", [16, 80])
def test_forward_exact_arithmetic(n, active):
    """Bit-exact forward: with every kernel sum exact, the output equals the
    bf16 oracle's to float64 rounding of the mean removal."""
    from paper_2405_19991_amd import Network
    p, layers = exact_params(active, 17 + n)
    rhof = np.round(synth.smoothed_noise(n, 0.0, 1.0, 19) * 16) / 16
    with Network(n_max=n, seed=0) as net:
        net.set_params(p)
        print(f"nn exact forward {n}^3 active {active}", flush=True)
        out = gpu_forward(net, rhof)
    out_ref, _ = C.net_forward_bf16(layers, rhof)
    err = np.abs(out - out_ref).max()
    print(f"exact forward {n}^3 {active}: max abs diff {err:.2e} (max |out| {np.abs(out_ref).max():.3f})", flush=True)
    assert np.abs(out_ref).max() > 1e-3
    assert err <= 1e-13


def test_forward_exact_arithmetic_128_sampled():
    """The bit-exact forward at 128^3 (8 bricks per block), at 256 voxels."""
    from paper_2405_19991_amd import Network
    n = 128
    p, layers = exact_params((0, 1), 23)
    rhof = np.round(synth.smoothed_noise(n, 0.0, 1.0, 24) * 16) / 16
    with Network(n_max=n, seed=0) as net:
        net.set_params(p)
        out = gpu_forward(net, rhof)
    g = synth.rng(25)
    vox = [tuple(int(c) for c in g.integers(0, n, size=3)) for _ in range(256)]
    vox[1:4] = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5)]
    ref = C.net_forward_bf16_at(layers, rhof, vox)
    got = np.array([out[:, z, y, x] for z, y, x in vox])
    assert np.abs((got[1:] - got[0]) - (ref[1:] - ref[0])).max() <= 1e-13


@pytest.mark.parametrize("n", [16, 32, 80])
def test_forward_matches_bf16_oracle(n):
    net, layers = setup(n, 3)
    rhof = synth.smoothed_noise(n, 0.1, 0.9, 5)
    print(f"nn forward {n}^3", flush=True)
    out = gpu_forward(net, rhof)
    net.close()
    out_ref, _ = C.net_forward_bf16(layers, rhof)
    close(out, out_ref, f"forward {n}^3")
    np.testing.assert_allclose(out.mean(axis=(1, 2, 3)), 0.0, atol=1e-12)


def test_forward_128_sampled_voxels():
    """The 128^3 forward (8192 bricks, 8 per block) at 256 seeded voxels,
    each against the oracle's output from that voxel's 11^3 receptive field;
    differences to the first sample cancel the global mean removal."""
    n = 128
    net, layers = setup(n, 7)
    rhof = synth.smoothed_noise(n, 0.1, 0.9, 8)
    print("nn forward 128^3 sampled", flush=True)
    out = gpu_forward(net, rhof)
    net.close()
    g = synth.rng(9)
    vox = [tuple(int(c) for c in g.integers(0, n, size=3)) for _ in range(256)]
    vox[1:4] = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5)]  # wrapped windows
    ref = C.net_forward_bf16_at(layers, rhof, vox)
    got = np.array([out[:, z, y, x] for z, y, x in vox])
    close(got[1:] - got[0], ref[1:] - ref[0], "forward 128^3 (sampled differences)")


@pytest.mark.parametrize("n", [16, 32, 80])
def test_gradients_match_bf16_oracle(n):
    """otm_nn_accumulate (loss, dL/dout in bf16, per-layer masked input
    gradients in bf16, weight and bias gradients in float32) against the bf16
    oracle's backward from the same forward."""
    import torch
    from paper_2405_19991_amd.api import compact_to_layers
    net, layers = setup(n, 11)
    rhof = synth.smoothed_noise(n, 0.1, 0.9, 12)
    chi = synth.random_vectors(n, 3, 13) * 0.1
    print(f"nn gradients {n}^3", flush=True)
    rd = torch.from_numpy(rhof.reshape(-1).copy()).cuda()
    cd = torch.from_numpy(chi.reshape(-1).copy()).cuda()
    net.zero_grads()
    L = net.accumulate(rd, cd)
    g = compact_to_layers(net.grads())
    net.close()
    out_ref, acts = C.net_forward_bf16(layers, rhof)
    L_ref, dout = C.loss_bf16(out_ref, chi)
    g_ref = C.net_backward_bf16(layers, acts, dout)
    assert L == pytest.approx(L_ref, rel=1e-5)
    for li in range(len(layers)):
        close(g[li]["W"], g_ref[li]["W"], f"dW layer {li} {n}^3", fro=3e-3, elem=5e-3)
        if li < len(layers) - 1:
            close(g[li]["b"], g_ref[li]["b"], f"db layer {li} {n}^3", fro=3e-3, elem=5e-3)
        else:
            # the exact gradient of the last bias is zero (mean removal); what
            # is left is the sum of the bf16-rounded loss gradient, on both sides
            scale = np.abs(g_ref[li]["W"]).max()
            assert np.abs(g[li]["b"] - g_ref[li]["b"]).max() <= 2e-3 * scale


def test_bf16_error_against_exact_network():
    """Size of what bf16 costs: the GPU forward and gradients against the
    exact float64 network on the same float32 parameters, at 16^3."""
    import torch
    from paper_2405_19991_amd.api import compact_to_layers
    n = 16
    net, layers = setup(n, 5)
    rhof = synth.smoothed_noise(n, 0.1, 0.9, 7)
    chi = synth.random_vectors(n, 3, 6) * 0.1
    out = gpu_forward(net, rhof)
    out_ref, acts = C.net_forward(layers, rhof[None])
    assert rel(out, out_ref) < 3e-2
    L_ref, dout = C.loss(out_ref, chi)
    g_ref = C.net_backward(layers, acts, dout)
    rd = torch.from_numpy(rhof.reshape(-1).copy()).cuda()
    cd = torch.from_numpy(chi.reshape(-1).copy()).cuda()
    net.zero_grads()
    L = net.accumulate(rd, cd)
    g = compact_to_layers(net.grads())
    net.close()
    assert L == pytest.approx(L_ref, rel=3e-2)
    for li in range(len(layers)):
        assert rel(g[li]["W"], g_ref[li]["W"]) < 6e-2, li
        if li < len(layers) - 1:
            assert rel(g[li]["b"], g_ref[li]["b"]) < 6e-2, li


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
