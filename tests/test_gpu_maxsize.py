"""The largest grid the library accepts (n = 1024: 3 n^3 > 2^31 node values
per vector, so every global offset must be 64-bit): the stand-alone operator
on caller device memory, checked against the oracle's node-by-node operator
at sampled nodes, every face and corner of the periodic cell among them."""
import itertools

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

N = 1024


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.empty_cache()


def sample_nodes(n, count, seed):
    edge = [0, 1, n - 2, n - 1]
    nodes = list(itertools.product(edge, edge, edge))  # every corner and face neighbourhood
    g = np.random.Generator(np.random.PCG64(seed))
    nodes += [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(count)]
    return nodes


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_operator_on_the_largest_grid(precision):
    import torch
    from paper_2405_19991_amd import apply_device
    n = N
    dtype = torch.float64 if precision == "fp64" else torch.float32
    print(f"operator n={n} {precision}: generating inputs", flush=True)
    g = torch.Generator(device="cuda").manual_seed(2024)
    k = torch.rand((n, n, n), generator=g, device="cuda", dtype=dtype).mul_(0.999).add_(0.001)
    x = torch.randn((3, n, n, n), generator=g, device="cuda", dtype=dtype)
    y = torch.empty_like(x)
    print(f"operator n={n} {precision}: apply", flush=True)
    apply_device(k, x, y, precision="fp64" if precision == "fp64" else "mixed")
    torch.cuda.synchronize()
    nodes = sample_nodes(n, 200, 7)
    i = torch.tensor([p[0] for p in nodes], device="cuda")
    j = torch.tensor([p[1] for p in nodes], device="cuda")
    kz = torch.tensor([p[2] for p in nodes], device="cuda")
    kp = torch.empty((len(nodes), 2, 2, 2), dtype=torch.float64)
    for cz, cy, cx in itertools.product((0, 1), repeat=3):
        kp[:, cz, cy, cx] = k[(kz + cz - 1) % n, (j + cy - 1) % n, (i + cx - 1) % n].double().cpu()
    xp = torch.empty((len(nodes), 3, 3, 3, 3), dtype=torch.float64)
    for dz, dy, dx in itertools.product(range(3), repeat=3):
        xp[:, :, dz, dy, dx] = x[:, (kz + dz - 1) % n, (j + dy - 1) % n, (i + dx - 1) % n].double().cpu().T
    got = y[:, kz, j, i].double().cpu().T.numpy()
    del k, x, y
    torch.cuda.empty_cache()
    ref = O.apply_at(kp.numpy(), xp.numpy())
    bound = O.apply_at(kp.numpy(), xp.numpy(), absolute=True)
    eps = np.finfo(np.float64 if precision == "fp64" else np.float32).eps
    err = np.abs(got - ref) / (bound * eps)
    print(f"operator n={n} {precision}: max error {err.max():.1f} ulp of sum |A||x|", flush=True)
    assert err.max() <= 64.0
