"""Device memory held by a context and by a batch (otm_device_bytes,
otm_batch_device_bytes): at least the per-node arrays the path needs, fixed
from creation on, and larger with the multigrid levels."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)
    from paper_2405_19991_amd import _native as N
    N.lib()
    yield


def held(n, **kw):
    from paper_2405_19991_amd import Homogenization
    rho = synth.smoothed_noise(n, 0.2, 0.6, 77)
    with Homogenization(n, (1.0, 1e-3), (0.3, 0.2, 0.1, 0, 0, 0), vf=0.4, tol=1e-6, **kw) as h:
        b0 = h.device_bytes()
        h.set_density(rho)
        h.step()
        h.prepare()
        h.apply(np.ones(3 * n ** 3))  # temporaries, freed again
        b1 = h.device_bytes()
    assert b0 == b1
    return b0


def test_context_bytes():
    n = 32
    nn = n ** 3
    fp64 = held(n, precision="fp64")
    # rho, filtered rho, k, D^-1, st, sensitivities, OC buffer (7 scalars per
    # element or node), b and x (3 loads each) and r, p (two), q: 25 doubles
    assert fp64 >= 25 * 8 * nn
    assert fp64 < 2 * 25 * 8 * nn + (64 << 20)
    mixed = held(n, precision="mixed")
    mg = held(n, precision="mixed", preconditioner="mg")
    mg64 = held(n, precision="fp64", preconditioner="mg")
    # the levels below the finest hold at most 1/7 of it again; level 0 adds
    # two float iterates and a scratch vector (9 floats per node)
    assert mg > mixed + 9 * 4 * nn
    assert mg64 > fp64 + 9 * 4 * nn
    print(f"32^3 context bytes: fp64 {fp64}, mixed {mixed}, mg {mg}, mg fp64 {mg64}", flush=True)
    assert held(2 * n, precision="fp64") > 4 * fp64


def test_batch_bytes():
    from paper_2405_19991_amd import Batch
    probs = [dict(n=n, target=(0.2, 0.2, 0.2, 0, 0, 0), vf=0.3) for n in (16, 24, 32)]
    with Batch(probs, tol=1e-6, autotune=False) as B:
        b = B.device_bytes()
    cells = sum(n ** 3 for n in (16, 24, 32))
    assert b >= 25 * 8 * cells
    print(f"batch bytes {b} for {cells} cells", flush=True)
