"""Caller-supplied streams: a context, a batch and the stateless operator
enqueue their work on the stream they are given, with the same results as
on the library's own streams."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TARGET = (0.3, 0.2, 0.1, 0.02, 0.01, 0.015)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)
    yield


def test_context_and_batch_on_a_caller_stream():
    """A context and a batch created on a torch stream give the tensors,
    iteration counts and updated densities of the same objects on their own
    streams, bit for bit (fixed tiles)."""
    import torch
    from paper_2405_19991_amd import Batch, Homogenization
    n = 16
    rho = synth.smoothed_noise(n, 0.05, 0.95, 71)
    side = torch.cuda.Stream()
    res = {}
    for key, stream in (("own", None), ("caller", side.cuda_stream)):
        print(f"context on the {key} stream", flush=True)
        with Homogenization(n, (1.0, 1e-3), TARGET, vf=0.4, tol=1e-11, autotune=False, kernel_variant=4,
                            stream=stream) as h:
            h.set_density(rho)
            r = h.step()
            res[key] = (np.array(r["kappa"]), list(r["pcg_iters"]), h.get_field("rho"))
    assert res["own"][1] == res["caller"][1]
    np.testing.assert_array_equal(res["own"][0], res["caller"][0])
    np.testing.assert_array_equal(res["own"][2], res["caller"][2])
    probs = [dict(n=8, target=TARGET, vf=0.3), dict(n=12, target=TARGET, vf=0.4)]
    rhos = [synth.smoothed_noise(p["n"], 0.1, 0.9, 72 + i) for i, p in enumerate(probs)]
    out = {}
    for key, stream in (("own", None), ("caller", side.cuda_stream)):
        print(f"batch on the {key} stream", flush=True)
        with Batch(probs, tol=1e-10, autotune=False, iteration="fused", stream=stream) as B:
            for d, r in enumerate(rhos):
                B.set_density(d, r)
            recs = B.step()
            out[key] = ([np.array(r["kappa"]) for r in recs], [B.get_field(d, "rho") for d in range(len(probs))])
    for a, b in zip(out["own"][0] + out["own"][1], out["caller"][0] + out["caller"][1]):
        np.testing.assert_array_equal(a, b)


def test_stateless_operator_is_ordered_on_the_caller_stream():
    """The operator enqueued on a side stream right after torch work on that
    stream sees that work's result (stream order, no host wait in between)
    and equals the operator on the current stream."""
    import torch
    from paper_2405_19991_amd import apply_device
    n = 24
    g = torch.Generator(device="cuda").manual_seed(5)
    k = (0.5 + torch.rand((n, n, n), generator=g, device="cuda", dtype=torch.float64)).contiguous()
    x0 = torch.randn((3, n, n, n), generator=g, device="cuda", dtype=torch.float64)
    ref = torch.empty_like(x0)
    apply_device(k, (2.0 * x0).contiguous(), ref, precision="fp64")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    y = torch.zeros_like(x0)
    side.wait_stream(torch.cuda.current_stream())  # y's fill and x0 come first
    with torch.cuda.stream(side):
        x = x0 * 2.0  # produced on the side stream
        apply_device(k, x, y, precision="fp64", stream=side.cuda_stream)
    side.synchronize()
    assert torch.equal(y, ref)
