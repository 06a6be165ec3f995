"""Warm starts scaled by the energy-minimising factor s = b.x / x.A x.

Closed forms: a multiple c chi* of the solution is scaled back to chi* (the
energy along chi* is minimal at s = 1/c), so the solve needs no iteration;
a guess with b.x <= 0 (here -chi*) gets s = 0 and the solve runs as from zero.
"""
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


def cell(guess, precision="fp64", tol=1e-10):
    from paper_2405_19991_amd import Homogenization
    n = 16
    rho = synth.smoothed_noise(n, 0.1, 0.9, 4242)
    h = Homogenization(n, (1.0, 1e-3), (0.2, 0.15, 0.1, 0.0, 0.0, 0.0), vf=0.5, tol=tol, precision=precision,
                       guess=guess)
    h.set_density(rho)
    return h


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_multiple_of_solution_is_rescaled(precision):
    with cell("zero", tol=1e-12) as h:
        kappa0, st0 = h.homogenize()
        chi = h.get_field("chi")
    with cell("user", precision=precision) as h:
        h.set_guess(3.5 * chi)
        kappa, st = h.homogenize()
    assert st["converged"]
    assert max(st["iterations"]) <= 1, st
    np.testing.assert_allclose(kappa, kappa0, rtol=1e-9, atol=1e-12)


def test_opposite_guess_starts_from_zero():
    with cell("zero", tol=1e-12) as h:
        h.homogenize()
        chi = h.get_field("chi")
    with cell("zero") as h:
        _, st_zero = h.homogenize()
    with cell("user") as h:
        h.set_guess(-chi)
        kappa, st = h.homogenize()
    assert st["converged"]
    assert st["iterations"] == st_zero["iterations"]
