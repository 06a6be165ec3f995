"""otm_oc_update_noalloc (the OC update that allocates nothing) against
otm_oc_update of a context, through the C ABI.

Both compute the Optimality Criteria update (Sec. 3.3, OCOptimizer) from the
same densities and sensitivities; the no-allocation call recomputes q_e from
(rho_e, s_e) with the same expression and reduces over the same grids, so
rho_new and lambda must agree to the OC bar of 1e-12 (in practice exactly).
Two calls in a row, the second on a smaller cell, check that what the first
call left in the shared scratch does not leak into the second; a third call
updates in place.  Inputs: densities 0.45 +- 0.4 (clamped to [rho_min, 1] by
the context, and clamped the same way here), sensitivities mostly negative
with ~15 % positive entries (those go to the lower move limit)."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RHO_MIN = 1e-3


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)
    from paper_2405_19991_amd import _native as N
    N.lib()
    yield


def inputs(n, seed):
    rho = np.clip(synth.uniform_noise(n, 0.45, 0.4, seed), RHO_MIN, 1.0)
    g = synth.rng(seed + 1)
    s = -g.uniform(0.0, 2e-3, size=(n, n, n)) / n ** 3
    s[g.uniform(size=(n, n, n)) < 0.15] *= -0.5
    return rho, s


def context_oc(n, rho, s, vstar):
    from paper_2405_19991_amd import Homogenization
    with Homogenization(n, (1.0, 1e-3), [0.1, 0.1, 0.1, 0, 0, 0], vf=0.3) as h:
        h.set_density(rho)
        h.set_field("sens", s)
        return h.oc_update(vstar)


def noalloc_oc(rho, s, vstar, in_place=False):
    import torch
    from paper_2405_19991_amd import oc_update_noalloc
    rd = torch.from_numpy(rho.ravel().copy()).cuda()
    sd = torch.from_numpy(s.ravel().copy()).cuda()
    lam = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    out = rd if in_place else torch.full_like(rd, -7.0)
    oc_update_noalloc(rd, sd, vstar, out=out, lam=lam, move=0.05, eta=0.5, rho_min=RHO_MIN)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(rho.shape), float(lam.item())


@pytest.mark.parametrize("n,seed,dv,in_place", [(40, 11, -0.02, False), (20, 12, 0.01, False), (24, 13, -0.005, True)])
def test_noalloc_matches_context_oc(n, seed, dv, in_place):
    rho, s = inputs(n, seed)
    vstar = float(rho.mean() + dv)
    ref_rho, ref_lam = context_oc(n, rho, s, vstar)
    got_rho, got_lam = noalloc_oc(rho, s, vstar, in_place=in_place)
    assert np.abs(got_rho - ref_rho).max() <= 1e-12
    assert abs(got_lam - ref_lam) <= 1e-12 * abs(ref_lam)
    assert abs(got_rho.mean() - vstar) < 1e-9  # volume constraint met (vstar reachable here)


def test_noalloc_two_calls_second_smaller():
    """Back-to-back calls on one stream, 48^3 then 16^3, each against its
    context result: the second call must not see the first one's scratch."""
    import torch
    from paper_2405_19991_amd import oc_update_noalloc
    cases = []
    for n, seed, dv in ((48, 21, -0.03), (16, 22, 0.02)):
        rho, s = inputs(n, seed)
        vstar = float(rho.mean() + dv)
        cases.append((n, rho, s, vstar, context_oc(n, rho, s, vstar)))
    outs = []
    for n, rho, s, vstar, _ in cases:
        rd = torch.from_numpy(rho.ravel().copy()).cuda()
        sd = torch.from_numpy(s.ravel().copy()).cuda()
        lam = torch.zeros(1, dtype=torch.float64, device="cuda")
        outs.append((oc_update_noalloc(rd, sd, vstar, lam=lam, rho_min=RHO_MIN), lam))
    torch.cuda.synchronize()
    for (n, rho, s, vstar, (ref_rho, ref_lam)), (out, lam) in zip(cases, outs):
        got = out.cpu().numpy().reshape(rho.shape)
        assert np.abs(got - ref_rho).max() <= 1e-12, n
        assert abs(float(lam.item()) - ref_lam) <= 1e-12 * abs(ref_lam), n


def test_noalloc_rejects_invalid_arguments():
    import torch
    from paper_2405_19991_amd import _native as N
    L = N.lib()
    oc = N.OcOpts(0.05, 0.5, RHO_MIN)
    rd = torch.full((8 ** 3,), 0.5, dtype=torch.float64, device="cuda")
    sd = torch.full((8 ** 3,), -1e-4, dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.otm_oc_update_noalloc(2000, p(rd), p(sd), 0.3, ctypes.byref(oc), p(rd), None, None) == N.OTM_EINVAL
    assert L.otm_oc_update_noalloc(8, p(rd), p(sd), 1.5, ctypes.byref(oc), p(rd), None, None) == N.OTM_EINVAL
    assert L.otm_oc_update_noalloc(8, p(rd), p(sd), 0.3, ctypes.byref(oc), p(sd), None, None) == N.OTM_EINVAL
    assert L.otm_oc_update_noalloc(8, p(rd), p(sd), 0.3, None, p(rd), None, None) == N.OTM_EINVAL
