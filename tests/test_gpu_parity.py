"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances follow from the arithmetic:
* operator: both sides sum <= 21 products per row in float64 (float32 for the
  mixed operator); compared entry-wise against eps * sum_u |A_vu| |x_u|;
* tensor: its error is second order in the solve error, so solves to 1e-11
  (FP64) give a relative Frobenius error far below 1e-9; the mixed path is
  held to 1e-5;
* fields from shared inputs (filter, SIMP, loads, diagonal, sensitivities
  from a given chi, OC from given sensitivities): 1e-12 relative.
Sizes span several 256-thread blocks and ragged tails (n = 5, 12, 13, 16).
"""
import numpy as np
import pytest

import oracle as O
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


def make(n, rho, precision="fp64", tol=1e-11, target=(0.3, 0.2, 0.1, 0.02, 0.01, 0.015), **kw):
    from paper_2405_19991_amd import Homogenization
    h = Homogenization(n, (1.0, 1e-3), target, vf=float(np.mean(rho)), precision=precision, tol=tol, **kw)
    h.set_density(rho)
    return h


def abs_scale(A: O.CSR27, x):
    """sum_u |A_vu| |x_u| per node, per load"""
    absA = O.CSR27(A.n, A.cols, np.abs(A.vals))
    return np.stack([absA.matvec(np.abs(x[i])) for i in range(3)])


# ------------------------------------------------------------------ operator

@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [5, 12, 13, 16, 33])
def test_apply_fp64(n, variant):
    rho = synth.random_field(n, 100 + n, 1e-3, 1.0)
    x = synth.random_vectors(n, 3, 200 + n)
    prm = O.Params()
    k = O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal)
    A = O.assemble(k)
    y_ref = np.stack([A.matvec(x[i]) for i in range(3)])
    with make(n, rho, kernel_variant=variant) as h:
        h.prepare()
        y = h.apply(x, "fp64")
    scale = abs_scale(A, x)
    assert np.all(np.abs(y - y_ref) <= 64 * np.finfo(float).eps * scale + 1e-300)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [5, 16, 40])
def test_apply_mixed(n, variant):
    rho = synth.random_field(n, 300 + n, 1e-3, 1.0)
    x = synth.random_vectors(n, 3, 400 + n)
    prm = O.Params()
    k = O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal)
    A = O.assemble(k)
    y_ref = np.stack([A.matvec(x[i]) for i in range(3)])
    with make(n, rho, precision="mixed", kernel_variant=variant) as h:
        h.prepare()
        y = h.apply(x, "mixed")
    scale = abs_scale(A, x)
    assert np.all(np.abs(y - y_ref) <= 64 * np.finfo(np.float32).eps * scale)


def test_stateless_apply_device_variants():
    """otm_apply_device on torch device memory: tiled and direct-gather kernels
    agree with the oracle at a size with several tiles and a ragged tail."""
    import torch
    from paper_2405_19991_amd import apply_device
    n = 38
    rho = synth.random_field(n, 41, 1e-3, 1.0)
    prm = O.Params()
    k = O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal)
    A = O.assemble(k)
    x = synth.random_vectors(n, 3, 42)
    y_ref = np.stack([A.matvec(x[i]) for i in range(3)])
    scale = abs_scale(A, x)
    for prec, dt, eps in (("fp64", torch.float64, np.finfo(float).eps), ("mixed", torch.float32, np.finfo(np.float32).eps)):
        kd = torch.from_numpy(k.reshape(-1)).to(dt).cuda()
        xd = torch.from_numpy(x.reshape(-1)).to(dt).cuda()
        for variant in (0, 1, 2, 3):
            yd = torch.full_like(xd, float("nan"))
            apply_device(kd, xd, yd, prec, variant=variant)
            torch.cuda.synchronize()
            y = yd.double().cpu().numpy().reshape(3, n, n, n)
            assert np.all(np.abs(y - y_ref) <= 64 * eps * scale), (prec, variant)


@pytest.mark.parametrize("tx,tz", [(16, 1), (32, 3), (64, 2), (64, 7), (16, 40), (32, 1)])
@pytest.mark.parametrize("n", [20, 37, 38])
def test_apply_tile_shapes(n, tx, tz):
    """The z-march and ring kernels for every tile width, plane counts that do
    and do not divide n, and tiles wider than the cell (n < tile width)."""
    rho = synth.random_field(n, 70 + n, 1e-3, 1.0)
    x = synth.random_vectors(n, 3, 71 + n)
    prm = O.Params()
    k = O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal)
    A = O.assemble(k)
    y_ref = np.stack([A.matvec(x[i]) for i in range(3)])
    scale = abs_scale(A, x)
    for variant in (0, 2, 3):
        with make(n, rho, kernel_variant=variant, tile_tx=tx, tile_tz=tz) as h:
            h.prepare()
            y = h.apply(x, "fp64")
        assert np.all(np.abs(y - y_ref) <= 64 * np.finfo(float).eps * scale), variant


def test_pcg_tile_shapes_agree():
    """Full FP64 solves with different z-march tiles give the same tensor."""
    n = 24
    rho = synth.smoothed_noise(n, 0.05, 0.95, 73)
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    for variant, tx, tz in ((0, 32, 5), (0, 64, 3), (3, 16, 5), (3, 32, 2), (3, 64, 24), (2, 32, 4)):
        with make(n, rho, tol=1e-11, tile_tx=tx, tile_tz=tz, kernel_variant=variant) as h:
            kappa, st = h.homogenize()
        assert st["converged"] and rel_fro(kappa, ref["kappa"]) <= 1e-9, (variant, tx, tz)


# ------------------------------------------------------------- setup fields

@pytest.mark.parametrize("n", [4, 13])
def test_prepare_fields(n):
    rho = synth.random_field(n, 500 + n, 1e-3, 1.0)
    prm = O.Params()
    rhof = O.density_filter(rho, prm.rfilter)
    k = O.simp(rhof, prm.k0, prm.kmin, prm.penal)
    b = O.macro_loads(k)
    b -= b.reshape(3, -1).mean(axis=1)[:, None, None, None]
    A = O.assemble(k)
    diag = A.vals[:, 13].reshape((n,) * 3)
    with make(n, rho) as h:
        h.prepare()
        np.testing.assert_allclose(h.get_field("rhof"), rhof, rtol=1e-14)
        np.testing.assert_allclose(h.get_field("k"), k, rtol=1e-13)
        np.testing.assert_allclose(h.get_field("b"), b, rtol=0, atol=1e-14 * np.abs(b).max())
        np.testing.assert_allclose(h.get_field("diag"), diag, rtol=1e-13)


def test_filter_radius_variants():
    n = 9
    rho = synth.random_field(n, 77, 1e-3, 1.0)
    for r in (0.0, 0.9, 1.5, 2.5):
        with make(n, rho, filter_radius=r) as h:
            h.prepare()
            np.testing.assert_allclose(h.get_field("rhof"), O.density_filter(rho, r), rtol=1e-13)


# ------------------------------------------------------------------- tensor

def rel_fro(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [6, 12, 16, 35])
def test_homogenize_fp64(n, variant):
    rho = synth.random_field(n, 600 + n, 0.05, 1.0)
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    with make(n, rho, tol=1e-11, kernel_variant=variant) as h:
        kappa, st = h.homogenize()
        assert st["converged"]
        assert max(st["rel_residual"]) <= 1e-11
        assert rel_fro(kappa, ref["kappa"]) <= 1e-9
        chi = h.get_field("chi")
    # chi is first order in the solve error
    assert np.abs(chi - ref["chi"]).max() <= 1e-8 * np.abs(ref["chi"]).max()
    assert np.abs(chi.reshape(3, -1).mean(axis=1)).max() < 1e-14


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [8, 16, 34])
def test_homogenize_mixed(n, variant):
    rho = synth.smoothed_noise(n, 0.1, 0.9, 700 + n)
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    with make(n, rho, precision="mixed", tol=1e-6, kernel_variant=variant) as h:
        kappa, st = h.homogenize()
        assert st["converged"]
        assert max(st["rel_residual"]) <= 1e-6
        assert rel_fro(kappa, ref["kappa"]) <= 1e-5


def test_uniform_and_laminate_closed_forms():
    n = 16
    with make(n, np.full((n, n, n), 0.37)) as h:
        kappa, st = h.homogenize()
        kc = 1e-3 + 0.37 ** 3 * (1 - 1e-3)
        np.testing.assert_allclose(kappa, [kc, kc, kc, 0, 0, 0], atol=1e-15)
        assert st["iterations"] == [0, 0, 0]
    prof = synth.rng(9).uniform(0.05, 1.0, size=n)
    rho = np.broadcast_to(prof[:, None, None], (n, n, n)).copy()
    with make(n, rho, tol=1e-12) as h:
        kappa, _ = h.homogenize()
        k = h.get_field("k")[:, 0, 0]
    np.testing.assert_allclose(kappa[:3], [k.mean(), k.mean(), 1 / np.mean(1 / k)], rtol=1e-10)
    np.testing.assert_allclose(kappa[3:], 0.0, atol=1e-12)


# ------------------------------------------------------- steps, shared inputs

@pytest.mark.parametrize("n", [5, 12])
def test_sensitivity_from_shared_chi(n):
    rho = synth.random_field(n, 800 + n, 0.1, 0.9)
    prm = O.Params(tol=1e-13)
    ref = O.homogenize(rho, prm)
    w = np.array([0.3, -0.2, 0.1, 0.05, -0.02, 0.01])
    s_ref = O.sensitivities(ref, w, prm)
    with make(n, rho) as h:
        h.prepare()
        h.set_field("chi", ref["chi"])
        s = h.sensitivity(w)
        st = h.get_field("sens_elem")
    st_ref = O.element_sensitivity(ref["rhof"], ref["E"], w, prm.k0, prm.kmin, prm.penal)
    assert np.abs(st - st_ref).max() <= 1e-12 * np.abs(st_ref).max()
    assert np.abs(s - s_ref).max() <= 1e-12 * np.abs(s_ref).max()


@pytest.mark.parametrize("n,vstar", [(6, 0.45), (13, 0.3), (16, 0.62)])
def test_oc_from_shared_sensitivities(n, vstar):
    g = synth.rng(900 + n)
    rho = g.uniform(0.05, 0.95, size=(n, n, n))
    s = g.standard_normal((n, n, n)) * 1e-4 - 5e-5
    rn_ref, lam_ref, _ = O.oc_update(rho, s, vstar)
    with make(n, rho) as h:
        h.set_field("sens", s)
        rn, lam = h.oc_update(vstar)
    assert lam == pytest.approx(lam_ref, rel=1e-12)
    np.testing.assert_allclose(rn, rn_ref, rtol=1e-12, atol=0)


def test_oc_degenerate_cases():
    n = 8
    rho = np.full((n, n, n), 0.5)
    with make(n, rho) as h:       # all sensitivities positive: lower move limit
        h.set_field("sens", np.full((n, n, n), 1e-3))
        rn, _ = h.oc_update(0.5)
    np.testing.assert_allclose(rn, 0.45, atol=1e-15)
    with make(n, rho) as h:       # unreachable V*: upper move limit where s < 0
        s = -np.ones((n, n, n)) * 1e-4
        h.set_field("sens", s)
        rn, _ = h.oc_update(0.99)
        rn_ref, _, _ = O.oc_update(rho, s, 0.99)
    np.testing.assert_allclose(rn, rn_ref, rtol=1e-12)


# ------------------------------------------------------------ full iterations

def test_first_iterations_track_oracle():
    w = synth.config1()
    prm = O.Params(tol=1e-10)
    gov = O.Governor(w.vf)
    rho_ref = w.rho0.copy()
    from paper_2405_19991_amd import Homogenization
    with Homogenization(w.n, (w.k0, w.kmin), w.target, vf=w.vf, tol=1e-10) as h:
        h.set_density(w.rho0)
        for it in range(3):
            rec = h.step()
            rho_ref, r_ref, _, _ = O.oc_iteration(rho_ref, w.target, gov, prm)
            assert rec["g"] == pytest.approx(r_ref.g, rel=1e-6)
            np.testing.assert_allclose(rec["kappa"], r_ref.kappa, rtol=1e-6, atol=1e-9)
            assert rec["vstar"] == pytest.approx(r_ref.vstar, rel=1e-9)
        rho = h.get_field("rho")
    assert np.abs(rho - rho_ref).max() < 1e-6


def test_errors_and_state():
    from paper_2405_19991_amd import Homogenization
    from paper_2405_19991_amd import _native as N
    n = 6
    with Homogenization(n) as h:
        with pytest.raises(N.OTMError) as e:
            h.sensitivity(np.zeros(6))
        assert e.value.status == N.OTM_ESTATE
        bad = np.full((n, n, n), 0.3)
        bad[1, 2, 3] = np.nan
        with pytest.raises(N.OTMError) as e:
            h.set_density(bad)
        assert e.value.status == N.OTM_ENONFINITE
        with pytest.raises(N.OTMError) as e:
            h.set_density(np.zeros(5))
        assert e.value.status == N.OTM_EINVAL
    # max_iter too small: not converged, outputs filled
    rho = synth.random_field(n, 5, 0.1, 0.9)
    with make(n, rho, max_iter=2, check_every=1) as h:
        kappa, st = h.homogenize()
        assert st["status"] == N.OTM_NOT_CONVERGED and not st["converged"]
        assert np.all(np.isfinite(kappa))


def test_clamp_on_entry():
    n = 5
    rho = synth.random_field(n, 3, -0.5, 1.5)
    with make(n, rho) as h:
        got = h.get_field("rho")
    np.testing.assert_array_equal(got, np.clip(rho, 1e-3, 1.0))
