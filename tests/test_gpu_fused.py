"""Fused PCG iteration (kernel_variant 4): one z-march pass and one reduction
per iteration, with the next r.D^-1 r taken from the expansion of
(r - a q)^T D^-1 (r - a q).  Its iterates are those of plain Jacobi-PCG in exact
arithmetic, so it is held to the same oracle tolerances as the other kernels
(tensor relative error 1e-9 in FP64 solved to 1e-11, 1e-5 mixed), and its
iteration counts to those of the two-pass iteration.
"""
import itertools

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


def rel_fro(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [4, 6, 12, 16, 34, 48])
def test_fused_fp64_matches_oracle(n):
    print(f"fused fp64 n={n}", flush=True)
    rho = synth.random_field(n, 900 + n, 0.05, 1.0)
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    with make(n, rho, tol=1e-11, kernel_variant=4) as h:
        assert h.tile()["variant"] == 4
        kappa, st = h.homogenize()
        chi = h.get_field("chi")
    assert st["converged"] and max(st["rel_residual"]) <= 1e-11
    assert rel_fro(kappa, ref["kappa"]) <= 1e-9
    assert np.abs(chi - ref["chi"]).max() <= 1e-8 * np.abs(ref["chi"]).max()
    assert np.abs(chi.reshape(3, -1).mean(axis=1)).max() < 1e-14


@pytest.mark.parametrize("n", [8, 16, 34, 64])
def test_fused_mixed_matches_oracle(n):
    print(f"fused mixed n={n}", flush=True)
    rho = synth.smoothed_noise(n, 0.1, 0.9, 950 + n)
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    with make(n, rho, precision="mixed", tol=1e-6, kernel_variant=4) as h:
        kappa, st = h.homogenize()
    assert st["converged"] and max(st["rel_residual"]) <= 1e-6
    assert rel_fro(kappa, ref["kappa"]) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_iterations_match_two_pass(precision):
    """Same Krylov iterates as the two-pass iteration: equal counts up to a
    couple of iterations of rounding (and the check interval's granularity)."""
    n = 32
    rho = synth.smoothed_noise(n, 0.05, 0.95, 31)
    tol = 1e-10 if precision == "fp64" else 1e-6
    res = {}
    for v in (0, 4):
        with make(n, rho, precision=precision, tol=tol, kernel_variant=v, autotune=0, check_every=1) as h:
            kappa, st = h.homogenize()
        res[v] = (np.array(st["iterations"]), np.array(kappa))
    assert np.all(np.abs(res[4][0] - res[0][0]) <= 2 + res[0][0] // 50), res
    assert rel_fro(res[4][1], res[0][1]) <= (1e-9 if precision == "fp64" else 1e-5)


def test_fused_tile_shapes_agree():
    n = 24
    rho = synth.smoothed_noise(n, 0.05, 0.95, 74)
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    for tx, tz in ((32, 5), (64, 3), (32, 24), (64, 7)):
        print(f"fused tile tx={tx} tz={tz}", flush=True)
        with make(n, rho, tol=1e-11, tile_tx=tx, tile_tz=tz, kernel_variant=4) as h:
            kappa, st = h.homogenize()
        assert st["converged"] and rel_fro(kappa, ref["kappa"]) <= 1e-9, (tx, tz)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_inactive_loads(precision):
    """Laminate along z: the x and y loads vanish (inactive from the start) and
    only the z load iterates -- the kernel's per-load skip path.  Closed forms:
    arithmetic mean across the layers' plane, harmonic mean along z."""
    n = 16
    layers = np.where(np.arange(n) % 4 < 2, 0.9, 0.2)
    rho = np.broadcast_to(layers[:, None, None], (n, n, n)).copy()
    prm = O.Params()
    k = O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal)[:, 0, 0]
    with make(n, rho, precision=precision, tol=1e-10 if precision == "fp64" else 1e-6, kernel_variant=4) as h:
        kappa, st = h.homogenize()
    assert st["converged"]
    assert st["iterations"][0] == 0 and st["iterations"][1] == 0
    tol = 1e-9 if precision == "fp64" else 1e-5
    np.testing.assert_allclose(kappa[:3], [k.mean(), k.mean(), 1.0 / np.mean(1.0 / k)], rtol=tol)
    assert np.abs(kappa[3:]).max() <= tol * k.mean()


def test_fused_uniform_density_needs_no_iteration():
    n = 12
    with make(n, np.full((n, n, n), 0.4), kernel_variant=4) as h:
        kappa, st = h.homogenize()
    k = 1e-3 + 0.4 ** 3 * (1.0 - 1e-3)
    assert st["converged"] and max(st["iterations"]) == 0
    np.testing.assert_allclose(kappa, [k, k, k, 0, 0, 0], rtol=0, atol=1e-14)


def test_fused_design_iterations_track_oracle():
    """Three design iterations with the previous solution as the start: the
    fused path follows the oracle's objective, tensor, bound and densities."""
    w = synth.config1()
    prm = O.Params(tol=1e-10)
    gov = O.Governor(w.vf)
    rho_ref = w.rho0.copy()
    from paper_2405_19991_amd import Homogenization
    with Homogenization(w.n, (w.k0, w.kmin), w.target, vf=w.vf, tol=1e-10, kernel_variant=4,
                        guess="previous") as h:
        h.set_density(w.rho0)
        for it in range(3):
            rec = h.step()
            rho_ref, r_ref, _, _ = O.oc_iteration(rho_ref, w.target, gov, prm)
            assert rec["g"] == pytest.approx(r_ref.g, rel=1e-6)
            np.testing.assert_allclose(rec["kappa"], r_ref.kappa, rtol=1e-6, atol=1e-9)
            assert rec["vstar"] == pytest.approx(r_ref.vstar, rel=1e-9)
        rho = h.get_field("rho")
    assert np.abs(rho - rho_ref).max() < 1e-6


def test_fused_rejects_odd_n():
    from paper_2405_19991_amd import Homogenization
    for v in (4, 5):
        with pytest.raises(Exception):
            Homogenization(13, (1.0, 1e-3), (0.1,) * 3 + (0.0,) * 3, vf=0.3, kernel_variant=v)


@pytest.mark.parametrize("precision,n", [("fp64", 16), ("fp64", 34), ("mixed", 32), ("mixed", 64)])
def test_chained_passes_equal_finalized_passes(precision, n):
    """Chained passes (each block reduces its predecessor's partial sums) sum
    the same values in the same order as the finalize kernel: the iterates,
    iteration counts and tensors are bit-identical."""
    rho = synth.smoothed_noise(n, 0.05, 0.95, 77 + n)
    tol = 1e-11 if precision == "fp64" else 1e-6
    res = {}
    for v in (4, 5):
        print(f"chain check {precision} n={n} variant={v}", flush=True)
        with make(n, rho, precision=precision, tol=tol, kernel_variant=v, check_every=8) as h:
            assert h.tile()["variant"] == v
            kappa, st = h.homogenize()
            res[v] = (st["iterations"], np.array(kappa), h.get_field("chi"))
        assert st["converged"]
    assert res[4][0] == res[5][0]
    assert np.array_equal(res[4][1], res[5][1])
    assert np.array_equal(res[4][2], res[5][2])


def test_chained_inactive_loads_and_oracle():
    """Chained passes with loads that are inactive from the start, against the
    laminate closed forms."""
    n = 16
    layers = np.where(np.arange(n) % 4 < 2, 0.9, 0.2)
    rho = np.broadcast_to(layers[:, None, None], (n, n, n)).copy()
    prm = O.Params()
    k = O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal)[:, 0, 0]
    with make(n, rho, tol=1e-10, kernel_variant=5) as h:
        kappa, st = h.homogenize()
    assert st["converged"] and st["iterations"][0] == 0 and st["iterations"][1] == 0
    np.testing.assert_allclose(kappa[:3], [k.mean(), k.mean(), 1.0 / np.mean(1.0 / k)], rtol=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_loads_stopping_together(precision):
    """A density symmetric under every permutation of the axes: the three
    loads converge within a couple of passes of each other, inside one check
    interval, so the all-loads passes still queued in that chunk (and the
    pass bridging the host's check) find every load stopped and return at
    once.  The tensor matches the oracle; in float64, where only the device
    decides when a load stops, checking every 16 passes and after every pass
    give the same iteration counts and the same tensor bit for bit."""
    n = 24
    base = synth.smoothed_noise(n, 0.05, 0.95, 91)
    rho = sum(np.transpose(base, p) for p in itertools.permutations(range(3))) / 6.0
    tol = 1e-11 if precision == "fp64" else 1e-6
    ref = O.homogenize(rho, O.Params(tol=1e-13))
    out = {}
    for ce in (16, 1):
        print(f"loads stopping together {precision} check_every={ce}", flush=True)
        with make(n, rho, precision=precision, tol=tol, kernel_variant=4, check_every=ce) as h:
            kappa, st = h.homogenize()
            out[ce] = (np.array(kappa), list(st["iterations"]), h.timings()[7])
        assert st["converged"]
    its = out[16][1]
    assert max(its) - min(its) <= 2, its
    assert out[16][2] > max(its)  # passes were launched after the last load stopped
    bar = 1e-9 if precision == "fp64" else 1e-5
    assert rel_fro(out[16][0], ref["kappa"]) <= bar
    assert rel_fro(out[1][0], ref["kappa"]) <= bar
    if precision == "fp64":
        assert out[16][1] == out[1][1]
        np.testing.assert_array_equal(out[16][0], out[1][0])
