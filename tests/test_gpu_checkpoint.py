"""Checkpoint / resume through the C ABI (otm_save_state / otm_load_state):
a design run interrupted after three design iterations, saved (density,
last solution, adaptive-bound state), loaded into a fresh context and
continued, repeats the uninterrupted run bit for bit, with either start
guess (the previous-iterate start resumes from the saved solution).  Bad
files are rejected with a status, never half-loaded.  Network weights go
through otm_nn_save / otm_nn_load as .npy files that numpy reads and writes
too."""
import os

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


def make(w, **kw):
    from paper_2405_19991_amd import Homogenization
    return Homogenization(w.n, (w.k0, w.kmin), w.target, vf=w.vf, tol=1e-9, **kw)


@pytest.mark.parametrize("guess", ["zero", "previous"])
def test_resume_matches_uninterrupted_run(guess, tmp_path):
    w = synth.config1()
    with make(w, guess=guess) as h:
        h.set_density(w.rho0)
        full = [h.step() for _ in range(5)]
        rho_full = h.get_field("rho")
    path = os.path.join(str(tmp_path), "ckpt.otm")
    with make(w, guess=guess) as h:
        h.set_density(w.rho0)
        for _ in range(3):
            h.step()
        h.save_state(path)
        gov_saved = h.governor_state()
    assert os.path.getsize(path) == 8 + 16 + 11 * 8 + 8 * 8 + 4 * w.n ** 3 * 8 + 8
    with make(w, guess=guess) as h:
        h.load_state(path)
        assert h.governor_state() == gov_saved
        rest = [h.step() for _ in range(2)]
        rho_rest = h.get_field("rho")
    for a, b in zip(full[3:], rest):
        assert (a["vstar"], a["g"], list(a["kappa"]), a["pcg_iters"]) == (b["vstar"], b["g"], list(b["kappa"]),
                                                                          b["pcg_iters"])
    np.testing.assert_array_equal(rho_rest, rho_full)


def test_state_file_without_solution(tmp_path):
    """Saved before any solve: density and bound only; loads and steps."""
    w = synth.config1()
    path = os.path.join(str(tmp_path), "fresh.otm")
    with make(w) as h:
        h.set_density(w.rho0)
        h.save_state(path)
    assert os.path.getsize(path) == 8 + 16 + 11 * 8 + 8 * 8 + w.n ** 3 * 8 + 8
    with make(w) as h:
        h.load_state(path)
        np.testing.assert_array_equal(h.get_field("rho"), np.clip(w.rho0, 1e-3, 1.0))
        h.step()


def test_bad_state_files_are_rejected(tmp_path):
    from paper_2405_19991_amd import Homogenization
    from paper_2405_19991_amd import _native as N
    w = synth.config1()
    good = os.path.join(str(tmp_path), "good.otm")
    with make(w) as h:
        h.set_density(w.rho0)
        h.step()
        h.save_state(good)
    data = open(good, "rb").read()
    cases = {"flipped": data[:200] + bytes([data[200] ^ 1]) + data[201:], "truncated": data[:-9],
             "magic": b"X" + data[1:], "empty": b""}
    for name, blob in cases.items():
        p = os.path.join(str(tmp_path), name + ".otm")
        open(p, "wb").write(blob)
        with make(w) as h:
            h.set_density(np.full((w.n,) * 3, 0.5))
            with pytest.raises(N.OTMError) as e:
                h.load_state(p)
            assert e.value.status == N.OTM_EIO, name
            assert np.all(h.get_field("rho") == 0.5), name  # nothing half-loaded
    with make(w) as h, pytest.raises(N.OTMError) as e:
        h.load_state(os.path.join(str(tmp_path), "missing.otm"))
    assert e.value.status == N.OTM_EIO
    # another resolution, another target
    with Homogenization(w.n + 2, (w.k0, w.kmin), w.target, vf=w.vf) as h, pytest.raises(N.OTMError) as e:
        h.load_state(good)
    assert e.value.status == N.OTM_EINVAL
    with Homogenization(w.n, (w.k0, w.kmin), [0.2, 0.1, 0.1, 0, 0, 0], vf=w.vf) as h, \
            pytest.raises(N.OTMError) as e:
        h.load_state(good)
    assert e.value.status == N.OTM_EINVAL


def test_network_weights_file_round_trip(tmp_path):
    """otm_nn_save writes a .npy that numpy reads back exactly; otm_nn_load
    reads numpy's own .npy (the shipped weights) and rejects other shapes and
    dtypes."""
    from paper_2405_19991_amd import Network
    from paper_2405_19991_amd import _native as N
    from paper_2405_19991_amd.warmstart import DEFAULT_WEIGHTS
    shipped = np.load(DEFAULT_WEIGHTS, allow_pickle=False)
    with Network(n_max=16, seed=3) as net:
        net.load(DEFAULT_WEIGHTS)
        np.testing.assert_array_equal(net.params(), shipped)
        p = os.path.join(str(tmp_path), "w.npy")
        rng = np.random.default_rng(5)
        w = rng.standard_normal(shipped.size).astype(np.float32)
        net.set_params(w)
        net.save(p)
        back = np.load(p, allow_pickle=False)
        assert back.dtype == np.float32 and back.shape == w.shape
        np.testing.assert_array_equal(back, w)
        net.set_params(shipped)
        net.load(p)
        np.testing.assert_array_equal(net.params(), w)
        for name, arr in (("f64", w.astype(np.float64)), ("2d", w.reshape(1, -1)), ("short", w[:-1])):
            q = os.path.join(str(tmp_path), name + ".npy")
            np.save(q, arr)
            with pytest.raises(N.OTMError) as e:
                net.load(q)
            assert e.value.status == N.OTM_EIO, name
        np.testing.assert_array_equal(net.params(), w)
