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
    assert os.path.getsize(path) == 8 + 16 + 11 * 8 + 8 * 8 + 8 + 4 * w.n ** 3 * 8 + 8
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
    assert os.path.getsize(path) == 8 + 16 + 11 * 8 + 8 * 8 + 8 + w.n ** 3 * 8 + 8
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


def fnv1a(data: bytes) -> int:
    h = 1469598103934665603
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def test_resume_with_adaptive_step_matches_uninterrupted_run(tmp_path):
    """With the adaptive OC step (move_min > 0) the step after a resume
    depends on the objective's last change, which the file keeps."""
    w = synth.config1()
    kw = dict(guess="previous", move=0.05, move_min=0.002)
    with make(w, **kw) as h:
        h.set_density(w.rho0)
        full = [h.step() for _ in range(8)]
    path = os.path.join(str(tmp_path), "adapt.otm")
    with make(w, **kw) as h:
        h.set_density(w.rho0)
        for _ in range(5):
            h.step()
        h.save_state(path)
    with make(w, **kw) as h:
        h.load_state(path)
        rest = [h.step() for _ in range(3)]
    assert len({r["move"] for r in full}) > 1, "the step adapted"
    for a, b in zip(full[5:], rest):
        assert (a["move"], a["vstar"], a["g"], list(a["kappa"])) == (b["move"], b["vstar"], b["g"], list(b["kappa"]))


def test_version1_state_file_loads(tmp_path):
    """A file in the earlier layout (no objective change; read as 0) loads."""
    w = synth.config1()
    path = os.path.join(str(tmp_path), "v2.otm")
    with make(w) as h:
        h.set_density(w.rho0)
        h.step()
        h.save_state(path)
        rho = h.get_field("rho")
    data = open(path, "rb").read()
    head1 = 8 + 16 + 11 * 8 + 8 * 8
    body = data[head1 + 8:-8]
    v1 = data[:8] + (1).to_bytes(4, "little") + data[12:head1] + body
    v1 += fnv1a(v1).to_bytes(8, "little")
    p1 = os.path.join(str(tmp_path), "v1.otm")
    open(p1, "wb").write(v1)
    with make(w) as h:
        h.load_state(p1)
        np.testing.assert_array_equal(h.get_field("rho"), rho)
        h.step()


def batch_problems():
    g = synth.rng(81)
    return [dict(n=n, target=synth.random_spd_target(g), vf=0.3, rho=synth.smoothed_noise(n, 0.15, 0.45, 810 + n))
            for n in (8, 12, 16)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_resume_matches_uninterrupted_run(precision, tmp_path):
    from paper_2405_19991_amd import Batch
    probs = batch_problems()
    kw = dict(tol=1e-9, precision=precision, autotune=False, iteration="fused", guess="previous", move_min=0.002)
    with Batch(probs, **kw) as B:
        for d, p in enumerate(probs):
            B.set_density(d, p["rho"])
        full = [B.step() for _ in range(5)]
        rho_full = [B.get_field(d, "rho") for d in range(len(probs))]
    path = os.path.join(str(tmp_path), "batch.otm")
    with Batch(probs, **kw) as B:
        for d, p in enumerate(probs):
            B.set_density(d, p["rho"])
        for _ in range(3):
            B.step()
        B.save_state(path)
        gov = [B.governor_state(d) for d in range(len(probs))]
    n3 = sum(p["n"] ** 3 for p in probs)
    assert os.path.getsize(path) == 8 + 16 + len(probs) * (8 + 11 * 8 + 8 * 8) + 4 * n3 * 8 + 8
    with Batch(probs, **kw) as B:
        B.load_state(path)
        assert [B.governor_state(d) for d in range(len(probs))] == gov
        rest = [B.step() for _ in range(2)]
        rho_rest = [B.get_field(d, "rho") for d in range(len(probs))]
    for a, b in zip(full[3:], rest):
        for ra, rb in zip(a, b):
            assert (ra["iter"], ra["vstar"], ra["move"], ra["g"], list(ra["kappa"]), ra["pcg_iters"]) == \
                (rb["iter"], rb["vstar"], rb["move"], rb["g"], list(rb["kappa"]), rb["pcg_iters"])
    for a, b in zip(rho_full, rho_rest):
        np.testing.assert_array_equal(a, b)


def test_bad_batch_state_files_are_rejected(tmp_path):
    from paper_2405_19991_amd import Batch
    from paper_2405_19991_amd import _native as N
    probs = batch_problems()
    good = os.path.join(str(tmp_path), "good.otm")
    with Batch(probs, tol=1e-8, autotune=False) as B:
        with pytest.raises(N.OTMError) as e:
            B.save_state(good)  # no densities yet
        assert e.value.status == N.OTM_ESTATE
        for d, p in enumerate(probs):
            B.set_density(d, p["rho"])
        B.step()
        B.save_state(good)
    data = open(good, "rb").read()
    cases = {"flipped": data[:300] + bytes([data[300] ^ 1]) + data[301:], "truncated": data[:-9],
             "magic": b"X" + data[1:], "context file": b"OTMSTATE" + data[8:]}
    for name, blob in cases.items():
        p = os.path.join(str(tmp_path), name.replace(" ", "_") + ".otm")
        open(p, "wb").write(blob)
        with Batch(probs, tol=1e-8, autotune=False) as B:
            for d in range(len(probs)):
                B.set_density(d, np.full((probs[d]["n"],) * 3, 0.5))
            with pytest.raises(N.OTMError) as e:
                B.load_state(p)
            assert e.value.status == N.OTM_EIO, name
            assert all(np.all(B.get_field(d, "rho") == 0.5) for d in range(len(probs))), name
    # other designs: one fewer, another n, another target
    others = [probs[:2], [dict(probs[0], n=10, rho=None)] + probs[1:], [dict(probs[0], target=[0.2, 0.1, 0.1, 0, 0, 0])]
              + probs[1:]]
    for q in others:
        with Batch(q, tol=1e-8, autotune=False) as B, pytest.raises(N.OTMError) as e:
            B.load_state(good)
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
