"""One context per host thread: contexts on their own streams run
concurrently without sharing state (the autotuner's process-wide choices
are the only shared data, behind a lock)."""
import threading

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

TARGET = (0.3, 0.2, 0.1, 0.02, 0.01, 0.015)


def solve(n, rho, out, key, errors, **kw):
    try:
        from paper_2405_19991_amd import Homogenization
        with Homogenization(n, (1.0, 1e-3), TARGET, vf=float(np.mean(rho)), tol=1e-11, **kw) as h:
            h.set_density(rho)
            kappa, st = h.homogenize()
            out[key] = (np.array(kappa), list(st["iterations"]), bool(st["converged"]))
    except Exception as e:  # re-raised on the main thread
        errors.append(e)


def run_threads(cases, **kw):
    out, errors = {}, []
    threads = [threading.Thread(target=solve, args=(n, rho, out, i, errors), kwargs=kw)
               for i, (n, rho) in enumerate(cases)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a solver thread did not finish"
    if errors:
        raise errors[0]
    return out


def test_two_contexts_on_two_threads():
    """Two contexts solving at the same time on two host threads give the
    tensors and iteration counts of the same contexts run one after the
    other (fixed tiles: bit for bit); with the autotuner on, each still
    matches the oracle."""
    cases = [(16, synth.smoothed_noise(16, 0.05, 0.95, 61)), (20, synth.smoothed_noise(20, 0.1, 0.9, 62))]
    fixed = dict(autotune=False, kernel_variant=4)
    seq, errors = {}, []
    for i, (n, rho) in enumerate(cases):
        print(f"sequential context n={n}", flush=True)
        solve(n, rho, seq, i, errors, **fixed)
    if errors:
        raise errors[0]
    print("two contexts on two threads", flush=True)
    par = run_threads(cases, **fixed)
    for i in range(len(cases)):
        assert par[i][2] and seq[i][2]
        assert par[i][1] == seq[i][1]
        np.testing.assert_array_equal(par[i][0], seq[i][0])
    print("two contexts on two threads, autotuned", flush=True)
    tuned = run_threads(cases)
    for i, (n, rho) in enumerate(cases):
        ref = O.homogenize(rho, O.Params(tol=1e-13))
        rel = np.linalg.norm(tuned[i][0] - ref["kappa"]) / np.linalg.norm(ref["kappa"])
        assert tuned[i][2] and rel <= 1e-9, (n, rel)
