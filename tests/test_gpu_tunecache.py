"""Persistent tuning choices (OTM_TUNE_CACHE): a context that tunes appends
its choice to the file; a context of the same configuration in a process
without that choice in memory adopts the stored line instead of timing; a
stored line the context could not have chosen itself is ignored.  Grid
sizes used nowhere else in the suite keep the in-process cache out of the
way."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)
    from paper_2405_19991_amd import _native as N
    N.lib()
    yield


@pytest.fixture
def cache_file(tmp_path, monkeypatch):
    path = os.path.join(str(tmp_path), "tune.txt")
    monkeypatch.setenv("OTM_TUNE_CACHE", path)
    return path


def arch_of_lines(path):
    return [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]


def test_tuning_appends_its_choice(cache_file):
    from paper_2405_19991_amd import Homogenization
    with Homogenization(22, (1.0, 1e-3), [0.1, 0.1, 0.1, 0, 0, 0], vf=0.3) as h:
        tile = h.tile()
    lines = arch_of_lines(cache_file)
    assert len(lines) == 1
    arch, key, pair, fused, chain, tx, tz, us = lines[0]
    assert arch.startswith("gfx950") and key == "context_n22_fp64"
    assert (int(float(tx)), int(float(tz))) == (tile["tx"], tile["tz"])
    assert float(us) > 0


def test_stored_choice_is_adopted_and_invalid_one_ignored(cache_file):
    from paper_2405_19991_amd import Homogenization
    import subprocess
    import sys
    # the architecture string as the library reports it: tune once in a child
    env = dict(os.environ, OTM_TUNE_CACHE=cache_file)
    code = ("import sys; sys.path.insert(0, %r); from paper_2405_19991_amd import Homogenization; "
            "Homogenization(26, (1.0, 1e-3), [0.1, 0.1, 0.1, 0, 0, 0], vf=0.3).close()") % ROOT
    subprocess.run([sys.executable, "-c", code], env=env, check=True, timeout=120)
    arch = arch_of_lines(cache_file)[0][0]
    # a later line for n=28: the fused pass, 32-wide, 4 planes (valid); for
    # n=30: a tile width the kernels do not have (ignored, so it tunes)
    with open(cache_file, "a") as f:
        f.write(f"{arch} context_n28_fp64 1 1 0 32 4 123.0\n")
        f.write(f"{arch} context_n30_fp64 1 1 0 48 4 1.0\n")
    with Homogenization(28, (1.0, 1e-3), [0.1, 0.1, 0.1, 0, 0, 0], vf=0.3) as h:
        t = h.tile()
        h.set_density(np.full((28, 28, 28), 0.4))
        _, st = h.homogenize()
    assert (t["variant"], t["tx"], t["tz"]) == (4, 32, 4) and st["converged"]
    with Homogenization(30, (1.0, 1e-3), [0.1, 0.1, 0.1, 0, 0, 0], vf=0.3) as h:
        t = h.tile()
    assert t["tx"] in (16, 32, 64)
    keys = [ln[1] for ln in arch_of_lines(cache_file)]
    assert keys.count("context_n30_fp64") == 2  # the tuned choice was appended after the bad line
