"""The adaptive volume bound (Algorithm 1) of the HIP path against the
oracle's, through every branch: shrink (objective tolerable), stall
counting, reset (volume off the bound), and rebound after `patience`
stalls, for a single context and for a batch.

Two checks per design iteration:
* replay: the oracle's transition is fed the GPU's own observations
  (g, mean(rho~^p), mean(rho)); the whole state (V*, Df, count, gap,
  g_prev, termination counter) must agree to rounding, since the governor
  is scalar float64 logic evaluated in the same order on both sides;
* trajectory: the oracle runs the same design iterations with its own
  solves (CSR + CG to 1e-12) and the per-iteration V*, objective and
  stall count must follow (V* to 1e-9 relative).

Workload: the 16^3 isotropic cell (0.3 +- 0.05 noise, seed 101), with the
target set to the oracle's tensor of the initial density, so the first
objective is ~0 and the bound shrinks at once; the governor thresholds are
chosen so that the twelve iterations contain shrinks, resets, stalls and
rebounds, with every objective at least 8 % away from the bound (the
branch decisions cannot flip on rounding)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

GOV = dict(bound=1e-3, dg_small=1.0, dv_small=0.06, patience=2)
GOV_B = dict(bound=1.2e-3, dg_small=1.0, dv_small=0.04, patience=2)
ITERS = 12


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)
    from paper_2405_19991_amd import _native as N
    N.lib()
    yield


@pytest.fixture(scope="module")
def workload():
    w = synth.config1()
    prm = O.Params(tol=1e-12)
    target = O.homogenize(w.rho0, prm)["kappa"].copy()
    return w, target, prm


def oracle_trajectory(w, target, prm, gov_opts):
    gov = O.Governor(w.vf, O.GovernorParams(**gov_opts))
    rho = w.rho0.copy()
    out = []
    for _ in range(ITERS):
        rho, rec, _, _ = O.oc_iteration(rho, target, gov, prm)
        out.append((rec, gov.state))
    return out


def replay_and_compare(recs, states, vf, gov_opts):
    """Feed the GPU's observations to the oracle's transition; compare states.
    Returns the branch labels seen (R shrink, s stall, B rebound, - reset)."""
    gp = O.GovernorParams(**gov_opts)
    st = O.GovernorState(vf)
    labels = []
    for rec, gpu_state in zip(recs, states):
        prev = st
        st = O.governor_transition(st, rec["g"], rec["low_bound"], rec["volume"], gp)
        assert rec["vstar"] == pytest.approx(st.vstar, rel=1e-14, abs=0)
        vstar, df, count, gap, g_prev, flat = gpu_state[:6]
        assert vstar == pytest.approx(st.vstar, rel=1e-14, abs=0)
        assert df == pytest.approx(st.df, rel=1e-14, abs=0)
        assert gap == pytest.approx(st.gap, rel=1e-14, abs=1e-300)
        assert g_prev == rec["g"]
        assert int(count) == st.count and int(flat) == st.small_steps
        if rec["g"] <= gp.bound:
            labels.append("R")
        elif st.count == 0 and prev.count + 1 >= gp.patience and st.vstar != prev.vstar:
            labels.append("B")
        else:
            labels.append("s" if st.count > 0 else "-")
        # branch decisions are far from the thresholds
        assert abs(rec["g"] - gp.bound) > 0.05 * gp.bound
    return "".join(labels)


def check_trajectory(recs, ref, bound):
    for it, (rec, (r_ref, st_ref)) in enumerate(zip(recs, ref)):
        assert rec["vstar"] == pytest.approx(r_ref.vstar, rel=1e-9), it
        assert rec["g"] == pytest.approx(r_ref.g, rel=1e-6, abs=1e-12 * bound), it
        assert rec["low_bound"] == pytest.approx(r_ref.low_bound, rel=1e-9), it


@pytest.mark.parametrize("gov_opts", [GOV, GOV_B], ids=["shrink-once-per-phase", "three-shrinks"])
def test_single_context_governor_all_branches(workload, gov_opts):
    from paper_2405_19991_amd import Homogenization
    w, target, prm = workload
    recs, states = [], []
    with Homogenization(w.n, (w.k0, w.kmin), target, vf=w.vf, tol=1e-10, governor=gov_opts) as h:
        h.set_density(w.rho0)
        for _ in range(ITERS):
            recs.append(h.step())
            states.append(h.governor_state())
    labels = replay_and_compare(recs, states, w.vf, gov_opts)
    print("single context branches:", labels, flush=True)
    assert labels.count("R") >= 2 and labels.count("B") >= 2 and "-" in labels and "s" in labels
    check_trajectory(recs, oracle_trajectory(w, target, prm, gov_opts), gov_opts["bound"])


def test_batch_governor_all_branches(workload):
    """Two designs in one batch: the workload above and its mirror image (the
    tensor is the same under x -> -x up to the signs of k12 and k13, so the
    target is mirrored too); each design's bound follows the oracle."""
    from paper_2405_19991_amd import Batch
    w, target, prm = workload
    mirror = w.rho0[:, :, ::-1].copy()
    t_mirror = target * np.array([1, 1, 1, -1, 1, -1])
    designs = [(w.rho0, target), (mirror, t_mirror)]
    with Batch([dict(n=w.n, target=tuple(t), vf=w.vf) for _, t in designs], tol=1e-10, governor=GOV) as B:
        for d, (rho, _) in enumerate(designs):
            B.set_density(d, rho)
        recs = [[], []]
        states = [[], []]
        for _ in range(ITERS):
            r = B.step()
            for d in range(2):
                recs[d].append(r[d])
                states[d].append(B.governor_state(d))
    for d, (rho, t) in enumerate(designs):
        labels = replay_and_compare(recs[d], states[d], w.vf, GOV)
        print(f"batch design {d} branches:", labels, flush=True)
        assert labels.count("R") >= 2 and labels.count("B") >= 2 and "-" in labels
    check_trajectory(recs[0], oracle_trajectory(w, target, prm, GOV), GOV["bound"])
    check_trajectory(recs[1], oracle_trajectory(dataclasses.replace(w, rho0=mirror), t_mirror, prm, GOV), GOV["bound"])
