#!/usr/bin/env python3
"""Benchmark: design iterations of the periodic thermal homogenization path
on one MI355X, for the 128^3 anisotropic cell.

One step = one full design iteration on one cell: filter + SIMP + macro loads
+ Jacobi-PCG for the three loads + homogenized tensor + sensitivities +
filter transpose + adaptive V* + OC bisection update.  The design state
(density, governor) carries over from step to step, as in the method.

Printed JSON line: `value` is PCG DOF-updates per second over the whole timed
region, (n^3 * sum over loads of PCG iterations) / wall time of the K steps;
`ms_per_step` is the mean wall time of a design iteration.
"""
from __future__ import annotations

import argparse
import functools
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def collected(fn):
    """Run a leg after a full garbage collection.  main() turns the
    automatic collector off, so that a collection pass (tens of ms in this
    process) never lands inside a timed region; each leg starts clean."""
    @functools.wraps(fn)
    def run(*a, **k):
        gc.collect()
        return fn(*a, **k)
    return run


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--guess", choices=["zero", "previous"], default="zero")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-design batch leg")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--apply-only", action="store_true",
                    help="run only the stand-alone operator (fixed tile) and a device copy of known size, for "
                         "hardware-counter profiling; prints one JSON line with their HIP-event timings")
    ap.add_argument("--apply-tx", type=int, default=64)
    ap.add_argument("--apply-tz", type=int, default=8)
    ap.add_argument("--weights", default=None,
                    help="network weights (.npy) for the warm-start leg (default: the package's trained weights)")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the warm-start leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the 16^3 / 64^3 legs")
    ap.add_argument("--no-gallery", action="store_true", help="skip the 61-target traversal leg")
    ap.add_argument("--no-full-run", action="store_true", help="skip the 150-iteration design runs")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 leg")
    ap.add_argument("--no-fused-sizes", action="store_true", help="skip the fused pass at 192^3 and 256^3")
    ap.add_argument("--gallery-iters", type=int, default=500)
    ap.add_argument("--gallery-n", type=int, default=32)
    ap.add_argument("--retune", action="store_true",
                    help="time the kernel candidates at start-up instead of using the shipped tuning file")
    ap.add_argument("--variant", type=int, default=0,
                    help="solver kernel: 0 automatic (autotuned), 4 fused iteration, 1-3 cross-check kernels")
    ap.add_argument("--solver-tx", type=int, default=0, help="solver tile width (0: automatic)")
    ap.add_argument("--solver-tz", type=int, default=0, help="solver planes per z-march (0: automatic)")
    ap.add_argument("--preconditioner", choices=["jacobi", "mg"], default="jacobi",
                    help="preconditioner of the timed design iterations")
    ap.add_argument("--no-mg", action="store_true", help="skip the multigrid leg")
    ap.add_argument("--mg-sweeps", type=int, default=1, help="relaxation steps per leg of the V-cycle, finest level")
    ap.add_argument("--mg-coarse-sweeps", type=int, default=2, help="the same on coarser levels (0: as --mg-sweeps)")
    ap.add_argument("--check-every", type=int, default=16,
                    help="PCG iterations between host convergence checks (at most 2 with multigrid)")
    ap.add_argument("--reliable-delta", type=float, default=None,
                    help="mixed precision: refresh the float64 residual after this relative drop "
                         "(default 1e-2, or 1e-3 with the multigrid preconditioner)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, run three 64 MiB device copies (a kernel of known traffic, "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


# Counter-measured HBM bytes of a kernel come from a committed rocprofv3
# summary; they stand only while the kernel's sources hash as they did when
# the counters were taken (else the traffic field is null).
TRAFFIC_RECORDS = {
    4: ("profiles/k_fused_f32_cell128_traffic.md",
        ("paper_2405_19991_amd/csrc/otm_fused.hip", "paper_2405_19991_amd/csrc/otm_device.h")),
}


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kind: int, tile_tx: int, tile_tz: int):
    """The counter record for this kernel and tile, if its sources still hash
    as they did when the counters were taken."""
    rec = TRAFFIC_RECORDS.get(kind)
    if rec is None or not os.path.exists(os.path.join(ROOT, rec[0])):
        return None
    digest = sources_sha256(rec[1])
    for line in open(os.path.join(ROOT, rec[0])):
        if line.startswith("record: "):
            d = json.loads(line[len("record: "):])
            if d.get("sha256") == digest and (d.get("tile_tx"), d.get("tile_tz")) == (tile_tx, tile_tz):
                return d
    return None


def oracle_tensor_error(w, kappa, tol):
    """Relative Frobenius error of the first design iteration's tensor against
    the CPU FP64 oracle's (stored by tests/golden/make_cell128_kappa.py, which
    runs the oracle alone), for the 128^3 cell's initial density."""
    path = os.path.join(ROOT, "tests", "golden", "cell128_kappa.json")
    if w.n != 128 or not os.path.exists(path):
        return None
    import numpy as np
    ref = json.load(open(path))
    k_ref = np.array(ref["kappa"])
    return {"value": float(np.linalg.norm(np.array(kappa) - k_ref) / np.linalg.norm(k_ref)),
            "oracle_tol": ref["tol"], "gpu_tol": tol, "reference": "tests/golden/cell128_kappa.json"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


@collected
def cpu_baseline(iters_128: int = 1, iters_64: int = 5, iters_16: int = 30):
    """The CPU FP64 oracle (CSR assembly + plain unpreconditioned CG, OpenMP
    on every host core) timed per design iteration on the three single-cell
    workloads: 16^3 (tol 1e-8) for all its 30 iterations, 64^3 (tol 1e-6) for
    5, 128^3 (tol 1e-6) for 1.  Each design iteration is the oracle's whole
    step: filter, SIMP, assembly, loads, three CG solves, tensor, objective,
    sensitivities, governor and OC.  value = the 128^3 leg's DOF-updates/s
    (n^3 x CG iterations summed over the loads / seconds of the whole step),
    the GPU metric's unit."""
    import synth
    import oracle as O
    legs = {}
    for name, w, tol, iters in (("cell16_iso_fp64", synth.config1(), 1e-8, iters_16),
                                ("cell64_ortho_fp64", synth.config2("fp64"), 1e-6, iters_64),
                                ("cell128_aniso_fp64", synth.config3("fp64"), 1e-6, iters_128)):
        prm = O.Params(tol=tol, k0=w.k0, kmin=w.kmin, penal=w.penal, rfilter=w.rfilter)
        gov = O.Governor(w.vf)
        rho = w.rho0.copy()
        cg_iters = 0
        t0 = time.perf_counter()
        for _ in range(iters):
            rho, rec, _, _ = O.oc_iteration(rho, w.target, gov, prm)
            cg_iters += sum(rec.pcg_iters)
        dt = time.perf_counter() - t0
        legs[name] = {"n": w.n, "tol": tol, "design_iterations": iters, "s_per_oc_iter": dt / iters,
                      "cg_iters_per_oc_iter": cg_iters / iters, "dof_updates_per_s": w.n ** 3 * cg_iters / dt}
    top = legs["cell128_aniso_fp64"]
    return {
        "value": top["dof_updates_per_s"],
        "unit": "DOF-updates/s",
        "cores": O.num_threads(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": (f"{iters_128} oracle design iteration(s) of the 128^3 anisotropic cell from its initial density "
                   f"(filter, SIMP, CSR assembly, 3 plain FP64 CG solves to 1e-6, tensor, sensitivities, OC; "
                   f"{top['s_per_oc_iter']:.1f} s each); also {iters_64} at 64^3 and {iters_16} at 16^3"),
        "per_config": legs,
    }


@collected
def batch_leg(steps: int, log, precision: str = "fp64"):
    """64 designs, n in {32, 48, 64} (seeded mix), FP64 or mixed, tol 1e-6: one
    batched design iteration per step (work-list launches, hipGraph PCG
    chunks)."""
    import time as _t
    import synth
    from paper_2405_19991_amd import Batch
    import torch
    ws = synth.config4()
    probs = [dict(n=w.n, target=w.target, vf=w.vf) for w in ws]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    B = Batch(probs, tol=1e-6, precision=precision)
    free_min = torch.cuda.mem_get_info()[0]
    for d, w in enumerate(ws):
        B.set_density(d, w.rho0)
    B.step()  # warm-up (graph capture)
    t0 = _t.perf_counter()
    iters = 0
    step_ms = []
    for _ in range(steps):
        ts = _t.perf_counter()
        recs = B.step()
        step_ms.append(1e3 * (_t.perf_counter() - ts))
        iters += sum(sum(r["pcg_iters"]) * ws[d].n ** 3 for d, r in enumerate(recs))
        inf = B.info()
        log(f"batch {precision} step: {step_ms[-1]:.1f} ms (library: step {inf['step_ms']:.1f}, solve {inf['solve_ms']:.1f}), "
            f"max pcg {max(max(r['pcg_iters']) for r in recs)}, mean g {sum(r['g'] for r in recs) / len(recs):.3e}")
    t1 = _t.perf_counter()
    free_min = min(free_min, torch.cuda.mem_get_info()[0])
    info = B.info()
    dev_bytes = B.device_bytes()
    B.close()
    return {"workload": f"batch64_n32-64_{precision}", "designs": len(ws), "cells": int(info["cells"]),
            "device_bytes": dev_bytes, "device_in_use_peak_bytes": int(free0 - free_min),
            "s_per_oc_iter": (t1 - t0) / steps, "pcg_dof_updates_per_s": iters / (t1 - t0),
            "iteration": "fused" if info["fused"] else "two_pass", "refreshes": int(info["refreshes"]),
            "tile_tx": int(info["tile_tx"]), "tile_tz": int(info["tile_tz"]), "work_items": int(info["work_items"]),
            "steps": steps, "step_ms": [round(x, 2) for x in step_ms]}


@collected
def multigrid_leg(w, steps: int, log, sweeps: int = 1, coarse_sweeps: int = 2, smoother: str = "jacobi"):
    """The timed workload's design iterations with one multigrid V-cycle as
    the preconditioner (mixed precision, same start and tolerance; damped
    Jacobi or 8-colour Gauss-Seidel relaxation): one warm-up design
    iteration, then `steps` timed ones."""
    import torch
    from paper_2405_19991_amd import Homogenization
    with Homogenization(w.n, (w.k0, w.kmin), w.target, vf=w.vf, penal=w.penal, filter_radius=w.rfilter,
                        precision="mixed", tol=w.tol, preconditioner="mg", mg_sweeps=sweeps,
                        mg_coarse_sweeps=coarse_sweeps, mg_smoother=smoother) as h:
        h.set_density(w.rho0)
        first = h.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = [h.step() for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        dev_bytes = h.device_bytes()
    iters = sum(sum(r["pcg_iters"]) for r in recs)
    out = {"device_bytes": dev_bytes, "workload": w.name + "_mixed_mg", "n": w.n, "tol": w.tol, "mg_sweeps": [sweeps, coarse_sweeps],
           "smoother": smoother, "s_per_oc_iter": dt / steps,
           "pcg_iters_per_step": iters / steps, "ms_solve_per_step": sum(r["ms_solve"] for r in recs) / steps,
           "pcg_dof_updates_per_s": w.n ** 3 * iters / dt, "first_kappa": first["kappa"],
           "first_pcg_iters": first["pcg_iters"], "steps": steps}
    log(f"multigrid ({smoother}): {1e3 * out['s_per_oc_iter']:.2f} ms per design iteration, "
        f"{out['pcg_iters_per_step']:.1f} PCG iterations per step")
    return out


@collected
def fp64_leg(steps: int, log):
    """The 128^3 anisotropic cell with every vector and the operator in
    float64 (tol 1e-6, zero start), once with the Jacobi and once with the
    multigrid preconditioner (float32 V-cycle inside float64 CG): one warm-up
    and `steps` timed design iterations each; PCG DOF-updates/s as for the
    headline value."""
    import synth
    import torch
    from paper_2405_19991_amd import Homogenization
    w = synth.config3("fp64")
    w.tol = 1e-6
    res = {}
    for pc in ("jacobi", "mg"):
        with Homogenization(w.n, (w.k0, w.kmin), w.target, vf=w.vf, penal=w.penal, filter_radius=w.rfilter,
                            precision="fp64", tol=w.tol, preconditioner=pc) as h:
            h.set_density(w.rho0)
            h.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs = [h.step() for _ in range(steps)]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            tile = h.tile()
            dev_bytes = h.device_bytes()
        iters = sum(sum(r["pcg_iters"]) for r in recs)
        res[pc] = {"device_bytes": dev_bytes, "pcg_dof_updates_per_s": w.n ** 3 * iters / dt, "s_per_oc_iter": dt / steps,
                   "pcg_iters_per_step": iters / steps, "solver_tile": tile}
        log(f"fp64 {pc}: {res[pc]['pcg_dof_updates_per_s']:.3e} DOF-updates/s, "
            f"{1e3 * res[pc]['s_per_oc_iter']:.2f} ms per design iteration")
    out = {"workload": w.name + "_fp64", "n": w.n, "tol": w.tol, "steps": steps}
    out.update(res["jacobi"])
    out["multigrid"] = res["mg"]
    return out


@collected
def full_run_leg(w, log, iters: int = 150):
    """The 128^3 configuration's whole design run (150 design iterations,
    previous solution as the start, mixed precision, tol 1e-6) with the
    multigrid and with the Jacobi preconditioner: seconds per design iteration
    over iterations 2..150, PCG iterations per solve, final objective."""
    import torch
    from paper_2405_19991_amd import Homogenization
    out = {}
    for pc in ("mg", "jacobi"):
        with Homogenization(w.n, (w.k0, w.kmin), w.target, vf=w.vf, penal=w.penal, filter_radius=w.rfilter,
                            precision="mixed", tol=w.tol, preconditioner=pc, guess="previous") as h:
            h.set_density(w.rho0)
            h.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs = [h.step() for _ in range(iters - 1)]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        its = [max(r["pcg_iters"]) for r in recs]
        out[pc] = {"s_per_oc_iter": dt / (iters - 1), "s_total": dt, "pcg_iters_max": max(its),
                   "pcg_iters_last": its[-1], "g_last": recs[-1]["g"],
                   "max_rel_residual": max(max(r["rel_residual"]) for r in recs)}
        log(f"full run {pc}: {1e3 * out[pc]['s_per_oc_iter']:.2f} ms per design iteration over {iters - 1}, "
            f"g {recs[-1]['g']:.4e}")
    return {"workload": w.name + "_mixed_150_iterations", "iterations": iters, **out}


@collected
def gallery_leg(iters: int, log, n: int = 32, move: float = 0.02, move_min: float = 0.0, governor=None):
    """Anisotropic-space traversal (Sec. 4.2): the 61 positive-definite targets
    with diagonal [0.3, 0.2, 0.1] as one batch of n^3 designs, IWP start at
    volume 0.3, volume bound starting at 1 (Algorithm 1), OC move limit `move`
    (adaptive down to `move_min` when that is positive), `iters` batched
    design iterations.  Reported per design: whether some iterate met the
    tolerable error g <= 1e-4 (model 3's answer is the last such iterate:
    the bound then keeps trading volume against the objective), that
    iterate's volume, and the final objectives."""
    import numpy as np
    import synth
    from paper_2405_19991_amd import Batch, init_density
    T = synth.gallery_targets()
    B = Batch([dict(n=n, target=tuple(t), vf=1.0) for t in T], tol=1e-6, guess="previous", move=move,
              move_min=move_min, governor=governor)
    rho0 = init_density(n, "IWP", 0.3)
    for d in range(len(T)):
        B.set_density(d, rho0)
    g0 = np.array([r["g"] for r in B.step()])
    gbest = g0.copy()
    # model 3's answer per design: the last design iterate whose objective met
    # the tolerable error (its volume; nan while none has)
    vol_ok = np.full(len(T), np.nan)
    t0 = time.perf_counter()
    for _ in range(iters):
        recs = B.step()
        g = np.array([r["g"] for r in recs])
        gbest = np.minimum(gbest, g)
        ok = g <= 1e-4
        vol_ok[ok] = np.array([r["volume"] for r in recs])[ok]
    dt = time.perf_counter() - t0
    B.close()
    g = np.array([r["g"] for r in recs])
    out = {"workload": f"gallery61_n{n}_fp64", "designs": len(T), "iterations": iters + 1, "move": move,
           "move_min": move_min,
           "s_per_oc_iter": dt / iters, "g_start_median": float(np.median(g0)), "g_median": float(np.median(g)),
           "g_max": float(g.max()), "designs_g_le_1e-4": int((g <= 1e-4).sum()),
           "best_g_median": float(np.median(gbest)), "designs_best_g_le_1e-4": int((gbest <= 1e-4).sum()),
           "feasible_volume_median": float(np.nanmedian(vol_ok)) if np.isfinite(vol_ok).any() else None,
           "mean_volume": float(np.mean([r["volume"] for r in recs]))}
    log(f"gallery: {1e3 * out['s_per_oc_iter']:.1f} ms per batched design iteration, g median "
        f"{out['g_start_median']:.2e} -> {out['g_median']:.2e}, {out['designs_best_g_le_1e-4']} of 61 reached "
        f"g <= 1e-4 (last feasible volume median {out['feasible_volume_median']})")
    return out


@collected
def config_legs(steps: int, log):
    """Seconds per design iteration of the smaller cells: 16^3 isotropic (FP64,
    tol 1e-8) and 64^3 orthotropic (FP64 and mixed, tol 1e-6); one warm-up
    design iteration each, then `steps` timed ones."""
    import synth
    import torch
    from paper_2405_19991_amd import Homogenization
    out = []
    for w in (synth.config1(), synth.config2("fp64"), synth.config2("mixed")):
        with Homogenization(w.n, (w.k0, w.kmin), w.target, vf=w.vf, penal=w.penal, filter_radius=w.rfilter,
                            precision=w.precision, tol=w.tol) as h:
            h.set_density(w.rho0)
            h.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iters = 0
            for _ in range(steps):
                iters += sum(h.step()["pcg_iters"])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            name = w.name if w.name.endswith(w.precision) else w.name + "_" + w.precision
            rec = {"workload": name, "n": w.n, "tol": w.tol, "s_per_oc_iter": dt / steps,
                   "pcg_dof_updates_per_s": w.n ** 3 * iters / dt, "solver_tile": h.tile(), "steps": steps}
        log(f"config {rec['workload']}: {1e3 * rec['s_per_oc_iter']:.2f} ms per design iteration")
        out.append(rec)
    return out


@collected
@collected
def fused_sizes_leg(log, sizes=(192, 256)):
    """The fused PCG pass on larger cells (mixed, Jacobi-PCG, the
    autotuner's tile): its live per-launch timing over two solves after one
    design iteration, against the minimum PCG-iteration bytes (76 B/node)
    and the pass's own schedule (104 B/node).  At 128^3 the pass's vectors
    largely stay in the 256 MB Infinity Cache between passes; at these
    sizes they stream from HBM."""
    import synth
    from paper_2405_19991_amd import Homogenization
    out = []
    for n in sizes:
        rho = synth.smoothed_noise(n, 0.15, 0.45, 301)
        with Homogenization(n, (1.0, 1e-3), (0.3, 0.2, 0.1, 0.1, 0.05, 0.05), vf=0.3, precision="mixed",
                            tol=1e-6) as h:
            h.set_density(rho)
            h.step()
            h.pass_timing(reset=True)
            h.homogenize()
            h.homogenize()
            pt, tile = h.pass_timing(), h.tile()
        rec = {"n": n, "tile": tile, "kernel": "k_fused_f32" if pt["kernel"] == 4 else "direction+operator",
               "sampled_launches": pt["launches"], "us_per_launch": pt["us"]}
        if pt["launches"] > 0 and pt["kernel"] == 4:
            alg = 76.0 * n ** 3
            rec.update(alg_bytes_per_launch=alg, frac=alg / (pt["us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                       schedule_frac=pt["bytes"] / (pt["us"] * 1e-6) / 1e9 / HBM_PEAK_GBS)
            log(f"fused pass {n}^3: {pt['us']:.1f} us, {rec['frac']:.3f} of peak on 76 B/node, "
                f"{rec['schedule_frac']:.3f} on its schedule")
        out.append(rec)
    return out


def warm_start_leg(weights, log):
    """Time to 1e-6 on the held-out 128^3 cell at design iteration 5: zero
    start (FP64, mixed), previous design iteration's solution, and the trained
    network's prediction (forward pass included)."""
    from paper_2405_19991_amd import Network
    from paper_2405_19991_amd import warmstart as W
    path = weights or W.DEFAULT_WEIGHTS
    if not os.path.exists(path):
        log(f"warm start: no weights at {path}, leg skipped")
        return None
    net = Network(n_max=128)
    net.load(path)
    ev = W.evaluate(net)
    for k, v in ev.items():
        if isinstance(v, dict):
            v.pop("kappa", None)
            log(f"warm start {k}: {v['pcg_iters']} PCG iterations, {v['ms']:.2f} ms")
    ev["weights"] = os.path.relpath(path, ROOT)
    return ev


@collected
def apply_sizes(reps: int):
    """Stand-alone operator (3 loads, two-node z-march) on random conductivities
    at 128^3 and 256^3 in float32 and float64: microseconds per launch and
    algorithmic GB/s (28 or 56 B per node) for the best of four tile shapes."""
    import torch
    from paper_2405_19991_amd import time_apply_device
    out = []
    for n in (128, 256):
        nn = n ** 3
        for prec, dt, bpn in (("mixed", torch.float32, 28), ("fp64", torch.float64, 56)):
            k = (torch.rand(nn, dtype=torch.float64, device="cuda") * 0.999 + 0.001).to(dt)
            x = torch.randn(3 * nn, dtype=dt, device="cuda")
            y = torch.empty_like(x)
            best = min((time_apply_device(k, x, y, prec, reps=reps, variant=0, tile_tx=64, tile_tz=tz), tz)
                       for tz in (8, 16, 32))
            ach = bpn * nn / (best[0] * 1e-6) / 1e9
            out.append({"n": n, "dtype": "f32" if prec == "mixed" else "f64", "tile": [64, best[1]],
                        "us_per_launch": best[0], "alg_bytes_per_launch": bpn * nn, "achieved": ach,
                        "frac": ach / HBM_PEAK_GBS})
            del k, x, y
    torch.cuda.empty_cache()
    return out


def apply_only(args):
    """Operator and copy launches for counter runs (rocprofv3 --pmc)."""
    import torch
    from paper_2405_19991_amd import time_apply_device
    torch.cuda.set_device(0)
    n = args.n
    nn = n ** 3
    dt = torch.float32 if args.precision == "mixed" else torch.float64
    k = (torch.rand(nn, dtype=torch.float64, device="cuda") * 0.999 + 0.001).to(dt)
    x = torch.randn(3 * nn, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    v = 0 if n % 2 == 0 else 3
    # warm-up launches first (about 50 ms of the operator): a GPU that has just
    # been idle runs its first milliseconds of work at lower clocks
    warm = max(1, int(50e3 / max(time_apply_device(k, x, y, args.precision, reps=2, variant=v, tile_tx=args.apply_tx,
                                                     tile_tz=args.apply_tz), 1.0)))
    time_apply_device(k, x, y, args.precision, reps=warm, variant=v, tile_tx=args.apply_tx, tile_tz=args.apply_tz)
    us = time_apply_device(k, x, y, args.precision, reps=args.apply_reps, variant=v, tile_tx=args.apply_tx,
                           tile_tz=args.apply_tz)
    src = torch.empty(64 * 1024 * 1024, dtype=torch.uint8, device="cuda")  # 64 MiB copy
    dst = torch.empty_like(src)
    for _ in range(args.apply_reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    bpn = 28 if args.precision == "mixed" else 56
    print(json.dumps({"apply_us": us, "alg_bytes": bpn * nn, "copy_bytes": src.numel(), "launches": args.apply_reps + 1,
                      "tile": [v, args.apply_tx, args.apply_tz]}), flush=True)


TUNE_FILE = os.path.join(ROOT, "paper_2405_19991_amd", "tuning", "gfx950.tune")


def use_shipped_tuning(retune: bool):
    """Kernel and tile choices: unless OTM_TUNE_CACHE is already set or
    --retune is given, the autotuners start from a private copy of the
    package's tuning file (choices timed on an MI355X), so that the timed
    configuration does not depend on the timing noise of one start-up; new
    configurations are tuned and added to the copy."""
    if "OTM_TUNE_CACHE" in os.environ:
        return {"source": "OTM_TUNE_CACHE", "path": os.environ["OTM_TUNE_CACHE"]}
    if retune or not os.path.exists(TUNE_FILE):
        return {"source": "timed at start-up"}
    import shutil
    import tempfile
    fd, path = tempfile.mkstemp(prefix="otm_tune_", suffix=".txt")
    os.close(fd)
    shutil.copyfile(TUNE_FILE, path)
    os.environ["OTM_TUNE_CACHE"] = path
    return {"source": os.path.relpath(TUNE_FILE, ROOT)}


def main():
    gc.disable()  # collections run only between legs (see collected)
    args = parse()
    if args.apply_only:
        apply_only(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    tuning = use_shipped_tuning(args.retune)
    import numpy as np
    import torch
    import synth
    from paper_2405_19991_amd import Homogenization, time_apply_device

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.n == 128:
        w = synth.config3(args.precision)
    else:
        w = synth.Workload(f"cell{args.n}_aniso", args.n, synth.smoothed_noise(args.n, 0.15, 0.45, 301),
                           np.array(synth.TARGET_ANISO), 0.3, precision=args.precision)
    w.tol = args.tol
    n = w.n
    nn = n ** 3
    # device memory in use (hipMemGetInfo, whole device: the library, the HIP
    # runtime and torch's cache) before the context exists, then sampled after
    # its creation (which includes the autotuner's timing) and after every
    # design iteration; the library allocates nothing per iteration
    torch.cuda.synchronize()
    free0, total_mem = torch.cuda.mem_get_info()
    free_min = [free0]

    def sample_mem():
        free_min[0] = min(free_min[0], torch.cuda.mem_get_info()[0])

    h = Homogenization(n, (w.k0, w.kmin), w.target, vf=w.vf, penal=w.penal, filter_radius=w.rfilter,
                       precision=args.precision, guess=args.guess, tol=w.tol, kernel_variant=args.variant,
                       tile_tx=args.solver_tx, tile_tz=args.solver_tz, preconditioner=args.preconditioner,
                       mg_sweeps=args.mg_sweeps, mg_coarse_sweeps=args.mg_coarse_sweeps,
                       reliable_delta=args.reliable_delta, check_every=args.check_every)
    h.set_density(w.rho0)
    sample_mem()
    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    log(f"bench: {w.name} n={n} precision={args.precision} warmup={args.warmup} steps={args.steps}")
    first_kappa = None
    for i in range(args.warmup):
        r = h.step()
        if first_kappa is None:
            first_kappa = r["kappa"]
        log(f"warmup {i}: g={r['g']:.4e} pcg={r['pcg_iters']} ms={r['ms_total']:.1f}")
        sample_mem()
    torch.cuda.synchronize()
    h.pass_timing(reset=True)
    recs = []
    gc.collect()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        recs.append(h.step())
        log(f"step: g={recs[-1]['g']:.4e} pcg={recs[-1]['pcg_iters']} ms={recs[-1]['ms_total']:.1f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    sample_mem()  # after the timed region (mem_get_info synchronises the device)
    if first_kappa is None:
        first_kappa = recs[0]["kappa"]
    pcg_iters = sum(sum(r["pcg_iters"]) for r in recs)
    dof = nn * pcg_iters
    solve_ms = sum(r["ms_solve"] for r in recs)
    live = h.pass_timing()

    # dominant kernel: the stencil operator, timed with HIP events on its stream
    k_field = torch.from_numpy(h.get_field("k").reshape(-1)).cuda()
    dt = torch.float32 if args.precision == "mixed" else torch.float64
    kd = k_field.to(dt).contiguous()
    x = torch.randn(3 * nn, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    tile = h.tile()
    dev_bytes = h.device_bytes()
    # the operator in the configuration the solver was tuned to, and the best
    # z-march shape for the stand-alone operator
    # (the fused iteration's operator is the two-node z-march)
    cands = [(0 if tile["variant"] in (4, 5) else tile["variant"], tile["tx"], tile["tz"])]
    for tx in ((32, 64) if n % 2 == 0 else (16, 32, 64)):
        for tz in (4, 5, 6, 8, 16):
            cands.append((0 if n % 2 == 0 else 3, tx, tz))
    best = None
    for v, tx, tz in cands:
        t_us = time_apply_device(kd, x, y, args.precision, reps=args.apply_reps, variant=v, tile_tx=tx, tile_tz=tz)
        if best is None or t_us < best[0]:
            best = (t_us, v, tx, tz)
    us, v_best, tx_best, tz_best = best
    us_gather = time_apply_device(kd, x, y, args.precision, reps=args.apply_reps, variant=1)
    # the same operator with five buffer sets in rotation (k, x, y per set;
    # 290 MB in FP32 at 128^3, above the 256 MB Infinity Cache), so that each
    # launch reads its inputs from HBM; timed with torch events on the stream
    # the launches use
    from paper_2405_19991_amd import apply_device_tiled
    sets = [(kd.clone(), torch.randn_like(x), torch.empty_like(y)) for _ in range(5)]
    for kk, xx, yy in sets:
        apply_device_tiled(kk, xx, yy, args.precision, tx_best, tz_best, variant=v_best)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rot_rounds = max(1, args.apply_reps // 5)
    e0.record()
    for _ in range(rot_rounds):
        for kk, xx, yy in sets:
            apply_device_tiled(kk, xx, yy, args.precision, tx_best, tz_best, variant=v_best)
    e1.record()
    torch.cuda.synchronize()
    us_rot = 1000.0 * e0.elapsed_time(e1) / (rot_rounds * len(sets))
    del sets
    bpn = 28 if args.precision == "mixed" else 56
    alg_bytes = bpn * nn
    achieved = alg_bytes / (us * 1e-6) / 1e9
    tname = "float" if args.precision == "mixed" else "double"
    kname = {0: "k_march2", 3: "k_march", 2: "k_tiled"}[v_best]
    operator = {"kernel": f"{kname}<{tname}, ..., DIR=false> tile {tx_best}x{256 // (tx_best // (2 if v_best == 0 else 1))}, tz={tz_best} (stencil apply, 3 loads)",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "us_per_launch": us, "alg_bytes_per_launch": alg_bytes, "direct_gather_us_per_launch": us_gather,
                "rotating_sets": {"sets": 5, "us_per_launch": us_rot,
                                  "achieved": alg_bytes / (us_rot * 1e-6) / 1e9,
                                  "frac": alg_bytes / (us_rot * 1e-6) / 1e9 / HBM_PEAK_GBS}}
    # dominant kernel of the timed design iterations, timed live (HIP events
    # around one sampled launch per check interval, on the solver's stream)
    if live["launches"] > 0:
        kdesc = ("k_fused_f32 (fused PCG pass: r -= a q, x += a p, p = D^-1 r + b p, q = A p, five dots; 3 loads)"
                 if live["kernel"] == 4 else
                 f"k_march2<{tname}, ..., DIR=true> (direction + operator pass, 3 loads)")
        if live["kernel"] == 4 and args.precision == "fp64":
            kdesc = kdesc.replace("k_fused_f32", "k_fused_f64")
        trec = (recorded_traffic(live["kernel"], tile["tx"], tile["tz"])
                if args.precision == "mixed" and n == 128 else None)
        # achieved/frac on the minimum state traffic of one PCG iteration: x, r, p
        # read and written per load plus k (152 B/node in float64, 76 B/node
        # with float32 vectors); the pass's own schedule bytes stand beside it
        if live["kernel"] == 4:
            min_bytes = (76 if args.precision == "mixed" else 152) * nn
        else:  # a two-pass iteration's first pass: its own bytes only
            min_bytes = live["bytes"]
        ach = min_bytes / (live["us"] * 1e-6) / 1e9
        roof = {"bound": "hbm", "kernel": kdesc, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": trec["traffic_bytes_per_launch"] if trec else None,
                "traffic_source": TRAFFIC_RECORDS[live["kernel"]][0] if trec else None,
                "us_per_launch": live["us"], "alg_bytes_per_launch": min_bytes,
                "alg_bytes_basis": ("minimum PCG-iteration state traffic: x, r, p read+write per load, k read "
                                    f"({min_bytes // nn} B/node)" if live["kernel"] == 4 else "pass bytes"),
                "schedule_bytes_per_launch": live["bytes"],
                "schedule_frac": live["bytes"] / (live["us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                "sampled_launches": live["launches"],
                "tile": {"tx": tile["tx"], "tz": tile["tz"], "blocks": tile["blocks"]}}
    else:
        roof = dict(operator, bound="hbm", traffic=None)

    out = {
        "metric": "128^3 PCG DOF-updates/s (whole design iteration, mixed precision)",
        "value": dof / wall,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-operator/f64-dots" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name + ("_" + args.precision), "n": n, "tol": w.tol, "loads": 3,
                   "guess": args.guess, "target": list(map(float, w.target)), "vf": w.vf,
                   "k0": w.k0, "kmin": w.kmin, "penal": w.penal, "filter_radius": w.rfilter},
        "s_per_oc_iter": wall / args.steps,
        "pcg_iters_per_step": pcg_iters / args.steps,
        "pcg_only_dof_per_s": dof / (solve_ms * 1e-3) if solve_ms > 0 else None,
        "solver_tile": tile,
        "tuning": tuning,
        "device_bytes": dev_bytes,
        "device_memory": {"context_bytes": dev_bytes, "device_in_use_peak_bytes": int(free0 - free_min[0]),
                          "device_total_bytes": int(total_mem),
                          "basis": "hipMemGetInfo (whole device) before the context exists, minus its minimum free "
                                   "memory sampled after creation, after each warm-up and after the timed "
                                   "iterations: the library, the HIP runtime and torch's cache"},
        "kappa_rel_err_vs_oracle": oracle_tensor_error(w, first_kappa, args.tol),
        "last_g": recs[-1]["g"],
        "last_kappa": recs[-1]["kappa"],
        "roofline": roof,
        "operator": operator,
    }
    h.close()
    if args.calib_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"apply kernel {us:.2f} us ({achieved:.0f} GB/s algorithmic); rotating 5 sets {us_rot:.2f} us")
    if not args.no_mg and args.preconditioner == "jacobi" and args.precision == "mixed" and n == 128:
        mg = multigrid_leg(w, args.steps, log, args.mg_sweeps, args.mg_coarse_sweeps)
        mg["kappa_rel_err_vs_oracle"] = oracle_tensor_error(w, mg.pop("first_kappa"), args.tol)
        out["multigrid"] = mg
        # the paper's relaxation: 8-colour Gauss-Seidel, one sweep per level and leg
        gs = multigrid_leg(w, args.steps, log, 1, 1, smoother="gs8")
        gs["kappa_rel_err_vs_oracle"] = oracle_tensor_error(w, gs.pop("first_kappa"), args.tol)
        out["multigrid_gs8"] = gs
    if not args.no_fp64 and args.precision == "mixed" and n == 128:
        out["fp64"] = fp64_leg(args.steps, log)
    if not args.no_full_run and args.precision == "mixed" and n == 128:
        out["full_run"] = full_run_leg(w, log)
    if not args.no_batch:
        out["batch"] = batch_leg(args.batch_steps, log)
        out["batch_mixed"] = batch_leg(args.batch_steps, log, "mixed")
    if not args.no_configs:
        out["configs"] = config_legs(5, log)
    if not args.no_gallery:
        # the paper's step 0.05 with the adaptive limit, the stall threshold at the bound
        out["gallery"] = gallery_leg(args.gallery_iters, log, n=args.gallery_n, move=0.05, move_min=0.002,
                                     governor={"dg_small": 1e-4})
    if not args.no_warm_start and n == 128:
        out["warm_start"] = warm_start_leg(args.weights, log)
    if not args.no_fused_sizes and args.preconditioner == "jacobi" and args.precision == "mixed" and n == 128:
        out["fused_sizes"] = fused_sizes_leg(log)
    # the operator in the other precision and at 256^3 (whose buffers exceed
    # the Infinity Cache), best of a few z-march shapes each; last, because
    # seconds of streaming at full bandwidth slow the GPU work right after it
    operator["sizes"] = apply_sizes(args.apply_reps)
    for a in operator["sizes"]:
        log(f"apply {a['n']}^3 {a['dtype']}: {a['us_per_launch']:.2f} us, {a['frac']:.3f} of peak")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
