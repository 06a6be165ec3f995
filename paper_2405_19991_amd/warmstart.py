"""Training and evaluation of the learned PCG warm start.

Pairs (filtered density, converged fluctuation fields) are produced by the
method itself: seeded design runs of the GPU optimizer dump one pair per
design iteration.  The network is trained on the GPU with the library's
forward/backward kernels and Adam; this module only sequences samples.

    python -m paper_2405_19991_amd.warmstart train --out weights.npy
    python -m paper_2405_19991_amd.warmstart eval --weights weights.npy
    python -m paper_2405_19991_amd.warmstart spectrum --weights weights.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart.npy")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def design_runs() -> List[Tuple[str, int, object, object, float, int]]:
    """(name, n, rho0, target, vf, iterations) for the training designs, about
    2000 (rho~, chi) pairs: 20 isotropic 16^3 cells x 30 design iterations,
    8 orthotropic 64^3 cells x 100, 4 anisotropic 128^3 cells x 150 (the
    evaluation cell, seed 303, is held out)."""
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    runs = []
    for s in range(20):
        runs.append((f"iso16_{s}", 16, synth.uniform_noise(16, 0.3, 0.05, 1000 + s), synth.TARGET_ISO, 0.3, 30))
    for s in range(8):
        runs.append((f"ortho64_{s}", 64, synth.smoothed_noise(64, 0.2, 0.5, 201 + s), synth.TARGET_ORTHO, 0.35, 100))
    for seed in (301, 302, 304, 305):
        runs.append((f"aniso128_{seed}", 128, synth.smoothed_noise(128, 0.15, 0.45, seed), synth.TARGET_ANISO, 0.3,
                     150))
    return runs


def generate(runs=None, tol: float = 1e-6):
    """Run the optimizer and keep (rho~, chi) of every design iteration on the GPU."""
    import torch
    from .api import Homogenization
    runs = runs or design_runs()
    data = []
    for name, n, rho0, target, vf, iters in runs:
        with Homogenization(n, (1.0, 1e-3), target, vf=vf, tol=tol, precision="mixed" if n >= 64 else "fp64",
                            guess="previous") as h:
            h.set_density(rho0)
            for _ in range(iters):
                h.step()
                # the fields of the iteration just solved: rho~ of the density it used and chi
                rf = torch.from_numpy(h.get_field("rhof").reshape(-1)).cuda()
                chi = torch.from_numpy(h.get_field("chi").reshape(-1)).cuda()
                data.append((n, rf, chi))
        _log(f"data: {name} done, {len(data)} pairs")
    return data


def train(data, epochs: int = 30, batch: int = 8, lr: float = 2e-3, seed: int = 0, n_max: int = 128,
          halve_every: int = 8):
    from .api import Network
    net = Network(n_max=n_max, seed=seed)
    g = np.random.Generator(np.random.PCG64(seed))
    history = []
    for ep in range(epochs):
        order = g.permutation(len(data))
        tot, cnt = 0.0, 0
        net.zero_grads()
        for q, idx in enumerate(order):
            n, rf, chi = data[idx]
            tot += net.accumulate(rf, chi)
            cnt += 1
            if cnt % batch == 0 or q == len(order) - 1:
                net.adam(lr * (0.5 ** (ep // halve_every)), min(batch, cnt % batch or batch))
        history.append(tot / len(order))
        _log(f"epoch {ep}: mean loss {history[-1]:.4e}")
    return net, history


def _solve_record(h, kappa, st, ms):
    return {"pcg_iters": int(sum(st["iterations"])), "max_load_iters": int(max(st["iterations"])),
            "ms": ms, "converged": bool(st["converged"]), "learned_used": bool(h.timings()[6]),
            "kappa": [float(v) for v in kappa]}


def time_to_tol(n: int, rho, target, vf: float, precision: str, guess: str, net=None,
                tol: float = 1e-6, preconditioner: str = "jacobi") -> Dict[str, float]:
    """PCG iterations and wall time of one homogenization of the density rho
    from a zero or learned start (a warm-up solve of the same state first).
    The time includes the network's forward pass for the learned start."""
    import torch
    from .api import Homogenization
    with Homogenization(n, (1.0, 1e-3), target, vf=vf, tol=tol, precision=precision, guess=guess,
                        preconditioner=preconditioner) as h:
        if net is not None:
            h.set_network(net)
        h.set_density(rho)
        h.homogenize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kappa, st = h.homogenize()
        ms = 1000.0 * (time.perf_counter() - t0)
        return _solve_record(h, kappa, st, ms)


def evaluate(net, n: int = 128, seed: int = 303, at_iter: int = 5, tol: float = 1e-6) -> Dict[str, Dict[str, float]]:
    """Time to tol on a held-out 128^3 anisotropic cell at design iteration
    `at_iter`: the previous design iteration's solution as the start (that
    solve, timed inside the design run), then zero and learned starts on the
    same density."""
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    from .api import Homogenization
    rho0 = synth.smoothed_noise(n, 0.15, 0.45, seed)
    tgt, vf = synth.TARGET_ANISO, 0.3
    with Homogenization(n, (1.0, 1e-3), tgt, vf=vf, tol=tol, precision="mixed", guess="previous") as h:
        h.set_density(rho0)
        for _ in range(at_iter):
            h.step()
        rho_k = h.get_field("rho")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kappa, st = h.homogenize()
        prev = _solve_record(h, kappa, st, 1000.0 * (time.perf_counter() - t0))
    return {
        "design_iteration": at_iter,
        "zero_fp64": time_to_tol(n, rho_k, tgt, vf, "fp64", "zero", tol=tol),
        "zero_mixed": time_to_tol(n, rho_k, tgt, vf, "mixed", "zero", tol=tol),
        "previous_mixed": prev,
        "learned_mixed": time_to_tol(n, rho_k, tgt, vf, "mixed", "learned", net, tol=tol),
        "learned_fp64": time_to_tol(n, rho_k, tgt, vf, "fp64", "learned", net, tol=tol),
        "zero_mixed_mg": time_to_tol(n, rho_k, tgt, vf, "mixed", "zero", tol=tol, preconditioner="mg"),
        "learned_mixed_mg": time_to_tol(n, rho_k, tgt, vf, "mixed", "learned", net, tol=tol, preconditioner="mg"),
    }


FLOP_FWD = 2 * 27 * (1 * 16 + 3 * 16 * 16 + 16 * 3)       # per voxel, forward
FLOP_TRAIN = FLOP_FWD + 2 * 27 * (3 * 16 * 16 + 16 * 3) + FLOP_FWD  # + input and weight gradients


def kernels(n: int = 128, reps: int = 5) -> Dict[str, float]:
    """Wall time of one forward pass and of one training sample (forward,
    input and weight gradients, loss) at n^3 on random inputs."""
    import torch
    from .api import Network
    net = Network(n_max=n, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    rf = torch.rand(n ** 3, dtype=torch.float64, device="cuda", generator=g)
    chi = torch.rand(3 * n ** 3, dtype=torch.float64, device="cuda", generator=g) - 0.5
    out = torch.empty_like(chi)
    net.forward(rf, out)
    net.accumulate(rf, chi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(rf, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        net.accumulate(rf, chi)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, trn = (t1 - t0) / reps, (t2 - t1) / reps
    vox = n ** 3
    return {"n": n, "forward_ms": 1e3 * fwd, "train_sample_ms": 1e3 * trn,
            "forward_tflops": FLOP_FWD * vox / fwd / 1e12, "train_tflops": FLOP_TRAIN * vox / trn / 1e12}


def error_spectrum(net, n: int = 128, seed: int = 303, at_iter: int = 5) -> Dict[str, object]:
    """Where the warm starts' errors lie, on the held-out anisotropic cell at
    design iteration `at_iter`: for the network's prediction and for the
    previous design iteration's solution, each scaled by its energy factor
    s = b.x / x.A x, per load the relative energy-norm and L2 errors against a
    float64 solve to 1e-10 and the fraction of the error's energy (its
    squared Fourier coefficients) at wavenumbers |k| <= 2, 4, 8, 16; and the
    same fractions for chi itself."""
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    from .api import Homogenization
    rho = synth.smoothed_noise(n, 0.15, 0.45, seed)
    kk = np.fft.fftfreq(n) * n
    K = np.sqrt(kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kk[None, None, :] ** 2)

    def bands(e):
        E = np.abs(np.fft.fftn(e)) ** 2
        return {f"|k|<={kc}": float(E[K <= kc].sum() / E.sum()) for kc in (2, 4, 8, 16)}

    out: Dict[str, object] = {"n": n, "seed": seed, "design_iteration": at_iter}
    with Homogenization(n, (1.0, 1e-3), synth.TARGET_ANISO, vf=0.3, tol=1e-10, guess="previous") as h:
        h.set_density(rho)
        for _ in range(at_iter):
            h.step()
        chi_prev = h.get_field("chi")
        h.homogenize()
        chi, b = h.get_field("chi"), h.get_field("b")
        rf = torch.from_numpy(h.get_field("rhof").reshape(-1).copy()).cuda()
        x0 = torch.empty(3 * n ** 3, dtype=torch.float64, device="cuda")
        net.forward(rf, x0)
        torch.cuda.synchronize()
        for name, x in (("learned", x0.cpu().numpy().reshape(3, n, n, n)), ("previous", chi_prev)):
            ax = h.apply(x).reshape(3, n, n, n)
            rec = []
            for l in range(3):
                xax, bx, bchi = float(np.sum(x[l] * ax[l])), float(np.sum(b[l] * x[l])), float(np.sum(b[l] * chi[l]))
                sc = max(bx, 0.0) / xax
                e = sc * x[l] - chi[l]
                rec.append({"scale": sc, "energy_err": float(np.sqrt(max(sc * sc * xax - 2 * sc * bx + bchi, 0.0) / bchi)),
                            "l2_err": float(np.linalg.norm(e) / np.linalg.norm(chi[l])), **bands(e)})
            out[name] = rec
        out["chi"] = [bands(chi[l]) for l in range(3)]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval", "kernels", "spectrum"])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--summary", default=None)
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    from .api import Network
    if a.cmd == "kernels":
        print(json.dumps(kernels()), flush=True)
        return
    if a.cmd == "spectrum":
        net = Network(n_max=128)
        net.load(a.weights)
        print(json.dumps(error_spectrum(net), indent=1), flush=True)
        return
    if a.cmd == "train":
        t0 = time.perf_counter()
        data = generate()
        t1 = time.perf_counter()
        net, hist = train(data, epochs=a.epochs)
        t2 = time.perf_counter()
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        net.save(a.out)
        ev = evaluate(net)
        summary = {"pairs": len(data), "data_s": t1 - t0, "train_s": t2 - t1, "loss_history": hist, "eval_128": ev}
        print(json.dumps(summary), flush=True)
        if a.summary:
            with open(a.summary, "w") as f:
                json.dump(summary, f, indent=1)
    else:
        net = Network(n_max=128)
        net.load(a.weights)
        print(json.dumps(evaluate(net)), flush=True)


if __name__ == "__main__":
    main()
