"""Writes cell128_kappa.json: the homogenized tensor of the 128^3 anisotropic
cell's initial density (first design iteration), computed by the CPU FP64
oracle alone (CSR stiffness, plain CG to a relative residual of 1e-10 per
load).  It is the full-size reference for the GPU paths' tensors.

    python tests/golden/make_cell128_kappa.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402


def main():
    w = synth.config3("fp64")
    prm = O.Params(tol=1e-10, max_iter=100000)
    t0 = time.time()
    out = O.homogenize(w.rho0, prm, with_energies=False)
    rec = {
        "what": "homogenized tensor [k11, k22, k33, k12, k23, k13] of the 128^3 anisotropic cell's initial density",
        "workload": w.name,
        "n": w.n,
        "k0": w.k0, "kmin": w.kmin, "penal": w.penal, "filter_radius": w.rfilter,
        "tol": prm.tol,
        "kappa": [float(v) for v in out["kappa"]],
        "cg_iterations": [int(v) for v in out["iters"]],
        "rel_residuals": [float(v) for v in out["residuals"]],
        "converged": [bool(v) for v in out["converged"]],
        "oracle_threads": O.num_threads(),
        "seconds": time.time() - t0,
        "script": "tests/golden/make_cell128_kappa.py",
    }
    with open(os.path.join(HERE, "cell128_kappa.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
