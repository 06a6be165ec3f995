"""Python front end over the C ABI (argument marshalling only).

Mirrors the paper's Python interface shape (Sec. 3.5): a homogenization
object configured with a resolution, the two conductivities [k0, kmin] and a
target 6-vector, given a density, then optimized; and a one-call
``run_instance``.  Host arrays are float64 numpy arrays of shape (n, n, n)
indexed [z][y][x]; device inputs may be float64 torch CUDA tensors.
"""
from __future__ import annotations

import ctypes
import json
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _native as N

_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


OBJECTIVES = {"mse": N.OTM_OBJ_MSE, "rel": N.OTM_OBJ_REL, "l1": N.OTM_OBJ_L1}
INITS = {"P": N.OTM_INIT_P, "D": N.OTM_INIT_D, "G": N.OTM_INIT_G, "IWP": N.OTM_INIT_IWP, "ball": N.OTM_INIT_BALL}


def init_density(n: int, kind: str = "IWP", vf: float = 0.3) -> np.ndarray:
    """Initial density field (n, n, n) indexed [k][j][i]: P, D, G, IWP or the
    centre ball, with exactly round(vf n^3) solid elements (otm_init_density)."""
    out = np.empty(int(n) ** 3, dtype=np.float64)
    N.check(N.lib().otm_init_density(int(n), INITS[kind], float(vf), _ptr(out)))
    return out.reshape((int(n),) * 3)


class Homogenization:
    """One periodic n^3 design cell on the current HIP device."""

    def __init__(self, n: int, heat_ratio: Sequence[float] = (1.0, 1e-3),
                 target: Sequence[float] = (0.1, 0.1, 0.1, 0.0, 0.0, 0.0), vf: float = 0.3,
                 penal: float = 3.0, filter_radius: float = 1.5, precision: Optional[str] = None,
                 guess: str = "zero", tol: float = 1e-8, max_iter: int = 20000, check_every: int = 16,
                 reliable_delta: Optional[float] = None, move: float = 0.05, eta: float = 0.5, rho_min: float = 1e-3,
                 move_min: float = 0.0, mg_smoother: str = "jacobi",
                 governor: Optional[Dict[str, float]] = None, stream=None, kernel_variant: int = 0,
                 tile_tz: int = 0, tile_tx: int = 0, autotune: bool = True, preconditioner: str = "jacobi",
                 mg_sweeps: int = 1, mg_coarse_sweeps: int = 2, objective: str = "mse", symmetry: str = "none",
                 stall_window: int = 0):
        L = N.lib()
        self.n = int(n)
        p = N.Problem()
        p.n = self.n
        p.k0, p.kmin = float(heat_ratio[0]), float(heat_ratio[1])
        p.penal = float(penal)
        p.filter_radius = float(filter_radius)
        for i, t in enumerate(target):
            p.target[i] = float(t)
        p.vf = float(vf)
        p.objective = OBJECTIVES[objective]
        p.symmetry = {"none": N.OTM_SYM_NONE, "central": N.OTM_SYM_CENTRAL}[symmetry]
        s, o, g = N.default_options()
        if precision is None:  # the V-cycle runs in float32: multigrid implies mixed precision
            precision = "mixed" if preconditioner == "mg" else "fp64"
        s.precision = {"fp64": N.OTM_FP64, "mixed": N.OTM_MIXED}[precision]
        s.guess = {"zero": N.OTM_GUESS_ZERO, "previous": N.OTM_GUESS_PREVIOUS, "user": N.OTM_GUESS_USER,
                   "learned": N.OTM_GUESS_LEARNED}[guess]
        if reliable_delta is None:  # a V-cycle iteration cuts the residual several-fold
            reliable_delta = 1e-3 if preconditioner == "mg" else 1e-2
        s.tol, s.max_iter, s.check_every, s.reliable_delta = float(tol), int(max_iter), int(check_every), float(reliable_delta)
        s.kernel_variant, s.tile_tz, s.tile_tx = int(kernel_variant), int(tile_tz), int(tile_tx)
        s.autotune = int(bool(autotune))
        s.preconditioner = {"jacobi": N.OTM_PRECOND_JACOBI, "mg": N.OTM_PRECOND_MG}[preconditioner]
        s.mg_sweeps, s.mg_coarse_sweeps = int(mg_sweeps), int(mg_coarse_sweeps)
        s.stall_window = int(stall_window)
        s.mg_smoother = {"jacobi": N.OTM_MG_JACOBI, "gs8": N.OTM_MG_GS8}[mg_smoother]
        o.move, o.eta, o.rho_min, o.move_min = float(move), float(eta), float(rho_min), float(move_min)
        for key, val in (governor or {}).items():
            setattr(g, key, val)
        self.problem, self.solver, self.oc, self.gov = p, s, o, g
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(int(stream)) if stream is not None else None
        N.check(L.otm_create(ctypes.byref(p), ctypes.byref(s), ctypes.byref(o), ctypes.byref(g), st,
                             ctypes.byref(h)))
        self._h = h
        self._L = L

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            self._L.otm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, status, allow_nc=True):
        return N.check(status, self._h, allow_nc)

    @property
    def nn(self) -> int:
        return self.n ** 3

    # -- inputs
    def set_density(self, rho) -> None:
        try:
            import torch
            if isinstance(rho, torch.Tensor) and rho.is_cuda:
                if rho.dtype != torch.float64 or not rho.is_contiguous():
                    raise ValueError("device density must be a contiguous float64 tensor")
                self._chk(self._L.otm_set_density_device(self._h, ctypes.c_void_p(rho.data_ptr()), rho.numel()))
                return
        except ImportError:
            pass
        a = _f64(rho).reshape(-1)
        self._chk(self._L.otm_set_density(self._h, _ptr(a), a.size))

    def set_guess(self, chi) -> None:
        a = _f64(chi).reshape(-1)
        self._chk(self._L.otm_set_guess(self._h, _ptr(a), a.size))

    # -- the hot path, one piece at a time
    def prepare(self) -> None:
        self._chk(self._L.otm_prepare(self._h))

    def homogenize(self):
        kappa = np.zeros(6)
        st = N.SolveStats()
        status = self._chk(self._L.otm_homogenize(self._h, _ptr(kappa), ctypes.byref(st)))
        return kappa, dict(iterations=list(st.iterations), rel_residual=list(st.rel_residual),
                           converged=bool(st.converged), refreshes=st.refreshes, ms_solve=st.ms_solve,
                           status=status, stalled=st.stalled, fallback=bool(st.fallback))

    def sensitivity(self, dg_dkappa) -> np.ndarray:
        w = _f64(dg_dkappa)
        out = np.empty(self.nn)
        self._chk(self._L.otm_sensitivity(self._h, _ptr(w), _ptr(out)))
        return out.reshape((self.n,) * 3)

    def oc_update(self, vstar: float):
        out = np.empty(self.nn)
        lam = ctypes.c_double()
        self._chk(self._L.otm_oc_update(self._h, float(vstar), _ptr(out), ctypes.byref(lam)))
        return out.reshape((self.n,) * 3), lam.value

    def step(self) -> Dict[str, object]:
        r = N.IterRecord()
        self._chk(self._L.otm_step(self._h, ctypes.byref(r)))
        return r.to_dict()

    def optimize(self, max_iter: int):
        out = np.empty(self.nn)
        log = (N.IterRecord * max(1, max_iter))()
        done = ctypes.c_int32()
        self._chk(self._L.otm_optimize(self._h, int(max_iter), _ptr(out), log, max(1, max_iter), ctypes.byref(done)))
        return out.reshape((self.n,) * 3), [log[i].to_dict() for i in range(done.value)]

    def get_field(self, name: str) -> np.ndarray:
        size = 3 * self.nn if name in N.FIELD3 else self.nn
        out = np.empty(size)
        self._chk(self._L.otm_get_field(self._h, N.FIELDS[name], _ptr(out), size))
        shape = (3, self.n, self.n, self.n) if name in N.FIELD3 else (self.n,) * 3
        return out.reshape(shape)

    def set_field(self, name: str, values) -> None:
        a = _f64(values).reshape(-1)
        self._chk(self._L.otm_set_field(self._h, N.FIELDS[name], _ptr(a), a.size))

    def apply(self, x, precision: str = "fp64") -> np.ndarray:
        a = _f64(x).reshape(-1)
        if a.size != 3 * self.nn:
            raise ValueError("x must hold 3 n^3 values")
        y = np.empty_like(a)
        self._chk(self._L.otm_apply(self._h, {"fp64": N.OTM_FP64, "mixed": N.OTM_MIXED}[precision], _ptr(a), _ptr(y)))
        return y.reshape(3, self.n, self.n, self.n)

    def set_network(self, net) -> None:
        """Attach a Network for guess='learned' (None detaches)."""
        self._net = net
        self._chk(self._L.otm_set_network(self._h, net._h if net is not None else None))

    def tile(self) -> Dict[str, int]:
        t = (ctypes.c_int32 * 4)()
        self._chk(self._L.otm_get_tile(self._h, t))
        return dict(variant=t[0], tx=t[1], tz=t[2], blocks=t[3])

    def pass_timing(self, reset: bool = False) -> Dict[str, float]:
        """Live HIP-event timing of the solver's dominant kernel since the last reset."""
        t = np.zeros(4)
        self._chk(self._L.otm_pass_timing(self._h, int(bool(reset)), _ptr(t)))
        return dict(launches=int(t[0]), us=float(t[1]), bytes=float(t[2]), kernel=int(t[3]))

    def timings(self) -> List[float]:
        t = np.zeros(8)
        self._chk(self._L.otm_get_timings(self._h, _ptr(t)))
        return t.tolist()

    def device_bytes(self) -> int:
        """Device memory the context holds, bytes."""
        b = ctypes.c_int64()
        self._chk(self._L.otm_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    # -- governor state, checkpoint / resume
    def governor_state(self) -> List[float]:
        s = np.zeros(8)
        self._chk(self._L.otm_get_governor(self._h, _ptr(s)))
        return s.tolist()

    def set_governor_state(self, s: Sequence[float]) -> None:
        a = _f64(s)
        self._chk(self._L.otm_set_governor(self._h, _ptr(a)))

    def save_state(self, path: str) -> None:
        """Checkpoint (otm_save_state): density, last solution (warm start)
        and governor state in the library's binary state file."""
        self._chk(self._L.otm_save_state(self._h, str(path).encode()))

    def load_state(self, path: str) -> None:
        """Resume from a file written by save_state (otm_load_state)."""
        self._chk(self._L.otm_load_state(self._h, str(path).encode()))


def _operator_args(k, x, y, precision: str, stream):
    """Validate the tensors of a stateless operator call before any pointer
    reaches the library: n^3 conductivities, 3 n^3 node values, contiguous
    CUDA tensors of the precision's dtype on one device, y not aliasing x."""
    import torch
    if precision not in ("fp64", "mixed", "fp32"):
        raise ValueError(f"unknown precision {precision!r}")
    n = round(k.numel() ** (1.0 / 3.0))
    if n < 4 or n ** 3 != k.numel() or x.numel() != 3 * n ** 3 or y.numel() != 3 * n ** 3:
        raise ValueError("shape mismatch: k needs n^3 values, x and y 3 n^3")
    want = torch.float64 if precision == "fp64" else torch.float32
    for t in (k, x, y):
        if t.dtype != want or not t.is_cuda or not t.is_contiguous() or t.device != k.device:
            raise ValueError("tensors must be contiguous CUDA tensors of the precision's dtype on one device")
    if y.data_ptr() == x.data_ptr():
        raise ValueError("y must not alias x")
    s = stream if stream is not None else torch.cuda.current_stream(k.device).cuda_stream
    prec = N.OTM_FP64 if precision == "fp64" else N.OTM_MIXED
    return n, prec, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), \
        ctypes.c_void_p(s)


def apply_device(k, x, y, precision: str = "fp64", stream=None, variant: int = 0) -> None:
    """y = A x on caller device memory (torch CUDA tensors, load-major 3 n^3)."""
    n, prec, kp, xp, yp, s = _operator_args(k, x, y, precision, stream)
    N.check(N.lib().otm_apply_device(n, prec, int(variant), kp, xp, yp, s))


def apply_device_tiled(k, x, y, precision: str, tile_tx: int, tile_tz: int, variant: int = 0, stream=None) -> None:
    """One y = A x launch with an explicit tile, on the given (default: the
    current torch) stream, not synchronised."""
    n, prec, kp, xp, yp, s = _operator_args(k, x, y, precision, stream)
    N.check(N.lib().otm_apply_device_tiled(n, prec, int(variant), int(tile_tx), int(tile_tz), kp, xp, yp, s))


def time_apply_device(k, x, y, precision: str = "fp64", reps: int = 50, stream=None, variant: int = 0,
                      tile_tx: int = 0, tile_tz: int = 0) -> float:
    n, prec, kp, xp, yp, s = _operator_args(k, x, y, precision, stream)
    us = ctypes.c_double()
    N.check(N.lib().otm_time_apply_device(n, prec, int(variant), int(tile_tx), int(tile_tz), kp, xp, yp, s,
                                          int(reps), ctypes.byref(us)))
    return us.value


def oc_update_noalloc(rho, sens, vstar: float, out=None, lam=None, move: float = 0.05, eta: float = 0.5,
                      rho_min: float = 1e-3, stream=None):
    """OC update on caller device memory with no device allocation in the
    library (otm_oc_update_noalloc): rho, sens and out are float64 CUDA
    tensors of n^3 values (out may be rho); lam, if given, a one-element
    float64 CUDA tensor for the multiplier.  Enqueued on the stream (default:
    the current torch stream), not synchronised.  Returns out."""
    import torch
    n = round(rho.numel() ** (1.0 / 3.0))
    if n ** 3 != rho.numel() or sens.numel() != rho.numel():
        raise ValueError("rho and sens need n^3 values each")
    if out is None:
        out = torch.empty_like(rho)
    ts = [rho, sens, out] + ([lam] if lam is not None else [])
    for t in ts:
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.device != rho.device:
            raise ValueError("tensors must be contiguous float64 CUDA tensors on one device")
    if out.numel() != rho.numel() or (lam is not None and lam.numel() != 1):
        raise ValueError("out needs n^3 values, lam one")
    oc = N.OcOpts(float(move), float(eta), float(rho_min))
    s = stream if stream is not None else torch.cuda.current_stream(rho.device).cuda_stream
    N.check(N.lib().otm_oc_update_noalloc(n, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(sens.data_ptr()),
                                          float(vstar), ctypes.byref(oc), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(lam.data_ptr() if lam is not None else None),
                                          ctypes.c_void_p(s)))
    return out


def run_instance(reso: int, heat_ratio: Sequence[float], target: Sequence[float], init="IWP", vf: float = 0.3,
                 max_iter: int = 500, **kw):
    """Design one structure: mirrors the paper's runInstance(reso, heatRatio,
    target, init, model) for the adaptive-volume model with OC.  `init` is an
    initializer name (P, D, G, IWP -- the paper's default -- or ball, at volume
    fraction vf) or a density array."""
    rho0 = init_density(reso, init, vf) if isinstance(init, str) else np.asarray(init, dtype=np.float64)
    with Homogenization(reso, heat_ratio, target, vf=vf, **kw) as h:
        h.set_density(rho0)
        rho, log = h.optimize(max_iter)
    return rho, log


def version() -> str:
    return N.lib().otm_version().decode()


def dumps_log(log) -> str:
    return "\n".join(json.dumps(r) for r in log)


class Batch:
    """Many independent cells of uneven (even) n, stepped together: every
    phase of a design iteration is one launch over all designs, and PCG
    chunks replay a captured hipGraph.  float64 or mixed precision.

    precision: "fp64", or "mixed" (float32 operator and Krylov vectors with
    float64 residual refreshes; fused iteration only; reliable_delta defaults
    to 1e-4 here, since a refresh covers every design).  iteration: "auto"
    (the autotuner picks the fused single-pass or the two-pass PCG
    iteration; with autotune off, the two-pass one), "fused" or "two_pass"."""

    ITERATIONS = {"auto": 0, "fused": 4, "two_pass": 1}

    def __init__(self, problems: Sequence[Dict[str, object]], tol: float = 1e-6, max_iter: int = 20000,
                 check_every: int = 16, guess: str = "zero", move: float = 0.05, eta: float = 0.5, move_min: float = 0.0,
                 rho_min: float = 1e-3, governor: Optional[Dict[str, float]] = None, autotune: bool = True,
                 tile_tx: int = 0, tile_tz: int = 0, iteration: str = "auto", precision: str = "fp64",
                 reliable_delta: Optional[float] = None, stall_window: int = 0, stream=None):
        L = N.lib()
        arr = (N.Problem * len(problems))()
        self.ns = []
        for i, pr in enumerate(problems):
            p = arr[i]
            p.n = int(pr["n"])
            hr = pr.get("heat_ratio", (1.0, 1e-3))
            p.k0, p.kmin = float(hr[0]), float(hr[1])
            p.penal = float(pr.get("penal", 3.0))
            p.filter_radius = float(pr.get("filter_radius", 1.5))
            for q, t in enumerate(pr["target"]):
                p.target[q] = float(t)
            p.vf = float(pr.get("vf", 0.3))
            p.objective = OBJECTIVES[pr.get("objective", "mse")]
            p.symmetry = N.OTM_SYM_NONE
            self.ns.append(p.n)
        s, o, g = N.default_options()
        s.precision = {"fp64": N.OTM_FP64, "mixed": N.OTM_MIXED}[precision]
        if reliable_delta is not None:
            s.reliable_delta = float(reliable_delta)
        elif precision == "mixed":
            # a batch refreshes every design at once: fewer, deeper refreshes
            # pay off (1e-4: 27.7 ms per 64-design iteration against 28.8 ms
            # at a context's 1e-2, same iterations)
            s.reliable_delta = 1e-4
        s.guess = {"zero": N.OTM_GUESS_ZERO, "previous": N.OTM_GUESS_PREVIOUS}[guess]
        s.tol, s.max_iter, s.check_every = float(tol), int(max_iter), int(check_every)
        s.autotune, s.tile_tx, s.tile_tz = int(bool(autotune)), int(tile_tx), int(tile_tz)
        s.kernel_variant = self.ITERATIONS[iteration]
        s.stall_window = int(stall_window)
        o.move, o.eta, o.rho_min, o.move_min = float(move), float(eta), float(rho_min), float(move_min)
        for key, val in (governor or {}).items():
            setattr(g, key, val)
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(int(stream)) if stream is not None else None
        N.check(L.otm_batch_create(arr, len(problems), ctypes.byref(s), ctypes.byref(o), ctypes.byref(g), st,
                                   ctypes.byref(h)))
        self._h, self._L, self.count = h, L, len(problems)

    def _chk(self, status, allow_nc=True):
        if status == N.OTM_OK or (status == N.OTM_NOT_CONVERGED and allow_nc):
            return status
        msg = self._L.otm_strerror(status).decode()
        raise N.OTMError(status, msg + " (" + self._L.otm_batch_last_error(self._h).decode() + ")")

    def close(self):
        if getattr(self, "_h", None):
            self._L.otm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_density(self, d: int, rho) -> None:
        a = _f64(rho).reshape(-1)
        self._chk(self._L.otm_batch_set_density(self._h, int(d), _ptr(a), a.size))

    def get_field(self, d: int, name: str) -> np.ndarray:
        n = self.ns[d]
        size = 3 * n ** 3 if name in N.FIELD3 else n ** 3
        out = np.empty(size)
        self._chk(self._L.otm_batch_get_field(self._h, int(d), N.FIELDS[name], _ptr(out), size))
        return out.reshape((3, n, n, n) if name in N.FIELD3 else (n, n, n))

    def set_graph(self, on: bool) -> None:
        self._chk(self._L.otm_batch_set_graph(self._h, int(bool(on))))

    def save_state(self, path: str) -> None:
        """Checkpoint (otm_batch_save_state): every design's density, last
        solution and governor state, and the iteration count."""
        self._chk(self._L.otm_batch_save_state(self._h, str(path).encode()))

    def load_state(self, path: str) -> None:
        """Resume from a file written by save_state for the same designs
        (otm_batch_load_state)."""
        self._chk(self._L.otm_batch_load_state(self._h, str(path).encode()))

    def step(self) -> List[Dict[str, object]]:
        recs = (N.IterRecord * self.count)()
        status = self._chk(self._L.otm_batch_step(self._h, recs))
        out = [recs[i].to_dict() for i in range(self.count)]
        for r in out:
            r["status"] = status
        return out

    def info(self) -> Dict[str, float]:
        a = np.zeros(10)
        self._chk(self._L.otm_batch_info(self._h, _ptr(a)))
        keys = ["designs", "cells", "work_items", "tile_tx", "tile_tz", "tuned_iteration_us", "solve_ms", "step_ms",
                "fused", "refreshes"]
        return dict(zip(keys, a.tolist()))

    def governor_state(self, d: int) -> List[float]:
        """Adaptive volume bound of design d: [V*, Df, stalls, gap, g_prev, flat, iter, OC step]."""
        s = np.zeros(8)
        self._chk(self._L.otm_batch_get_governor(self._h, int(d), _ptr(s)))
        return s.tolist()

    def device_bytes(self) -> int:
        """Device memory the batch holds, bytes."""
        b = ctypes.c_int64()
        self._chk(self._L.otm_batch_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)


class Network:
    """The learned warm start: periodic 3x3x3 CNN (1-16-16-16-16-3) on bf16 MFMA.
    Training runs on the GPU through forward/backward kernels; Python only
    sequences samples.  Device inputs are float64 torch CUDA tensors."""

    def __init__(self, n_max: int = 128, seed: int = 0, stream=None):
        L = N.lib()
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(int(stream)) if stream is not None else None
        N.check(L.otm_nn_create(int(n_max), int(seed), st, ctypes.byref(h)))
        self._h, self._L, self.n_max = h, L, n_max
        self.count = int(L.otm_nn_param_count())

    def _chk(self, status):
        if status != N.OTM_OK:
            raise N.OTMError(status, self._L.otm_strerror(status).decode() + " (" +
                             self._L.otm_nn_last_error(self._h).decode() + ")")

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            self._L.otm_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        a = np.empty(self.count, dtype=np.float32)
        self._chk(self._L.otm_nn_get_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
        return a

    def set_params(self, a) -> None:
        a = np.ascontiguousarray(a, dtype=np.float32)
        self._chk(self._L.otm_nn_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))

    def grads(self) -> np.ndarray:
        a = np.empty(self.count, dtype=np.float32)
        self._chk(self._L.otm_nn_get_grads(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
        return a

    @staticmethod
    def _n(t, k=1):
        n = round((t.numel() // k) ** (1.0 / 3.0))
        return n

    def forward(self, rhof_dev, chi0_dev) -> None:
        import torch
        n = self._n(rhof_dev)
        assert rhof_dev.dtype == torch.float64 and chi0_dev.dtype == torch.float64 and chi0_dev.numel() == 3 * n ** 3
        self._chk(self._L.otm_nn_forward(self._h, n, ctypes.c_void_p(rhof_dev.data_ptr()),
                                         ctypes.c_void_p(chi0_dev.data_ptr())))

    def accumulate(self, rhof_dev, chi_dev) -> float:
        n = self._n(rhof_dev)
        loss = ctypes.c_double()
        self._chk(self._L.otm_nn_accumulate(self._h, n, ctypes.c_void_p(rhof_dev.data_ptr()),
                                            ctypes.c_void_p(chi_dev.data_ptr()), ctypes.byref(loss)))
        return loss.value

    def adam(self, lr: float, batch: int) -> None:
        self._chk(self._L.otm_nn_adam(self._h, float(lr), int(batch)))

    def zero_grads(self) -> None:
        self._chk(self._L.otm_nn_zero_grads(self._h))

    def save(self, path: str) -> None:
        """Weights as a float32 .npy file (otm_nn_save)."""
        self._chk(self._L.otm_nn_save(self._h, str(path).encode()))

    def load(self, path: str) -> None:
        """Weights from a float32 .npy file (otm_nn_load)."""
        self._chk(self._L.otm_nn_load(self._h, str(path).encode()))


def compact_to_layers(a: np.ndarray, channels=(1, 16, 16, 16, 16, 3)):
    """Split the compact parameter vector into [{'W': (cout, cin, 27), 'b': (cout,)}]."""
    out, q = [], 0
    for cin, cout in zip(channels[:-1], channels[1:]):
        W = a[q:q + cout * cin * 27].reshape(cout, cin, 27)
        q += cout * cin * 27
        b = a[q:q + cout]
        q += cout
        out.append({"W": W.astype(np.float64), "b": b.astype(np.float64)})
    return out
