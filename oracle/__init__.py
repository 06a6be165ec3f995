"""CPU FP64 oracle for the periodic thermal homogenization design step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``.  The product library never
imports, links or calls anything here, and this package imports nothing from
the product package; the only shared code is the seeded input generator
module ``synth``, which holds none of the method's arithmetic.

What it computes (paper: Quan, Zhai, Fu, "OpenTM", arXiv 2405.19991):

* ``homogenize``: density filter (Sec. 2.3 filter equation) -> SIMP
  conductivity (Sec. 2.2) -> assembled periodic stiffness and the three macro
  loads (Sec. 2.2, K T^(i) = f^(i); Sec. 2.4 enforceMacroLoad) -> plain
  conjugate gradients on the zero-mean subspace -> homogenized tensor
  (discrete homogenization formula, Sec. 2.2) as the 6-vector of Sec. 2.2.
* ``objective``: the six-term squared error (Sec. 4.4, MSE objective), and
  the relative and l1 objectives of the same section.
* ``symmetrize_central``: the central-symmetry constraint (Sec. 4.3).
* ``init_density``: the TPMS and centre-ball initial densities (Sec. 4.3).
* ``sensitivities``: chain rule of Sec. 2.3 through the tensor, SIMP and the
  filter transpose.
* ``oc_update``: Optimality Criteria bisection (Sec. 3.3, OCOptimizer).
* ``Governor``: adaptive volume bound, Algorithm 1, plus the three-iteration
  stall test of Sec. 2.3.

Pins (tests/test_oracle_*.py): element matrix against the hand-derived
pattern and spectrum; dense direct solve on 4^3; closed forms for uniform,
laminate and checkerboard cells; Voigt/Reuss bounds; symmetry and
permutation covariance; finite differences of the full objective; filter
Fourier symbol; OC closed form; hand-traced governor tables.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OTM_ORACLE_LIB may name another build of the same source (the sanitizer
# check runs the oracle from an instrumented copy)
_LIBPATH = os.environ.get("OTM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.c_int64
_d = ctypes.c_double


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    sig = {
        "ora_num_threads": ([], ctypes.c_int),
        "ora_element_matrix": ([_dp], None),
        "ora_filter": ([_i64, _d, _dp, _dp], None),
        "ora_filter_transpose": ([_i64, _d, _dp, _dp], None),
        "ora_simp": ([_i64, _dp, _d, _d, _d, _dp], None),
        "ora_assemble": ([_i64, _dp, _ip, _dp], None),
        "ora_rhs": ([_i64, _dp, _dp], None),
        "ora_spmv": ([_i64, _ip, _dp, _dp, _dp], None),
        "ora_cg": ([_i64, _ip, _dp, _dp, _d, _i64, _dp, _dp], ctypes.c_int),
        "ora_cg_fixed": ([_i64, _ip, _dp, _dp, _i64, _dp], None),
        "ora_energy": ([_i64, _dp, _dp], None),
        "ora_kappa": ([_i64, _dp, _dp, _dp], None),
        "ora_sens": ([_i64, _dp, _dp, _dp, _d, _d, _d, _dp], None),
        "ora_oc_update": ([_i64, _dp, _dp, _d, _d, _d, _d, _dp, _ip], ctypes.c_double),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _c(a: np.ndarray, dtype=np.float64) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_ip)
    raise TypeError(a.dtype)


def num_threads() -> int:
    return int(_load().ora_num_threads())


# ---------------------------------------------------------------- primitives

def element_matrix() -> np.ndarray:
    """8x8 unit-voxel conduction matrix (trilinear hex, Gauss quadrature)."""
    K = np.zeros(64)
    _load().ora_element_matrix(_ptr(K))
    return K.reshape(8, 8)


def density_filter(rho: np.ndarray, r: float) -> np.ndarray:
    rho = _c(rho)
    n = rho.shape[0]
    out = np.empty_like(rho)
    _load().ora_filter(n, float(r), _ptr(rho), _ptr(out))
    return out


def density_filter_T(y: np.ndarray, r: float) -> np.ndarray:
    y = _c(y)
    n = y.shape[0]
    out = np.empty_like(y)
    _load().ora_filter_transpose(n, float(r), _ptr(y), _ptr(out))
    return out


def simp(rhof: np.ndarray, k0: float, kmin: float, p: float) -> np.ndarray:
    rhof = _c(rhof)
    out = np.empty_like(rhof)
    _load().ora_simp(rhof.size, _ptr(rhof), float(k0), float(kmin), float(p), _ptr(out))
    return out


@dataclasses.dataclass
class CSR27:
    """Periodic stiffness with 27 slots per row (slot = 9(dz+1)+3(dy+1)+(dx+1))."""
    n: int
    cols: np.ndarray   # (n^3, 27) int32
    vals: np.ndarray   # (n^3, 27) float64

    def matvec(self, x: np.ndarray) -> np.ndarray:
        x = _c(x).reshape(-1)
        y = np.empty_like(x)
        _load().ora_spmv(x.size, _ptr(self.cols), _ptr(self.vals), _ptr(x), _ptr(y))
        return y.reshape((self.n,) * 3)

    def dense(self) -> np.ndarray:
        nn = self.n ** 3
        A = np.zeros((nn, nn))
        for v in range(nn):
            for s in range(27):
                A[v, self.cols[v, s]] += self.vals[v, s]
        return A


def assemble(k: np.ndarray) -> CSR27:
    k = _c(k)
    n = k.shape[0]
    if n < 3:
        raise ValueError("assembly needs n >= 3")
    nn = n ** 3
    cols = np.empty((nn, 27), dtype=np.int32)
    vals = np.empty((nn, 27))
    _load().ora_assemble(n, _ptr(k), _ptr(cols), _ptr(vals))
    return CSR27(n, cols, vals)


def apply_at(k_patch: np.ndarray, x_patch: np.ndarray, absolute: bool = False) -> np.ndarray:
    """(A x) at single nodes from their neighbourhoods, by the definition of
    the assembled operator A = sum_e k_e P_e^T K P_e (Sec. 2, the discrete
    periodic cell problem; vertex order l = a + 2b + 4c): the node is vertex
    (1-cx, 1-cy, 1-cz) of the element whose lower corner sits at
    node + (cx-1, cy-1, cz-1), and that element's vertex (a, b, c) is the
    neighbour node + (cx-1+a, cy-1+b, cz-1+c).

    k_patch: (m, 2, 2, 2) conductivities of those eight elements, [cz][cy][cx].
    x_patch: (m, L, 3, 3, 3) values at node + (dx-1, dy-1, dz-1), [dz][dy][dx].
    absolute: use |K| entries and |x| (the bound sum_b |A_vb| |x_b| for
    rounding tolerances).  Returns (m, L).  Plain loops, for sampled nodes of
    grids too large to assemble."""
    K = element_matrix()
    if absolute:
        K = np.abs(K)
        x_patch = np.abs(x_patch)
    k_patch = np.asarray(k_patch, dtype=np.float64)
    x_patch = np.asarray(x_patch, dtype=np.float64)
    m, L = x_patch.shape[0], x_patch.shape[1]
    out = np.zeros((m, L))
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                lv = (1 - cx) + 2 * (1 - cy) + 4 * (1 - cz)
                ke = k_patch[:, cz, cy, cx][:, None]
                for l in range(8):
                    a, b, c = l & 1, (l >> 1) & 1, (l >> 2) & 1
                    out += ke * K[lv, l] * x_patch[:, :, cz + c, cy + b, cx + a]
    return out


def macro_loads(k: np.ndarray) -> np.ndarray:
    """(3, n, n, n) right-hand sides b^i."""
    k = _c(k)
    n = k.shape[0]
    b = np.empty((3, n, n, n))
    _load().ora_rhs(n, _ptr(k), _ptr(b))
    return b


def cg(A: CSR27, b: np.ndarray, tol: float, max_iter: int = 100000):
    """Plain CG on the zero-mean subspace; returns (x, iterations, true_rel_residual, converged)."""
    b = _c(b).reshape(-1)
    x = np.empty_like(b)
    st = np.zeros(2)
    rc = _load().ora_cg(b.size, _ptr(A.cols), _ptr(A.vals), _ptr(b), float(tol), int(max_iter), _ptr(x), _ptr(st))
    return x.reshape((A.n,) * 3), int(st[0]), float(st[1]), rc == 0


def cg_fixed(A: CSR27, b: np.ndarray, iters: int) -> np.ndarray:
    b = _c(b).reshape(-1)
    x = np.empty_like(b)
    _load().ora_cg_fixed(b.size, _ptr(A.cols), _ptr(A.vals), _ptr(b), int(iters), _ptr(x))
    return x.reshape((A.n,) * 3)


def element_energies(chi: np.ndarray) -> np.ndarray:
    """(6, n, n, n) E_e,c for c in [11,22,33,12,23,13]."""
    chi = _c(chi)
    n = chi.shape[1]
    E = np.empty((6, n, n, n))
    _load().ora_energy(n, _ptr(chi), _ptr(E))
    return E


def kappa_from_energies(k: np.ndarray, E: np.ndarray) -> np.ndarray:
    k = _c(k)
    E = _c(E)
    out = np.zeros(6)
    _load().ora_kappa(k.size, _ptr(k), _ptr(E), _ptr(out))
    return out


def element_sensitivity(rhof, E, w6, k0, kmin, p) -> np.ndarray:
    rhof = _c(rhof)
    E = _c(E)
    w6 = _c(w6)
    out = np.empty_like(rhof)
    _load().ora_sens(rhof.size, _ptr(rhof), _ptr(E), _ptr(w6), float(k0), float(kmin), float(p), _ptr(out))
    return out


def oc_update(rho, s, vstar, move=0.05, eta=0.5, rho_min=1e-3):
    """Returns (rho_new, lambda, bisection_steps)."""
    rho = _c(rho)
    s = _c(s)
    out = np.empty_like(rho)
    steps = np.zeros(1, dtype=np.int32)
    lam = _load().ora_oc_update(rho.size, _ptr(rho), _ptr(s), float(vstar), float(move), float(eta),
                                float(rho_min), _ptr(out), _ptr(steps))
    return out, float(lam), int(steps[0])


# ------------------------------------------------------------- composites

@dataclasses.dataclass
class Params:
    k0: float = 1.0
    kmin: float = 1e-3
    penal: float = 3.0
    rfilter: float = 1.5
    tol: float = 1e-12
    max_iter: int = 200000
    move: float = 0.05
    eta: float = 0.5
    rho_min: float = 1e-3


def homogenize(rho: np.ndarray, prm: Params, with_energies: bool = True) -> Dict[str, object]:
    """Filter -> SIMP -> assemble -> 3 CG solves -> tensor.  Everything FP64."""
    rhof = density_filter(rho, prm.rfilter)
    k = simp(rhof, prm.k0, prm.kmin, prm.penal)
    A = assemble(k)
    b = macro_loads(k)
    n = rho.shape[0]
    chi = np.empty((3, n, n, n))
    iters, res, conv = [], [], []
    for i in range(3):
        chi[i], it, rr, ok = cg(A, b[i], prm.tol, prm.max_iter)
        iters.append(it)
        res.append(rr)
        conv.append(ok)
    E = element_energies(chi)
    kappa = kappa_from_energies(k, E)
    out = dict(rhof=rhof, k=k, b=b, chi=chi, kappa=kappa, iters=iters, residuals=res, converged=conv)
    if with_energies:
        out["E"] = E
    out["A"] = A
    return out


OBJ_MSE = 0
OBJ_REL = 1
OBJ_L1 = 2


def objective(kappa: np.ndarray, target: np.ndarray, kind: int = OBJ_MSE):
    """The objective over the six tensor components and dg/dkappa.

    OBJ_MSE: sum_c (kappa_c - target_c)^2 (Sec. 4.4, MSE objective).
    OBJ_REL: sum_c (kappa_c / target_c - 1)^2 (the relative objective of
    Sec. 4.4; every target component must be nonzero).
    OBJ_L1:  sum_c |kappa_c - target_c| (the l1 objective of Sec. 4.4), with
    d|a|/da taken as 0 at a = 0 as the paper states."""
    kap = np.asarray(kappa, dtype=np.float64)
    tgt = np.asarray(target, dtype=np.float64)
    if kind == OBJ_MSE:
        d = kap - tgt
        return float(np.sum(d * d)), 2.0 * d
    if kind == OBJ_REL:
        if np.any(tgt == 0.0):
            raise ValueError("the relative objective needs every target component nonzero")
        d = kap / tgt - 1.0
        return float(np.sum(d * d)), 2.0 * d / tgt
    if kind == OBJ_L1:
        d = kap - tgt
        return float(np.sum(np.abs(d))), np.sign(d)
    raise ValueError(f"unknown objective {kind}")


INIT_KINDS = ("P", "D", "G", "IWP", "ball")


def init_level(kind: str, n: int) -> np.ndarray:
    """Level-set values at element centres, X = 2 pi (i + 1/2) / n, shape
    (n, n, n) indexed [k][j][i]: the standard trigonometric approximations of
    the Schwarz P and D surfaces, the gyroid and Schoen's IWP surface (the
    classic initializations of Sec. 4.3), or minus the distance from the cell
    centre for the centre ball."""
    c = (np.arange(n) + 0.5)
    Z, Y, X = np.meshgrid(2 * np.pi * c / n, 2 * np.pi * c / n, 2 * np.pi * c / n, indexing="ij")
    if kind == "P":
        return np.cos(X) + np.cos(Y) + np.cos(Z)
    if kind == "D":
        return np.cos(X) * np.cos(Y) * np.cos(Z) - np.sin(X) * np.sin(Y) * np.sin(Z)
    if kind == "G":
        return np.sin(X) * np.cos(Y) + np.sin(Y) * np.cos(Z) + np.sin(Z) * np.cos(X)
    if kind == "IWP":
        return (2 * (np.cos(X) * np.cos(Y) + np.cos(Y) * np.cos(Z) + np.cos(Z) * np.cos(X))
                - (np.cos(2 * X) + np.cos(2 * Y) + np.cos(2 * Z)))
    if kind == "ball":
        zc, yc, xc = np.meshgrid(c - n / 2, c - n / 2, c - n / 2, indexing="ij")
        return -np.sqrt(xc * xc + yc * yc + zc * zc)
    raise ValueError(kind)


def init_density(kind: str, n: int, vf: float) -> np.ndarray:
    """Solid (1) on the round(vf n^3) elements with the smallest level-set
    values (stable order of the flat index for ties), void (0) elsewhere."""
    phi = init_level(kind, n).reshape(-1)
    order = np.argsort(phi, kind="stable")
    rho = np.zeros(n ** 3)
    rho[order[:int(round(vf * n ** 3))]] = 1.0
    return rho.reshape(n, n, n)


def symmetrize_central(field: np.ndarray) -> np.ndarray:
    """Central symmetry (Sec. 4.3, customized microstructures): each element
    and its image under the point reflection through the cell centre,
    (i, j, k) -> (n-1-i, n-1-j, n-1-k), both take the mean of their two values."""
    f = np.asarray(field, dtype=np.float64)
    return 0.5 * (f + f[::-1, ::-1, ::-1])


def sensitivities(h: Dict[str, object], w6: np.ndarray, prm: Params) -> np.ndarray:
    """dg/drho = F^T [ N^-3 p rho~^(p-1) (k0-kmin) sum_c w_c E_e,c ]."""
    st = element_sensitivity(h["rhof"], h["E"], w6, prm.k0, prm.kmin, prm.penal)
    return density_filter_T(st, prm.rfilter)


# ----------------------------------------------------------------- governor

@dataclasses.dataclass
class GovernorParams:
    bound: float = 1e-4        # tolerable objective value (Sec. 4.2: 1e-4)
    dg_small: float = 1e-6     # |g^(I-1) - g^I| below this is "little progress" (1e-2 * bound)
    dv_small: float = 1e-3     # |V - V*| below this is "at the boundary"
    decay: float = 0.8         # Df <- 0.8 Df after each reduction
    rebound: float = 0.3       # V* <- V* + 0.3 gap Df after a stall
    patience: int = 5          # stalls needed before a rebound
    g_tol: float = 1e-6        # termination: |dg| below this ...
    stall_iters: int = 3       # ... for this many consecutive iterations
    rho_min: float = 1e-3


@dataclasses.dataclass(frozen=True)
class GovernorState:
    """What Algorithm 1 carries from one OC iteration to the next, in the
    paper's notation: V*, the decrease factor Df, the stall counter `count`,
    the last measured `gap`, g^[I-1]; plus the count of consecutive small
    objective changes used by the termination test."""
    vstar: float
    df: float = 1.0
    count: int = 0
    gap: float = 0.0
    g_prev: float = 1.0      # g^[0] = 1
    small_steps: int = 0


def governor_transition(st: GovernorState, g: float, low_bound: float, volume: float,
                        gp: GovernorParams) -> GovernorState:
    """Algorithm 1 on one OC iteration's observations: the objective g^[I],
    lowBound = mean(rho~^p) and the volume V = mean(rho).  Returns the next
    state; V* is clamped to [rho_min, 1] at the end."""
    vstar, df, gap = st.vstar, st.df, st.gap
    # Reduce V* only when the objective is tolerable: V* loses the fraction
    # Df of its distance to lowBound, and Df decays for the next reduction.
    if g <= gp.bound:
        gap = vstar - low_bound
        vstar, df = vstar - gap * df, gp.decay * df
    # Little progress, still too large an objective, volume on the bound:
    # all three (judged after the reduction) make a stalled iteration.
    tests = (abs(st.g_prev - g) < gp.dg_small, g > gp.bound, abs(volume - vstar) < gp.dv_small)
    count = st.count + 1 if all(tests) else 0
    # Rebound V* once the stalls reach the patience.
    if count >= gp.patience:
        vstar, count = vstar + gp.rebound * gap * df, 0
    vstar = min(1.0, max(gp.rho_min, vstar))
    small = st.small_steps + 1 if abs(st.g_prev - g) < gp.g_tol else 0
    return GovernorState(vstar, df, count, gap, g, small)


class Governor:
    """Adaptive volume bound V*(rho) (Sec. 2.3, model 3; Algorithm 1): holds a
    GovernorState and advances it once per OC iteration.

    The state starts at Df = 1, count = 0, g^[0] = 1, gap = 0; V*_0 is the
    configured volume fraction (vstar0 = 1 reproduces the algorithm's own
    initial value)."""

    def __init__(self, vstar0: float, gp: Optional[GovernorParams] = None):
        self.gp = gp or GovernorParams()
        self.state = GovernorState(float(vstar0))

    def update(self, g: float, low_bound: float, volume: float) -> float:
        self.state = governor_transition(self.state, g, low_bound, volume, self.gp)
        return self.state.vstar

    vstar = property(lambda self: self.state.vstar)
    df = property(lambda self: self.state.df)
    count = property(lambda self: self.state.count)
    gap = property(lambda self: self.state.gap)
    g_prev = property(lambda self: self.state.g_prev)
    small_steps = property(lambda self: self.state.small_steps)

    @property
    def converged(self) -> bool:
        """Termination: |g^[I-1] - g^[I]| < g_tol for stall_iters consecutive iterations."""
        return self.small_steps >= self.gp.stall_iters


# --------------------------------------------------------------- OC driver

@dataclasses.dataclass
class IterRecord:
    g: float
    kappa: np.ndarray
    volume: float
    low_bound: float
    vstar: float
    lam: float
    pcg_iters: List[int]


def oc_iteration(rho: np.ndarray, target: np.ndarray, gov: Governor, prm: Params, objective_kind: int = OBJ_MSE,
                 central_symmetry: bool = False):
    """One OC iteration in the order: homogenize -> objective -> sensitivities
    -> governor(g, mean(rho~^p), mean(rho)) -> OC update with the new V*.
    With central symmetry the densities are averaged over symmetric element
    pairs before the evaluation and the sensitivities after it."""
    if central_symmetry:
        rho = symmetrize_central(rho)
    h = homogenize(rho, prm)
    g, w = objective(h["kappa"], target, objective_kind)
    s = sensitivities(h, w, prm)
    if central_symmetry:
        s = symmetrize_central(s)
    low = float(np.mean(np.power(h["rhof"], prm.penal)))
    vol = float(np.mean(rho))
    vstar = gov.update(g, low, vol)
    rho_new, lam, _ = oc_update(rho, s, vstar, prm.move, prm.eta, prm.rho_min)
    rec = IterRecord(g, h["kappa"].copy(), vol, low, vstar, lam, list(h["iters"]))
    return rho_new, rec, h, s


def run(rho0: np.ndarray, target: Sequence[float], vstar0: float, iters: int, prm: Params,
        gp: Optional[GovernorParams] = None):
    gov = Governor(vstar0, gp)
    rho = np.array(rho0, dtype=np.float64)
    log = []
    for _ in range(iters):
        rho, rec, _, _ = oc_iteration(rho, np.asarray(target, dtype=np.float64), gov, prm)
        log.append(rec)
    return rho, log
