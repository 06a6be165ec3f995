"""Seeded synthetic inputs shared by the test oracle and the HIP path.

This module draws random numbers and shapes them into design densities and
target tensors; it contains none of the homogenization method's arithmetic
(no filter, no SIMP law, no stiffness, no solver).  Both sides receive the
same float64 arrays from here.

Layout convention: a grid of N x N x N voxels is a C-ordered numpy array of
shape (N, N, N) indexed ``[k][j][i]``, i.e. flat index ``i + N*(j + N*k)``
with x fastest.

The paper has no public dataset: its designs start from named TPMS shapes
whose formulas it does not give.  The workloads below stand in for them with
seeded noise of the same sizes and density ranges (Sec. 4, "Optimization
parameters"; Fig. 1 targets).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

# Target tensors are stored as the 6-vector [k11, k22, k33, k12, k23, k13]
# (the paper's tensor-to-vector correspondence, Sec. 2.2).

TARGET_ISO = (0.1, 0.1, 0.1, 0.0, 0.0, 0.0)
TARGET_ORTHO = (0.3, 0.2, 0.1, 0.0, 0.0, 0.0)
TARGET_ANISO = (0.3, 0.2, 0.1, 0.1, 0.05, 0.05)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_noise(n: int, center: float, half_width: float, seed: int) -> np.ndarray:
    """center + U(-half_width, half_width) per voxel, float64, shape (n,n,n)."""
    g = rng(seed)
    return center + g.uniform(-half_width, half_width, size=(n, n, n))


def smoothed_noise(n: int, lo: float, hi: float, seed: int, sigma: float = 1.5) -> np.ndarray:
    """U(0,1) white noise low-passed by a periodic Gaussian of width ``sigma``
    voxels (applied in Fourier space), then mapped affinely onto [lo, hi].

    The smoothing is deliberately not the design filter of the method: it only
    gives the initial density spatial correlation."""
    g = rng(seed)
    w = g.uniform(0.0, 1.0, size=(n, n, n))
    f = np.fft.fftfreq(n)
    k2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    h = np.exp(-2.0 * (np.pi * sigma) ** 2 * k2)
    s = np.real(np.fft.ifftn(np.fft.fftn(w) * h))
    smin, smax = s.min(), s.max()
    if smax - smin <= 0:
        return np.full((n, n, n), 0.5 * (lo + hi))
    return lo + (hi - lo) * (s - smin) / (smax - smin)


def random_spd_target(g: np.random.Generator, lam_lo=0.05, lam_hi=0.35) -> np.ndarray:
    """kappa* = Q diag(lam) Q^T with lam ~ U[lam_lo, lam_hi]^3 and Q a
    Haar-random rotation (QR of a Gaussian matrix, signs fixed, det +1).
    Returned as the 6-vector [11, 22, 33, 12, 23, 13]."""
    lam = g.uniform(lam_lo, lam_hi, size=3)
    a = g.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    m = q @ np.diag(lam) @ q.T
    return np.array([m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[1, 2], m[0, 2]])


@dataclasses.dataclass
class Workload:
    """One design problem: initial density plus the problem constants."""
    name: str
    n: int
    rho0: np.ndarray            # (n,n,n) float64
    target: np.ndarray          # (6,) float64
    vf: float                   # initial volume bound V*_0
    k0: float = 1.0
    kmin: float = 1e-3
    penal: float = 3.0
    rfilter: float = 1.5
    tol: float = 1e-8
    oc_iters: int = 30
    precision: str = "fp64"     # "fp64" or "mixed"


def config1() -> Workload:
    """16^3 cell, FP64, isotropic target, 0.3 +- 0.05 noise, tol 1e-8, 30 OC iterations."""
    return Workload("cell16_iso_fp64", 16, uniform_noise(16, 0.3, 0.05, 101),
                    np.array(TARGET_ISO), 0.3, tol=1e-8, oc_iters=30)


def config2(precision: str = "fp64") -> Workload:
    """64^3 cell, orthotropic target, smoothed noise on [0.2, 0.5], tol 1e-6, 100 OC iterations."""
    return Workload("cell64_ortho", 64, smoothed_noise(64, 0.2, 0.5, 201),
                    np.array(TARGET_ORTHO), 0.35, tol=1e-6, oc_iters=100, precision=precision)


def config3(precision: str = "mixed") -> Workload:
    """128^3 cell, anisotropic target, smoothed noise on [0.15, 0.45], tol 1e-6, 150 OC iterations."""
    return Workload("cell128_aniso", 128, smoothed_noise(128, 0.15, 0.45, 301),
                    np.array(TARGET_ANISO), 0.3, tol=1e-6, oc_iters=150, precision=precision)


def config4(count: int = 64, sizes=(32, 48, 64), seed: int = 401) -> List[Workload]:
    """Batch of designs with uneven N, random SPD targets, vf ~ U[0.2, 0.4]."""
    g = rng(seed)
    out = []
    for d in range(count):
        n = int(g.choice(sizes))
        vf = float(g.uniform(0.2, 0.4))
        tgt = random_spd_target(g)
        sub = int(g.integers(0, 2**31 - 1))
        rho = smoothed_noise(n, vf - 0.15, vf + 0.15, sub)
        out.append(Workload(f"batch{d}_n{n}", n, rho, tgt, vf, tol=1e-6, oc_iters=1))
    return out


def random_field(n: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Plain i.i.d. uniform field (used for operator-level parity inputs)."""
    return rng(seed).uniform(lo, hi, size=(n, n, n))


def random_vectors(n: int, count: int, seed: int) -> np.ndarray:
    """(count, n, n, n) standard-normal vectors (operator-level parity inputs)."""
    return rng(seed).standard_normal((count, n, n, n))


# Anisotropic-space traversal (Sec. 4.2): the diagonal fixed at [0.3, 0.2, 0.1]
# and the off-diagonal entries stepped below the 2x2 principal-minor limits.
# The printed k23 and k13 sets are swapped (their stated limits, sqrt(0.2*0.1)
# and sqrt(0.3*0.1), only fit the other way round); swapped, 61 of the 96
# combinations are positive definite, as the paper states.
GALLERY_DIAG = (0.3, 0.2, 0.1)
GALLERY_K12 = (0.0, 0.05, 0.1, 0.15, 0.2, 0.24)
GALLERY_K23 = (0.0, 0.05, 0.1, 0.14)
GALLERY_K13 = (0.0, 0.05, 0.1, 0.15)


def gallery_targets() -> List[np.ndarray]:
    """The positive-definite targets of the traversal, [k11,k22,k33,k12,k23,k13]."""
    out = []
    for k12 in GALLERY_K12:
        for k23 in GALLERY_K23:
            for k13 in GALLERY_K13:
                t = np.array([*GALLERY_DIAG, k12, k23, k13])
                m = np.array([[t[0], t[3], t[5]], [t[3], t[1], t[4]], [t[5], t[4], t[2]]])
                if np.all(np.linalg.eigvalsh(m) > 0.0):
                    out.append(t)
    return out
