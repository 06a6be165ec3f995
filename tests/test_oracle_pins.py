"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each checks a closed form, an
invariant, a hand derivation or a brute-force computation that a mistake in
the oracle (dropped term, wrong sign or index, transposed operand) breaks.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PRM = O.Params(tol=1e-13)


def popcount(x):
    return bin(x).count("1")


# ------------------------------------------------------------ element matrix

def test_element_matrix_hand_pattern():
    """Hand derivation: 12 K = 4 on the diagonal, 0 between edge-adjacent
    vertices (one coordinate differs), -1 for face and body diagonals."""
    K = O.element_matrix()
    hand = np.zeros((8, 8))
    for l in range(8):
        for m in range(8):
            d = popcount(l ^ m)
            hand[l, m] = {0: 4.0, 1: 0.0, 2: -1.0, 3: -1.0}[d] / 12.0
    np.testing.assert_allclose(K, hand, rtol=0, atol=1e-15)


def test_element_matrix_spectrum():
    ev = np.sort(np.linalg.eigvalsh(O.element_matrix())) * 12.0
    np.testing.assert_allclose(ev, [0, 2, 4, 4, 4, 6, 6, 6], atol=1e-13)


def test_element_matrix_linear_fields():
    """A unit gradient along axis i has energy delta_ij against axis j
    (|grad| = 1 over a unit voxel), and K X gives the +-1/4 load template."""
    K = O.element_matrix()
    X = np.array([[(l >> i) & 1 for i in range(3)] for l in range(8)], dtype=float)
    np.testing.assert_allclose(X.T @ K @ X, np.eye(3), atol=1e-15)
    np.testing.assert_allclose(K @ X, (2 * X - 1) / 4.0, atol=1e-15)


# ------------------------------------------------------------------ assembly

@pytest.mark.parametrize("n", [3, 4, 5])
def test_assembly_structure(n):
    k = synth.random_field(n, 7, 0.001, 1.0)
    A = O.assemble(k)
    D = A.dense()
    np.testing.assert_allclose(D, D.T, atol=1e-15)
    np.testing.assert_allclose(D @ np.ones(n ** 3), 0.0, atol=1e-14)
    # stencil from counting shared elements: face neighbours 0, edge-diagonal
    # -(k_a + k_b)/12 over the two shared elements, corners -k/12, centre sum k/3
    kk = k  # indexed [z][y][x]
    for v in [0, n ** 3 // 2, n ** 3 - 1]:
        vi, vj, vk = v % n, (v // n) % n, v // (n * n)
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            u = ((vi + dx) % n) + n * (((vj + dy) % n) + n * ((vk + dz) % n))
            shared = []
            for a, b, c in itertools.product((0, 1), repeat=3):
                ex, ey, ez = vi - 1 + a, vj - 1 + b, vk - 1 + c   # incident element origin
                # element spans [ex, ex+1]; it contains the neighbour iff ex <= vi+dx <= ex+1
                if ex <= vi + dx <= ex + 1 and ey <= vj + dy <= ey + 1 and ez <= vk + dz <= ez + 1:
                    shared.append(kk[ez % n, ey % n, ex % n])
            nz = abs(dx) + abs(dy) + abs(dz)
            coef = {0: 4.0, 1: 0.0, 2: -1.0, 3: -1.0}[nz] / 12.0
            assert D[v, u] == pytest.approx(coef * sum(shared), abs=1e-15)


def test_macro_loads_sum_to_zero_and_uniform():
    n = 5
    k = synth.random_field(n, 3, 0.001, 1.0)
    b = O.macro_loads(k)
    assert np.abs(b.reshape(3, -1).sum(axis=1)).max() < 1e-13
    bu = O.macro_loads(np.full((n, n, n), 0.7))
    assert np.abs(bu).max() < 1e-15


def test_macro_load_single_element():
    """One element with k=1, others 0: its 8 vertices get (2 l_i - 1)/4."""
    n = 4
    k = np.zeros((n, n, n))
    k[1, 2, 3] = 1.0  # element origin x=3, y=2, z=1
    b = O.macro_loads(k)
    for l in range(8):
        a, bb, c = l & 1, (l >> 1) & 1, (l >> 2) & 1
        x, y, z = (3 + a) % n, (2 + bb) % n, (1 + c) % n
        for i, bit in enumerate((a, bb, c)):
            assert b[i, z, y, x] == pytest.approx((2 * bit - 1) / 4.0, abs=1e-15)
    assert np.count_nonzero(np.abs(b) > 1e-15) == 24


# --------------------------------------------------------------------- solve

def test_dense_direct_solve_4cube():
    """CG on the zero-mean subspace equals a dense direct solve with node 0
    pinned, then mean-removed (4^3 grid)."""
    n = 4
    k = O.simp(synth.random_field(n, 11, 0.0, 1.0), 1.0, 1e-3, 3.0)
    A = O.assemble(k)
    D = A.dense()
    b = O.macro_loads(k).reshape(3, -1)
    for i in range(3):
        x_cg, it, res, ok = O.cg(A, b[i], 1e-14)
        assert ok and res < 1e-12
        Dp = D[1:, 1:]
        xd = np.zeros(n ** 3)
        xd[1:] = np.linalg.solve(Dp, b[i][1:])
        xd -= xd.mean()
        np.testing.assert_allclose(x_cg.reshape(-1), xd, atol=1e-10 * np.abs(xd).max())


# -------------------------------------------------------------- closed forms

@pytest.mark.parametrize("c", [0.0, 0.3, 1.0])
def test_uniform_cell(c):
    n = 6
    h = O.homogenize(np.full((n, n, n), c), PRM)
    kc = 1e-3 + c ** 3 * (1.0 - 1e-3)
    np.testing.assert_allclose(h["kappa"], [kc, kc, kc, 0, 0, 0], atol=1e-15)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate(axis):
    """Density varying along one axis only: along the layers the tensor is the
    arithmetic mean of k, across them the harmonic mean; off-diagonals vanish.
    (Exact for the discrete model: the problem reduces to 1D linear FE.)"""
    n = 8
    prof = synth.rng(5).uniform(0.05, 1.0, size=n)
    shape = [1, 1, 1]
    shape[axis] = n
    rho = np.broadcast_to(prof.reshape(shape), (n, n, n)).copy()
    h = O.homogenize(rho, PRM)
    k = h["k"]
    layers = np.moveaxis(k, axis, 0)[:, 0, 0]
    ar, hm = layers.mean(), 1.0 / np.mean(1.0 / layers)
    # numpy axis 0 is z (component 2), axis 2 is x (component 0)
    comp = 2 - axis
    diag = [ar, ar, ar]
    diag[comp] = hm
    np.testing.assert_allclose(h["kappa"][:3], diag, rtol=1e-11)
    np.testing.assert_allclose(h["kappa"][3:], 0.0, atol=1e-13)


def checkerboard(n):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return ((x + y + z) % 2 == 0).astype(float)


def test_checkerboard_filter_off():
    n = 6
    prm = O.Params(tol=1e-13, rfilter=0.0)
    h = O.homogenize(checkerboard(n), prm)
    kc = 0.5 * (1.0 + 1e-3)
    assert np.abs(h["b"]).max() < 1e-15
    np.testing.assert_allclose(h["kappa"], [kc, kc, kc, 0, 0, 0], atol=1e-15)


def test_checkerboard_filter_on():
    """The filter's symbol at the Nyquist wave is 0.2^3: rho~ = 0.5 +- 0.004."""
    n = 6
    h = O.homogenize(checkerboard(n), PRM)
    cb = checkerboard(n)
    np.testing.assert_allclose(h["rhof"], 0.5 + 0.5 * 0.008 * (2 * cb - 1), atol=1e-15)
    km = h["k"].mean()
    np.testing.assert_allclose(h["kappa"], [km, km, km, 0, 0, 0], atol=1e-14)


def kappa_matrix(k6):
    a, b, c, d, e, f = k6
    return np.array([[a, d, f], [d, b, e], [f, e, c]])


def test_bounds_symmetry_spd():
    n = 6
    rho = synth.random_field(n, 21, 0.0, 1.0)
    h = O.homogenize(rho, PRM)
    K = kappa_matrix(h["kappa"])
    assert np.all(np.linalg.eigvalsh(K) > 0)
    k = h["k"]
    voigt, reuss = k.mean(), 1.0 / np.mean(1.0 / k)
    g = synth.rng(1)
    for _ in range(20):
        e = g.standard_normal(3)
        e /= np.linalg.norm(e)
        val = e @ K @ e
        assert reuss * (1 - 1e-12) <= val <= voigt * (1 + 1e-12)
    # symmetric energies: E_12 computed from (1,2) equals the (2,1) pairing by construction of kappa
    # short formula at convergence: kappa_ij = mean(k) delta_ij - N^-3 chi^i . b^j
    chi, b = h["chi"].reshape(3, -1), h["b"].reshape(3, -1)
    b = b - b.mean(axis=1, keepdims=True)
    short = k.mean() * np.eye(3) - chi @ b.T / n ** 3
    np.testing.assert_allclose(short, K, atol=1e-11)
    np.testing.assert_allclose(short, short.T, atol=1e-11)


def test_permutation_reflection_shift():
    n = 5
    rho = synth.random_field(n, 31, 0.0, 1.0)
    K = kappa_matrix(O.homogenize(rho, PRM)["kappa"])
    # cyclic shift leaves kappa unchanged
    Ks = kappa_matrix(O.homogenize(np.roll(rho, (1, 2, 3), axis=(0, 1, 2)), PRM)["kappa"])
    np.testing.assert_allclose(Ks, K, atol=1e-12)
    # swapping numpy axes 1 and 2 swaps physical x and y
    Kp = kappa_matrix(O.homogenize(np.ascontiguousarray(rho.transpose(0, 2, 1)), PRM)["kappa"])
    P = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1.0]])
    np.testing.assert_allclose(Kp, P @ K @ P.T, atol=1e-12)
    # reflection x -> -x flips the sign of k12 and k13
    Kr = kappa_matrix(O.homogenize(np.ascontiguousarray(rho[:, :, ::-1]), PRM)["kappa"])
    Rm = np.diag([-1.0, 1.0, 1.0])
    np.testing.assert_allclose(Kr, Rm @ K @ Rm, atol=1e-12)


# --------------------------------------------------------------- sensitivity

def objective_of(rho, target, prm):
    h = O.homogenize(rho, prm, with_energies=False)
    return O.objective(h["kappa"], target)[0]


def test_sensitivity_finite_differences():
    n = 4
    prm = O.Params(tol=1e-14)
    rho = synth.random_field(n, 41, 0.2, 0.8)
    target = np.array([0.3, 0.2, 0.1, 0.02, 0.01, 0.015])
    h = O.homogenize(rho, prm)
    g, w = O.objective(h["kappa"], target)
    s = O.sensitivities(h, w, prm)
    delta = 1e-4
    idx = synth.rng(2).choice(n ** 3, size=6, replace=False)
    for e in idx:
        rp = rho.copy().reshape(-1)
        rm = rho.copy().reshape(-1)
        rp[e] += delta
        rm[e] -= delta
        fd = (objective_of(rp.reshape(rho.shape), target, prm) - objective_of(rm.reshape(rho.shape), target, prm)) / (2 * delta)
        assert abs(fd - s.reshape(-1)[e]) <= 1e-6 * np.abs(s).max()


def test_sensitivity_permutation():
    n = 4
    rho = synth.random_field(n, 43, 0.2, 0.8)
    target = np.array([0.2, 0.2, 0.1, 0.0, 0.0, 0.0])  # symmetric in x <-> y
    h = O.homogenize(rho, PRM)
    s = O.sensitivities(h, O.objective(h["kappa"], target)[1], PRM)
    rt = np.ascontiguousarray(rho.transpose(0, 2, 1))
    ht = O.homogenize(rt, PRM)
    st = O.sensitivities(ht, O.objective(ht["kappa"], target)[1], PRM)
    np.testing.assert_allclose(st, s.transpose(0, 2, 1), atol=1e-12 * np.abs(s).max())


# -------------------------------------------------------------------- filter

@pytest.mark.parametrize("r,w", [(1.5, [0.2, 0.6, 0.2]), (2.5, [0.5 / 6.5, 1.5 / 6.5, 2.5 / 6.5, 1.5 / 6.5, 0.5 / 6.5])])
def test_filter_fourier_symbol(r, w):
    """A plane wave is an eigenvector of the periodic filter with eigenvalue
    prod_a sum_d w_d cos(2 pi m_a d / N)."""
    n = 8
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    R = len(w) // 2
    for m in [(0, 0, 0), (1, 0, 0), (1, 2, 3), (4, 4, 4), (3, 0, 1)]:
        wave = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / n)
        sym = 1.0
        for ma in m:
            sym *= sum(w[d + R] * np.cos(2 * np.pi * ma * d / n) for d in range(-R, R + 1))
        np.testing.assert_allclose(O.density_filter(wave, r), sym * wave, atol=1e-14)


def test_filter_partition_transpose_identity():
    n = 6
    x = synth.random_field(n, 51)
    y = synth.random_field(n, 52)
    np.testing.assert_allclose(O.density_filter(np.ones((n, n, n)), 1.5), 1.0, atol=1e-15)
    assert np.sum(O.density_filter(x, 1.5) * y) == pytest.approx(np.sum(x * O.density_filter_T(y, 1.5)), rel=1e-13)
    assert O.density_filter(x, 1.5).mean() == pytest.approx(x.mean(), rel=1e-14)
    np.testing.assert_allclose(O.density_filter(x, 0.8), x, rtol=4e-16)   # radius below one voxel: identity weights
    np.testing.assert_array_equal(O.density_filter(x, 0.0), x)


# ------------------------------------------------------------------------ OC

def test_oc_closed_form_interior():
    """With move limits that never bind, rho_new = q lam^-eta and the volume
    equation gives lam = (mean(q)/V*)^(1/eta) exactly."""
    n = 5
    g = synth.rng(61)
    rho = g.uniform(0.3, 0.5, size=(n, n, n))
    s = -g.uniform(0.5, 1.5, size=(n, n, n)) / n ** 3
    vstar = 0.4
    eta = 0.5
    q = rho * (np.maximum(0.0, -s) * n ** 3) ** eta
    lam_exact = (q.mean() / vstar) ** (1.0 / eta)
    assert np.all(q / lam_exact ** eta > 1e-3) and np.all(q / lam_exact ** eta < 1.0)
    rho_new, lam, steps = O.oc_update(rho, s, vstar, move=1.0, eta=eta, rho_min=1e-3)
    assert lam == pytest.approx(lam_exact, rel=1e-12)
    assert rho_new.mean() == pytest.approx(vstar, rel=1e-12)
    np.testing.assert_allclose(rho_new, q / lam_exact ** eta, rtol=1e-12)


def test_oc_bounds_and_volume():
    n = 6
    g = synth.rng(62)
    rho = g.uniform(0.0, 1.0, size=(n, n, n)).clip(1e-3, 1)
    s = g.standard_normal((n, n, n)) * 1e-4   # mixed signs
    for vstar in [0.3, 0.5, 0.6]:
        rn, lam, _ = O.oc_update(rho, s, vstar)
        lo = np.maximum(1e-3, rho - 0.05)
        hi = np.minimum(1.0, rho + 0.05)
        assert np.all(rn >= lo - 1e-15) and np.all(rn <= hi + 1e-15)
        hi_reach = np.where(s < 0, hi, lo)
        if lo.mean() < vstar < hi_reach.mean():
            assert rn.mean() == pytest.approx(vstar, rel=1e-12)


def test_oc_positive_sensitivities_go_to_lower_limit():
    n = 4
    rho = np.full((n, n, n), 0.5)
    s = np.full((n, n, n), 1e-3)
    rn, _, _ = O.oc_update(rho, s, 0.5)
    np.testing.assert_allclose(rn, 0.45, atol=1e-15)


# ------------------------------------------------------------------ governor

def test_governor_hand_trace():
    """Hand-traced run of Algorithm 1 with bound 1e-4 and V*_0 = 0.5."""
    gov = O.Governor(0.5)
    seq = [  # (g, lowBound, V) -> expected V*, count, Df
        ((5e-5, 0.30, 0.50), 0.30, 0, 0.8),     # reduce: gap 0.2
        ((2e-4, 0.25, 0.30), 0.30, 0, 0.8),     # progress 1.5e-4: not small
        ((2e-4, 0.25, 0.30), 0.30, 1, 0.8),     # stalled at the bound
        ((2e-4, 0.25, 0.30), 0.30, 2, 0.8),
        ((2e-4, 0.25, 0.30), 0.30, 3, 0.8),
        ((2e-4, 0.25, 0.30), 0.30, 4, 0.8),
        ((2e-4, 0.25, 0.30), 0.348, 0, 0.8),    # fifth stall: rebound by 0.3*0.2*0.8
        ((2e-4, 0.25, 0.30), 0.348, 0, 0.8),    # |V - V*| = 0.048: not at the bound
        ((9e-5, 0.20, 0.348), 0.2296, 0, 0.64),  # reduce: gap 0.148, Df 0.8 -> 0.64
    ]
    for (g, low, vol), vs, count, df in seq:
        assert gov.update(g, low, vol) == pytest.approx(vs, abs=1e-15)
        assert gov.count == count
        assert gov.df == pytest.approx(df, abs=1e-15)


def test_governor_clamp_and_termination():
    gov = O.Governor(0.002)
    assert gov.update(1e-5, 0.0, 0.002) == 1e-3   # V* would reach 0: clamped to rho_min
    gov = O.Governor(0.3)
    flags = []
    for g in [1e-3, 1e-3, 1e-3, 1e-3, 5e-3]:
        gov.update(g, 0.1, 0.3)
        flags.append(gov.converged)
    assert flags == [False, False, False, True, False]


def test_governor_rebound_uses_decayed_factor_and_resets_count():
    """Algorithm 1 with patience 2, all stall tests passing: the second stall
    raises V* by 0.3 * gap * Df with the Df left by the last reduction
    (0.8 after one), and the count starts again."""
    gp = O.GovernorParams(bound=1e-4, dg_small=1.0, dv_small=1.0, patience=2)
    gov = O.Governor(0.6, gp)
    assert gov.update(1e-5, 0.2, 0.6) == pytest.approx(0.2, abs=1e-15)    # reduce: gap 0.4, Df 1 -> 0.8
    assert gov.count == 0
    assert gov.update(1e-3, 0.1, 0.2) == pytest.approx(0.2, abs=1e-15)    # first stall
    assert gov.count == 1
    assert gov.update(1e-3, 0.1, 0.2) == pytest.approx(0.296, abs=1e-15)  # rebound 0.3 * 0.4 * 0.8
    assert (gov.count, gov.gap, gov.df) == (0, pytest.approx(0.4), pytest.approx(0.8))


def _checkerboard(n, a, d):
    i = np.arange(n)
    par = (i[:, None, None] + i[None, :, None] + i[None, None, :]) % 2
    return a + d * (1 - 2 * par)


def test_oc_iteration_low_bound_is_mean_of_filtered_density_power():
    """The composition of one OC iteration (reading R15/R17): the governor's
    lowBound is mean(rho~^p) over elements, with rho~ the filtered density,
    and the OC update of the same iteration enforces the V* it produced.

    Element-parity checkerboard rho = a + d (-1)^(i+j+k): the r = 1.5 filter
    has the 1-D symbol 0.6 - 0.4 = 0.2 on the alternating mode, so
    rho~ = a + 0.008 d (-1)^(i+j+k) and mean(rho~^3) = a^3 + 3 a (0.008 d)^2.
    With the bound so large that the first iteration reduces and Df = 1, V*
    lands exactly on lowBound.  mean(rho^3) (no filter) gives a^3 + 3 a d^2,
    mean(k_e) gives kmin + mean(rho~^3)(k0 - kmin): both differ here.  The
    target exceeds every reachable conductivity, so every sensitivity is
    negative and, with move 1, V* is reachable: mean(rho_new) = V*."""
    n, a, d = 6, 0.5, 0.4
    rho = _checkerboard(n, a, d)
    prm = O.Params(k0=2.0, kmin=0.1, tol=1e-12, move=1.0)
    gov = O.Governor(0.9, O.GovernorParams(bound=1e9))
    rho_new, rec, h, s = O.oc_iteration(rho, np.array([10.0, 10.0, 10.0, 0.0, 0.0, 0.0]), gov, prm)
    low = a ** 3 + 3 * a * (0.008 * d) ** 2
    assert rec.low_bound == pytest.approx(low, rel=1e-13)
    assert rec.vstar == pytest.approx(low, rel=1e-13)
    assert abs(rec.vstar - (a ** 3 + 3 * a * d ** 2)) > 0.1
    assert abs(rec.vstar - (0.1 + low * 1.9)) > 0.1
    assert rec.volume == pytest.approx(a, rel=1e-15)
    assert np.all(s < 0)
    assert np.mean(rho_new) == pytest.approx(low, rel=1e-12)
    assert gov.df == pytest.approx(0.8, abs=1e-15)


# -------------------------------------------------------------- golden data

def test_gallery_positive_definite_count():
    d = json.load(open(os.path.join(GOLDEN, "gallery_sets.json")))
    count = 0
    for a, b, c in itertools.product(d["k12"], d["k23"], d["k13"]):
        K = kappa_matrix([*d["diagonal"], a, b, c])
        count += bool(np.all(np.linalg.eigvalsh(K) > 0))
    assert len(d["k12"]) * len(d["k23"]) * len(d["k13"]) == d["combinations"]
    assert count == d["positive_definite"]


def test_oracle_defaults_match_paper_parameters():
    d = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    p = O.Params()
    gp = O.GovernorParams()
    assert (p.penal, p.rfilter, p.move, p.eta, p.rho_min, p.k0) == (
        d["penal"], d["filter_radius"], d["oc_move"], d["oc_damping"], d["rho_min"], d["k0"])
    assert (gp.decay, gp.rebound, gp.patience, gp.bound) == (
        d["governor_decay"], d["governor_rebound"], d["governor_patience"], d["tolerable_error"])


# ------------------------------------------- objective variants, symmetry

TGT6 = np.array([0.3, 0.2, 0.1, 0.05, 0.05, 0.05])


def _fd_grad(f, x, h=1e-7):
    g = np.zeros_like(x)
    for q in range(x.size):
        e = np.zeros_like(x)
        e[q] = h
        g[q] = (f(x + e) - f(x - e)) / (2 * h)
    return g


def test_relative_objective_closed_form_and_gradient():
    """kappa = target (1 + delta) gives g = sum delta^2 and dg/dkappa = 2 delta / target."""
    delta = np.array([0.1, -0.2, 0.05, 0.3, -0.1, 0.0])
    kap = TGT6 * (1.0 + delta)
    g, w = O.objective(kap, TGT6, O.OBJ_REL)
    assert g == pytest.approx(np.sum(delta ** 2), rel=1e-13)
    np.testing.assert_allclose(w, 2.0 * delta / TGT6, rtol=1e-12, atol=1e-14)
    fd = _fd_grad(lambda k: O.objective(k, TGT6, O.OBJ_REL)[0], kap)
    np.testing.assert_allclose(w, fd, rtol=1e-6, atol=1e-7)
    with pytest.raises(ValueError):
        O.objective(kap, np.array([0.3, 0.2, 0.1, 0.0, 0.05, 0.05]), O.OBJ_REL)


def test_l1_objective_value_gradient_and_kink_convention():
    d = np.array([0.02, -0.01, 0.0, 0.03, -0.04, 0.005])
    kap = TGT6 + d
    g, w = O.objective(kap, TGT6, O.OBJ_L1)
    assert g == pytest.approx(np.sum(np.abs(d)), rel=1e-13)
    np.testing.assert_array_equal(w, [1.0, -1.0, 0.0, 1.0, -1.0, 1.0])  # d|a|/da = 0 at a = 0
    away = kap + np.array([0, 0, 0.001, 0, 0, 0])
    fd = _fd_grad(lambda k: O.objective(k, TGT6, O.OBJ_L1)[0], away, 1e-6)
    np.testing.assert_allclose(O.objective(away, TGT6, O.OBJ_L1)[1], fd, atol=1e-8)
    # MSE reduces to the six-term squared error
    g2, w2 = O.objective(kap, TGT6, O.OBJ_MSE)
    assert g2 == pytest.approx(np.sum(d * d), rel=1e-13)


def test_central_pairing_is_the_reversed_flat_index():
    """The point reflection (i,j,k) -> (n-1-i, n-1-j, n-1-k) maps flat index e
    to n^3 - 1 - e; averaging is idempotent and keeps the mean."""
    n = 5
    f = synth.random_field(n, 7, 0.0, 1.0)
    s = O.symmetrize_central(f)
    flat = s.reshape(-1)
    np.testing.assert_array_equal(flat, flat[::-1])
    i, j, k = 1, 3, 4
    assert s[k, j, i] == 0.5 * (f[k, j, i] + f[n - 1 - k, n - 1 - j, n - 1 - i])
    np.testing.assert_array_equal(O.symmetrize_central(s), s)
    assert s.mean() == pytest.approx(f.mean(), rel=1e-15)


def test_sensitivities_of_a_centrally_symmetric_design_are_symmetric():
    """kappa is invariant under the point reflection (R = -I maps kappa to
    R kappa R^T = kappa), so a design equal to its reflection has a reflected-
    symmetric gradient, for any objective of kappa; a generic design does not."""
    n = 6
    prm = O.Params(tol=1e-13)
    for sym in (True, False):
        rho = synth.random_field(n, 11, 0.1, 0.9)
        if sym:
            rho = O.symmetrize_central(rho)
        h = O.homogenize(rho, prm)
        for kind in (O.OBJ_MSE, O.OBJ_REL, O.OBJ_L1):
            _, w = O.objective(h["kappa"], TGT6, kind)
            s = O.sensitivities(h, w, prm)
            asym = np.abs(s - s[::-1, ::-1, ::-1]).max() / np.abs(s).max()
            if sym:
                assert asym < 1e-9, (kind, asym)
            else:
                assert asym > 1e-3, (kind, asym)


def test_symmetric_oc_iteration_output_is_exactly_symmetric():
    n = 6
    rho = synth.random_field(n, 12, 0.2, 0.5)
    gov = O.Governor(0.35)
    rho_new, rec, _, s = O.oc_iteration(rho, TGT6, gov, O.Params(tol=1e-12), O.OBJ_REL, central_symmetry=True)
    flat = rho_new.reshape(-1)
    np.testing.assert_array_equal(flat, flat[::-1])
    np.testing.assert_array_equal(s.reshape(-1), s.reshape(-1)[::-1])


def patches(k, x, nodes):
    """Neighbourhoods of the given nodes (i, j, kz) for oracle.apply_at, with
    periodic wrap: k of the eight incident elements, x of the 27 nodes."""
    n = k.shape[0]
    kp = np.empty((len(nodes), 2, 2, 2))
    xp = np.empty((len(nodes), x.shape[0], 3, 3, 3))
    for q, (i, j, kz) in enumerate(nodes):
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    kp[q, cz, cy, cx] = k[(kz + cz - 1) % n, (j + cy - 1) % n, (i + cx - 1) % n]
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    xp[q, :, dz, dy, dx] = x[:, (kz + dz - 1) % n, (j + dy - 1) % n, (i + dx - 1) % n]
    return kp, xp


@pytest.mark.parametrize("n", [3, 5, 6])
def test_apply_at_equals_assembled_operator(n):
    """The node-by-node operator equals the assembled CSR operator at every
    node (periodic wrap included), and its absolute form bounds it."""
    g = synth.rng(300 + n)
    k = g.uniform(1e-3, 1.0, size=(n, n, n))
    x = g.standard_normal((2, n, n, n))
    A = O.assemble(k)
    nodes = [(i, j, kz) for kz in range(n) for j in range(n) for i in range(n)]
    kp, xp = patches(k, x, nodes)
    got = O.apply_at(kp, xp)
    for l in range(2):
        ref = A.matvec(x[l]).reshape(-1)
        np.testing.assert_allclose(got[:, l], ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    bound = O.apply_at(kp, xp, absolute=True)
    assert np.all(np.abs(got) <= bound * (1 + 1e-12))
