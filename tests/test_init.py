"""Initial densities (Sec. 4.3): the library's host initializer against the
oracle's, and the oracle's level sets against identities of the surfaces
(no GPU needed)."""
import ctypes
import os

import numpy as np
import pytest

import oracle as O


def test_level_set_identities():
    """Half-period shifts and the point reflection act on the published
    surfaces as they must: P changes sign under a half-period shift of all
    three axes, D under a shift of one axis, the gyroid under the point
    reflection; IWP is invariant under axis permutations; the ball is radial."""
    n = 16
    h = n // 2
    P = O.init_level("P", n)
    np.testing.assert_allclose(np.roll(P, (h, h, h), axis=(0, 1, 2)), -P, atol=1e-14)
    D = O.init_level("D", n)
    np.testing.assert_allclose(np.roll(D, h, axis=2), -D, atol=1e-14)
    G = O.init_level("G", n)
    np.testing.assert_allclose(G[::-1, ::-1, ::-1], -G, atol=1e-14)
    I = O.init_level("IWP", n)
    for perm in ((0, 2, 1), (1, 0, 2), (2, 1, 0)):
        np.testing.assert_allclose(np.transpose(I, perm), I, atol=1e-13)
    B = O.init_level("ball", n)
    np.testing.assert_allclose(B, B[::-1, :, :], atol=0)
    assert B[h, h, h] == B.max() and B[0, 0, 0] == B.min()


@pytest.mark.parametrize("kind", O.INIT_KINDS)
def test_oracle_init_counts_and_ball_shape(kind):
    n, vf = 12, 0.3
    rho = O.init_density(kind, n, vf)
    assert set(np.unique(rho)) <= {0.0, 1.0}
    assert rho.sum() == round(vf * n ** 3)
    if kind == "ball":
        d = -O.init_level("ball", n)
        assert d[rho == 0].max() <= d[rho == 1].min()  # the void is a central ball


@pytest.fixture(scope="module")
def L():
    from paper_2405_19991_amd import _native as N
    if not os.path.exists(N.LIBPATH):
        pytest.fail("libopentm_amd.so is not built; run __graft_entry__.build()")
    return N.lib()


@pytest.mark.parametrize("kind", O.INIT_KINDS)
@pytest.mark.parametrize("n,vf", [(8, 0.3), (16, 0.25), (24, 0.5)])
def test_library_initializer_matches_oracle(L, kind, n, vf):
    """Same solid set except where two level-set values tie to rounding at the
    threshold (the two implementations evaluate the sums in their own order)."""
    from paper_2405_19991_amd import init_density
    got = init_density(n, kind, vf)
    ref = O.init_density(kind, n, vf)
    assert got.sum() == ref.sum() == round(vf * n ** 3)
    diff = np.flatnonzero(got.reshape(-1) != ref.reshape(-1))
    if diff.size:
        phi = O.init_level(kind, n).reshape(-1)
        thr = np.sort(phi)[int(round(vf * n ** 3)) - 1]
        assert np.abs(phi[diff] - thr).max() < 1e-12


def test_library_initializer_rejects_bad_arguments(L):
    from paper_2405_19991_amd import _native as N
    out = np.empty(8 ** 3)
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.otm_init_density(8, 5, 0.3, ptr) == N.OTM_EINVAL
    assert L.otm_init_density(8, 0, 0.0, ptr) == N.OTM_EINVAL
    assert L.otm_init_density(2, 0, 0.3, ptr) == N.OTM_EINVAL
    assert L.otm_init_density(8, 0, 0.3, None) == N.OTM_EINVAL
