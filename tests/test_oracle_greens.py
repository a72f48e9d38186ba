"""Pins of the oracle's Green's-function derivatives (Sec. 2).

D .. D_ijk are printed in the paper; D_ijkl is the fourth derivative named in
the text of eq. 7; D'_ijkl is the tensor of eq. 8.  They are pinned here by
finite differences of g(R) = -1/R, by the harmonic property of 1/R (every
trace vanishes), by index symmetry, and by the torque property that defines
D' (it differs from D_ijkl only by terms along R_i, which exert no torque).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc


def g(R):
    return -1.0 / np.sqrt(np.dot(R, R))


def num_grad(f, R, h):
    """Fourth-order central difference of f (scalar or array valued)."""
    out = []
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        out.append((-f(R + 2 * e) + 8 * f(R + e) - 8 * f(R - e) + f(R - 2 * e)) / (12 * h))
    return np.stack(out, axis=0)


RS = [np.array([1.0, 2.0, 2.0]), np.array([-0.7, 0.3, 1.9]), np.array([3.1, -2.2, -0.4])]


@pytest.mark.parametrize("R", RS)
def test_derivatives_match_finite_differences(R):
    D0, D1, D2, D3, D4, _ = orc.greens(R)
    assert D0 == pytest.approx(g(R), rel=1e-15)
    h = 1e-3 * np.linalg.norm(R)
    # each derivative is the finite difference of the one below it
    d1 = num_grad(g, R, h)
    d2 = num_grad(lambda r: orc.greens(r)[1], R, h)
    d3 = num_grad(lambda r: orc.greens(r)[2], R, h)
    d4 = num_grad(lambda r: orc.greens(r)[3], R, h)
    for ana, num in ((D1, d1), (D2, d2), (D3, d3), (D4, d4)):
        scale = np.max(np.abs(ana))
        assert np.max(np.abs(ana - num)) <= 1e-8 * scale


@pytest.mark.parametrize("R", RS)
def test_derivatives_traceless_and_symmetric(R):
    _, D1, D2, D3, D4, _ = orc.greens(R)
    # Laplace's equation: every pair of indices contracts to zero
    assert abs(np.trace(D2)) <= 1e-14 * np.abs(D2).max()
    assert np.max(np.abs(np.einsum("iik->k", D3))) <= 1e-14 * np.abs(D3).max()
    assert np.max(np.abs(np.einsum("iikl->kl", D4))) <= 1e-14 * np.abs(D4).max()
    for T in (D2, D3, D4):
        for perm in itertools.permutations(range(T.ndim)):
            # products of R components in another order round differently
            assert np.max(np.abs(T - np.transpose(T, perm))) <= 1e-15 * np.abs(T).max()


def test_printed_closed_forms_at_a_pythagorean_point():
    # R = (1,2,2), |R| = 3: the printed expressions give exact small rationals
    R = np.array([1.0, 2.0, 2.0])
    D0, D1, D2, D3, D4, D4p = orc.greens(R)
    assert D0 == pytest.approx(-1.0 / 3.0, rel=1e-15)
    np.testing.assert_allclose(D1, R / 27.0, rtol=1e-15)
    # D_xx = -(3*1 - 9)/243 = 6/243; D_yz = -(3*4)/243
    assert D2[0, 0] == pytest.approx(6.0 / 243.0, rel=1e-14)
    assert D2[1, 2] == pytest.approx(-12.0 / 243.0, rel=1e-14)
    # D_xyz = 15*1*2*2/3^7 = 60/2187
    assert D3[0, 1, 2] == pytest.approx(60.0 / 2187.0, rel=1e-14)
    # D_xxx = (15 - 3*3*1*9)/2187 = -66/2187
    assert D3[0, 0, 0] == pytest.approx(-66.0 / 2187.0, rel=1e-14)
    # fourth derivative: D_xxxx = -105/3^9 + 15*6/3^7 - 9/3^5 = -24/19683
    assert D4[0, 0, 0, 0] == pytest.approx(-24.0 / 19683.0, rel=1e-13)
    # eq. 8 tensor: only terms with a delta on the first index survive
    assert D4p[0, 1, 1, 2] == 0.0
    assert D4p[0, 0, 1, 2] == pytest.approx(60.0 / 2187.0, rel=1e-14)
    assert D4p[0, 0, 0, 0] == pytest.approx(-36.0 / 2187.0, rel=1e-14)


@pytest.mark.parametrize("R", RS)
def test_eq8_tensor_exerts_the_same_torque(R):
    """D' keeps exactly the parts of D_ijkl that produce a torque about R."""
    _, _, _, _, D4, D4p = orc.greens(R)
    rng = np.random.default_rng(5)
    Q = rng.normal(size=(3, 3, 3))
    Q = sum(np.transpose(Q, p) for p in itertools.permutations(range(3))) / 6.0
    F = np.einsum("ijkl,jkl->i", D4, Q)
    Fp = np.einsum("ijkl,jkl->i", D4p, Q)
    tau = np.cross(R, F)
    taup = np.cross(R, Fp)
    assert np.max(np.abs(tau - taup)) <= 1e-13 * np.max(np.abs(tau))
    # and the difference is parallel to R
    diff = F - Fp
    assert np.linalg.norm(np.cross(diff, R)) <= 1e-13 * np.linalg.norm(diff) * np.linalg.norm(R)
