"""Pins of one accepted cell pair in the oracle: eqs. 2-4, the pairwise force
balance (eq. "unit"), the net torque of the uncorrected pair (eq. "nettorque",
at the appendix's expansion order P = 3) and its cancellation by the
corrections of eq. 7 (TC) and eq. 8 (TCO).

The reference for the accelerations is direct summation between the two
clusters written out in numpy here.
"""
import numpy as np
import pytest

from oracle import oracle as orc


def cluster(rng, n, centre, size):
    X = centre[:, None] + size * rng.uniform(-1, 1, size=(3, n))
    m = rng.uniform(0.5, 1.5, size=n)
    return X, m


def direct_cross(XA, mA, XB, mB):
    """Acceleration on every particle of A caused by B, and potential."""
    d = XB[:, None, :] - XA[:, :, None]  # [3, nA, nB]
    r = np.sqrt((d ** 2).sum(axis=0))
    g = (mB[None, None, :] * d / r ** 3).sum(axis=2)
    p = -(mB[None, :] / r).sum(axis=1)
    return g.T, p


def far(XA, mA, XB, mB, variant):
    return orc.pair_far((XA[0], XA[1], XA[2], mA), (XB[0], XB[1], XB[2], mB), variant)


@pytest.mark.parametrize("variant", [orc.UC, orc.TC, orc.TCO])
def test_force_error_scales_as_third_power(variant):
    """Quadrupole-order expansion: the force error falls as (size/d)^3."""
    rng = np.random.default_rng(11)
    dirn = np.array([0.6, -0.48, 0.64])
    UA = rng.uniform(-1, 1, size=(3, 40))
    UB = rng.uniform(-1, 1, size=(3, 30))
    mA = rng.uniform(0.5, 1.5, 40)
    mB = rng.uniform(0.5, 1.5, 30)
    errs = []
    for s in (0.08, 0.04, 0.02):
        XA = UA * s
        XB = dirn[:, None] * 1.0 + UB * s
        gA, _, gB, _ = far(XA, mA, XB, mB, variant)
        tA, _ = direct_cross(XA, mA, XB, mB)
        tB, _ = direct_cross(XB, mB, XA, mA)
        e = max(np.abs(gA - tA).max() / np.abs(tA).max(), np.abs(gB - tB).max() / np.abs(tB).max())
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.0 < r1 < 10.5 and 6.0 < r2 < 10.5, errs


def test_potential_error_scales_as_fourth_power():
    rng = np.random.default_rng(12)
    UA = rng.uniform(-1, 1, size=(3, 25))
    UB = rng.uniform(-1, 1, size=(3, 35))
    mA = rng.uniform(0.5, 1.5, 25)
    mB = rng.uniform(0.5, 1.5, 35)
    errs = []
    for s in (0.08, 0.04, 0.02):
        XA = UA * s
        XB = np.array([[0.0], [1.0], [0.0]]) + UB * s
        _, pA, _, pB = far(XA, mA, XB, mB, orc.UC)
        _, qA = direct_cross(XA, mA, XB, mB)
        _, qB = direct_cross(XB, mB, XA, mA)
        # the dropped octupole constant (M_ijk D_ijk / 6) is O(s^3) but the same
        # for every particle of a cell, so compare after removing the cell mean
        e = max(np.abs((pA - qA) - (pA - qA).mean()).max(),
                np.abs((pB - qB) - (pB - qB).mean()).max()) / np.abs(qA).max()
        errs.append(e)
    assert 12.0 < errs[0] / errs[1] < 20.0 and 12.0 < errs[1] / errs[2] < 20.0, errs


def test_point_masses_are_exact():
    XA = np.array([[0.1], [0.2], [0.3]])
    XB = np.array([[1.3], [-0.4], [0.9]])
    mA = np.array([2.0])
    mB = np.array([0.5])
    for v in (orc.UC, orc.TC, orc.TCO):
        gA, pA, gB, pB = far(XA, mA, XB, mB, v)
        tA, qA = direct_cross(XA, mA, XB, mB)
        tB, qB = direct_cross(XB, mB, XA, mA)
        np.testing.assert_allclose(gA, tA, rtol=1e-15)
        np.testing.assert_allclose(gB, tB, rtol=1e-15)
        np.testing.assert_allclose(pA, qA, rtol=1e-15)
        np.testing.assert_allclose(pB, qB, rtol=1e-15)


def test_two_body_closed_form():
    # unit masses two apart: |g| = 1/4 towards the other body, potential -1/2
    gA, pA, gB, pB = orc.pair_far(([0.0], [0.0], [0.0], [1.0]), ([2.0], [0.0], [0.0], [1.0]), orc.TC)
    assert np.array_equal(gA, [[0.25, 0.0, 0.0]])
    assert np.array_equal(gB, [[-0.25, 0.0, 0.0]])
    assert pA[0] == -0.5 and pB[0] == -0.5


@pytest.mark.parametrize("variant", [orc.UC, orc.TC, orc.TCO])
def test_pair_force_balance(variant):
    """eq. "unit": the pair's forces cancel to round-off for every variant."""
    rng = np.random.default_rng(13)
    XA, mA = cluster(rng, 37, np.array([0.0, 0.0, 0.0]), 0.2)
    XB, mB = cluster(rng, 23, np.array([1.1, 0.7, -0.4]), 0.3)
    gA, _, gB, _ = far(XA, mA, XB, mB, variant)
    F = (mA[:, None] * gA).sum(axis=0) + (mB[:, None] * gB).sum(axis=0)
    scale = (mA[:, None] * np.abs(gA)).sum(axis=0).max()
    assert np.abs(F).max() <= 1e-14 * scale


def moments_full(X, m):
    M = m.sum()
    Z = (X * m).sum(axis=1) / M
    x = X - Z[:, None]
    return M, Z, np.einsum("n,in,jn,kn->ijk", m, x, x, x)


@pytest.mark.parametrize("offset", [np.array([1.1, 0.7, -0.4]), np.array([-0.3, 1.4, 0.9])])
def test_uncorrected_pair_torque_and_its_correction(offset):
    """The uncorrected pair exerts a net torque; eq. 7 (prefactor 1/6 of the
    appendix at P = 3, applied +F_c/M_A to A and -F_c/M_B to B) and eq. 8 remove it.

    The torque is measured from the particle accelerations (sum of X x m g);
    for UC it must equal R x F with F = (1/6) Q_jkl D_ijkl, Q = M_A,jkl M_B -
    M_A M_B,jkl: eq. "nettorque" of the paper written at P = 3 of the
    appendix's net-torque sum.  Half the prefactor, or the opposite sign, would
    leave a torque of the same size."""
    rng = np.random.default_rng(14)
    XA, mA = cluster(rng, 41, np.array([0.0, 0.0, 0.0]), 0.25)
    XB, mB = cluster(rng, 29, offset, 0.35)
    torques = {}
    for v in (orc.UC, orc.TC, orc.TCO):
        gA, _, gB, _ = far(XA, mA, XB, mB, v)
        tau = np.cross(XA.T, mA[:, None] * gA).sum(axis=0) + np.cross(XB.T, mB[:, None] * gB).sum(axis=0)
        torques[v] = tau
    MA, ZA, OA = moments_full(XA, mA)
    MB, ZB, OB = moments_full(XB, mB)
    R = ZA - ZB
    D4 = orc.greens(R)[4]
    Q = OA * MB - MA * OB
    expected = np.cross(R, np.einsum("ijkl,jkl->i", D4, Q) / 6.0)
    uc = torques[orc.UC]
    assert np.linalg.norm(uc) > 1e-6
    np.testing.assert_allclose(uc, expected, rtol=1e-9, atol=1e-12 * np.linalg.norm(uc))
    # corrected variants: residual at round-off relative to the removed torque
    gscale = np.linalg.norm(R) * MA * MB / np.dot(R, R)
    for v in (orc.TC, orc.TCO):
        assert np.linalg.norm(torques[v]) <= 1e-13 * gscale, (v, torques[v], uc)
