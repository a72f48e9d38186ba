"""Pins of the oracle's Sec. 3 metrics on hand-computed cases: the net force
and torque balance, X x g, and the relative force and torque errors.

Each expected value below is worked out by hand in the comment beside it, so
a dropped absolute value, a swapped cross product or a wrong normalisation
fails here and not only against the device twin of the same metric."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W


def test_balance_hand_values():
    # every acceleration the same: sum m A = sum m |A|, balance 1
    m = np.array([1.0, 1.0])
    A = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    assert orc.balance(m, A) == 1.0
    # m = (1, 3), A_x = (3, -1), A_y = (0, 2), A_z = 0:
    #   sum m A_x = 3 - 3 = 0, sum m |A_x| = 6; sum m A_y = 6, sum m |A_y| = 6
    #   balance = sqrt((0 + 36 + 0) / (36 + 36 + 0)) = sqrt(1/2)
    m = np.array([1.0, 3.0])
    A = np.array([[3.0, -1.0], [0.0, 2.0], [0.0, 0.0]])
    assert orc.balance(m, A) == pytest.approx(math.sqrt(0.5), rel=1e-15)
    # equal and opposite forces: m A sums to zero exactly
    m = np.array([2.0, 0.5])
    A = np.array([[0.25, -1.0], [-3.0, 12.0], [1.0, -4.0]])
    assert orc.balance(m, A) == 0.0


def test_balance_cancels_large_terms_exactly():
    # 1e16 + 1 - 1e16 sums to 1 with exact (fsum) summation, to 0 or 2 with
    # plain left-to-right doubles: the metric must not add round-off
    m = np.ones(3)
    A = np.array([[1e16, 1.0, -1e16], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    assert orc.balance(m, A) == pytest.approx(1.0 / (2e16 + 1.0), rel=1e-15)


def test_angular_hand_values():
    pos = np.array([[1.0, 0.0, 2.0], [0.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    acc = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 3.0], [0.0, 1.0, 0.0]])
    # (1,0,0) x (0,1,0) = (0,0,1); (0,1,0) x (0,0,1) = (1,0,0); (2,0,0) x (0,3,0) = (0,0,6)
    expect = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 6.0]])
    assert np.array_equal(orc.angular(pos, acc), expect)


def test_rel_force_error_hand_values():
    true = np.array([[3.0, 0.0, 0.0], [4.0, 0.0, 1.0], [0.0, 0.0, 0.0]])
    acc = np.array([[3.0, 1.0, 0.0], [4.0, 0.0, 1.5], [1.0, 0.0, 0.0]])
    # particle 0: |(0,0,1)| / |(3,4,0)| = 1/5; particle 1: zero truth, skipped;
    # particle 2: |(0,0.5,0)| / 1 = 0.5
    e = orc.rel_force_error(acc, true)
    assert np.array_equal(e, np.array([0.2, 0.5]))


def test_rel_torque_error_hand_values():
    pos = np.array([[0.0], [0.0], [2.0]])
    true = np.array([[1.0], [0.0], [0.0]])
    acc = np.array([[1.0], [1.0], [5.0]])
    # X x g_true = (0,0,2) x (1,0,0) = (0,2,0); X x g = (0,0,2) x (1,1,5) = (-2,2,0)
    # |(-2,0,0)| / |(0,2,0)| = 1 (the radial part of g carries no torque)
    assert np.array_equal(orc.rel_torque_error(pos, acc, true), np.array([1.0]))


def test_two_body_direct_sum_balances_to_zero():
    # the exact pair forces of two bodies: m1 g1 = -m2 g2 and both act along
    # the line joining them, so force and torque balances vanish (to rounding)
    x, y, z = np.array([0.3, -1.1]), np.array([0.2, 0.7]), np.array([-0.5, 0.4])
    m = np.array([2.0, 0.5])
    a, _, _ = orc.direct(x, y, z, m)
    pos = np.stack([x, y, z])
    assert orc.balance(m, a) <= 1e-16
    assert orc.balance(m, orc.angular(pos, a)) <= 1e-15
    # and the pull on body 0 is m_1 / d^2 towards body 1
    d = pos[:, 1] - pos[:, 0]
    r = np.linalg.norm(d)
    assert np.allclose(a[:, 0], m[1] * d / r**3, rtol=1e-15, atol=0)


def test_direct_sum_errors_are_zero_against_themselves():
    x, y, z, m = W.plummer(300, seed=3)
    a, _, _ = orc.direct(x, y, z, m)
    assert np.all(orc.rel_force_error(a, a) == 0.0)
    e = orc.rel_force_error(1.001 * a, a)
    assert np.allclose(e, 1e-3, rtol=1e-9)
