"""Pins of the oracle's uniform-step leapfrog (the time integration over which
Sec. 1 and Sec. 4 measure angular momentum conservation).

Against: the closed two-body circular orbit (one period returns the bodies
to their start to the integrator's second-order error, energy and angular
momentum held), time reversibility (reversed velocities retrace the steps to
round-off), and the paper's claim: with the torque correction the total
angular momentum of a many-body integration stays at round-off, without it it
drifts; linear momentum is kept by every variant."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W


def ang(x, y, z, vx, vy, vz, m):
    return np.array([np.sum(m * (y * vz - z * vy)), np.sum(m * (z * vx - x * vz)), np.sum(m * (x * vy - y * vx))])


def test_two_body_circular_orbit_closes():
    # masses 2 and 1 at distance 1, circular orbit about the centre of mass:
    # angular speed sqrt(M/d^3) = sqrt(3), period 2 pi / sqrt(3)
    m = np.array([2.0, 1.0])
    x = np.array([-1.0 / 3.0, 2.0 / 3.0])
    y = np.zeros(2)
    z = np.zeros(2)
    w = np.sqrt(3.0)
    vx = np.zeros(2)
    vy = w * x
    vz = np.zeros(2)
    T = 2.0 * np.pi / w
    steps = 4000
    X, Y, Z, VX, VY, VZ, _ = orc.leapfrog(x, y, z, vx, vy, vz, m, 0.5, T / steps, steps)
    # leapfrog's phase error over one period is O(dt^2): (T/steps)^2 ~ 1e-7
    assert np.max(np.abs(X - x)) < 1e-5 and np.max(np.abs(Y - y)) < 1e-5
    E0 = 0.5 * np.sum(m * (vx**2 + vy**2)) - m[0] * m[1] / 1.0
    d = np.hypot(X[1] - X[0], Y[1] - Y[0])
    E1 = 0.5 * np.sum(m * (VX**2 + VY**2 + VZ**2)) - m[0] * m[1] / d
    assert abs(E1 - E0) < 1e-6 * abs(E0)
    L0, L1 = ang(x, y, z, vx, vy, vz, m), ang(X, Y, Z, VX, VY, VZ, m)
    assert np.linalg.norm(L1 - L0) <= 1e-13 * np.linalg.norm(L0)
    # doubled accelerations (as if each half kick took a whole dt) do not close it
    Xb, Yb, *_ = orc.leapfrog(x, y, z, vx, vy, vz, 2.0 * m, 0.5, T / steps, steps)
    assert np.max(np.abs(Xb - x)) > 1e-2


def test_time_reversibility():
    x, y, z, m, vx, vy, vz = W.two_plummer_binary(400, seed=5)
    X, Y, Z, VX, VY, VZ, A = orc.leapfrog(x, y, z, vx, vy, vz, m, 0.6, 1e-3, 15)
    assert np.max(np.abs(X - x)) > 1e-4  # it moved
    X2, Y2, Z2, VX2, VY2, VZ2, _ = orc.leapfrog(X, Y, Z, -VX, -VY, -VZ, m, 0.6, 1e-3, 15, acc=A)
    scale = np.max(np.abs(x))
    for a, b in ((X2, x), (Y2, y), (Z2, z)):
        assert np.max(np.abs(a - b)) <= 1e-12 * scale
    vs = np.max(np.abs(vx))
    for a, b in ((VX2, -vx), (VY2, -vy), (VZ2, -vz)):
        assert np.max(np.abs(a - b)) <= 1e-11 * vs


@pytest.mark.parametrize("variant", [orc.UC, orc.TC, orc.TCO])
def test_momentum_and_angular_momentum_over_steps(variant):
    x, y, z, m, vx, vy, vz = W.two_plummer_binary(1500, seed=9)
    L0 = ang(x, y, z, vx, vy, vz, m)
    P0 = np.array([np.sum(m * vx), np.sum(m * vy), np.sum(m * vz)])
    X, Y, Z, VX, VY, VZ, _ = orc.leapfrog(x, y, z, vx, vy, vz, m, 0.6, 2e-3, 20, n_crit=8, variant=variant)
    L1 = ang(X, Y, Z, VX, VY, VZ, m)
    P1 = np.array([np.sum(m * VX), np.sum(m * VY), np.sum(m * VZ)])
    dl = np.linalg.norm(L1 - L0) / np.linalg.norm(L0)
    # linear momentum: zero net force in every variant (scale: the orbital momentum)
    pscale = np.sum(m * np.abs(vy))
    assert np.linalg.norm(P1 - P0) <= 1e-14 * pscale
    if variant == orc.UC:
        assert dl > 1e-11, dl
    else:
        assert dl <= 1e-14, dl
