"""Time integration through the library (amfmm_leapfrog: uniform-step
kick-drift-kick, Sec. 1 and Sec. 4) on two Plummer spheres in equilibrium on a
circular orbit about each other (workloads.two_plummer_binary).

* Against the oracle's leapfrog: 4096 particles, 8 steps, FP64, TC: positions
  and velocities agree to round-off (1e-12 of their scale).
* One whole orbit (period 2 pi sqrt(27) = 32.6) of the 2^16 binary with
  dt = 0.02 (1633 steps), FP64, theta 0.5: a drift leaves the total angular
  momentum L unchanged and a kick changes it by dt times the net torque, so
  with the torque correction (TC) L stays at round-off over the orbit, while
  without it (UC) it drifts; the drift per orbit of both is reported.  The
  net momentum stays at round-off in both.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1706_06989_amd import amfmm
from paper_1706_06989_amd import workloads as W
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def ang(X, Y, Z, VX, VY, VZ, M):
    return torch.stack([(M * (Y * VZ - Z * VY)).sum(), (M * (Z * VX - X * VZ)).sum(),
                        (M * (X * VY - Y * VX)).sum()]).cpu().numpy()


def test_leapfrog_matches_oracle():
    x, y, z, m, vx, vy, vz = W.two_plummer_binary(4096, seed=11)
    say("leapfrog parity 4096")
    X, Y, Z, M, VX, VY, VZ = to_dev(x, y, z, m, vx, vy, vz)
    s = amfmm.Solver()
    ax, ay, az, _ = s.solve_gravity(X, Y, Z, M, 0.5, pot=False)
    s.leapfrog(X, Y, Z, VX, VY, VZ, M, 0.5, 5e-3, 8, (ax, ay, az))
    ox, oy, oz, ovx, ovy, ovz, _ = orc.leapfrog(x, y, z, vx, vy, vz, m, 0.5, 5e-3, 8)
    pscale = np.max(np.abs(x))
    vscale = np.max(np.abs(vy))
    dp = max(np.max(np.abs(A.cpu().numpy() - B)) for A, B in ((X, ox), (Y, oy), (Z, oz))) / pscale
    dv = max(np.max(np.abs(A.cpu().numpy() - B)) for A, B in ((VX, ovx), (VY, ovy), (VZ, ovz))) / vscale
    say(f"  max position difference / scale {dp:.2e}, velocity {dv:.2e}")
    assert dp <= 1e-12 and dv <= 1e-12
    s.close()


def orbit(variant, n=1 << 16, dt=0.02):
    x, y, z, m, vx, vy, vz = W.two_plummer_binary(n, seed=7)
    X, Y, Z, M, VX, VY, VZ = to_dev(x, y, z, m, vx, vy, vz)
    period = 2.0 * np.pi * np.sqrt(27.0)
    steps = int(round(period / dt))
    s = amfmm.Solver(variant=variant)
    L0 = ang(X, Y, Z, VX, VY, VZ, M)
    P0 = torch.stack([(M * VX).sum(), (M * VY).sum(), (M * VZ).sum()]).cpu().numpy()
    acc = s.solve_gravity(X, Y, Z, M, 0.5, pot=False)[:3]
    drift = []
    done = 0
    for chunk in (steps // 4,) * 3 + (steps - 3 * (steps // 4),):
        s.leapfrog(X, Y, Z, VX, VY, VZ, M, 0.5, dt, chunk, acc)
        done += chunk
        L = ang(X, Y, Z, VX, VY, VZ, M)
        drift.append(float(np.linalg.norm(L - L0) / np.linalg.norm(L0)))
        say(f"  {variant=} {done}/{steps} steps: relative change of L {drift[-1]:.3e}")
    P = torch.stack([(M * VX).sum(), (M * VY).sum(), (M * VZ).sum()]).cpu().numpy()
    pscale = (M * VY.abs()).sum().item()
    s.close()
    return drift, float(np.linalg.norm(P - P0) / pscale), steps


@pytest.mark.timeout(600)
def test_angular_momentum_over_one_orbit():
    say("one orbit of the 2^16 binary, UC and TC")
    uc, puc, steps = orbit(amfmm.UC)
    tc, ptc, _ = orbit(amfmm.TC)
    say(f"relative change of L over one orbit ({steps} steps): UC {uc[-1]:.3e}, TC {tc[-1]:.3e}; "
        f"net momentum UC {puc:.1e}, TC {ptc:.1e}")
    assert max(tc) <= 1e-12
    assert uc[-1] >= 1e3 * max(tc[-1], 1e-16)
    assert puc <= 1e-12 and ptc <= 1e-12
