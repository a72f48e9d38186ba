"""Mixed precision (FP32 pair terms, FP64 accumulation, FP64 correction)
against the FP64 oracle, through the C ABI.

There is no paper value for this mode; the FP64 oracle is the judge.  Bounds,
with u = 2^-24 the FP32 unit round-off:
  * per particle, |g_mixed - g_oracle| <= 2e-6 * gabs at the 99th percentile
    and <= 1e-4 * gabs at worst (measured: about 1.6e-7 and 3e-6).  A pair term carries a few u of rounding
    plus the rounding of the FP32 offsets, u |x - Z| / |x - y| relative; the
    worst case is a close pair far from its leaf's centre, so the bound on the
    maximum is loose and the percentile is the meaningful one.
  * potentials: 1e-6 relative at the 99th percentile (every term one sign).
  * force and torque balances: below 1e-7 (FP32 terms are no longer exactly
    antisymmetric; the correction is still FP64; measured about 1e-9).
The tests print what they measure.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1706_06989_amd import amfmm
from paper_1706_06989_amd import workloads as W
from tests.gpu_util import gpu_solve, say, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "uniform4k": lambda: W.uniform_cube(4096, seed=1),
    "plummer16k": lambda: W.plummer(16384, seed=2),
    "twoplummer20k": lambda: W.two_plummer(20000, seed=3),
    "sphere5001": lambda: W.uniform_sphere(5001, seed=4),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("variant", [amfmm.UC, amfmm.TC, amfmm.TCO])
def test_mixed_against_fp64_oracle(name, variant):
    x, y, z, m = CASES[name]()
    for theta in (0.35, 0.7):
        say("mixed", name, len(x), variant, theta)
        acc, pot, _ = gpu_solve(x, y, z, m, theta, variant=variant, precision=amfmm.MIXED)
        t = orc.Tree(x, y, z, m)
        t.compute_moments()
        t.walk(theta)
        oacc, opot = t.evaluate(variant)
        _, _, gabs = orc.direct(x, y, z, m)
        err = np.linalg.norm(acc - oacc, axis=0) / gabs
        perr = np.abs(pot - opot) / np.abs(opot)
        say(f"  accel err/gabs p99 {np.percentile(err, 99):.3e} max {err.max():.3e}; "
            f"pot p99 {np.percentile(perr, 99):.3e}")
        assert np.percentile(err, 99) <= 2e-6
        assert err.max() <= 1e-4
        assert np.percentile(perr, 99) <= 1e-6


def test_mixed_balances_and_truth():
    """Residual total force and torque of the mixed solve, and its error against
    direct summation next to the FP64 solve's."""
    x, y, z, m = W.two_plummer(60000, seed=9)
    X, Y, Z, M = to_dev(x, y, z, m)
    idx = W.sample_targets(len(x), 2048, seed=99)
    truth, _, _ = orc.direct(x, y, z, m, idx)
    res = {}
    for prec in (amfmm.FP64, amfmm.MIXED):
        s = amfmm.Solver(precision=prec)
        ax, ay, az, _ = s.solve_gravity(X, Y, Z, M, 0.5)
        fb, tb = s.balance(X, Y, Z, M, ax, ay, az)
        acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])[:, idx]
        e = np.linalg.norm(acc - truth, axis=0) / np.linalg.norm(truth, axis=0)
        res[prec] = (fb, tb, np.percentile(e, 99))
        say(f"precision {prec}: force balance {fb:.3e} torque balance {tb:.3e} p99 vs truth {res[prec][2]:.3e}")
    fb, tb, p99 = res[amfmm.MIXED]
    assert fb <= 1e-7 and tb <= 1e-7
    # FP32 rounding stays far below the method's own error
    assert abs(p99 - res[amfmm.FP64][2]) <= 0.01 * res[amfmm.FP64][2]


def test_mixed_batched_matches_whole():
    """The batched walk selects the same pairs as the whole walk (the same
    counts); a cell's pairs may be summed in another order (the frontier of a
    level is cut into work chunks by its size), which under mixed precision
    moves results by FP32 rounding only: p99 2e-6 and max 1e-5 of gabs."""
    x, y, z, m = W.plummer(1 << 16, seed=12)
    X, Y, Z, M = to_dev(x, y, z, m)
    s1 = amfmm.Solver(precision=amfmm.MIXED)
    a1 = s1.solve_gravity(X, Y, Z, M, 0.4)
    s2 = amfmm.Solver(precision=amfmm.MIXED, list_bytes=1 << 20)
    a2 = s2.solve_gravity(X, Y, Z, M, 0.4)
    c1, c2 = s1.get_counts(), s2.get_counts()
    for k in ("near_interactions", "far_evaluations"):
        assert c1[k] == c2[k] > 0
    idx = W.sample_targets(len(x), 1024, seed=99)
    _, _, gabs = orc.direct(x, y, z, m, idx)
    h1 = np.stack([v.cpu().numpy() for v in a1[:3]])[:, idx]
    h2 = np.stack([v.cpu().numpy() for v in a2[:3]])[:, idx]
    e = np.linalg.norm(h1 - h2, axis=0) / gabs
    say(f"batched against whole (mixed): p99 {np.percentile(e, 99):.2e}, max {e.max():.2e}")
    assert np.percentile(e, 99) <= 2e-6 and e.max() <= 1e-5
