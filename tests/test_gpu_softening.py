"""The softened Green's function g = -1/sqrt(R^2 + eps^2) on the GPU (Sec. 4:
the torque correction holds for any Green's function of the distance alone),
through the C ABI, against the oracle with the same softening: FP64
accelerations and potentials to 1e-12 of gabs (the softened magnitude scale),
mixed precision within its bounds, the direct sum to round-off, and the
balances (zero net force for every variant, zero net torque with TC and
TCO)."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1706_06989_amd import amfmm
from paper_1706_06989_amd import workloads as W
from tests.gpu_util import dup_points, say, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "uniform4k": lambda: W.uniform_cube(4096, seed=1),
    "plummer16k": lambda: W.plummer(16384, seed=2),
    "twoplummer20k": lambda: W.two_plummer(20000, seed=3),
    "duplicates": dup_points,
}


def host(o):
    return np.stack([v.cpu().numpy() for v in o])


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("eps", [0.003, 0.05])
def test_softened_solve_matches_oracle(name, eps):
    x, y, z, m = CASES[name]()
    say("softened", name, len(x), eps)
    X, Y, Z, M = to_dev(x, y, z, m)
    _, _, gabs = orc.direct(x, y, z, m, softening=eps)
    pos = np.stack([x, y, z])
    for variant in (amfmm.UC, amfmm.TC, amfmm.TCO):
        oa, op = orc.solve(x, y, z, m, theta=0.5, variant=variant, softening=eps)
        for prec in (amfmm.FP64, amfmm.MIXED):
            s = amfmm.Solver(variant=variant, precision=prec, softening=eps)
            o = s.solve_gravity(X, Y, Z, M, 0.5)
            a = host(o)
            err = np.linalg.norm(a[:3] - oa, axis=0) / gabs
            perr = np.abs(a[3] - op) / np.abs(op)
            fb, tb = s.balance(X, Y, Z, M, o[0], o[1], o[2])
            s.close()
            if prec == amfmm.FP64:
                assert err.max() <= 1e-12 and perr.max() <= 1e-12, (variant, err.max(), perr.max())
                assert fb <= 1e-13, (variant, fb)
                if variant != amfmm.UC:
                    assert tb <= 1e-13, (variant, tb)
            else:
                assert err.max() <= 1e-4 and np.percentile(err, 99) <= 2e-6, (variant, err.max())
                assert np.percentile(perr, 99) <= 1e-6
                assert fb <= 1e-7, (variant, fb)
                if variant != amfmm.UC:
                    assert tb <= 1e-7, (variant, tb)
        # the oracle's own balances for the record
        if variant == amfmm.TC:
            say(f"  oracle TC torque balance {orc.balance(m, orc.angular(pos, oa)):.1e}")


def test_softened_direct_sum_matches_oracle():
    x, y, z, m = W.plummer(8192, seed=9)
    eps = 0.01
    X, Y, Z, M = to_dev(x, y, z, m)
    s = amfmm.Solver(softening=eps)
    idx = W.sample_targets(len(x), 500, seed=3)
    T = torch.from_numpy(idx).cuda()
    ax, ay, az, p, g = s.direct(X, Y, Z, M, T)
    oa, op, og = orc.direct(x, y, z, m, idx, softening=eps)
    a = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
    assert np.max(np.linalg.norm(a - oa, axis=0) / og) <= 1e-13
    assert np.max(np.abs(p.cpu().numpy() - op) / np.abs(op)) <= 1e-13
    assert np.max(np.abs(g.cpu().numpy() - og) / og) <= 1e-13
    s.close()


def test_negative_softening_is_rejected():
    with pytest.raises(amfmm.AmfmmError) as e:
        amfmm.Solver(softening=-1.0)
    assert e.value.code == amfmm.E_INVALID
