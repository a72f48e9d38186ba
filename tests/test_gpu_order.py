"""The appendix's expansion order P = 4 on the GPU (FP64, UC and TC) through
the C ABI, against the oracle's general form at P = 4: accelerations to
1e-12 of gabs and potentials to 1e-12 relative, plain and softened; the
balances at round-off (zero net torque with the correction at this order);
the error against direct summation below the order-3 solve's; the option
checks."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("name,softening,n_crit", [(n, 0.0, 25) for n in sorted(CASES)] +
                         [("plummer16k", 0.01, 25), ("plummer16k", 0.0, 64), ("twoplummer20k", 0.0, 64)])
def test_order4_matches_oracle(name, softening, n_crit):
    """Plain and softened, with the configuration's leaves (25) and the
    benchmark's order-4 leaves (64)."""
    x, y, z, m = CASES[name]()
    say("order 4", name, len(x), softening, n_crit)
    X, Y, Z, M = to_dev(x, y, z, m)
    _, _, gabs = orc.direct(x, y, z, m, softening=softening)
    for variant in (amfmm.UC, amfmm.TC):
        oa, op = orc.solve(x, y, z, m, theta=0.5, n_crit=n_crit, variant=variant, softening=softening, order=4)
        s = amfmm.Solver(variant=variant, softening=softening, order=4, n_crit=n_crit)
        o = s.solve_gravity(X, Y, Z, M, 0.5)
        a = host(o)
        err = np.linalg.norm(a[:3] - oa, axis=0) / gabs
        perr = np.abs(a[3] - op) / np.abs(op)
        fb, tb = s.balance(X, Y, Z, M, o[0], o[1], o[2])
        s.close()
        say(f"  variant {variant}: max {err.max():.1e}, pot {perr.max():.1e}, balances {fb:.1e} {tb:.1e}")
        assert err.max() <= 1e-12 and perr.max() <= 1e-12, (variant, err.max(), perr.max())
        assert fb <= 1e-13
        if variant == amfmm.TC:
            assert tb <= 1e-13


@pytest.mark.parametrize("name", ["plummer16k", "twoplummer20k"])
def test_order4_mixed_near_field_within_mixed_bounds(name):
    """Order 4 with the mixed near field (FP32 pair terms, compensated FP64
    sums; the order-4 far field stays FP64): against the oracle at order 4
    within the mixed-precision bounds, balances at FP32 round-off."""
    x, y, z, m = CASES[name]()
    X, Y, Z, M = to_dev(x, y, z, m)
    _, _, gabs = orc.direct(x, y, z, m)
    oa, op = orc.solve(x, y, z, m, theta=0.5, variant=amfmm.TC, order=4)
    s = amfmm.Solver(variant=amfmm.TC, precision=amfmm.MIXED, order=4)
    o = s.solve_gravity(X, Y, Z, M, 0.5)
    a = host(o)
    err = np.linalg.norm(a[:3] - oa, axis=0) / gabs
    perr = np.abs(a[3] - op) / np.abs(op)
    fb, tb = s.balance(X, Y, Z, M, o[0], o[1], o[2])
    s.close()
    say(f"order 4 mixed {name}: max {err.max():.1e} p99 {np.percentile(err, 99):.1e}, balances {fb:.1e} {tb:.1e}")
    assert err.max() <= 1e-4 and np.percentile(err, 99) <= 2e-6
    assert np.percentile(perr, 99) <= 1e-6
    assert fb <= 1e-7 and tb <= 1e-7


def test_order4_is_more_accurate_and_conserves():
    x, y, z, m = W.plummer(65536, seed=7)
    say("order 4 against order 3, plummer 65536")
    X, Y, Z, M = to_dev(x, y, z, m)
    idx = W.sample_targets(len(x), 2048, seed=99)
    at, _, _ = orc.direct(x, y, z, m, idx)
    p99 = {}
    for order in (3, 4):
        for variant in (amfmm.UC, amfmm.TC):
            s = amfmm.Solver(variant=variant, order=order)
            o = s.solve_gravity(X, Y, Z, M, 0.5, pot=False)
            a = np.stack([o[k].cpu().numpy()[idx] for k in range(3)])
            e = np.linalg.norm(a - at, axis=0) / np.linalg.norm(at, axis=0)
            fb, tb = s.balance(X, Y, Z, M, o[0], o[1], o[2])
            s.close()
            p99[(order, variant)] = np.percentile(e, 99)
            say(f"  order {order} variant {variant}: p99 {p99[(order, variant)]:.2e}, balances {fb:.1e} {tb:.1e}")
            assert fb <= 1e-13
            if variant == amfmm.TC:
                assert tb <= 1e-13
            else:
                assert tb >= 1e-9
    assert p99[(4, amfmm.TC)] <= 0.5 * p99[(3, amfmm.TC)]


def test_order_option_checks():
    for kw in ({"order": 5}, {"order": 2}, {"order": 4, "variant": amfmm.TCO}):
        with pytest.raises(amfmm.AmfmmError) as e:
            amfmm.Solver(**kw)
        assert e.value.code == amfmm.E_INVALID


def test_order4_batched_matches_whole():
    """At order 4 the batched solve (forced by a tiny list budget: the walk
    and the evaluation cut into subtrees, the order-4 expansions of the top
    levels kept across batches) selects the same pairs and gives the whole
    solve's results up to summation order."""
    x, y, z, m = W.plummer(1 << 17, seed=12)
    say("order 4 batched", len(x))
    X, Y, Z, M = to_dev(x, y, z, m)
    whole = amfmm.Solver(order=4)
    a1 = host(whole.solve_gravity(X, Y, Z, M, 0.5))
    c1 = whole.get_counts()
    part = amfmm.Solver(order=4, list_bytes=1 << 20)
    a2 = host(part.solve_gravity(X, Y, Z, M, 0.5))
    c2 = part.get_counts()
    for k in ("near_interactions", "far_evaluations", "walk_candidates"):
        assert c1[k] == c2[k] > 0, k
    assert c2["walk_pass_launches"] > c1["walk_pass_launches"]
    idx = W.sample_targets(len(x), 256, seed=99)
    _, _, gabs = orc.direct(x, y, z, m, idx)
    assert np.max(np.linalg.norm(a1[:3, idx] - a2[:3, idx], axis=0) / gabs) <= 1e-13
    assert np.max(np.abs(a1[3] - a2[3]) / np.abs(a1[3])) <= 1e-13
    whole.close()
    part.close()
