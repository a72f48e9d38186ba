"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: keys, permutation, cells and both interaction lists bit-exact; mass,
centre of mass and R_max bit-exact (they decide the walk); quadrupole and
octupole to 1e-12 of M R^k; accelerations to 1e-12 of the per-particle
magnitude scale gabs_i = sum_j m_j / r_ij^2 (the sum of the magnitudes the
result is made of, so the bound is meaningful also where the field cancels);
potentials to 1e-12 relative (every term of a potential has the same sign).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1706_06989_amd import amfmm
from paper_1706_06989_amd import workloads as W
from tests.gpu_util import dup_points, gpu_solve, say, to_dev, tree_parts

pytestmark = pytest.mark.gpu


CASES = {
    "uniform4k": lambda: W.uniform_cube(4096, seed=1),
    "plummer16k": lambda: W.plummer(16384, seed=2),
    "twoplummer20k": lambda: W.two_plummer(20000, seed=3),
    "sphere5001": lambda: W.uniform_sphere(5001, seed=4),
    "n1": lambda: (np.array([0.3]), np.array([0.1]), np.array([-0.2]), np.array([1.0])),
    "n25": lambda: W.uniform_cube(25, seed=5),
    "n26": lambda: W.uniform_cube(26, seed=6),
    "duplicates": dup_points,
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    x, y, z, m = CASES[request.param]()
    return request.param, (x, y, z, m)


def test_tree_bit_exact(case):
    name, (x, y, z, m) = case
    say("tree", name, len(x))
    s, _ = tree_parts(x, y, z, m)
    g = s.get_tree()
    t = orc.Tree(x, y, z, m)
    k, p = t.keys()
    assert np.array_equal(g["keys"], k)
    assert np.array_equal(g["perm"], p)
    c = t.cells()
    for f in ("level", "begin", "count", "parent", "child0", "nchild"):
        assert np.array_equal(g[f], c[f]), f


def test_moments(case):
    name, (x, y, z, m) = case
    say("moments", name, len(x))
    s, _ = tree_parts(x, y, z, m)
    s.compute_moments()
    gm = s.get_moments()
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    om = t.moments()
    # mass, centre of mass and R_max decide the walk: bit for bit
    assert np.array_equal(gm[:, :5], om[:, :5])
    M, R = om[:, 0:1], om[:, 4:5]
    tiny = 1e-300
    assert np.all(np.abs(gm[:, 5:11] - om[:, 5:11]) <= 1e-12 * M * R**2 + tiny)
    assert np.all(np.abs(gm[:, 11:21] - om[:, 11:21]) <= 1e-12 * M * R**3 + tiny)


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7, 1.0])
def test_lists_bit_exact(case, theta):
    name, (x, y, z, m) = case
    say("lists", name, len(x), theta)
    s, _ = tree_parts(x, y, z, m)
    s.compute_moments()
    s.walk(theta)
    far, near = s.get_lists()
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk(theta)
    ofar, onear = t.lists()
    assert np.array_equal(far, ofar)
    assert np.array_equal(near, onear)


@pytest.mark.parametrize("variant", [amfmm.UC, amfmm.TC, amfmm.TCO])
def test_accelerations_fp64(case, variant):
    name, (x, y, z, m) = case
    say("fp64 accel", name, len(x), variant)
    for theta in (0.5, 0.8):
        acc, pot, _ = gpu_solve(x, y, z, m, theta, variant=variant)
        t = orc.Tree(x, y, z, m)
        t.compute_moments()
        t.walk(theta)
        oacc, opot = t.evaluate(variant)
        _, _, gabs = orc.direct(x, y, z, m)
        if len(x) == 1:
            assert np.all(acc == 0) and np.all(pot == 0)
            continue
        err = np.linalg.norm(acc - oacc, axis=0) / gabs
        assert err.max() <= 1e-12, (theta, err.max())
        perr = np.abs(pot - opot) / np.abs(opot)
        assert perr.max() <= 1e-12, (theta, perr.max())


def test_direct_sum_parity():
    x, y, z, m = W.two_plummer(6000, seed=8)
    say("direct", len(x))
    s = amfmm.Solver()
    X, Y, Z, M = to_dev(x, y, z, m)
    idx = W.sample_targets(len(x), 700, seed=3)
    ax, ay, az, p, g = s.direct(X, Y, Z, M, torch.from_numpy(idx).to("cuda"))
    acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
    oacc, opot, ogabs = orc.direct(x, y, z, m, idx)
    assert np.max(np.linalg.norm(acc - oacc, axis=0) / ogabs) <= 1e-14
    assert np.max(np.abs(p.cpu().numpy() - opot) / np.abs(opot)) <= 1e-14
    assert np.max(np.abs(g.cpu().numpy() - ogabs) / ogabs) <= 1e-14


def test_balances_on_gpu():
    x, y, z, m = W.two_plummer(30000, seed=9)
    say("balance", len(x))
    X, Y, Z, M = to_dev(x, y, z, m)
    res = {}
    for v in (amfmm.UC, amfmm.TC, amfmm.TCO):
        s = amfmm.Solver(variant=v)
        ax, ay, az, _ = s.solve_gravity(X, Y, Z, M, 0.6)
        res[v] = s.balance(X, Y, Z, M, ax, ay, az)
        # the device metric agrees with the oracle's metric on the same field
        acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
        pos = np.stack([x, y, z])
        assert abs(res[v][0] - orc.balance(m, acc)) <= 1e-3 * res[v][0] + 1e-18
        assert abs(res[v][1] - orc.balance(m, orc.angular(pos, acc))) <= 1e-3 * res[v][1] + 1e-18
    for v in res:
        assert res[v][0] <= 1e-13, res
    assert res[amfmm.TC][1] <= 1e-13 and res[amfmm.TCO][1] <= 1e-13, res
    assert res[amfmm.UC][1] >= 1e3 * res[amfmm.TC][1], res


def test_deterministic():
    x, y, z, m = W.plummer(50000, seed=10)
    say("determinism", len(x))
    a1, p1, s = gpu_solve(x, y, z, m, 0.5)
    a2, p2, _ = gpu_solve(x, y, z, m, 0.5, solver=s)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)


def test_error_paths():
    say("errors")
    x, y, z, m = W.uniform_cube(100, seed=1)
    s = amfmm.Solver()
    X, Y, Z, M = to_dev(x, y, z, m)
    with pytest.raises(amfmm.AmfmmError) as e:
        s.compute_moments()
    assert e.value.code == amfmm.E_STATE
    with pytest.raises(amfmm.AmfmmError) as e:
        s.walk(0.5)
    assert e.value.code == amfmm.E_STATE
    for th in (0.0, -1.0, 1.5, float("nan")):
        with pytest.raises(amfmm.AmfmmError) as e:
            s.solve_gravity(X, Y, Z, M, th)
        assert e.value.code == amfmm.E_INVALID
    bad = x.copy()
    bad[17] = np.nan
    Xb, = to_dev(bad)
    with pytest.raises(amfmm.AmfmmError) as e:
        s.solve_gravity(Xb, Y, Z, M, 0.5)
    assert e.value.code == amfmm.E_NONFINITE
    mb = m.copy()
    mb[3] = 0.0
    Mb, = to_dev(mb)
    with pytest.raises(amfmm.AmfmmError) as e:
        s.solve_gravity(X, Y, Z, Mb, 0.5)
    assert e.value.code == amfmm.E_INVALID
    # no particles; arrays of different lengths are refused before the call
    e0 = torch.empty(0, dtype=torch.float64, device="cuda")
    with pytest.raises(amfmm.AmfmmError) as e:
        s.solve_gravity(e0, e0, e0, e0, 0.5)
    assert e.value.code == amfmm.E_INVALID
    with pytest.raises(ValueError):
        s.solve_gravity(X, Y[:50], Z, M, 0.5)
    with pytest.raises(ValueError):
        s.solve_gravity(X, Y, Z, M, 0.5, out=s._outputs(99, True))
    fe = amfmm.Solver(criterion=amfmm.MULTIPOLE, error_tol=1e-6, theta_max=0.5)
    fe.set_field_estimate(torch.ones(99, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        fe.solve_gravity(X, Y, Z, M, 0.5)
    fe.close()
    # a capped context reports out-of-memory instead of allocating
    small = amfmm.Solver(max_bytes=1 << 12)
    with pytest.raises(amfmm.AmfmmError) as e:
        small.solve_gravity(X, Y, Z, M, 0.5)
    assert e.value.code == amfmm.E_OOM
    # the context still works after errors
    ax, ay, az, p = s.solve_gravity(X, Y, Z, M, 0.5)
    assert torch.isfinite(ax).all()


@pytest.mark.parametrize("theta", [0.35, 0.7])
def test_batched_walk_matches_whole_walk(theta):
    """Walking and evaluating batch by batch (forced by a tiny list budget)
    selects the same pairs (the same interaction counts) and gives the same
    results up to the order in which a cell's pairs are summed."""
    x, y, z, m = W.plummer(1 << 17, seed=12)
    say("batched", len(x), theta)
    X, Y, Z, M = to_dev(x, y, z, m)
    whole = amfmm.Solver()
    a1 = host4(whole.solve_gravity(X, Y, Z, M, theta))
    c1 = whole.get_counts()
    part = amfmm.Solver(list_bytes=1 << 20)
    a2 = host4(part.solve_gravity(X, Y, Z, M, theta))
    c2 = part.get_counts()
    for k in ("near_interactions", "far_evaluations", "walk_candidates"):
        assert c1[k] == c2[k] > 0, k
    assert c2["walk_pass_launches"] > c1["walk_pass_launches"]  # batches walk the lower levels again
    idx = W.sample_targets(len(x), 256, seed=99)
    _, _, gabs = orc.direct(x, y, z, m, idx)
    assert np.max(np.linalg.norm(a1[:3, idx] - a2[:3, idx], axis=0) / gabs) <= 1e-13
    assert np.max(np.abs(a1[3] - a2[3]) / np.abs(a1[3])) <= 1e-13
    ph = part.get_phase_times()
    assert ph["near+eval"] > 0 and ph["walk"] > 0


FIELD_CASES = ["uniform4k", "plummer16k", "twoplummer20k", "duplicates"]


CRITERIA = {"estimate": (amfmm.ESTIMATE, "walk_field"), "multipole": (amfmm.MULTIPOLE, "walk_multipole")}


@pytest.mark.parametrize("crit", sorted(CRITERIA))
@pytest.mark.parametrize("name", FIELD_CASES)
@pytest.mark.parametrize("eps,tmax", [(1e-4, 0.7), (1e-6, 0.5)])
def test_field_criterion_lists_and_accelerations(crit, name, eps, tmax):
    """Error-estimate criteria: with the same per-particle field input both
    sides select the same pairs bit for bit, and the accelerations agree."""
    x, y, z, m = CASES[name]()
    say("field", crit, name, len(x), eps, tmax)
    at, _, gabs = orc.direct(x, y, z, m)
    gmag = np.linalg.norm(at, axis=0)
    code, walk = CRITERIA[crit]
    s = amfmm.Solver(criterion=code, error_tol=eps, theta_max=tmax)
    X, Y, Z, M = to_dev(x, y, z, m)
    G, = to_dev(gmag)
    s.set_field_estimate(G)
    s.build_tree(X, Y, Z, M)
    s.compute_moments()
    s.walk(0.5)
    far, near = s.get_lists()
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    getattr(t, walk)(eps, tmax, gmag)
    ofar, onear = t.lists()
    assert np.array_equal(far, ofar)
    assert np.array_equal(near, onear)
    ax, ay, az, p = s.evaluate()
    acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
    oacc, opot = t.evaluate(orc.TC)
    assert np.max(np.linalg.norm(acc - oacc, axis=0) / gabs) <= 1e-12
    assert np.max(np.abs(p.cpu().numpy() - opot) / np.abs(opot)) <= 1e-12


def test_multipole_criterion_batched_matches_whole():
    """The multipole criterion walked batch by batch (tiny list budget) selects
    the same pairs (the same interaction counts) and gives the same
    accelerations up to rounding: a cell's pairs may be summed in another order,
    since how a level's frontier is cut into work chunks depends on its size."""
    x, y, z, m = W.plummer(1 << 17, seed=13)
    say("batched multipole", len(x))
    X, Y, Z, M = to_dev(x, y, z, m)
    r = np.sqrt(x * x + y * y + z * z)
    G, = to_dev(r / (r * r + 1.0) ** 1.5)  # Plummer field magnitude (unit mass and scale)
    outs = []
    for lb in (0, 1 << 20):
        s = amfmm.Solver(criterion=amfmm.MULTIPOLE, error_tol=1e-6, theta_max=0.7, list_bytes=lb)
        s.set_field_estimate(G)
        o = s.solve_gravity(X, Y, Z, M, 0.5)
        outs.append((host4(o), s.get_counts()))
    for k in ("near_interactions", "far_evaluations", "walk_candidates"):
        assert outs[0][1][k] == outs[1][1][k] > 0, k
    idx = W.sample_targets(len(x), 256, seed=99)
    _, _, gabs = orc.direct(x, y, z, m, idx)
    a0, a1 = outs[0][0][:3, idx], outs[1][0][:3, idx]
    assert np.max(np.linalg.norm(a0 - a1, axis=0) / gabs) <= 1e-13
    p0, p1 = outs[0][0][3], outs[1][0][3]
    assert np.max(np.abs(p0 - p1) / np.abs(p0)) <= 1e-13


def host4(o):
    return np.stack([v.cpu().numpy() for v in o])


@pytest.mark.parametrize("windows", ["0", "0.02"])
def test_walk_staging_paths(windows, monkeypatch):
    """The walk writes each chunk's pairs to a window, then to spill regions,
    and walks a chunk again when both are full.  Windows shrunk by a test
    factor push chunks into the spill regions and, once the spill pool is
    drained, into the second pass: the lists still equal the oracle's bit for
    bit and the accelerations agree."""
    monkeypatch.setenv("AMFMM_WALK_WINDOWS", windows)
    for name in ("plummer16k", "twoplummer20k"):
        x, y, z, m = CASES[name]()
        say("staging paths", windows, name)
        at, _, gabs = orc.direct(x, y, z, m)
        gmag = np.linalg.norm(at, axis=0)
        X, Y, Z, M = to_dev(x, y, z, m)
        G, = to_dev(gmag)
        t = orc.Tree(x, y, z, m)
        t.compute_moments()
        for crit in ("geometric", "multipole"):
            if crit == "geometric":
                s = amfmm.Solver()
                t.walk(0.5)
            else:
                s = amfmm.Solver(criterion=amfmm.MULTIPOLE, error_tol=1e-6, theta_max=0.5)
                s.set_field_estimate(G)
                t.walk_multipole(1e-6, 0.5, gmag)
            s.build_tree(X, Y, Z, M)
            s.compute_moments()
            s.walk(0.5)
            far, near = s.get_lists()
            ofar, onear = t.lists()
            assert np.array_equal(far, ofar) and np.array_equal(near, onear), (name, crit)
            ax, ay, az, _ = s.evaluate()
            acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
            oacc, _ = t.evaluate(orc.TC)
            assert np.max(np.linalg.norm(acc - oacc, axis=0) / gabs) <= 1e-12, (name, crit)
