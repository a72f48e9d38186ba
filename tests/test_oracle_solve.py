"""Whole-solve pins of the oracle (Sec. 2 method, Sec. 3 metrics).

Against: exact direct summation (tiny N and the 4096-particle uniform cube),
the cases where the method reduces to direct summation (one leaf; tiny
theta), coverage of every particle pair exactly once, closed forms (two
distant clusters, uniform-sphere and Plummer radial accelerations), and the
paper's invariants (zero net force for every variant, zero net torque for the
corrected ones, error shrinking with theta, TC error close to UC error).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W

from .walk_check import check_walk, geometric_accept


def test_single_leaf_equals_direct_sum():
    x, y, z, m = W.uniform_cube(25, seed=3)
    a, p = orc.solve(x, y, z, m, theta=0.5)
    at, pt, gabs = orc.direct(x, y, z, m)
    assert np.max(np.abs(a - at) / gabs) <= 1e-14
    assert np.max(np.abs(p - pt) / np.abs(pt)) <= 1e-14


def test_tiny_theta_equals_direct_sum():
    # with theta this small only single-particle pairs (exact) are accepted
    x, y, z, m = W.plummer(600, seed=5)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk(1e-6)
    a, p = t.evaluate(orc.TC)
    at, pt, gabs = orc.direct(x, y, z, m)
    assert np.max(np.linalg.norm(a - at, axis=0) / gabs) <= 1e-13
    assert np.max(np.abs(p - pt) / np.abs(pt)) <= 1e-13


@pytest.mark.parametrize("theta", [0.3, 0.7, 1.0])
def test_every_particle_pair_covered_once(theta):
    x, y, z, m = W.two_plummer(700, seed=6)
    t = orc.Tree(x, y, z, m, n_crit=8)
    t.compute_moments()
    t.walk(theta)
    m2l, p2p = t.lists()
    c = t.cells()
    keys, perm = t.keys()
    n = len(x)
    cover = np.zeros((n, n), np.int32)

    def rng_(ci):
        return slice(c["begin"][ci], c["begin"][ci] + c["count"][ci])

    for a, b in m2l:
        assert a < b
        cover[rng_(a), rng_(b)] += 1
        cover[rng_(b), rng_(a)] += 1
    for a, b in p2p:
        assert a <= b
        cover[rng_(a), rng_(b)] += 1
        if a != b:
            cover[rng_(b), rng_(a)] += 1
    off = ~np.eye(n, dtype=bool)
    assert np.all(cover[off] == 1)
    # the lists are sorted and free of duplicates
    assert len({tuple(v) for v in m2l}) == len(m2l)
    assert len({tuple(v) for v in p2p}) == len(p2p)
    # every accepted pair meets the opening criterion
    mo = t.moments()
    for a, b in m2l:
        d = np.linalg.norm(mo[a, 1:4] - mo[b, 1:4])
        assert d >= (mo[a, 4] + mo[b, 4]) / theta


@pytest.mark.parametrize("theta", [0.3, 0.7, 1.0])
def test_walk_is_complete(theta):
    """The lists hold exactly the walk's terminal pairs: no pair is split that
    the criterion accepts, and no leaf pair that it accepts goes to the near
    field (checked bottom-up, see walk_check)."""
    x, y, z, m = W.two_plummer(700, seed=6)
    t = orc.Tree(x, y, z, m, n_crit=8)
    t.compute_moments()
    t.walk(theta)
    m2l, p2p = t.lists()
    mo = t.moments()
    check_walk(t.cells(), mo, m2l, p2p, geometric_accept(mo, theta))
    # the lists of a walk 1.25 times more conservative than the criterion
    # (a covering, self-consistent walk at a smaller angle) fail the check
    t.walk(theta / 1.25)
    m2l_c, p2p_c = t.lists()
    with pytest.raises(AssertionError):
        check_walk(t.cells(), mo, m2l_c, p2p_c, geometric_accept(mo, theta))


@pytest.fixture(scope="module")
def cube4k():
    x, y, z, m = W.make("uniform4k")
    at, pt, gabs = orc.direct(x, y, z, m)
    return (x, y, z, m), at, pt, gabs


def test_uniform4k_against_direct_sum(cube4k):
    (x, y, z, m), at, pt, gabs = cube4k
    eps = {}
    for th in (0.3, 0.5, 0.7, 0.9):
        a, p = orc.solve(x, y, z, m, theta=th, variant=orc.TC)
        e = orc.rel_force_error(a, at)
        eps[th] = (e.mean(), np.percentile(e, 99))
        # potentials: one order looser than forces, relative to |phi|
        assert np.percentile(np.abs(p - pt) / np.abs(pt), 99) < 10 * eps[th][1]
    means = [eps[t][0] for t in (0.3, 0.5, 0.7, 0.9)]
    assert all(a < b for a, b in zip(means, means[1:])), eps
    assert eps[0.5][0] < 1e-2 and eps[0.3][0] < 2e-3, eps


def test_balances_uniform4k(cube4k):
    (x, y, z, m), at, pt, gabs = cube4k
    pos = np.stack([x, y, z])
    res = {}
    for v in (orc.UC, orc.TC, orc.TCO):
        a, _ = orc.solve(x, y, z, m, theta=0.5, variant=v)
        res[v] = (orc.balance(m, a), orc.balance(m, orc.angular(pos, a)),
                  orc.rel_force_error(a, at).mean())
    for v in res:
        assert res[v][0] <= 1e-14, res  # net force: every variant
    assert res[orc.TC][1] <= 1e-14 and res[orc.TCO][1] <= 1e-14, res
    assert res[orc.UC][1] >= 1e3 * res[orc.TC][1], res
    # the correction costs no accuracy (TC ~ UC); TCO is no better than TC
    assert 0.8 < res[orc.TC][2] / res[orc.UC][2] < 1.25, res
    assert res[orc.TCO][2] >= 0.99 * res[orc.TC][2], res


def test_distant_clusters_act_as_point_masses():
    x1, y1, z1, _ = W.uniform_sphere(400, seed=1, radius=0.05)
    x2, y2, z2, _ = W.uniform_sphere(300, seed=2, radius=0.05)
    D = 10.0
    x = np.concatenate([x1, x2 + D])
    y = np.concatenate([y1, y2])
    z = np.concatenate([z1, z2])
    m = np.concatenate([np.full(400, 2.0 / 400), np.full(300, 1.0 / 300)])
    a, _ = orc.solve(x, y, z, m, theta=0.5)
    # cluster 1 (mass 2) is pulled towards +x with 1/D^2, cluster 2 with 2/D^2
    g1 = a[0, :400]
    g2 = a[0, 400:]
    # internal fields average out over the cluster (force balance within it)
    assert abs(np.average(g1, weights=m[:400]) - 1.0 / D**2) <= 1e-3 / D**2
    assert abs(np.average(g2, weights=m[400:]) + 2.0 / D**2) <= 1e-3 / D**2


def test_uniform_sphere_radial_field():
    """Inside a uniform ball of mass 1, g_r = -r (radius 1), in shell means."""
    x, y, z, m = W.uniform_sphere(40000, seed=21)
    a, _ = orc.solve(x, y, z, m, theta=0.5)
    r = np.sqrt(x * x + y * y + z * z)
    gr = (a[0] * x + a[1] * y + a[2] * z) / r
    for lo, hi in ((0.3, 0.4), (0.5, 0.6), (0.7, 0.8)):
        s = (r >= lo) & (r < hi)
        rm = r[s].mean()
        assert abs(gr[s].mean() + rm) <= 0.03 * rm


def test_plummer_radial_field():
    """Truncated Plummer sphere: g_r = -M(<r)/r^2 with M(<r) = r^3/(1+r^2)^{3/2}
    divided by the mass fraction inside the truncation radius."""
    x, y, z, m = W.plummer(40000, seed=22)
    a, _ = orc.solve(x, y, z, m, theta=0.5)
    r = np.sqrt(x * x + y * y + z * z)
    gr = (a[0] * x + a[1] * y + a[2] * z) / r
    frac = 20.0**3 / (1 + 20.0**2) ** 1.5
    for lo, hi in ((0.5, 0.6), (1.0, 1.2), (2.0, 2.5)):
        s = (r >= lo) & (r < hi)
        rm = r[s].mean()
        expect = -(rm**3 / (1 + rm * rm) ** 1.5) / frac / rm**2
        assert abs(gr[s].mean() - expect) <= 0.04 * abs(expect)


def test_coincident_particles_are_skipped():
    x, y, z, m = W.uniform_cube(200, seed=9)
    x = np.concatenate([x, x[:5]])
    y = np.concatenate([y, y[:5]])
    z = np.concatenate([z, z[:5]])
    m = np.full(len(x), 1.0 / len(x))
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk(0.5)
    a, p = t.evaluate()
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(p))
    assert t.coincident == 5


def test_sampled_evaluation_matches_full():
    x, y, z, m = W.two_plummer(5000, seed=31)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk(0.6)
    for v in (orc.UC, orc.TC):
        a, p = t.evaluate(v)
        idx = W.sample_targets(len(x), 300, seed=4)
        s, q = t.evaluate_sample(idx, v)
        _, _, gabs = orc.direct(x, y, z, m, idx)
        assert np.max(np.linalg.norm(s - a[:, idx], axis=0) / gabs) <= 1e-14
        assert np.max(np.abs(q - p[idx]) / np.abs(p[idx])) <= 1e-14


def test_target_ordered_evaluation_matches():
    """The target-ordered evaluation (the CPU baseline's, on all cores in the
    OpenMP build) equals the pair-ordered one up to summation order, and the
    OpenMP build gives the serial build's result bit for bit."""
    import os
    import subprocess
    import sys

    x, y, z, m = W.two_plummer(3000, seed=8)
    x = np.concatenate([x, x[:3]])  # coincident points: counted once per pair
    y = np.concatenate([y, y[:3]])
    z = np.concatenate([z, z[:3]])
    m = np.full(len(x), 1.0 / len(x))
    t = orc.Tree(x, y, z, m, n_crit=12)
    t.compute_moments()
    t.walk(0.6)
    _, _, gabs = orc.direct(x, y, z, m)
    for v in (orc.UC, orc.TC, orc.TCO):
        a, p = t.evaluate(v)
        c1 = t.coincident
        b, q = t.evaluate_targets(v)
        assert t.coincident == c1 == 3
        assert np.max(np.linalg.norm(a - b, axis=0) / gabs) <= 1e-14
        assert np.max(np.abs(p - q) / np.abs(p)) <= 1e-14
    from oracle.build import ensure_built_omp
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, numpy as np; sys.path.insert(0, %r)\n"
            "from oracle import oracle as orc\nfrom paper_1706_06989_amd import workloads as W\n"
            "x, y, z, m = W.two_plummer(3000, seed=8)\n"
            "t = orc.Tree(x, y, z, m, n_crit=12); t.compute_moments(); t.walk(0.6)\n"
            "a, p = t.evaluate_targets(orc.TC)\n"
            "sys.stdout.buffer.write(np.concatenate([a.ravel(), p]).tobytes())\n" % root)
    outs = []
    for lib in (None, ensure_built_omp()):
        env = dict(os.environ, OMP_NUM_THREADS="4")
        env.pop("AMFMM_ORACLE_LIB", None)
        if lib:
            env["AMFMM_ORACLE_LIB"] = lib
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                   check=True).stdout)
    assert len(outs[0]) == 8 * 4 * 3000 and outs[0] == outs[1]
