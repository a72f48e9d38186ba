"""Pins of the oracle's error-estimate walk (the error-based pair selection the
paper's Sec. 2 refers to, in the symmetric form used here): coverage of every
particle pair exactly once, every accepted pair meeting the criterion for both
of its cells (recomputed here from particle data), the tolerance controlling the
accuracy, and the limit of a vanishing tolerance (direct summation)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W


def field_scale(t, gmag):
    """Per-cell scale from the particles of each cell, computed in numpy."""
    c = t.cells()
    keys, perm = t.keys()
    g = np.abs(gmag)[perm]
    s = np.empty(t.num_cells)
    for ci in range(t.num_cells):
        v = g[c["begin"][ci]:c["begin"][ci] + c["count"][ci]]
        s[ci] = max(v.min(), 0.1 * v.mean())
    return s


@pytest.mark.parametrize("eps,tmax", [(1e-3, 0.7), (1e-5, 0.5)])
def test_field_walk_covers_pairs_and_meets_criterion(eps, tmax):
    x, y, z, m = W.two_plummer(800, seed=17)
    a, _, _ = orc.direct(x, y, z, m)
    gmag = np.linalg.norm(a, axis=0)
    t = orc.Tree(x, y, z, m, n_crit=8)
    t.compute_moments()
    t.walk_field(eps, tmax, gmag)
    m2l, p2p = t.lists()
    c = t.cells()
    n = len(x)
    cover = np.zeros((n, n), np.int32)
    rng = lambda ci: slice(c["begin"][ci], c["begin"][ci] + c["count"][ci])
    for A, B in m2l:
        cover[rng(A), rng(B)] += 1
        cover[rng(B), rng(A)] += 1
    for A, B in p2p:
        cover[rng(A), rng(B)] += 1
        if A != B:
            cover[rng(B), rng(A)] += 1
    assert np.all(cover[~np.eye(n, dtype=bool)] == 1)
    mo = t.moments()
    s = field_scale(t, gmag)
    for A, B in m2l:
        d = np.linalg.norm(mo[A, 1:4] - mo[B, 1:4])
        r = mo[A, 4] + mo[B, 4]
        e = (r / d) ** 3 / d**2
        assert r <= tmax * d * (1 + 1e-12)
        assert e * mo[B, 0] <= eps * s[A] * (1 + 1e-9)
        assert e * mo[A, 0] <= eps * s[B] * (1 + 1e-9)
    assert len(m2l) > 0


def test_field_tolerance_controls_error():
    x, y, z, m = W.plummer(6000, seed=18)
    at, _, gabs = orc.direct(x, y, z, m)
    gmag = np.linalg.norm(at, axis=0)
    res = []
    for eps in (1e-3, 1e-4, 1e-5, 1e-6):
        t = orc.Tree(x, y, z, m)
        t.compute_moments()
        t.walk_field(eps, 0.7, gmag)
        a, _ = t.evaluate(orc.TC)
        res.append(np.percentile(orc.rel_force_error(a, at), 99))
    assert all(u > v for u, v in zip(res, res[1:])), res


def test_field_walk_vanishing_tolerance_is_direct_sum():
    x, y, z, m = W.plummer(500, seed=19)
    at, pt, gabs = orc.direct(x, y, z, m)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk_field(1e-30, 1.0, np.linalg.norm(at, axis=0))
    a, p = t.evaluate(orc.TC)
    assert np.max(np.linalg.norm(a - at, axis=0) / gabs) <= 1e-13


def test_field_walk_rejects_bad_arguments():
    x, y, z, m = W.uniform_cube(100, seed=1)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    g = np.ones(100)
    for eps, tm in ((0.0, 0.5), (1e-3, 0.0), (1e-3, 1.5)):
        with pytest.raises(orc.OracleError):
            t.walk_field(eps, tm, g)
