"""Pins of the oracle's upward pass: M (eq. 1), the centre of mass Z, the
dipole about Z (which must vanish, Sec. 2), M_ij (eq. quad), the octupole
M_ijk, and R_max (Sec. 2, opening criterion).  The reference is a vectorised
numpy evaluation of the definitions over each cell's particle range.
"""
import numpy as np

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W

IDX2 = [(i, j) for i in range(3) for j in range(i, 3)]
IDX3 = [(i, j, k) for i in range(3) for j in range(i, 3) for k in range(j, 3)]


def test_moments_match_definitions():
    x, y, z, m = W.two_plummer(6000, seed=4)
    t = orc.Tree(x, y, z, m, n_crit=25)
    t.compute_moments()
    mo = t.moments()
    keys, perm = t.keys()
    P = np.stack([x, y, z])[:, perm]
    ms = m[perm]
    c = t.cells()
    for ci in range(t.num_cells):
        b, n = c["begin"][ci], c["count"][ci]
        X = P[:, b:b + n]
        mu = ms[b:b + n]
        M = mu.sum()
        Z = (X * mu).sum(axis=1) / M
        assert abs(mo[ci, 0] - M) <= 1e-14 * M
        np.testing.assert_allclose(mo[ci, 1:4], Z, rtol=0, atol=1e-13 * (1 + np.abs(Z).max()))
        x_ = X - mo[ci, 1:4, None]
        # dipole about the centre of mass vanishes to round-off
        dip = (x_ * mu).sum(axis=1)
        assert np.abs(dip).max() <= 1e-13 * M * (np.abs(X).max() + 1e-300)
        r = np.sqrt((x_ ** 2).sum(axis=0))
        assert abs(mo[ci, 4] - r.max()) <= 1e-14 * (r.max() + 1e-300)
        M2 = np.einsum("n,in,jn->ij", mu, x_, x_)
        M3 = np.einsum("n,in,jn,kn->ijk", mu, x_, x_, x_)
        s2 = M * r.max() ** 2 + 1e-300
        s3 = M * r.max() ** 3 + 1e-300
        for q, (i, j) in enumerate(IDX2):
            assert abs(mo[ci, 5 + q] - M2[i, j]) <= 1e-13 * s2
        for q, (i, j, k) in enumerate(IDX3):
            assert abs(mo[ci, 11 + q] - M3[i, j, k]) <= 1e-13 * s3


def test_single_particle_cell_has_no_extent():
    x, y, z, m = W.uniform_cube(3, seed=2)
    t = orc.Tree(x, y, z, m, n_crit=1)
    t.compute_moments()
    mo = t.moments()
    c = t.cells()
    single = c["count"] == 1
    assert single.sum() == 3
    assert np.all(mo[single, 4] == 0.0)
    assert np.all(mo[single, 5:] == 0.0)


def test_parent_mass_is_sum_of_children():
    x, y, z, m = W.plummer(5000, seed=8)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    mo = t.moments()
    c = t.cells()
    for ci in np.where(c["nchild"] > 0)[0]:
        kids = range(c["child0"][ci], c["child0"][ci] + c["nchild"][ci])
        assert abs(sum(mo[k, 0] for k in kids) - mo[ci, 0]) <= 1e-15 * mo[ci, 0] * 8
