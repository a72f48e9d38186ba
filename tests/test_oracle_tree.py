"""Pins of the oracle's keys, sort and octree (Sec. 2: cells of at most
n_crit particles; Morton order, 21 bits per coordinate over the bounding cube).

The reference here is a brute-force recursive octant partition written in
Python on the raw coordinates, independent of the oracle's key arithmetic.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W


def brute_keys(x, y, z):
    lo = np.array([x.min(), y.min(), z.min()])
    side = max(x.max() - lo[0], y.max() - lo[1], z.max() - lo[2])
    if side == 0:
        side = 1.0
    scale = float(1 << 21) / side
    keys = []
    for X in zip(x, y, z):
        q = [min(int(np.floor((X[d] - lo[d]) * scale)), (1 << 21) - 1) for d in range(3)]
        q = [max(v, 0) for v in q]
        bits = ""
        for b in range(20, -1, -1):
            bits += f"{(q[0] >> b) & 1}{(q[1] >> b) & 1}{(q[2] >> b) & 1}"
        keys.append(int(bits, 2))
    return np.array(keys, dtype=np.uint64)


def brute_tree(keys_sorted, n_crit, max_level=21):
    """Return the set of (level, begin, count) of every cell, built by recursive
    partition of index ranges by the octant digit."""
    cells = set()

    def rec(level, b, e):
        cells.add((level, b, e - b))
        if e - b <= n_crit or level >= max_level:
            return
        shift = 3 * (21 - level - 1)
        digits = [(int(k) >> shift) & 7 for k in keys_sorted[b:e]]
        start = b
        for i in range(1, e - b + 1):
            if i == e - b or digits[i] != digits[i - 1]:
                rec(level + 1, start, b + i)
                start = b + i

    rec(0, 0, len(keys_sorted))
    return cells


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (300, 2), (2000, 3)])
def test_keys_and_tree_brute_force(n, seed):
    x, y, z, m = W.plummer(n, seed=seed) if n > 1 else (np.zeros(1),) * 3 + (np.ones(1),)
    t = orc.Tree(x, y, z, m, n_crit=25)
    keys, perm = t.keys()
    bk = brute_keys(x, y, z)
    # stable sort by key: ties keep caller order
    order = np.argsort(bk, kind="stable")
    assert np.array_equal(perm, order)
    assert np.array_equal(keys, bk[order])
    c = t.cells()
    got = set(zip(c["level"].tolist(), c["begin"].tolist(), c["count"].tolist()))
    assert got == brute_tree(bk[order], 25)


def test_tree_invariants_plummer():
    x, y, z, m = W.plummer(20000, seed=7)
    t = orc.Tree(x, y, z, m, n_crit=25)
    c = t.cells()
    nc = t.num_cells
    lev, beg, cnt = c["level"], c["begin"], c["count"]
    par, ch0, nch = c["parent"], c["child0"], c["nchild"]
    # (level, begin) order
    assert np.all(np.diff(lev) >= 0)
    for L in np.unique(lev):
        assert np.all(np.diff(beg[lev == L]) > 0)
    assert lev[0] == 0 and beg[0] == 0 and cnt[0] == len(x)
    for ci in range(nc):
        if nch[ci] == 0:
            assert cnt[ci] <= 25 or lev[ci] == 21
        else:
            assert cnt[ci] > 25
            kids = range(ch0[ci], ch0[ci] + nch[ci])
            assert sum(cnt[k] for k in kids) == cnt[ci]
            assert beg[ch0[ci]] == beg[ci]
            for k in kids:
                assert par[k] == ci and lev[k] == lev[ci] + 1
            for a, b in zip(kids, list(kids)[1:]):
                assert beg[b] == beg[a] + cnt[a]
    # leaves tile the particle range
    leaves = np.where(nch == 0)[0]
    order = np.argsort(beg[leaves])
    lb, lc = beg[leaves][order], cnt[leaves][order]
    assert lb[0] == 0 and np.all(lb[1:] == (lb + lc)[:-1]) and lb[-1] + lc[-1] == len(x)


def test_depth_cap_with_identical_points():
    # 40 copies of one point cannot be separated: the leaf at level 21 keeps them
    x = np.concatenate([np.full(40, 0.5), np.linspace(0, 1, 10)])
    y = np.concatenate([np.full(40, 0.5), np.linspace(0, 1, 10)])
    z = np.concatenate([np.full(40, 0.5), np.linspace(0, 1, 10)])
    m = np.full(50, 0.02)
    t = orc.Tree(x, y, z, m, n_crit=25)
    c = t.cells()
    assert c["count"][c["level"] == 21].max() >= 40
    assert t.depth == 21


@pytest.mark.parametrize("bad", ["nan", "inf", "zero_mass", "neg_mass"])
def test_invalid_inputs_rejected(bad):
    x, y, z, m = W.uniform_cube(64, seed=1)
    x = x.copy()
    m = m.copy()
    if bad == "nan":
        x[3] = np.nan
    elif bad == "inf":
        x[3] = np.inf
    elif bad == "zero_mass":
        m[5] = 0.0
    else:
        m[5] = -1.0
    with pytest.raises(orc.OracleError) as e:
        orc.Tree(x, y, z, m)
    assert e.value.code == (-2 if bad in ("nan", "inf") else -1)


def test_theta_out_of_range_rejected():
    x, y, z, m = W.uniform_cube(64, seed=1)
    for th in (0.0, -0.5, 1.5):
        with pytest.raises(orc.OracleError):
            orc.solve(x, y, z, m, theta=th)
