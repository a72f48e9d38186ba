"""Pins of the oracle's general expansion order (the appendix: the expansion
of the Green's function to order P in both cells' offsets and the corrective
force that cancels the pair torque at that order).

The derivatives of any order are pinned against the printed tensors (order
<= 4, plain and softened), finite differences and harmonicity; the general
form at P = 3 against the printed equations; the order of convergence
against direct sums; and at every P the two conservation laws: zero net force
for UC and TC, zero net torque with the correction (and not without it)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W


def tuple_of(e):
    return tuple([0] * int(e[0]) + [1] * int(e[1]) + [2] * int(e[2]))


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_general_derivatives_match_printed_tensors(eps):
    rng = np.random.default_rng(5)
    mi = orc.multi_indices(4)
    for _ in range(5):
        R = rng.normal(size=3) * 2.0
        D = orc.greens_general(R, 4, eps)
        ref = orc.greens_softened(R, eps) if eps else orc.greens(R)
        full = ref[:5]  # D0, D1, D2, D3, D4
        for k, e in enumerate(mi):
            t = tuple_of(e)
            want = full[0] if len(t) == 0 else full[len(t)][t]
            assert abs(D[k] - want) <= 1e-13 * max(1.0, abs(want)), (e, D[k], want)


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_higher_derivatives_by_finite_differences(eps):
    """Orders 5-7: D_(gamma + e_k) against central differences of D_gamma."""
    mi = orc.multi_indices(7)
    index = {tuple(e): k for k, e in enumerate(mi)}
    R = np.array([1.3, -0.7, 0.9])
    h = 1e-5
    D = orc.greens_general(R, 7, eps)
    for k, e in enumerate(mi):
        n = int(e.sum())
        if n < 4 or n > 6:
            continue
        for d in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[d] += h
            Rm[d] -= h
            fd = (orc.greens_general(Rp, n, eps)[k] - orc.greens_general(Rm, n, eps)[k]) / (2 * h)
            up = list(e)
            up[d] += 1
            exact = D[index[tuple(up)]]
            assert abs(fd - exact) <= 1e-6 * max(1.0, abs(exact)), (e, d, fd, exact)


def test_plain_derivatives_are_harmonic():
    """1/R is harmonic: sum_k D_(gamma + 2 e_k) = 0 at every order."""
    mi = orc.multi_indices(7)
    index = {tuple(e): k for k, e in enumerate(mi)}
    R = np.array([0.8, 1.1, -0.6])
    D = orc.greens_general(R, 7)
    for e in mi:
        if e.sum() > 5:
            continue
        terms = []
        for d in range(3):
            up = list(e)
            up[d] += 2
            terms.append(D[index[tuple(up)]])
        assert abs(sum(terms)) <= 1e-12 * max(abs(v) for v in terms)


def clusters(seed=0):
    rng = np.random.default_rng(seed)

    def cluster(n, c, r):
        p = rng.normal(size=(3, n))
        p *= r * rng.random(n) ** (1 / 3) / np.linalg.norm(p, axis=0)
        return (p[0] + c[0], p[1] + c[1], p[2] + c[2], rng.uniform(0.5, 1.5, n))

    return cluster


@pytest.mark.parametrize("variant", [orc.UC, orc.TC])
def test_general_form_at_order_three_is_the_printed_one(variant):
    cluster = clusters(1)
    A = cluster(40, (0.0, 0.0, 0.0), 1.0)
    B = cluster(30, (5.0, 1.0, -2.0), 0.8)
    ref = orc.pair_far(A, B, variant, 3)
    gen = orc.pair_far(A, B, variant, 3, general=True)
    for k in range(4):
        assert np.max(np.abs(gen[k] - ref[k])) <= 1e-14 * np.max(np.abs(ref[k]))
    # and through a whole tree
    x, y, z, m = W.plummer(4096, seed=3)
    _, _, gabs = orc.direct(x, y, z, m)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk(0.5)
    a3, p3 = t.evaluate(variant)
    t.set_order(3, general=True)
    ag, pg = t.evaluate(variant)
    assert np.max(np.linalg.norm(ag - a3, axis=0) / gabs) <= 1e-14
    assert np.max(np.abs(pg - p3) / np.abs(p3)) <= 1e-14


def direct_on(A, B):
    xa, xb = np.stack(A[:3]), np.stack(B[:3])
    d = xb[:, None, :] - xa[:, :, None]
    r3 = np.sqrt((d ** 2).sum(0)) ** 3
    return (B[3][None, :] * d / r3).sum(2).T


@pytest.mark.parametrize("P", [2, 3, 4, 5])
def test_force_error_falls_as_the_order(P):
    """The forces keep the terms m + n <= P - 1, so the relative error of a
    pair falls as (r/d)^P: from d = 16 to 32 by 2^P (within a factor 2^0.6)."""
    cluster = clusters(2)
    A = cluster(40, (0.0, 0.0, 0.0), 1.0)
    err = []
    for d in (16.0, 32.0):
        B = cluster(30, (0.6 * d, 0.64 * d, 0.48 * d), 0.8)
        g = orc.pair_far(A, B, orc.UC, P)[0]
        t = direct_on(A, B)
        err.append(np.max(np.linalg.norm(g - t, axis=1)) / np.max(np.linalg.norm(t, axis=1)))
    slope = np.log2(err[0] / err[1])
    assert abs(slope - P) <= 0.6, (P, err, slope)


@pytest.mark.parametrize("P", [2, 4, 5])
def test_conservation_at_any_order(P):
    """Zero net force for UC and TC; zero net torque with the correction at
    order P, a visible one without it; and order 4 more accurate than 3."""
    x, y, z, m = W.plummer(4096, seed=3)
    at, _, _ = orc.direct(x, y, z, m)
    pos = np.stack([x, y, z])
    res = {}
    for v in (orc.UC, orc.TC):
        a, _ = orc.solve(x, y, z, m, 0.5, variant=v, order=P)
        F = (m * a).sum(1)
        T = (m * np.cross(pos.T, a.T).T).sum(1)
        fs = (m * np.linalg.norm(a, axis=0)).sum()
        ts = (m * np.linalg.norm(pos, axis=0) * np.linalg.norm(a, axis=0)).sum()
        res[v] = (np.linalg.norm(F) / fs, np.linalg.norm(T) / ts,
                  np.percentile(np.linalg.norm(a - at, axis=0) / np.linalg.norm(at, axis=0), 99))
    assert res[orc.UC][0] <= 1e-15 and res[orc.TC][0] <= 1e-15
    assert res[orc.TC][1] <= 1e-15
    assert res[orc.UC][1] >= 1e-7
    if P == 4:
        a3, _ = orc.solve(x, y, z, m, 0.5, variant=orc.TC)
        e3 = np.percentile(np.linalg.norm(a3 - at, axis=0) / np.linalg.norm(at, axis=0), 99)
        assert res[orc.TC][2] <= 0.5 * e3


def test_tco_only_in_the_printed_form():
    x, y, z, m = W.uniform_cube(512, seed=1)
    t = orc.Tree(x, y, z, m, order=4)
    t.compute_moments()
    t.walk(0.5)
    with pytest.raises(orc.OracleError):
        t.evaluate(orc.TCO)
    with pytest.raises(orc.OracleError):
        t.set_order(7)
