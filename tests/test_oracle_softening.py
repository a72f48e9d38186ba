"""Pins of the oracle's softened Green's function, g = -1/sqrt(R^2 + eps^2)
(Sec. 4: the torque correction carries over to any Green's function of the
distance alone).

Against: finite differences of g (each derivative is the difference of the one
below it), the unsoftened tensors at eps = 0, the closed two-body force
m d / (d^2 + eps^2)^{3/2}, a brute-force numpy direct sum, the direct sum
itself at a vanishing opening angle, and the paper's invariants with
softening (zero net force in every variant, zero net torque with the
correction, error shrinking with theta)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W

from .test_oracle_greens import num_grad

RS = [np.array([1.0, 2.0, 2.0]), np.array([-0.07, 0.03, 0.19]), np.array([3.1, -2.2, -0.4])]


def gs(R, eps):
    return -1.0 / np.sqrt(np.dot(R, R) + eps * eps)


@pytest.mark.parametrize("R", RS)
@pytest.mark.parametrize("eps", [0.05, 0.4])
def test_softened_derivatives_match_finite_differences(R, eps):
    D0, D1, D2, D3, D4, D4p = orc.greens_softened(R, eps)
    assert D0 == pytest.approx(gs(R, eps), rel=1e-15)
    h = 1e-3 * np.sqrt(np.dot(R, R) + eps * eps)
    d1 = num_grad(lambda r: gs(r, eps), R, h)
    d2 = num_grad(lambda r: orc.greens_softened(r, eps)[1], R, h)
    d3 = num_grad(lambda r: orc.greens_softened(r, eps)[2], R, h)
    d4 = num_grad(lambda r: orc.greens_softened(r, eps)[3], R, h)
    for ana, num in ((D1, d1), (D2, d2), (D3, d3), (D4, d4)):
        scale = np.max(np.abs(ana))
        assert np.max(np.abs(ana - num)) <= 1e-8 * scale
    # softened g is not harmonic: the trace of D_ij is -3 eps^2 / s^{5/2} (= lap g)
    s = np.dot(R, R) + eps * eps
    assert np.trace(D2) == pytest.approx(3.0 * eps * eps / s**2.5, rel=1e-12)
    # D' differs from D_ijkl only by terms along R_i (no torque): R x (D - D')_i.. = 0
    diff = D4 - D4p
    t = np.einsum("pkr,p,kjlm->rjlm", np.array([[[0, 0, 0], [0, 0, 1], [0, -1, 0]],
                                               [[0, 0, -1], [0, 0, 0], [1, 0, 0]],
                                               [[0, 1, 0], [-1, 0, 0], [0, 0, 0]]], float), R, diff)
    assert np.max(np.abs(t)) <= 1e-13 * np.abs(D4).max()


@pytest.mark.parametrize("R", RS)
def test_zero_softening_is_the_plain_kernel(R):
    a = orc.greens_softened(R, 0.0)
    b = orc.greens(R)
    for u, v in zip(a, b):
        assert np.allclose(u, v, rtol=1e-14, atol=1e-14 * np.max(np.abs(v)))


def test_two_body_softened_closed_form():
    eps = 0.3
    x, y, z = np.array([0.2, 1.4]), np.array([-0.1, 0.5]), np.array([0.0, 0.3])
    m = np.array([2.0, 0.5])
    a, p = orc.solve(x, y, z, m, theta=0.5, softening=eps)
    d = np.array([x[1] - x[0], y[1] - y[0], z[1] - z[0]])
    s = np.dot(d, d) + eps * eps
    assert np.allclose(a[:, 0], m[1] * d / s**1.5, rtol=1e-14, atol=0)
    assert np.allclose(a[:, 1], -m[0] * d / s**1.5, rtol=1e-14, atol=0)
    assert p[0] == pytest.approx(-m[1] / np.sqrt(s), rel=1e-14)


def test_softened_direct_sum_brute_force():
    x, y, z, m = W.plummer(300, seed=4)
    eps = 0.02
    a, p, gabs = orc.direct(x, y, z, m, softening=eps)
    P = np.stack([x, y, z])
    d = P[:, None, :] - P[:, :, None]  # d[:, i, j] = X_j - X_i
    r2 = (d**2).sum(0)
    s = r2 + eps * eps
    np.fill_diagonal(s, np.inf)
    ref = (m[None, None, :] * d / s[None] ** 1.5).sum(2)
    assert np.max(np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)) <= 1e-13
    assert np.max(np.abs(p - (-(m[None, :] / np.sqrt(s)).sum(1))) / np.abs(p)) <= 1e-13
    assert np.max(np.abs(gabs - (m[None, :] / s).sum(1)) / gabs) <= 1e-13


def test_softened_solve_at_tiny_theta_is_direct():
    x, y, z, m = W.plummer(600, seed=5)
    eps = 0.01
    t = orc.Tree(x, y, z, m, softening=eps)
    t.compute_moments()
    t.walk(1e-6)
    a, p = t.evaluate(orc.TC)
    at, pt, gabs = orc.direct(x, y, z, m, softening=eps)
    assert np.max(np.linalg.norm(a - at, axis=0) / gabs) <= 1e-13
    assert np.max(np.abs(p - pt) / np.abs(pt)) <= 1e-13


def test_zero_softening_is_bitwise_the_plain_solve():
    x, y, z, m = W.two_plummer(3000, seed=3)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk(0.5)
    a, p = t.evaluate(orc.TC)
    t.set_softening(0.0)
    b, q = t.evaluate(orc.TC)
    assert np.array_equal(a, b) and np.array_equal(p, q)


def test_softened_invariants_and_convergence():
    x, y, z, m = W.two_plummer(4000, seed=12)
    eps = 0.02
    at, _, _ = orc.direct(x, y, z, m, softening=eps)
    pos = np.stack([x, y, z])
    t = orc.Tree(x, y, z, m, softening=eps)
    t.compute_moments()
    means = []
    for th in (0.3, 0.5, 0.8):
        t.walk(th)
        res = {}
        for v in (orc.UC, orc.TC, orc.TCO):
            a, _ = t.evaluate(v)
            res[v] = (orc.balance(m, a), orc.balance(m, orc.angular(pos, a)), orc.rel_force_error(a, at).mean())
        for v in res:
            assert res[v][0] <= 1e-14, (th, res)
        assert res[orc.TC][1] <= 1e-14 and res[orc.TCO][1] <= 1e-14, (th, res)
        assert res[orc.UC][1] >= 1e3 * res[orc.TC][1], (th, res)
        means.append(res[orc.TC][2])
    assert means[0] < means[1] < means[2], means
