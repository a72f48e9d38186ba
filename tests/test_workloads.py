"""The seeded input generators draw what their docstrings state: Plummer radii
follow the truncated cumulative mass profile M(<r) = r^3/(1+r^2)^{3/2} (a
Kolmogorov-Smirnov distance within the 99.9 % bound), directions are
isotropic, the two-sphere set has the stated counts, centres and centre of
mass, masses are equal, and every draw is reproducible from its seed."""
import numpy as np

from paper_1706_06989_amd import workloads as W


def plummer_cdf(r, a=1.0, rt=W.PLUMMER_RTRUNC):
    m = lambda s: (s / a) ** 3 / (1.0 + (s / a) ** 2) ** 1.5
    return m(r) / m(rt)


def ks_distance(samples, cdf):
    s = np.sort(samples)
    n = len(s)
    f = cdf(s)
    return max(np.max(np.arange(1, n + 1) / n - f), np.max(f - np.arange(n) / n))


def test_plummer_radii_follow_the_truncated_mass_profile():
    n = 20000
    for a in (1.0, 2.5):
        r = W._plummer_radii(np.random.default_rng(7), n, a, W.PLUMMER_RTRUNC * a)
        assert r.max() <= W.PLUMMER_RTRUNC * a * (1 + 1e-12) and r.min() > 0.0
        assert ks_distance(r, lambda s: plummer_cdf(s, a, W.PLUMMER_RTRUNC * a)) <= 1.95 / np.sqrt(n)
    # half of the mass lies within r = a / sqrt(2^{2/3} - 1) = 1.305 a (1.300 a
    # with the truncation at 20 a)
    r = W._plummer_radii(np.random.default_rng(8), 200000)
    assert abs(np.median(r) - 1.0 / np.sqrt(2.0 ** (2.0 / 3.0) - 1.0)) <= 0.02
    # a sphere of scale radius 2.5 is truncated at 20 of its own scale radii
    x, y, z, _ = W.plummer(20000, seed=9, a=2.5)
    r = np.sqrt(x * x + y * y + z * z)
    assert r.max() <= 50.0 * 1.01 and np.sum(r > 20.0) > 100


def test_plummer_sphere_is_isotropic_and_centred():
    x, y, z, m = W.plummer(20000, seed=2)
    r = np.sqrt(x * x + y * y + z * z)
    for c in (x, y, z):
        assert abs(np.mean(c)) <= 1e-14 * np.max(np.abs(c))  # recentred on its centre of mass
        assert abs(np.mean(c / r)) <= 4.0 / np.sqrt(3 * len(x))
    assert np.all(m == 1.0 / len(x)) and abs(m.sum() - 1.0) <= 1e-12


def test_two_spheres_counts_centres_and_centre_of_mass():
    n = 30001
    x, y, z, m = W.two_plummer(n, seed=3)
    n2 = n // 3
    n1 = n - n2
    assert len(x) == n and np.all(m == 1.0 / n)
    # the heavier sphere (first n1 particles) about x = -1, the lighter about x = +2
    assert abs(np.median(x[:n1]) + 1.0) <= 0.05 and abs(np.median(x[n1:]) - 2.0) <= 0.05
    assert abs(np.median(y[:n1])) <= 0.05 and abs(np.median(z[n1:])) <= 0.05
    # centre of mass near the origin: (n1 (-1) + n2 (2)) / n plus sampling noise
    com = np.array([np.mean(x), np.mean(y), np.mean(z)])
    assert abs(com[0] - (-n1 + 2 * n2) / n) <= 0.1 and np.all(np.abs(com[1:]) <= 0.1)


def test_uniform_sets_and_sample_targets():
    x, y, z, m = W.uniform_cube(5000, seed=1)
    for c in (x, y, z):
        assert c.min() >= 0.0 and c.max() < 1.0 and abs(c.mean() - 0.5) <= 0.02
    x, y, z, _ = W.uniform_sphere(5000, seed=4)
    r = np.sqrt(x * x + y * y + z * z)
    assert r.max() <= 1.0 and ks_distance(r, lambda s: s ** 3) <= 1.95 / np.sqrt(5000)
    t = W.sample_targets(1000, 300, seed=99)
    assert t.dtype == np.int64 and len(np.unique(t)) == 300 and np.all(np.diff(t) > 0)
    assert t.min() >= 0 and t.max() < 1000
    assert np.array_equal(W.sample_targets(10, 300), np.arange(10))


def test_draws_are_reproducible_and_named_workloads_have_their_sizes():
    a = W.make("twoplummer4m", n=4096)
    b = W.two_plummer(4096, seed=3)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert not np.array_equal(W.plummer(4096, seed=4)[0], W.plummer(4096, seed=5)[0])
    assert W.CONFIGS["plummer16m"]["n"] == 1 << 24 and W.CONFIGS["twoplummer16m"]["seed"] == 5
