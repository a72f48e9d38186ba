"""Seeded synthetic particle sets (host, FP64).

This module only draws inputs; it holds none of the solver's arithmetic and is
shared by the GPU tests, the oracle tests and the benchmark.  Every generator
uses numpy's PCG64 ``default_rng(seed)`` and returns ``(x, y, z, m)`` as
contiguous float64 arrays with equal masses 1/N (total mass 1).

The paper's own test problem (a double white dwarf of two Lane-Emden
polytropes, Sec. 3) is not fully specified (no separation, no Roche-lobe
volume); the two-Plummer set stands in for its two-component, unequal-mass,
centrally condensed structure.
"""
import numpy as np

PLUMMER_RTRUNC = 20.0


def _equal_masses(n):
    return np.full(n, 1.0 / n)


def uniform_cube(n, seed=1):
    """Uniform in [0,1)^3: three arrays x, y, z drawn in that order."""
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    y = rng.random(n)
    z = rng.random(n)
    return x, y, z, _equal_masses(n)


def uniform_sphere(n, seed=1, radius=1.0):
    """Uniform ball of the given radius about the origin."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    c = rng.uniform(-1.0, 1.0, n)
    p = rng.uniform(0.0, 2.0 * np.pi, n)
    r = radius * np.cbrt(u)
    s = np.sqrt(1.0 - c * c)
    return r * s * np.cos(p), r * s * np.sin(p), r * c, _equal_masses(n)


def _plummer_radii(rng, n, a=1.0, rtrunc=PLUMMER_RTRUNC):
    # cumulative mass fraction of a Plummer sphere, M(<r) = r^3 / (r^2 + a^2)^{3/2}
    # (scale radius a, unit mass), inverted for a uniform draw below the
    # truncation radius
    xmax = (rtrunc / a) ** 3 / (1.0 + (rtrunc / a) ** 2) ** 1.5
    X = rng.uniform(0.0, xmax, n)
    X = np.maximum(X, np.finfo(np.float64).tiny)
    return a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)


def _plummer_points(rng, n, a=1.0):
    r = _plummer_radii(rng, n, a, PLUMMER_RTRUNC * a)  # truncated at 20 scale radii
    c = rng.uniform(-1.0, 1.0, n)
    p = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - c * c)
    return r * s * np.cos(p), r * s * np.sin(p), r * c


def plummer(n, seed=2, a=1.0):
    """Plummer sphere, scale radius a, truncated at 20 a, centred on its own
    centre of mass (so torques about the origin are torques about the COM)."""
    rng = np.random.default_rng(seed)
    x, y, z = _plummer_points(rng, n, a)
    x -= x.mean()
    y -= y.mean()
    z -= z.mean()
    return x, y, z, _equal_masses(n)


def two_plummer(n, seed=3, a=1.0, a2=None):
    """Two Plummer spheres (truncated at 20 scale radii) with particle counts
    N - N//3 and N//3 (mass ratio ~0.5), centred at (-a, 0, 0) and (+2a, 0, 0),
    i.e. three scale radii apart with the combined centre of mass near the
    origin.  ``a2`` optionally gives the lighter sphere its own scale radius."""
    rng = np.random.default_rng(seed)
    n2 = n // 3
    n1 = n - n2
    x1, y1, z1 = _plummer_points(rng, n1, a)
    x2, y2, z2 = _plummer_points(rng, n2, a if a2 is None else a2)
    x = np.concatenate([x1 - a, x2 + 2.0 * a])
    y = np.concatenate([y1, y2])
    z = np.concatenate([z1, z2])
    return x, y, z, _equal_masses(n)


def _plummer_speeds(rng, r, mass, a):
    """Speeds of an isotropic Plummer sphere in equilibrium (G = 1) at radii r:
    q v_esc(r), v_esc^2 = 2 mass / sqrt(r^2 + a^2), with q drawn from the
    density q^2 (1 - q^2)^{7/2} on [0, 1] by rejection under the constant 0.1
    (Aarseth, Henon & Wielen 1974)."""
    q = np.empty(len(r))
    todo = np.arange(len(r))
    while len(todo):
        x = rng.random(len(todo))
        y = 0.1 * rng.random(len(todo))
        ok = y < x * x * (1.0 - x * x) ** 3.5
        q[todo[ok]] = x[ok]
        todo = todo[~ok]
    return q * np.sqrt(2.0 * mass / np.sqrt(r * r + a * a))


def _isotropic(rng, v):
    c = rng.uniform(-1.0, 1.0, len(v))
    p = rng.uniform(0.0, 2.0 * np.pi, len(v))
    s = np.sqrt(1.0 - c * c)
    return v * s * np.cos(p), v * s * np.sin(p), v * c


def two_plummer_binary(n, seed=7, a=1.0):
    """Positions and velocities of a bound binary: the two spheres of
    ``two_plummer`` (same seed stream for the positions), each given isotropic
    equilibrium velocities about its own centre, the two centres on a circular
    orbit about their common centre of mass in the x-y plane (separation 3a,
    angular speed sqrt(M / (3a)^3)).  Returns (x, y, z, m, vx, vy, vz); the
    orbital period is 2 pi / sqrt(M / (3a)^3), about 32.6 for a = 1, M = 1."""
    x, y, z, m = two_plummer(n, seed=seed, a=a)
    n2 = n // 3
    n1 = n - n2
    rng = np.random.default_rng(seed + 1000)
    vel = []
    for lo, hi, cx in ((0, n1, -a), (n1, n, 2.0 * a)):
        r = np.sqrt((x[lo:hi] - cx) ** 2 + y[lo:hi] ** 2 + z[lo:hi] ** 2)
        vel.append(_isotropic(rng, _plummer_speeds(rng, r, m[lo:hi].sum(), a)))
    vx, vy, vz = (np.concatenate([vel[0][k], vel[1][k]]) for k in range(3))
    m1, m2 = m[:n1].sum(), m[n1:].sum()
    d = 3.0 * a
    w = np.sqrt((m1 + m2) / d**3)
    com = (m1 * -a + m2 * 2.0 * a) / (m1 + m2)
    cx = np.concatenate([np.full(n1, -a), np.full(n2, 2.0 * a)])
    vy += w * (cx - com)
    # no net momentum
    vx -= np.average(vx, weights=m)
    vy -= np.average(vy, weights=m)
    vz -= np.average(vz, weights=m)
    return x, y, z, m, vx, vy, vz


# The five workloads the solver is specified on (sizes, seeds, shapes).
CONFIGS = {
    "uniform4k": dict(gen=uniform_cube, n=4096, seed=1),
    "plummer1m": dict(gen=plummer, n=1 << 20, seed=2),
    "twoplummer4m": dict(gen=two_plummer, n=1 << 22, seed=3),
    "plummer16m": dict(gen=plummer, n=1 << 24, seed=4),
    "twoplummer16m": dict(gen=two_plummer, n=1 << 24, seed=5),
}


def make(name, n=None, seed=None):
    c = CONFIGS[name]
    return c["gen"](c["n"] if n is None else n, seed=c["seed"] if seed is None else seed)


def sample_targets(n, k, seed=99):
    """k distinct target indices (sorted) for sampled error measurement."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
