"""Fit of the multipole error estimate's weights (test infrastructure: calls
the oracle only).

The estimate of the force error that an accepted pair causes on field cell T
from source S (not in the paper; it stands in for the error-based pair
selection Sec. 2 cites) is

    e_T = (w1 a1 + w2 a2 + w3 a3 + w4 a4 + w5 a5) M_S / d^6,
    a1 = R_T^3 d, a2 = k2_S R_S^2 R_T d, a3 = k3_S R_S^3 d, a4 = R_S^4, a5 = R_T^4,

with k2, k3 the traceless quadrupole and octupole norms of S in units of
M R_max^2 and M R_max^3 (the oracle's levels / 128).  The weights are chosen
by least squares in log space: over the accepted pairs of geometric walks of
a Plummer sphere (both cells of each pair as the field cell), minimise the sum
of (ln E - ln e)^2, E the method's largest error from the pair alone on T's
particles (the oracle's pair_errors, TC variant).  Sides with E = 0, or with
every term zero (point masses, exact up to rounding), are left out.

    python oracle/fit_multipole.py [--n 65536] [--thetas 0.4,0.6,0.8] [--pairs N]

prints the fitted weights (all accepted pairs by default: the weights the
oracle and the kernels carry come from that run, rounded to four digits),
the carried weights, and the spread of log2(E / e) under each.
"""
import argparse
import os
import sys

import numpy as np
from scipy.optimize import least_squares

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as orc  # noqa: E402
from paper_1706_06989_amd import workloads as W  # noqa: E402  (seeded inputs only)

KQ = 128.0  # the norm levels are held to the nearest 1/128


def pair_terms(mom, k2, k3, pairs):
    """Per side (field cell first, then swapped): the five terms a1..a5 times
    M_S / d^6, shape (2 n, 5)."""
    rows = []
    for t_col, s_col in ((0, 1), (1, 0)):
        T, S = pairs[:, t_col], pairs[:, s_col]
        zt, zs = mom[T, 1:4], mom[S, 1:4]
        d = np.sqrt(np.sum((zt - zs) ** 2, axis=1))
        rt, rs, ms = mom[T, 4], mom[S, 4], mom[S, 0]
        a = np.stack([rt ** 3 * d, (k2[S] / KQ) * rs ** 2 * rt * d, (k3[S] / KQ) * rs ** 3 * d, rs ** 4, rt ** 4],
                     axis=1)
        rows.append(a * (ms / d ** 6)[:, None])
    return np.concatenate(rows)


def collect(n=65536, thetas=(0.4, 0.6, 0.8), pairs_per_theta=None, seed=3, sample_seed=17):
    """Terms and measured errors of the accepted pairs of geometric walks of an
    n-particle Plummer sphere (seed 3), all of them or a seeded sample of
    pairs_per_theta per angle."""
    x, y, z, m = W.plummer(n, seed=seed)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    mom = t.moments()
    k2, k3 = t.multipole_levels()
    rng = np.random.default_rng(sample_seed)
    A, E = [], []
    for th in thetas:
        t.walk(th)
        far, _ = t.lists()
        far = far[far[:, 0] != far[:, 1]]
        pick = far
        if pairs_per_theta is not None and pairs_per_theta < len(far):
            pick = far[rng.choice(len(far), pairs_per_theta, replace=False)]
        err = t.pair_errors(pick, orc.TC)
        A.append(pair_terms(mom, k2, k3, pick))
        E.append(np.concatenate([err[:, 0], err[:, 1]]))
    A = np.concatenate(A)
    E = np.concatenate(E)
    # sides whose terms all vanish (two point masses) are exact up to rounding
    ok = (E > 0) & np.all(np.isfinite(A), axis=1) & (A.sum(axis=1) > 0)
    return A[ok], E[ok]


def residuals(w, A, E):
    return np.log(E) - np.log(A @ w)


def fit(A, E, w0=None):
    """Least squares in log space over positive weights."""
    v0 = np.log(w0 if w0 is not None else np.ones(A.shape[1]))
    r = least_squares(lambda v: residuals(np.exp(v), A, E), v0, method="lm")
    return np.exp(r.x)


def spread(w, A, E):
    """rms, median and 90th percentile of log2(E / e)."""
    r = residuals(w, A, E) / np.log(2.0)
    return float(np.sqrt(np.mean(r ** 2))), float(np.median(r)), float(np.percentile(r, 90))


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--n", type=int, default=65536)
    p.add_argument("--thetas", default="0.4,0.6,0.8")
    p.add_argument("--pairs", type=int, default=None, help="accepted pairs sampled per angle (default: all)")
    a = p.parse_args()
    A, E = collect(a.n, tuple(float(v) for v in a.thetas.split(",")), a.pairs)
    w = fit(A, E)
    cur = orc.multipole_weights()
    print(f"sides fitted: {len(E)}")
    print("fitted  w1..w5:", " ".join(f"{v:.4g}" for v in w), " log2 ratio rms/median/p90: %.3f %.3f %.3f" % spread(w, A, E))
    print("carried w1..w5:", " ".join(f"{v:.4g}" for v in cur), " log2 ratio rms/median/p90: %.3f %.3f %.3f" % spread(cur, A, E))


if __name__ == "__main__":
    main()
