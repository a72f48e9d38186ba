"""Completeness of a dual walk's lists, checked bottom-up (Sec. 2 opening rule,
the symmetric split rule of the walk).

The walk starts from the root's self pair; a cell's self pair yields its
children's self pairs and every pair of two of its children; a pair that the
criterion rejects and that is not two leaves is replaced by the pairs of one
cell's children with the other cell, where the opened cell is the one with the
larger R_max (ties: the lower index; never a leaf).  So a cell pair {a, b}
(a != b) is visited exactly when a and b are siblings, or when one of the two
pairs it can come from, {parent(a), b} or {a, parent(b)}, is visited, is
rejected, and opens the parent.  Far-field pairs must be accepted and visited;
near-field pairs must be two leaves, rejected and visited.

This is a different formulation from the oracle's top-down recursion (it asks,
for each listed pair, whether its ancestry is legal) and shares no code with
it.  Together with the coverage test (every particle pair exactly once) it
pins the lists to the walk's: an acceptance test stricter than the criterion
leaves visited pairs whose parent pair the criterion would have accepted, and
near-field pairs the criterion accepts.

`accept(a, b)` returns True, False, or None where rounding may decide (such a
pair is allowed either way).
"""
import math
import sys

import numpy as np


def geometric_accept(mo, theta):
    """The opening criterion as the walk evaluates it: d = sqrt((dx dx + dy dy)
    + dz dz), accept when d > 0 and d >= (R_A + R_B) / theta (IEEE double, the
    same operation order, so the decision is exact)."""
    Z = mo[:, 1:4]
    R = mo[:, 4]

    def accept(a, b):
        dx = float(Z[a, 0]) - float(Z[b, 0])
        dy = float(Z[a, 1]) - float(Z[b, 1])
        dz = float(Z[a, 2]) - float(Z[b, 2])
        d = math.sqrt((dx * dx + dy * dy) + dz * dz)
        return d > 0.0 and d >= (float(R[a]) + float(R[b])) / theta

    return accept


def check_walk(cells, mo, far, near, accept):
    """Assert that the far and near lists are exactly the visited terminal
    pairs of the walk under `accept` (see the module docstring)."""
    parent = np.asarray(cells["parent"])
    nchild = np.asarray(cells["nchild"])
    begin = np.asarray(cells["begin"])
    count = np.asarray(cells["count"])
    leaf = nchild == 0
    R = mo[:, 4]

    def nested(a, b):
        # one cell's particle range inside the other's: never a pair of the walk
        return (begin[a] <= begin[b] and begin[b] + count[b] <= begin[a] + count[a]) or \
               (begin[b] <= begin[a] and begin[a] + count[a] <= begin[b] + count[b])

    def opens(p, o):
        # the cell the split rule opens in the rejected pair (p, o), p not a leaf
        if leaf[o]:
            return p
        if R[p] > R[o] or (R[p] == R[o] and p < o):
            return p
        return o

    memo = {}
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 10000))

    def visited(a, b):
        key = (min(a, b), max(a, b))
        if key in memo:
            return memo[key]
        ok = parent[a] >= 0 and parent[a] == parent[b]
        for p, o in ((parent[a], b), (parent[b], a)):
            if ok:
                break
            if p < 0 or p == o or nested(p, o):
                continue
            acc = accept(p, o)
            if acc is True:
                continue
            if opens(p, o) != p:
                continue
            ok = visited(p, o)
        memo[key] = ok
        return ok

    try:
        for a, b in far:
            assert a != b
            assert accept(a, b) is not False, f"far pair {(a, b)} fails the criterion"
            assert visited(a, b), f"far pair {(a, b)} lies below a pair the criterion accepts"
        for a, b in near:
            if a == b:
                assert leaf[a], f"self pair of the non-leaf {a}"
                continue
            assert leaf[a] and leaf[b], f"near pair {(a, b)} is not two leaves"
            assert accept(a, b) is not True, f"near pair {(a, b)} meets the criterion"
            assert visited(a, b), f"near pair {(a, b)} lies below a pair the criterion accepts"
    finally:
        sys.setrecursionlimit(old)
