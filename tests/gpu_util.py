"""Helpers shared by the GPU tests: moving seeded host inputs to the device and
running the HIP solver through the C ABI binding."""
import sys

import numpy as np
import torch

from paper_1706_06989_amd import amfmm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda") for a in arrays]


def gpu_solve(x, y, z, m, theta, variant=amfmm.TC, precision=amfmm.FP64, n_crit=25, solver=None):
    s = solver or amfmm.Solver(n_crit=n_crit, variant=variant, precision=precision)
    X, Y, Z, M = to_dev(x, y, z, m)
    ax, ay, az, p = s.solve_gravity(X, Y, Z, M, theta)
    torch.cuda.synchronize()
    acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
    return acc, p.cpu().numpy(), s


def dup_points():
    """300 uniform points plus 40 coincident ones (a leaf deeper than the key
    resolution allows to split)."""
    from paper_1706_06989_amd import workloads as W
    x, y, z, m = W.uniform_cube(300, seed=7)
    x = np.concatenate([x, np.full(40, 0.25)])
    y = np.concatenate([y, np.full(40, 0.5)])
    z = np.concatenate([z, np.full(40, 0.75)])
    return x, y, z, np.full(len(x), 1.0 / len(x))


def tree_parts(x, y, z, m, n_crit=25):
    s = amfmm.Solver(n_crit=n_crit)
    X, Y, Z, M = to_dev(x, y, z, m)
    s.build_tree(X, Y, Z, M)
    return s, (X, Y, Z, M)
