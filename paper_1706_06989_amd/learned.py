"""Training schedule of the learned pair selection (argument marshalling and
bookkeeping only: labels, features, forward, backward and Adam run in the
library's GPU kernels through the C ABI).

Training data: cell pairs accepted by multipole error-estimate walks at
several tolerances on seeded synthetic particle sets (the field estimate from
a geometric pilot solve), each labelled by the library with log2 of the ratio
of the method's largest error on the pair (against direct summation) to the
multipole estimate (``Solver.pair_labels``).  Only pairs large enough for the
walk to ask the network (N_A N_B >= MIN_PAIR_WORK) are kept.  The network
predicts that ratio at the 0.9 quantile (pinball loss), so that it errs on
the safe side.
"""
import numpy as np
import torch

from . import amfmm
from . import workloads as W

TAU = 0.9
TRAIN_EPS = (1e-5, 1e-6, 3e-7)
TRAIN_THETA_MAX = 0.5
MIN_PAIR_WORK = 1024


def collect(x, y, z, m, eps_list=TRAIN_EPS, per_eps=20000, seed=11, variant=amfmm.TC):
    """Features and labels of pairs sampled from the far-field lists of
    multipole-estimate walks at each tolerance (host numpy arrays)."""
    dev = torch.device("cuda")
    X, Y, Z, M = (torch.from_numpy(np.ascontiguousarray(v, np.float64)).to(dev) for v in (x, y, z, m))
    pilot = amfmm.Solver(variant=variant)
    gx, gy, gz, _ = pilot.solve_gravity(X, Y, Z, M, 0.5, pot=False)
    rng = np.random.default_rng(seed)
    feats, labels = [], []
    for eps in eps_list:
        s = amfmm.Solver(variant=variant, criterion=amfmm.MULTIPOLE, error_tol=eps, theta_max=TRAIN_THETA_MAX)
        s.set_field_estimate(gx, gy, gz)
        s.build_tree(X, Y, Z, M)
        s.compute_moments()
        s.walk(0.5)
        far, _ = s.get_lists()
        cnt = np.asarray(s.get_tree()["count"])
        far = far[cnt[far[:, 0]].astype(np.int64) * cnt[far[:, 1]] >= MIN_PAIR_WORK]
        if len(far):
            pick = far[rng.choice(len(far), min(per_eps, len(far)), replace=False)]
            P = torch.from_numpy(np.ascontiguousarray(pick, np.int32)).to(dev)
            feats.append(s.pair_features(P).cpu().numpy())
            labels.append(s.pair_labels(P, variant).cpu().numpy())
        s.close()
    pilot.close()
    if not feats:
        return np.zeros((0, 8), np.float32), np.zeros(0, np.float32)
    f = np.concatenate(feats)
    lab = np.concatenate(labels)
    ok = np.isfinite(lab) & np.all(np.isfinite(f), axis=1) & (f[:, 0] > 0)
    return f[ok], lab[ok].astype(np.float32)


def training_set(n=1 << 18, per_eps=20000):
    """Pairs of the uniform 4096-particle cube (seed 1), a Plummer sphere
    (seed 2) and two Plummer spheres (seed 13; the benchmark's two-sphere
    workload uses seed 5)."""
    f1, l1 = collect(*W.uniform_cube(4096, seed=1), per_eps=per_eps, seed=11)
    f2, l2 = collect(*W.plummer(n, seed=2), per_eps=per_eps, seed=12)
    f3, l3 = collect(*W.two_plummer(n, seed=13), per_eps=per_eps, seed=14)
    return np.concatenate([f1, f2, f3]), np.concatenate([l1, l2, l3])


def init_model(feats, seed=7):
    """He-initialised network with the feature normalisation and training
    range of `feats` (float32 numpy, MLP_MODEL entries)."""
    rng = np.random.default_rng(seed)
    P = np.zeros(amfmm.MLP_MODEL, np.float32)
    P[0:512] = rng.normal(0.0, np.sqrt(2.0 / 8), 512)
    P[576:4672] = rng.normal(0.0, np.sqrt(2.0 / 64), 4096)
    P[4736:4800] = rng.normal(0.0, np.sqrt(1.0 / 64), 64)
    mu = feats.mean(axis=0).astype(np.float64)
    sd = feats.std(axis=0).astype(np.float64)
    sd[sd == 0] = 1.0
    P[4801:4809] = (1.0 / sd).astype(np.float32)
    P[4809:4817] = (-mu / sd).astype(np.float32)
    P[4817:4825] = feats.min(axis=0)
    P[4825:4833] = feats.max(axis=0)
    return P


def train(feats, labels, steps=3000, batch=4096, lr=2e-3, seed=7, solver=None, log=None):
    """Trains on the GPU; returns (model as float32 numpy, list of losses)."""
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed + 1)
    order = rng.permutation(len(labels))
    F = torch.from_numpy(np.ascontiguousarray(feats[order], np.float32)).to(dev)
    L = torch.from_numpy(np.ascontiguousarray(labels[order], np.float32)).to(dev)
    P = torch.from_numpy(init_model(feats, seed)).to(dev)
    Am = torch.zeros(amfmm.MLP_PARAMS, dtype=torch.float32, device=dev)
    Av = torch.zeros_like(Am)
    s = solver or amfmm.Solver()
    losses = []
    chunk = 250
    for s0 in range(0, steps, chunk):
        k = min(chunk, steps - s0)
        # step size halves over the last third of the schedule
        rate = lr if s0 < 2 * steps // 3 else lr / 4
        losses.append(s.mlp_train(F, L, P, Am, Av, s0, k, min(batch, len(labels)), rate, TAU))
        if log:
            log(f"train step {s0 + k}: loss {losses[-1]:.4f}")
    return P.cpu().numpy(), losses


def coverage(model, feats, labels, solver=None):
    """Fraction of labels at or below the prediction (target: TAU)."""
    s = solver or amfmm.Solver()
    dev = torch.device("cuda")
    y = s.mlp_predict(torch.from_numpy(np.ascontiguousarray(model, np.float32)).to(dev),
                      torch.from_numpy(np.ascontiguousarray(feats, np.float32)).to(dev)).cpu().numpy()
    return float(np.mean(labels <= y)), y
