"""Pins of the oracle's learned pair selection (not in the paper): the BF16
rounding and piecewise-linear log2 against their definitions, the network and
its gradient against torch (a library implementation of the same layers),
Adam against torch.optim.Adam, labels (the ratio of the method's largest pair
error to the multipole estimate) against an independent assembly from the
pair evaluation, numpy direct sums and the estimate recomputed from particle
sums, features' symmetry, and the walk's gating against the multipole
error-estimate walk."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1706_06989_amd import workloads as W

from .test_oracle_multipole import estimate, levels_from_particles


def random_model(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    P = np.zeros(orc.MLP_MODEL, np.float32)
    P[: orc.MLP_PARAMS] = rng.normal(0.0, scale, orc.MLP_PARAMS)
    P[4801:4809] = rng.uniform(0.5, 2.0, 8)   # normalisation a
    P[4809:4817] = rng.uniform(-1.0, 1.0, 8)  # normalisation b
    P[4817:4825] = -1e30                       # training range: everything
    P[4825:4833] = 1e30
    return P


def torch_forward(P, F, round_bf16):
    """The network written with torch layers (FP64 sums)."""
    def rd(t):
        return t.float().to(torch.bfloat16).double() if round_bf16 else t

    P = torch.from_numpy(P.astype(np.float64))
    F = torch.from_numpy(F.astype(np.float64))
    W1 = rd(P[0:512].reshape(64, 8))
    b1 = P[512:576]
    W2 = rd(P[576:4672].reshape(64, 64))
    b2 = P[4672:4736]
    w3 = rd(P[4736:4800])
    b3 = P[4800]
    x = F * P[4801:4809] + P[4809:4817]
    if round_bf16:
        x = rd(x)
    h1 = rd(torch.relu(torch.nn.functional.linear(x, W1, b1)))
    h2 = rd(torch.relu(torch.nn.functional.linear(h1, W2, b2)))
    return h2 @ w3 + b3


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(1)
    vals = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-3, 500) * 1e-20,
                           [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.75, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(vals).to(torch.bfloat16).float().numpy()
    got = np.array([orc.bf16_round(v) for v in vals], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_plog2_definition():
    # exact at powers of two, linear in between, never above log2 and at most
    # 1 - (1 + ln ln 2) / ln 2 = 0.0861 below it
    for e in range(-60, 61):
        assert orc.plog2(2.0 ** e) == e
        assert orc.plog2(1.5 * 2.0 ** e) == e + 0.5
    rng = np.random.default_rng(2)
    xs = np.exp(rng.uniform(-80, 80, 5000))
    gap = np.log2(xs) - np.array([orc.plog2(v) for v in xs])
    assert gap.min() >= -1e-12 and gap.max() <= 0.0861
    assert orc.plog2(0.0) == -2048.0 and orc.plog2(-1.0) == -2048.0


def test_predict_matches_torch_layers():
    P = random_model(3)
    rng = np.random.default_rng(4)
    F = rng.normal(0, 1, (400, 8)).astype(np.float32)
    y = orc.mlp_predict(P, F)
    ref = torch_forward(P, F, True).numpy()
    # FP32 sums against FP64 sums: a BF16 rounding of a hidden value may land on
    # the other side of a tie, so compare with a tolerance of a few BF16 ulps
    assert np.max(np.abs(y - ref)) <= 2e-2 * max(1.0, np.abs(ref).max())
    assert np.median(np.abs(y - ref)) <= 1e-5 * max(1.0, np.abs(ref).max())


def test_gradient_matches_torch_autograd_and_finite_differences():
    P = random_model(5)
    rng = np.random.default_rng(6)
    F = rng.normal(0, 1, (64, 8)).astype(np.float32)
    L = rng.normal(0, 1, 64).astype(np.float32)
    tau = 0.9
    loss, g = orc.mlp_grad(P, F, L, tau=tau, round=False)
    # autograd of the unrounded function
    Pt = torch.tensor(P.astype(np.float64), requires_grad=True)
    Ft = torch.from_numpy(F.astype(np.float64))
    x = Ft * Pt[4801:4809] + Pt[4809:4817]
    h1 = torch.relu(x @ Pt[0:512].reshape(64, 8).T + Pt[512:576])
    h2 = torch.relu(h1 @ Pt[576:4672].reshape(64, 64).T + Pt[4672:4736])
    y = h2 @ Pt[4736:4800] + Pt[4800]
    r = torch.from_numpy(L.astype(np.float64)) - y
    lt = torch.where(r < 0, (tau - 1) * r, tau * r).mean()
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-12 * abs(lt.item())
    ag = Pt.grad.numpy()[: orc.MLP_PARAMS]
    assert np.max(np.abs(g - ag)) <= 1e-12 * np.abs(ag).max()
    # central differences on a few parameters (the loss is piecewise linear in
    # each parameter away from kinks, so a small step is exact up to rounding)
    for k in [0, 7, 300, 520, 600, 3000, 4680, 4700, 4740, 4800]:
        h = 1e-3 * max(1.0, abs(float(P[k])))
        Pp, Pm = P.astype(np.float64).copy(), P.astype(np.float64).copy()
        Pp[k] += h
        Pm[k] -= h
        lp, _ = orc.mlp_grad(Pp.astype(np.float32), F, L, tau=tau, round=False)
        lm, _ = orc.mlp_grad(Pm.astype(np.float32), F, L, tau=tau, round=False)
        hp = float(np.float32(Pp[k])) - float(P[k])
        hm = float(P[k]) - float(np.float32(Pm[k]))
        fd = (lp - lm) / (hp + hm)
        assert abs(fd - g[k]) <= 1e-3 * np.abs(g).max() + 1e-6, (k, fd, g[k])


def test_rounded_gradient_close_to_unrounded():
    P = random_model(7)
    rng = np.random.default_rng(8)
    F = rng.normal(0, 1, (256, 8)).astype(np.float32)
    L = rng.normal(0, 1, 256).astype(np.float32)
    _, g0 = orc.mlp_grad(P, F, L, round=False)
    _, g1 = orc.mlp_grad(P, F, L, round=True)
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)


def test_adam_matches_torch():
    rng = np.random.default_rng(9)
    p = rng.normal(0, 1, orc.MLP_PARAMS).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pt = torch.tensor(p.astype(np.float64), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 4):
        g = rng.normal(0, 1, orc.MLP_PARAMS).astype(np.float32)
        orc.mlp_adam(p, g, m, v, t, 1e-3)
        pt.grad = torch.from_numpy(g.astype(np.float64))
        opt.step()
        assert np.max(np.abs(p - pt.detach().numpy())) <= 1e-6


@pytest.fixture(scope="module")
def plummer_tree():
    x, y, z, m = W.plummer(6000, seed=21)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    a, _, _ = orc.direct(x, y, z, m)
    return (x, y, z, m), t, np.linalg.norm(a, axis=0)


def test_features_symmetric_and_in_range(plummer_tree):
    (x, y, z, m), t, _ = plummer_tree
    t.walk(0.7)
    far, _ = t.lists()
    f = t.pair_features(far)
    fr = t.pair_features(far[:, ::-1])
    assert np.array_equal(f.view(np.uint32), fr.view(np.uint32))
    assert np.all(f[:, 0] <= 0.7 * (1 + 1e-6)) and np.all(f[:, 0] >= 0)
    assert np.all((f[:, 1:7] >= 0) & (f[:, 1:7] <= 1))
    # the norm-level features are the traceless levels recomputed from particles
    k2, k3 = levels_from_particles(t, x, y, z, m)
    a, b = far[:, 0], far[:, 1]
    assert np.array_equal(f[:, 2], ((k2[a] + k2[b]) / 256.0).astype(np.float32))
    assert np.array_equal(f[:, 5], (np.abs(k3[a] - k3[b]) / 128.0).astype(np.float32))
    # the counts feature is the plog2 of N_A N_B (counts saturated at 1024)
    c = t.cells()
    na, nb = np.minimum(c["count"][a], 1024), np.minimum(c["count"][b], 1024)
    ref = np.array([orc.plog2(float(u) * float(v)) for u, v in zip(na, nb)], np.float32)
    assert np.array_equal(f[:, 7], ref)


def test_labels_against_independent_assembly(plummer_tree):
    (x, y, z, m), t, _ = plummer_tree
    t.walk(0.6)
    far, _ = t.lists()
    c = t.cells()
    mo = t.moments()
    _, perm = t.keys()
    xs, ys, zs, ms = x[perm], y[perm], z[perm], m[perm]
    k2, k3 = levels_from_particles(t, x, y, z, m)
    rng = np.random.default_rng(3)
    small = far[(c["count"][far[:, 0]] <= 64) & (c["count"][far[:, 1]] <= 64)
                & (mo[far[:, 0], 4] > 0) & (mo[far[:, 1], 4] > 0)]
    sel = small[rng.choice(len(small), 40, replace=False)]
    lab = t.pair_labels(sel, orc.TC)
    for (A, B), L in zip(sel, lab):
        def parts(cell):
            b, n = c["begin"][cell], c["count"][cell]
            return xs[b:b + n], ys[b:b + n], zs[b:b + n], ms[b:b + n]
        PA, PB = parts(A), parts(B)
        gA, _, gB, _ = orc.pair_far(PA, PB, orc.TC)

        def direct(T, S):
            d = np.stack([S[k][None, :] - T[k][:, None] for k in range(3)])
            r3 = np.sqrt((d ** 2).sum(0)) ** 3
            return (S[3][None, :] * d / r3).sum(2).T

        d = np.linalg.norm(mo[A, 1:4] - mo[B, 1:4])
        eA = np.linalg.norm(gA - direct(PA, PB), axis=1).max()
        eB = np.linalg.norm(gB - direct(PB, PA), axis=1).max()
        estA = estimate(mo[A, 4], mo[B, 4], k2[B], k3[B], d, mo[B, 0])
        estB = estimate(mo[B, 4], mo[A, 4], k2[A], k3[A], d, mo[A, 0])
        ref = math.log2(max(eA / estA, eB / estB))
        assert abs(L - ref) <= 1e-6, (A, B, L, ref)


def test_labels_follow_the_expansion_order():
    """Two clusters of fixed shape, each one leaf, at a fixed distance: the
    method's error and the estimate both fall like (r/d)^3, so as the
    clusters shrink the label (their log ratio) settles to a constant of
    order one, the next order fading linearly: each halving of the size
    halves the change of the label."""
    rng = np.random.default_rng(11)
    base = rng.uniform(-1, 1, (2, 40, 3))
    labs = []
    m = None
    for r in (0.1, 0.05, 0.025, 0.0125, 0.00625):
        A = base[0] * r
        B = base[1] * r + np.array([1.0, 0.8, 0.6])
        P = np.concatenate([A, B])
        m = rng.uniform(0.5, 1.5, 80) if m is None else m
        t = orc.Tree(P[:, 0], P[:, 1], P[:, 2], m, n_crit=64)
        t.compute_moments()
        c = t.cells()
        leaves = np.nonzero(c["nchild"] == 0)[0]
        assert len(leaves) == 2 and sorted(c["count"][leaves]) == [40, 40]
        labs.append(t.pair_labels(leaves.reshape(1, 2))[0])
    steps = np.diff(labs)
    assert abs(labs[-1]) < 2.0, labs
    assert np.all(np.abs(steps) < 0.5), labs
    ratios = steps[1:] / steps[:-1]
    assert np.all((ratios > 0.35) & (ratios < 0.65)), labs


def test_learned_walk_without_model_is_geometric(plummer_tree):
    _, t, g = plummer_tree
    t.walk(0.55)
    ref = t.lists()
    t.walk_learned(1e-5, 0.7, 0.55, g, None)
    got = t.lists()
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])


def constant_model(out, in_range=True):
    P = np.zeros(orc.MLP_MODEL, np.float32)
    P[4800] = out
    P[4817:4825] = -1e30 if in_range else 1e30
    P[4825:4833] = 1e30 if in_range else -1e30
    return P


def test_learned_walk_gating(plummer_tree):
    """A network that always predicts a tiny ratio accepts every pair in the
    band (rho <= 2): the multipole walk at 2 eps.  One that always predicts a
    huge ratio accepts only below the band (rho <= 1/4): eps/4.  Bit for bit
    (the gates scale eps by powers of two)."""
    _, t, g = plummer_tree
    eps = 2e-5
    for out, factor in ((-1000.0, 2.0), (1000.0, 0.25)):
        t.walk_learned(eps, 0.7, 0.5, g, constant_model(out), min_work=1)
        got = t.lists()
        t.walk_multipole(eps * factor, 0.7, g)
        ref = t.lists()
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_learned_walk_small_pairs_take_the_multipole_estimate(plummer_tree):
    """With min_work above every N_A N_B the network is never asked: the
    decision is rho <= 1, the multipole error-estimate walk."""
    _, t, g = plummer_tree
    t.walk_learned(2e-5, 0.7, 0.5, g, constant_model(-1000.0), min_work=1 << 40)
    got = t.lists()
    t.walk_multipole(2e-5, 0.7, g)
    ref = t.lists()
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_learned_walk_out_of_range_takes_the_multipole_estimate(plummer_tree):
    """With an empty training range every band pair takes rho <= 1: the
    multipole error-estimate walk."""
    _, t, g = plummer_tree
    t.walk_learned(2e-5, 0.7, 0.4, g, constant_model(-1000.0, in_range=False), min_work=1)
    got = t.lists()
    t.walk_multipole(2e-5, 0.7, g)
    ref = t.lists()
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_learned_walk_follows_the_prediction(plummer_tree):
    """A constant integer prediction c (log2 of the error ratio) accepts a band
    pair when plog2(rho) <= -c, i.e. rho <= 2^-c (plog2 is exact at powers of
    two): the multipole walk at the tolerance eps 2^-c."""
    _, t, g = plummer_tree
    eps = 2e-5
    for c in (2.0, 1.0, 0.0, -1.0):
        t.walk_learned(eps, 0.7, 0.5, g, constant_model(c), min_work=1)
        got = t.lists()
        t.walk_multipole(eps * 2.0 ** -c, 0.7, g)
        ref = t.lists()
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), c
