"""Learned pair selection on the GPU, through the C ABI, against the oracle:
features and inference bit for bit, labels to round-off, gradients and Adam
to FP32 accuracy, the learned walk's lists bit for bit and its accelerations
to 1e-12."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1706_06989_amd import amfmm
from paper_1706_06989_amd import workloads as W
from tests.gpu_util import dup_points, say, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "uniform4k": lambda: W.uniform_cube(4096, seed=1),
    "plummer16k": lambda: W.plummer(16384, seed=2),
    "twoplummer20k": lambda: W.two_plummer(20000, seed=3),
}


def random_model(seed, feats=None, b3=0.0):
    rng = np.random.default_rng(seed)
    P = np.zeros(amfmm.MLP_MODEL, np.float32)
    P[:amfmm.MLP_PARAMS] = rng.normal(0.0, 0.3, amfmm.MLP_PARAMS)
    P[4800] = b3
    if feats is None:
        P[4801:4809] = rng.uniform(0.5, 2.0, 8)
        P[4809:4817] = rng.uniform(-1.0, 1.0, 8)
        P[4817:4825] = -1e30
        P[4825:4833] = 1e30
    else:
        sd = feats.std(0) + 1e-3
        P[4801:4809] = 1.0 / sd
        P[4809:4817] = -feats.mean(0) / sd
        P[4817:4825] = feats.min(0)
        P[4825:4833] = feats.max(0)
    return P


def cuda32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to("cuda")


@pytest.mark.parametrize("name", sorted(CASES))
def test_features_and_labels_match_oracle(name):
    x, y, z, m = CASES[name]()
    say("features/labels", name)
    s = amfmm.Solver()
    X, Y, Z, M = to_dev(x, y, z, m)
    s.build_tree(X, Y, Z, M)
    s.compute_moments()
    s.walk(0.7)
    far, _ = s.get_lists()
    rng = np.random.default_rng(5)
    pick = far[rng.choice(len(far), min(3000, len(far)), replace=False)]
    P = torch.from_numpy(np.ascontiguousarray(pick, np.int32)).to("cuda")
    gf = s.pair_features(P).cpu().numpy()
    gl = s.pair_labels(P, amfmm.TC).cpu().numpy()
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    of = t.pair_features(pick)
    ol = t.pair_labels(pick, orc.TC)
    bad = np.nonzero(np.any(gf.view(np.uint32) != of.view(np.uint32), axis=1))[0]
    assert len(bad) == 0, (len(bad), pick[bad[:5]], gf[bad[:5]], of[bad[:5]])
    # A label is log2 of an error that is a difference of nearly equal forces,
    # over the estimate: its relative rounding is about 1e-16 |g| / error, with
    # the error near (R/d)^3 |g|.  Compare to 1e-6 where (R/d)^3 > 1e-9; exact
    # pairs (point masses) give -inf on both sides.
    exact = ~np.isfinite(ol)
    assert np.array_equal(exact, ~np.isfinite(gl))
    big = ~exact & (of[:, 0].astype(np.float64) ** 3 > 1e-9)
    assert np.max(np.abs(gl[big] - ol[big])) <= 1e-6
    say(f"  {len(pick)} pairs, labels {np.percentile(ol[big], [5, 50, 95])}, exact {np.sum(exact)}")
    # pairs naming no cell of the tree come back as NaN, the others unchanged
    nc = s.get_counts()["cells"]
    odd = np.array([pick[0], [nc, pick[0][1]], [pick[1][0], -1], pick[1]], np.int32)
    Po = torch.from_numpy(odd).to("cuda")
    fo = s.pair_features(Po).cpu().numpy()
    lo = s.pair_labels(Po, amfmm.TC).cpu().numpy()
    assert np.all(np.isnan(fo[1:3])) and np.all(np.isnan(lo[1:3]))
    assert np.array_equal(fo[[0, 3]], gf[:2]) and np.array_equal(lo[[0, 3]], gl[:2])


def test_predict_bit_exact():
    rng = np.random.default_rng(3)
    P = random_model(4)
    F = rng.normal(0, 1, (5000, 8)).astype(np.float32)
    s = amfmm.Solver()
    y = s.mlp_predict(cuda32(P), cuda32(F)).cpu().numpy()
    ref = orc.mlp_predict(P, F)
    assert np.array_equal(y.view(np.uint32), ref.view(np.uint32))


def test_gradient_matches_oracle():
    rng = np.random.default_rng(6)
    P = random_model(7)
    F = rng.normal(0, 1, (1000, 8)).astype(np.float32)
    L = rng.normal(0, 2, 1000).astype(np.float32)
    s = amfmm.Solver()
    loss, g = s.mlp_grad(cuda32(P), cuda32(F), cuda32(L), 0.9)
    g = g.cpu().numpy().astype(np.float64)
    oloss, og = orc.mlp_grad(P, F, L, tau=0.9, round=True)
    rel = np.linalg.norm(g - og) / np.linalg.norm(og)
    say(f"grad: loss {loss:.6f} vs {oloss:.6f}, relative gradient difference {rel:.3e}")
    assert abs(loss - oloss) <= 1e-5 * abs(oloss)
    assert rel <= 1e-4
    # block by block (each layer's weights and biases)
    for lo, hi in ((0, 512), (512, 576), (576, 4672), (4672, 4736), (4736, 4800), (4800, 4801)):
        assert np.linalg.norm(g[lo:hi] - og[lo:hi]) <= 1e-3 * np.linalg.norm(og[lo:hi]) + 1e-9


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(8)
    P = random_model(9)
    F = rng.normal(0, 1, (512, 8)).astype(np.float32)
    L = rng.normal(0, 2, 512).astype(np.float32)
    s = amfmm.Solver()
    _, g = s.mlp_grad(cuda32(P), cuda32(F), cuda32(L), 0.9)
    Pd, Am, Av = cuda32(P), torch.zeros(amfmm.MLP_PARAMS, device="cuda"), torch.zeros(amfmm.MLP_PARAMS,
                                                                                          device="cuda")
    s.mlp_train(cuda32(F), cuda32(L), Pd, Am, Av, 0, 1, 512, 1e-3, 0.9)
    p = P[:amfmm.MLP_PARAMS].copy()
    m = np.zeros(amfmm.MLP_PARAMS, np.float32)
    v = np.zeros(amfmm.MLP_PARAMS, np.float32)
    orc.mlp_adam(p, g.cpu().numpy(), m, v, 1, 1e-3)
    got = Pd.cpu().numpy()
    assert np.max(np.abs(got[:amfmm.MLP_PARAMS] - p)) <= 1e-6
    assert np.array_equal(got[amfmm.MLP_PARAMS:], P[amfmm.MLP_PARAMS:])


LIST_CASES = {
    "uniform4k": lambda: W.uniform_cube(4096, seed=1),
    "plummer16k": lambda: W.plummer(16384, seed=2),
    "twoplummer20k": lambda: W.two_plummer(20000, seed=3),
    "duplicates": dup_points,
}


@pytest.mark.parametrize("name", sorted(LIST_CASES))
@pytest.mark.parametrize("eps,b3,min_work", [(1e-5, 0.0, 1), (1e-4, 1.0, 1), (1e-5, -1.0, 4096)])
def test_learned_walk_bit_exact(name, eps, b3, min_work):
    """Same model and field input on both sides: the same pairs, bit for bit,
    and the same accelerations to 1e-12."""
    x, y, z, m = LIST_CASES[name]()
    say("learned walk", name, len(x), eps, b3)
    at, _, gabs = orc.direct(x, y, z, m)
    gmag = np.linalg.norm(at, axis=0)
    t = orc.Tree(x, y, z, m)
    t.compute_moments()
    t.walk(0.8)
    far0, _ = t.lists()
    feats = t.pair_features(far0) if len(far0) else None
    P = random_model(10, feats, b3)
    t.walk_learned(eps, 0.8, 0.5, gmag, P, min_work)
    ofar, onear = t.lists()
    s = amfmm.Solver(criterion=amfmm.LEARNED, error_tol=eps, theta_max=0.8, learned_min_work=min_work)
    s.set_model(P)
    X, Y, Z, M = to_dev(x, y, z, m)
    G, = to_dev(gmag)
    s.set_field_estimate(G)
    s.build_tree(X, Y, Z, M)
    s.compute_moments()
    s.walk(0.5)
    far, near = s.get_lists()
    assert np.array_equal(far, ofar)
    assert np.array_equal(near, onear)
    ax, ay, az, p = s.evaluate()
    acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()])
    oacc, opot = t.evaluate(orc.TC)
    assert np.max(np.linalg.norm(acc - oacc, axis=0) / gabs) <= 1e-12
    # the network's decisions against the multipole walk at the tolerance
    # and at both gates
    counts = []
    for f in (0.25, 1.0, 2.0):
        t.walk_multipole(eps * f, 0.8, gmag)
        counts.append(len(t.lists()[0]))
    say(f"  far pairs: learned {len(ofar)}, multipole at eps/4, eps, 2 eps: {counts}")


def test_learned_without_model_is_geometric():
    x, y, z, m = W.plummer(8000, seed=13)
    X, Y, Z, M = to_dev(x, y, z, m)
    s = amfmm.Solver(criterion=amfmm.LEARNED, error_tol=1e-5, theta_max=0.8)
    G = torch.ones_like(X)
    s.set_field_estimate(G)
    a1 = s.solve_gravity(X, Y, Z, M, 0.6)
    a2 = amfmm.Solver().solve_gravity(X, Y, Z, M, 0.6)
    for u, v in zip(a1, a2):
        assert torch.equal(u, v)
