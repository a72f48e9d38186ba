"""What the trained network gains over the method without it.

The network is trained on the GPU (library kernels: labels, forward,
backward, Adam) from pairs of the uniform 4096-particle cube and a
2^20-particle Plummer sphere, then used on a different problem: two Plummer
spheres of 2^18 particles.  For each error tolerance the error-estimate walk
(the method without the network) and the learned walk are run from the same
field estimate; the test prints p99 relative force error against direct
summation, the work (far-field evaluations and near-field interactions) and
the time of each, and the work ratio at matched p99.

Asserted: training lowers the loss and reaches the 0.9 quantile on held-out
pairs; the learned walk stays accurate (p99 within 2x of the error-estimate
walk at the same tolerance, since out-of-range pairs and small pairs keep the
analytic factor).  The gain itself is reported, not asserted.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1706_06989_amd import amfmm, learned
from paper_1706_06989_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def work(c):
    # directed far-field evaluations cost about 15 near interactions each
    # (about 300 flops against 20)
    return c["near_interactions"] + 15 * c["far_evaluations"]


def test_trained_network_gain():
    f, lab = learned.training_set(n_plummer=1 << 20, per_theta=20000)
    rng = np.random.default_rng(0)
    idx = rng.permutation(len(lab))
    ntr = int(0.85 * len(lab))
    P, losses = learned.train(f[idx[:ntr]], lab[idx[:ntr]], steps=3000, batch=4096, lr=2e-3)
    cov, _ = learned.coverage(P, f[idx[ntr:]], lab[idx[ntr:]])
    say(f"pairs {len(lab)}, loss {losses[0]:.4f} -> {losses[-1]:.4f}, held-out coverage {cov:.3f}")
    assert losses[-1] < losses[0]
    assert 0.85 <= cov <= 0.95

    n = 1 << 18
    x, y, z, m = W.two_plummer(n, seed=5)
    X, Y, Z, M = (torch.from_numpy(v).cuda() for v in (x, y, z, m))
    pilot = amfmm.Solver()
    gx, gy, gz, _ = pilot.solve_gravity(X, Y, Z, M, 0.5, pot=False)
    tg = torch.from_numpy(W.sample_targets(n, 4096, seed=99)).cuda()
    tx, ty, tz, _, _ = pilot.direct(X, Y, Z, M, tg, pot=False, gabs=False)
    T = torch.stack([tx, ty, tz])

    def p99(o):
        A = torch.stack([o[0][tg], o[1][tg], o[2][tg]])
        e = (torch.linalg.norm(A - T, dim=0) / torch.linalg.norm(T, dim=0)).cpu().numpy()
        return float(np.percentile(e, 99))

    rows = []
    for crit in (amfmm.ESTIMATE, amfmm.LEARNED):
        for eps in (1e-5, 3e-6, 1e-6):
            s = amfmm.Solver(criterion=crit, error_tol=eps, theta_max=0.5)
            if crit == amfmm.LEARNED:
                s.set_model(P)
            s.set_field_estimate(gx, gy, gz)
            s.solve_gravity(X, Y, Z, M, 0.5, pot=False)  # warm-up (allocation)
            o = s.solve_gravity(X, Y, Z, M, 0.5, pot=False)
            torch.cuda.synchronize()
            c = s.get_counts()
            r = dict(criterion="learned" if crit == amfmm.LEARNED else "estimate", eps=eps, p99=p99(o),
                     ms=s.get_phase_times()["total"], work=work(c), far=c["far_evaluations"],
                     near=c["near_interactions"])
            rows.append(r)
            say(json.dumps(r))
    est = [r for r in rows if r["criterion"] == "estimate"]
    lea = [r for r in rows if r["criterion"] == "learned"]
    for a, b in zip(est, lea):
        assert b["p99"] <= 2.0 * a["p99"], (a, b)

    # work and time at matched p99: interpolate log(work) against log(p99)
    def at(rs, key, p):
        xs = np.log([r["p99"] for r in rs])
        ys = np.log([r[key] for r in rs])
        o = np.argsort(xs)
        return float(np.exp(np.interp(np.log(p), xs[o], ys[o])))

    p_ref = float(np.median([r["p99"] for r in est]))
    gain_work = at(est, "work", p_ref) / at(lea, "work", p_ref)
    gain_time = at(est, "ms", p_ref) / at(lea, "ms", p_ref)
    say(f"at p99 {p_ref:.3e}: learned needs 1/{gain_work:.3f} of the work and 1/{gain_time:.3f} of the time")
    out = os.environ.get("AMFMM_GAIN_OUT")
    if out:
        json.dump(dict(rows=rows, p99_ref=p_ref, gain_work=gain_work, gain_time=gain_time), open(out, "w"))
