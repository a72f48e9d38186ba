"""The allocation-free solve (amfmm_solve_gravity_noalloc), through the C ABI,
against the solve that allocates (amfmm_solve_gravity): the same inputs give
the same accelerations and potentials to the FP64 parity bar (1e-12 of
gabs; a cell's pairs may be summed in another order), on two calls in a row
(the second smaller), for the geometric and the multipole criterion and for
mixed precision; the call takes no device memory; 2^18 particles solve and
one more is refused with an error."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1706_06989_amd import amfmm
from paper_1706_06989_amd import workloads as W
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def outputs(n):
    return tuple(torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4))


def host4(o):
    return np.stack([v.cpu().numpy() for v in o])


@pytest.mark.parametrize("mode", ["geometric", "multipole", "mixed"])
def test_noalloc_matches_solve_on_two_calls(mode):
    kw = {}
    if mode == "multipole":
        kw = dict(criterion=amfmm.MULTIPOLE, error_tol=1e-5, theta_max=0.5)
    if mode == "mixed":
        kw = dict(precision=amfmm.MIXED)
    s = amfmm.Solver(**kw)
    for n, seed in ((1 << 15, 3), (1 << 12, 4)):
        x, y, z, m = W.plummer(n, seed=seed)
        say("no-alloc", mode, n)
        X, Y, Z, M = to_dev(x, y, z, m)
        if mode == "multipole":
            r = np.sqrt(x * x + y * y + z * z)
            G, = to_dev(r / (r * r + 1.0) ** 1.5)
            s.set_field_estimate(G)
        ref = host4(s.solve_gravity(X, Y, Z, M, 0.5))
        got = host4(s.solve_gravity_noalloc(X, Y, Z, M, 0.5, outputs(n)))
        torch.cuda.synchronize()
        _, _, gabs = orc.direct(x, y, z, m)
        err = np.max(np.linalg.norm(got[:3] - ref[:3], axis=0) / gabs)
        perr = np.max(np.abs(got[3] - ref[3]) / np.abs(ref[3]))
        say(f"  max |dg|/gabs {err:.2e}, max |dphi|/|phi| {perr:.2e}")
        assert err <= 1e-12 and perr <= 1e-12
        # the solve that allocates still works after it, with its own buffers
        again = host4(s.solve_gravity(X, Y, Z, M, 0.5))
        assert np.array_equal(again, ref)
    s.close()


def test_noalloc_takes_no_device_memory():
    x, y, z, m = W.plummer(1 << 14, seed=5)
    X, Y, Z, M = to_dev(x, y, z, m)
    out = outputs(len(x))
    s = amfmm.Solver()
    s.solve_gravity_noalloc(X, Y, Z, M, 0.5, out)  # first launch loads the code objects
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        s.solve_gravity_noalloc(X, Y, Z, M, 0.5, out)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    say(f"no-alloc: free device memory {free0 - free1} bytes lower after three calls")
    assert free0 - free1 < (4 << 20)
    # a context that has only run allocation-free solves holds no tree
    with pytest.raises(amfmm.AmfmmError) as e:
        s.get_lists()
    assert e.value.code == amfmm.E_STATE
    s.close()


def test_noalloc_at_and_beyond_its_maximum():
    """2^18 particles (the maximum) solve and match; one more is refused with
    an error, and the context still solves afterwards."""
    n = 1 << 18
    x, y, z, m = W.plummer(n, seed=7)
    X, Y, Z, M = to_dev(x, y, z, m)
    s = amfmm.Solver()
    say("no-alloc at the maximum", n)
    got = host4(s.solve_gravity_noalloc(X, Y, Z, M, 0.5, outputs(n)))
    ref = host4(s.solve_gravity(X, Y, Z, M, 0.5))
    idx = W.sample_targets(n, 512, seed=99)
    _, _, gabs = orc.direct(x, y, z, m, idx)
    err = np.max(np.linalg.norm(got[:3, idx] - ref[:3, idx], axis=0) / gabs)
    assert err <= 1e-12
    x1, y1, z1, m1 = W.uniform_cube(n + 1, seed=6)
    X1, Y1, Z1, M1 = to_dev(x1, y1, z1, m1)
    with pytest.raises(amfmm.AmfmmError) as e:
        s.solve_gravity_noalloc(X1, Y1, Z1, M1, 0.5, outputs(n + 1))
    assert e.value.code == amfmm.E_INVALID
    a = s.solve_gravity(X1, Y1, Z1, M1, 0.5)
    assert torch.isfinite(a[0]).all()
    s.close()
