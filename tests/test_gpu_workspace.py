"""H psi with a caller-supplied work space (abacus_pw_workspace_size +
abacus_pw_apply_h_ws): the very first H psi call for a problem, made inside a
HIP graph capture, allocates nothing, and every replay of the graph equals the
allocating entry point's eager result bit for bit, with unrelated eager work
between replays (every precision, several uneven k-points). A work space one
byte too small is refused before anything is enqueued."""
import numpy as np
import pytest

import oracle
from paper_2501_08697_amd import workload as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def B():
    from paper_2501_08697_amd import binding
    return binding


def problem(seed):
    return W.make_problem(W.tiny_config(fft=24, ecut=24.0, a=8.0, nb=20, natom=4, lmax=2, dfull=True, seed=seed,
                                        kfrac=((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (0.5, 0.5, 0.5))))


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_first_call_captured_in_graph(prec):
    b = B()
    b.set_tuning()
    # Every seed has the same cell, cutoff and k-points, so the same sphere: without a reset
    # a cached plan could be found again (its key holds the Miller array's address, which a
    # new host array may reuse), together with reduced-precision operator copies that a
    # static operator at a reused device address would leave stale. The first call of the
    # test must build its plan.
    b.plan_reset()
    p = problem(40 + prec)
    dp = b.DeviceProblem(p, static=True)
    x = torch.from_numpy(p.psi).cuda()
    if prec == b.FP32:
        x = x.to(torch.complex64)
    nbytes = b.workspace_size(dp, prec)
    print(f"[workspace] prec={prec} npw={list(p.npw)} bytes={nbytes}", flush=True)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.apply_h_ws(dp, x, ws, prec, out=y)
    torch.cuda.synchronize()
    ref = b.apply_h(dp, x, prec)   # the allocating entry point, eager
    torch.cuda.synchronize()
    for rep in range(3):
        y.zero_()
        ws.fill_(0xA5)                                        # scratch contents must not matter
        junk = torch.randn(1 << 16, device="cuda").sum()     # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), rep
        del junk
    tol = {0: 1e-12, 1: 1e-5, 2: 2e-2, 3: 1e-5}[prec]
    r = oracle.apply_h(p, p.psi)
    assert np.max(np.abs(ref.to(torch.complex128).cpu().numpy() - r)) / np.max(np.abs(r)) < tol


def test_too_small_work_space_is_refused():
    b = B()
    p = problem(50)
    dp = b.DeviceProblem(p)
    x = torch.from_numpy(p.psi).cuda()
    nbytes = b.workspace_size(dp)
    ws = torch.empty(nbytes - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(b.AbacusPwError) as e:
        b.apply_h_ws(dp, x, ws)
    assert e.value.name == "EBAD_SHAPE"
