"""H psi over several uneven k-points in one call, captured in a HIP graph.

After a warm-up call (which builds the plan and its work space), abacus_pw_apply_h
only enqueues kernels on the caller's stream: no allocation, no memset, no
synchronisation. So torch.cuda.graph can capture it. Each replay is compared
bit for bit with the eager result, with other eager work on the device between
replays.
"""
import numpy as np
import pytest

import oracle
from paper_2501_08697_amd import workload as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def B():
    from paper_2501_08697_amd import binding
    return binding


def multi_k():
    return W.make_problem(W.tiny_config(fft=24, ecut=24.0, a=8.0, nb=20, natom=4,
                                        kfrac=((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.5, 0.5))))


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_is_bitwise_eager(prec):
    b = B()
    p = multi_k()
    print(f"[graph] fft={p.fft} npw={list(p.npw)} nb={p.nb} prec={prec}", flush=True)
    dp = b.DeviceProblem(p, static=True)   # kept alive and unchanged through the replays
    x = torch.from_numpy(p.psi).cuda()
    if prec == b.FP32:
        x = x.to(torch.complex64)
    ref = b.apply_h(dp, x, prec)           # warm-up + eager reference
    torch.cuda.synchronize()
    y = torch.empty_like(x)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.apply_h(dp, x, prec, out=y)
    for rep in range(4):
        y.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()   # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), rep
        del junk
    tol = 1e-12 if prec == b.FP64 else 1e-5
    r = oracle.apply_h(p, p.psi)
    assert np.max(np.abs(ref.cpu().numpy() - r)) / np.max(np.abs(r)) < tol


def test_batched_k_equals_single_k_calls():
    """All k-points in one call (one launch per pass) == each k-point alone, bit for bit."""
    b = B()
    p = multi_k()
    dp = b.DeviceProblem(p)
    x = torch.from_numpy(p.psi).cuda()
    y = b.apply_h(dp, x).cpu().numpy()
    for k in range(p.nk):
        sub = p.single_k(k)
        dk = b.DeviceProblem(sub)
        yk = b.apply_h(dk, torch.from_numpy(sub.psi).cuda()).cpu().numpy()
        assert np.array_equal(yk, p.psi_k(k, y).reshape(-1)), k
