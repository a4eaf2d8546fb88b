"""GPU band density (abacus_pw_density) against the FP64 oracle.

Small cases compare every grid point. At the full grids of the larger
workloads a weight vector that is zero except on a few sampled bands keeps the
oracle's work small while the GPU still runs the full launch configuration
(adding zero-weight terms is exact); Parseval's identity checks the sum over
all bands at any size.
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


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def gpu_density(prob, occ, prec=0, psi=None):
    b = B()
    x = prob.psi if psi is None else psi
    print(f"[density] {prob.name} fft={prob.fft} npw={list(prob.npw)} nb={prob.nb} prec={prec}", flush=True)
    dp = b.DeviceProblem(prob)
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    if prec == b.FP32:
        t = t.to(torch.complex64)
    rho = b.density(dp, t, occ, precision=prec)
    torch.cuda.synchronize()
    return rho.cpu().numpy()


def parseval(prob, occ):
    n = np.prod(prob.fft)
    return n * sum(float(occ[k] @ np.sum(np.abs(prob.psi_k(k)) ** 2, axis=1)) for k in range(prob.nk))


@pytest.mark.parametrize("fft", [8, 12, 20])
def test_tiny_two_kpoints(fft):
    p = W.make_problem(W.tiny_config(fft=fft, ecut=9.0, kfrac=((0.1, 0.2, -0.1), (0.5, 0.0, 0.0)), natom=2, nb=3))
    occ = W.band_weights(p, 1)
    assert rel(gpu_density(p, occ), oracle.density(p, p.psi, occ)) < 1e-12


def test_c1():
    p = W.make_problem("C1")
    occ = W.band_weights(p, 2)
    assert rel(gpu_density(p, occ), oracle.density(p, p.psi, occ)) < 1e-12


@pytest.mark.parametrize("nb", [128, 37, 1])
def test_c2_bands(nb):
    """All 128 bands of the benchmark cell, a ragged band count and a single band."""
    p = W.make_problem("C2", nb=nb)
    occ = W.band_weights(p, 3)
    rho = gpu_density(p, occ)
    ref = oracle.density(p, p.psi, occ)
    assert rel(rho, ref) < 1e-12
    assert abs(np.sum(rho) - parseval(p, occ)) < 1e-12 * parseval(p, occ)


def test_c2_fp32_bound():
    """complex64 psi, FP32 transforms, FP64 accumulation: relative max-norm error below 5e-6."""
    p = W.make_problem("C2", nb=32)
    occ = W.band_weights(p, 4)
    err = rel(gpu_density(p, occ, prec=B().FP32), oracle.density(p, p.psi, occ))
    print(f"[density] FP32 relative max-norm error {err:.2e}")
    assert err < 5e-6


@pytest.mark.parametrize("name", ["C5", "C3", "C4"])
def test_full_grids_sampled_bands(name):
    """Full grid and spheres (uneven k-points for C3/C5); the oracle covers two sampled bands per k."""
    nb = {"C5": 256, "C3": 8, "C4": 8}[name]
    p = W.make_problem(name, nb=nb)
    occ = np.zeros((p.nk, p.nb))
    rng = np.random.default_rng(7)
    for k in range(p.nk):
        occ[k, rng.choice(p.nb, size=2, replace=False)] = rng.uniform(0.5, 2.0, size=2)
    rho = gpu_density(p, occ)
    assert rel(rho, oracle.density(p, p.psi, occ)) < 1e-12
    if name == "C5":
        full = W.band_weights(p, 5)
        tot = float(np.sum(gpu_density(p, full)))
        assert abs(tot - parseval(p, full)) < 1e-12 * parseval(p, full)


def test_zero_weights_and_repeatable():
    p = W.make_problem("C1")
    assert np.all(gpu_density(p, np.zeros((p.nk, p.nb))) == 0.0)
    occ = W.band_weights(p, 6)
    occ[0, ::2] *= -1.0   # any real weights
    a, b2 = gpu_density(p, occ), gpu_density(p, occ)
    assert np.array_equal(a, b2)
    assert rel(a, oracle.density(p, p.psi, occ)) < 1e-12


def test_rejects_bad_arguments():
    b = B()
    p = W.make_problem(W.tiny_config(fft=8, ecut=6.0, nb=2))
    dp = b.DeviceProblem(p)
    x = torch.from_numpy(p.psi).cuda()
    with pytest.raises(b.AbacusPwError) as e:
        b.density(dp, x, np.ones((p.nk, p.nb)), precision=b.MIXED_BF16)
    assert e.value.name == "EBAD_PRECISION"
    with pytest.raises(b.AbacusPwError) as e:
        b.density(dp, x, np.ones(p.nb + 1))
    assert e.value.name == "EBAD_SHAPE"
    cp = dp.c()
    rho = torch.empty(dp.fft, dtype=torch.float64, device="cuda")
    import ctypes as C
    code = b.lib().abacus_pw_density(C.byref(cp), 0, p.nb, x.data_ptr(), None, rho.data_ptr(), b._stream())
    assert b.ERRORS[code] == "ENULL_ARG"
