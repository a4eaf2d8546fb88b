"""GPU nonlocal force (abacus_pw_force_nl) against the FP64 oracle.

The force is a weighted sum over bands: at full size, weights that are zero except
on sampled bands keep the oracle's work small while the GPU runs every band
(zero-weight terms add exactly nothing).
"""
import dataclasses

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


def gpu_force(prob, occ, psi=None):
    b = B()
    print(f"[force] {prob.name} fft={prob.fft} npw={list(prob.npw)} nb={prob.nb} natom={prob.natom} "
          f"nproj={prob.nproj}", flush=True)
    dp = b.DeviceProblem(prob)
    x = torch.from_numpy(np.ascontiguousarray(prob.psi if psi is None else psi)).cuda()
    f = b.force_nl(dp, x, occ)
    torch.cuda.synchronize()
    return f.cpu().numpy()


@pytest.mark.parametrize("lmax,dfull", [(0, False), (1, False), (2, True)])
def test_tiny_two_kpoints(lmax, dfull):
    p = W.make_problem(W.tiny_config(fft=12, ecut=9.0, kfrac=((0.1, 0.2, -0.1), (0.5, 0.0, 0.0)), lmax=lmax,
                                     natom=3, nb=3, dfull=dfull))
    occ = W.band_weights(p, 1)
    assert rel(gpu_force(p, occ), oracle.force_nl(p, p.psi, occ)) < 1e-12


def test_c1():
    p = W.make_problem("C1")
    occ = W.band_weights(p, 2)
    assert rel(gpu_force(p, occ), oracle.force_nl(p, p.psi, occ)) < 1e-12


def test_c2_all_bands():
    p = W.make_problem("C2")
    occ = W.band_weights(p, 3)
    assert rel(gpu_force(p, occ), oracle.force_nl(p, p.psi, occ)) < 1e-12


def sampled(p, nsamp, seed):
    """Weights zero except nsamp bands per k; the oracle's problem restricted to those bands."""
    rng = np.random.default_rng(seed)
    occ = np.zeros((p.nk, p.nb))
    rows = [np.sort(rng.choice(p.nb, size=nsamp, replace=False)) for _ in range(p.nk)]
    off = p.pw_offsets
    sub_psi = []
    sub_occ = np.zeros((p.nk, nsamp))
    for k in range(p.nk):
        w = rng.uniform(0.5, 2.0, size=nsamp)
        occ[k, rows[k]] = w
        sub_occ[k] = w
        sub_psi.append(p.psi[p.nb * off[k]: p.nb * off[k + 1]].reshape(p.nb, -1)[rows[k]].reshape(-1))
    return occ, dataclasses.replace(p, nb=nsamp), np.concatenate(sub_psi), sub_occ


@pytest.mark.parametrize("name,nb", [("C5", 256), ("C4", 8)])
def test_full_size_sampled_bands(name, nb):
    """C5: four uneven k-points, 256 bands; C4: 9 projectors per atom with full D blocks, 128^3."""
    p = W.make_problem(name, nb=nb)
    occ, sub, sub_psi, sub_occ = sampled(p, 3, 7)
    assert rel(gpu_force(p, occ), oracle.force_nl(sub, sub_psi, sub_occ)) < 1e-12


def test_zero_weights_and_repeatable():
    p = W.make_problem("C1")
    assert np.all(gpu_force(p, np.zeros((p.nk, p.nb))) == 0.0)
    occ = W.band_weights(p, 4)
    a, b2 = gpu_force(p, occ), gpu_force(p, occ)
    assert np.array_equal(a, b2)


def test_rejects_bad_arguments():
    b = B()
    p = W.make_problem(W.tiny_config(fft=8, ecut=6.0, nb=2))
    dp = b.DeviceProblem(p)
    x = torch.from_numpy(p.psi).cuda()
    with pytest.raises(b.AbacusPwError) as e:
        b.force_nl(dp, x, np.ones(p.nb + 3))
    assert e.value.name == "EBAD_SHAPE"


def test_no_projectors_gives_zero_force():
    p = W.make_problem(W.tiny_config(fft=8, ecut=6.0, nb=2, natom=2))
    q = dataclasses.replace(p, nproj=0, beta=np.zeros(0, dtype=np.complex128), dmat=np.zeros(0),
                            proj_atom_offset=np.zeros(p.natom + 1, dtype=np.int32))
    f = gpu_force(q, np.ones((q.nk, q.nb)))
    assert f.shape == (q.natom, 3) and np.all(f == 0.0)
