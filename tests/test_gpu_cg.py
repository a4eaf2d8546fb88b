"""GPU band-by-band preconditioned CG (abacus_pw_cg) against the FP64 oracle's
CG (same steps), the explicit H's dense eigenvalues, and the GPU Davidson.

Both CGs start from the same vectors and take the same steps, so their
eigenvalues agree to rounding and their per-band step counts to within a
step or two (a residual that lands near tol may cross it one step earlier or
later).
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


def gpu_cg(prob, tol, max_iter, nb=None):
    b = B()
    nb = prob.nb if nb is None else nb
    print(f"[cg] {prob.name} fft={prob.fft} npw={list(prob.npw)} nb={nb} tol={tol}", flush=True)
    dp = b.DeviceProblem(prob)
    x = torch.from_numpy(np.ascontiguousarray(prob.psi)).cuda()
    eig, res, its, st = b.cg(dp, x, tol=tol, max_iter=max_iter, nb=nb)
    return eig, x.cpu().numpy(), res, its, st


def tiny(**kw):
    cfg = dict(fft=12, ecut=12.0, a=6.0, nb=6, natom=2)
    cfg.update(kw)
    return W.make_problem(W.tiny_config(**cfg))


@pytest.mark.parametrize("kfrac", [((0.0, 0.0, 0.0),), ((0.25, 0.0, 0.5),)])
def test_tiny_against_oracle_cg_and_dense(kfrac):
    p = tiny(kfrac=kfrac)
    eig, psi, res, its, st = gpu_cg(p, 1e-9, 300)
    assert st == 0
    e_o, psi_o, res_o, its_o = oracle.cg(p, tol=1e-9, max_iter=300)
    H = oracle.dense_h(p, 0, direct=True)
    ev = np.linalg.eigvalsh(H)[:p.nb]
    assert np.max(np.abs(eig[0] - ev)) < 1e-11
    assert np.max(np.abs(eig[0] - e_o[0])) < 1e-11
    assert np.max(np.abs(its[0] - its_o[0])) <= 2, (its, its_o)
    x = psi.reshape(p.nb, -1)
    assert np.max(np.abs(x.conj() @ x.T - np.eye(p.nb))) < 1e-12
    r = np.linalg.norm(x @ H.T - eig[0][:, None] * x, axis=1)
    assert np.max(r) < 1.5e-9 and np.max(res) < 1e-9


def test_two_uneven_kpoints():
    p = tiny(nb=4, kfrac=((0.0, 0.0, 0.0), (0.5, 0.5, 0.0)))
    eig, psi, res, its, st = gpu_cg(p, 1e-9, 300)
    assert st == 0
    for k in range(p.nk):
        H = oracle.dense_h(p, k, direct=True)
        assert np.max(np.abs(eig[k] - np.linalg.eigvalsh(H)[:p.nb])) < 1e-11


def test_c1_against_dense_and_davidson():
    p = W.make_problem(W.CONFIGS["C1"])
    eig, psi, res, its, st = gpu_cg(p, 1e-8, 400)
    assert st == 0
    H = oracle.dense_h(p, 0)
    ev = np.linalg.eigvalsh(H)[:p.nb]
    # Kato-Temple: |eps - eps_exact| <= ||r||^2 / gap, far below 1e-10 here
    assert np.max(np.abs(eig[0] - ev)) < 1e-10
    b = B()
    dp = b.DeviceProblem(p)
    x = torch.from_numpy(np.ascontiguousarray(p.psi)).cuda()
    e_dav, r_dav, it_dav, st_dav = b.davidson(dp, x, tol=1e-8, max_iter=200)
    assert st_dav == 0
    assert np.max(np.abs(np.sort(eig[0]) - e_dav[0])) < 1e-10


def test_rejects_bad_arguments():
    b = B()
    p = tiny(nb=4)
    dp = b.DeviceProblem(p)
    x = torch.from_numpy(np.ascontiguousarray(p.psi)).cuda()
    with pytest.raises(b.AbacusPwError) as e:
        b.cg(dp, x, tol=0.0)
    assert e.value.name == "EBAD_SHAPE"
    with pytest.raises(b.AbacusPwError) as e:
        b.cg(dp, x, nb=int(p.npw[0]) + 1)
    assert e.value.name == "EBAD_SHAPE"
