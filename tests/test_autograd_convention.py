"""Pins the oracle's adjoint to PyTorch's complex-gradient convention, on the
CPU, with H as an explicit dense matrix built by the oracle (no FFT, so the
autograd graph is plain torch matmuls)."""
import numpy as np
import torch

import oracle
from paper_2501_08697_amd import workload as W


def test_grad_psi_matches_torch_autograd():
    p = W.make_problem(W.tiny_config(fft=8, ecut=9.0, nb=3, kfrac=((0.1, 0.2, 0.0),), lmax=2, natom=2,
                                     with_grad_inputs=True))
    h = torch.from_numpy(oracle.dense_h(p, 0))
    x = torch.from_numpy(p.psi.reshape(p.nb, -1).copy()).requires_grad_(True)
    g = torch.from_numpy(p.dy.reshape(p.nb, -1).copy())
    y = x @ h.T                                  # rows: H x_n
    loss = torch.real(torch.sum(torch.conj(g) * y))
    loss.backward()
    gp, _, _ = oracle.apply_h_backward(p, p.psi, p.dy, want=("psi",))
    assert np.max(np.abs(x.grad.numpy().reshape(-1) - gp)) < 1e-13


def test_grad_v_and_d_match_torch_autograd():
    """H built in torch from V(r) and D: autograd of L = Re <g, H psi> against the oracle adjoint."""
    p = W.make_problem(W.tiny_config(fft=8, ecut=9.0, nb=2, kfrac=((0.1, 0.0, -0.2),), lmax=1, natom=2,
                                     with_grad_inputs=True))
    n = np.prod(p.fft)
    v = torch.from_numpy(p.vloc.copy()).requires_grad_(True)
    d = torch.from_numpy(p.dmat.copy()).requires_grad_(True)
    m = p.miller_k(0)
    kin = torch.from_numpy(oracle.kinetic(p, 0))
    vt = torch.fft.fftn(v.to(torch.complex128)) / n
    dm = (m[:, None, :] - m[None, :, :]) % np.array(p.fft)
    hloc = vt[dm[..., 0], dm[..., 1], dm[..., 2]]
    bk = torch.from_numpy(p.beta_k(0))
    dfull = torch.zeros((p.nproj, p.nproj), dtype=torch.float64)
    o = 0
    for a in range(p.natom):
        lo, hi = p.proj_atom_offset[a], p.proj_atom_offset[a + 1]
        k = hi - lo
        dfull = dfull.index_put((torch.arange(lo, hi)[:, None], torch.arange(lo, hi)[None, :]),
                                d[o:o + k * k].reshape(k, k))
        o += k * k
    hnl = bk.T @ dfull.to(torch.complex128) @ bk.conj()
    h = torch.diag(kin).to(torch.complex128) + hloc + hnl
    x = torch.from_numpy(p.psi.reshape(p.nb, -1).copy())
    g = torch.from_numpy(p.dy.reshape(p.nb, -1).copy())
    loss = torch.real(torch.sum(torch.conj(g) * (x @ h.T)))
    loss.backward()
    _, gv, gd = oracle.apply_h_backward(p, p.psi, p.dy, want=("v", "d"))
    assert np.max(np.abs(v.grad.numpy() - gv)) < 1e-14
    assert np.max(np.abs(d.grad.numpy() - gd)) < 1e-13
