"""Pins for the oracle's band density rho(r_j) = sum_{k,n} occ[k][n] |psi_nk(r_j)|^2:
a direct sum over the sphere at every grid point (no transform), Parseval's
identity, single plane waves, and agreement with the adjoint's grid gradient."""
import numpy as np

import oracle
from paper_2501_08697_amd import workload as W


def problem(fft=8, nb=3):
    cfg = W.tiny_config(fft=fft, ecut=9.0, kfrac=((0.1, 0.2, -0.1), (0.5, 0.0, 0.0)), lmax=1, natom=2, nb=nb)
    return W.make_problem(cfg)


def direct_density(p, occ):
    """psi(r_j) = sum_G c(G) exp(2 pi i sum_l m_l j_l / N_l), summed term by term."""
    n1, n2, n3 = p.fft
    j = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 3)
    frac = j / np.array(p.fft, dtype=float)
    rho = np.zeros(len(j))
    for k in range(p.nk):
        m = p.miller_k(k).astype(float)
        ph = np.exp(2j * np.pi * (frac @ m.T))         # [N][npw]
        vals = ph @ p.psi_k(k).T                         # [N][nb]
        rho += np.abs(vals) ** 2 @ occ[k]
    return rho.reshape(p.fft)


def test_matches_direct_sum_every_point():
    p = problem()
    occ = W.band_weights(p, 1)
    rho = oracle.density(p, p.psi, occ)
    ref = direct_density(p, occ)
    assert np.max(np.abs(rho - ref)) < 1e-13 * np.max(ref)


def test_direct_sum_radix3_grid():
    p = problem(fft=12, nb=2)
    occ = W.band_weights(p, 2)
    rho = oracle.density(p, p.psi, occ)
    np.testing.assert_allclose(rho, direct_density(p, occ), rtol=0, atol=1e-13 * np.max(rho))


def test_parseval():
    """sum_j |psi(r_j)|^2 = N sum_G |c(G)|^2 for the unnormalised inverse transform."""
    p = W.make_problem("C1")
    occ = W.band_weights(p, 3)
    rho = oracle.density(p, p.psi, occ)
    n = np.prod(p.fft)
    norms = np.array([[np.sum(np.abs(p.psi_k(k)[b]) ** 2) for b in range(p.nb)] for k in range(p.nk)])
    assert abs(np.sum(rho) - n * np.sum(occ * norms)) < 1e-12 * n * np.sum(occ * norms)


def test_single_plane_waves_are_uniform():
    """One coefficient per band: |exp(i G.r)|^2 = 1 at every grid point, so rho = sum occ."""
    p = problem()
    psi = np.zeros_like(p.psi)
    off = p.pw_offsets
    for k in range(p.nk):
        blk = psi[p.nb * off[k]: p.nb * off[k + 1]].reshape(p.nb, -1)
        for b in range(p.nb):
            blk[b, (7 * b + 3 * k + 1) % p.npw[k]] = 1.0
    occ = W.band_weights(p, 4)
    rho = oracle.density(p, psi, occ)
    np.testing.assert_allclose(rho, np.full(p.fft, np.sum(occ)), rtol=1e-14, atol=0)


def test_equals_adjoint_grid_gradient():
    """The adjoint's grad_V for upstream occ * psi is rho / N."""
    p = problem()
    occ = W.band_weights(p, 5)
    off = p.pw_offsets
    dy = np.empty_like(p.psi)
    for k in range(p.nk):
        dy[p.nb * off[k]: p.nb * off[k + 1]] = (occ[k][:, None] * p.psi_k(k)).reshape(-1)
    _, gv, _ = oracle.apply_h_backward(p, p.psi, dy, want=("v",))
    rho = oracle.density(p, p.psi, occ)
    assert np.max(np.abs(gv * np.prod(p.fft) - rho)) < 1e-13 * np.max(rho)
