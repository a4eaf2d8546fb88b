"""Pins for the oracle's density transform rho(G) = (1/N) sum_j rho(r_j) e^{-iG.r_j}
(the grid form of the density transform of Sec. III.A), applied to the band
density of the oracle.

Independent of the oracle's FFT: the coefficient autocorrelation
rho(G) = sum_{k,n} occ sum_{G1 - G2 = G (mod grid)} c(G1) conj(c(G2)), summed
pair by pair over the sphere (|psi(r)|^2 expanded in plane waves); a direct
O(N^2) sum of the definition on 8^3 and 6x10x15 grids; the G = 0 value equal
to sum occ ||c||^2 (Parseval); Hermitian symmetry rho(-G) = conj(rho(G)) of a
real density; a single plane wave giving a uniform density. A wrong sign in
the exponent, a missing 1/N or a transposed axis fails the autocorrelation and
the direct sum; a conjugation slip fails the symmetry check.
"""
import numpy as np
import pytest

import oracle
from paper_2501_08697_amd import workload as W


def problem(fft=8, nb=3, kfrac=((0.1, 0.2, -0.1), (0.5, 0.0, 0.0)), ecut=9.0):
    return W.make_problem(W.tiny_config(fft=fft, ecut=ecut, kfrac=kfrac, lmax=1, natom=2, nb=nb))


def autocorrelation(p, occ):
    """rho(G) on the grid from pairs of sphere coefficients, no transform."""
    n = np.array(p.fft)
    out = np.zeros(tuple(p.fft), dtype=np.complex128)
    for k in range(p.nk):
        m = p.miller_k(k)
        c = p.psi_k(k)
        # G1 - G2 for every pair, wrapped onto the grid
        d = (m[:, None, :] - m[None, :, :]) % n
        flat = (d[..., 0] * n[1] + d[..., 1]) * n[2] + d[..., 2]
        for b in range(p.nb):
            pair = occ[k, b] * np.outer(c[b], c[b].conj())      # c(G1) conj(c(G2))
            np.add.at(out.reshape(-1), flat.reshape(-1), pair.reshape(-1))
    return out


def direct_transform(rho):
    n1, n2, n3 = rho.shape
    out = np.zeros(rho.shape, dtype=np.complex128)
    j = [np.arange(x) for x in rho.shape]
    e1 = np.exp(-2j * np.pi * np.outer(j[0], j[0]) / n1)
    e2 = np.exp(-2j * np.pi * np.outer(j[1], j[1]) / n2)
    e3 = np.exp(-2j * np.pi * np.outer(j[2], j[2]) / n3)
    # out[q1,q2,q3] = sum_j rho[j1,j2,j3] e1[q1,j1] e2[q2,j2] e3[q3,j3] / N, term by term over j1
    for q1 in range(n1):
        acc = np.zeros((n2, n3), dtype=np.complex128)
        for j1 in range(n1):
            acc += e1[q1, j1] * (e2 @ rho[j1] @ e3.T)
        out[q1] = acc
    return out / rho.size


@pytest.mark.parametrize("fft", [8, 12])
def test_density_g_matches_coefficient_autocorrelation(fft):
    p = problem(fft=fft)
    occ = W.band_weights(p, 3)
    rg = oracle.density_g(oracle.density(p, p.psi, occ))
    ref = autocorrelation(p, occ)
    assert np.max(np.abs(rg - ref)) < 1e-13 * np.max(np.abs(ref))


def test_density_g_matches_direct_sum():
    rng = np.random.default_rng(7)
    for shape in ((8, 8, 8), (6, 10, 15)):
        rho = rng.standard_normal(shape)
        rg = oracle.density_g(rho)
        ref = direct_transform(rho)
        assert np.max(np.abs(rg - ref)) < 1e-14 * np.max(np.abs(ref)) * 10


def test_density_g_zero_and_hermitian():
    p = problem(fft=12, nb=4)
    occ = W.band_weights(p, 4)
    rg = oracle.density_g(oracle.density(p, p.psi, occ))
    norm = sum(float(occ[k] @ np.sum(np.abs(p.psi_k(k)) ** 2, axis=1)) for k in range(p.nk))
    assert abs(rg[0, 0, 0] - norm) < 1e-13 * norm
    # rho(-G) at index (-i) mod N
    neg = rg[np.ix_(*[(-np.arange(n)) % n for n in rg.shape])]
    assert np.max(np.abs(neg - rg.conj())) < 1e-15 * np.max(np.abs(rg)) * 10


def test_density_g_of_one_plane_wave_is_uniform():
    p = problem(fft=8, nb=1, kfrac=((0.0, 0.0, 0.0),))
    psi = np.zeros_like(p.psi)
    psi[5] = 0.6 - 0.8j                    # one sphere point, |c| = 1
    occ = np.array([[1.7]])
    rg = oracle.density_g(oracle.density(p, psi, occ))
    ref = np.zeros_like(rg)
    ref[0, 0, 0] = 1.7
    assert np.max(np.abs(rg - ref)) < 1e-15


def test_grid_values_at_wraps_negative_indices():
    g = np.arange(4 * 5 * 6).reshape(4, 5, 6).astype(np.complex128)
    m = np.array([[0, 0, 0], [-1, 2, -3], [1, -2, 5]], dtype=np.int32)
    v = oracle.grid_values_at(g, m)
    assert v[0] == g[0, 0, 0] and v[1] == g[3, 2, 3] and v[2] == g[1, 3, 5]
