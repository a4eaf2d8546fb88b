"""Pins for the oracle's H psi (Sec. III.A plane-wave KS equation with the
local + Kleinman-Bylander split of Sec. II.A) against closed forms, an
FFT-free explicit matrix, physical invariances and third-party routines."""
import dataclasses
import math
import os

import numpy as np
import pytest

import oracle
from paper_2501_08697_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(**kw):
    return W.make_problem(W.tiny_config(**kw))


def zeroed(p, v=True, d=True):
    q = dataclasses.replace(p)
    if v:
        q.vloc = np.zeros_like(p.vloc)
    if d:
        q.dmat = np.zeros_like(p.dmat)
    return q


def kinetic_closed_form(p, k):
    """|k+G|^2 from the Miller indices, with b = 2 pi A^{-T} computed by numpy."""
    b = 2 * np.pi * np.linalg.inv(p.lattice).T
    q = p.kpts[k][None, :] + p.miller_k(k) @ b
    return np.sum(q * q, axis=1)


def test_free_electron_h_is_diagonal_kinetic():
    p = zeroed(tiny(kfrac=((0.1, -0.2, 0.3),), nb=3))
    y = oracle.apply_h(p, p.psi).reshape(p.nb, -1)
    want = kinetic_closed_form(p, 0)[None, :] * p.psi.reshape(p.nb, -1)
    assert np.max(np.abs(y - want)) <= 1e-14 * np.max(np.abs(want))


def test_free_electron_c1_shells_match_golden():
    """V=0, D=0 at C1: the spectrum is the sorted (2 pi / a)^2 |m|^2 (golden table)."""
    p = zeroed(W.make_problem("C1"))
    h = oracle.dense_h(p, 0)
    ev = np.linalg.eigvalsh(h)[:20]
    gold = np.loadtxt(os.path.join(GOLDEN, "free_electron_c1.txt"))
    np.testing.assert_allclose(ev, gold, atol=1e-13)


def test_constant_potential_shifts_spectrum():
    p = tiny(nb=4)
    c = -0.731
    q = dataclasses.replace(p, vloc=p.vloc + c)
    y0 = oracle.apply_h(p, p.psi)
    y1 = oracle.apply_h(q, p.psi)
    assert np.max(np.abs(y1 - y0 - c * p.psi)) < 1e-13


@pytest.mark.parametrize("kw", [
    dict(),
    dict(kfrac=((0.25, 0.1, -0.3),)),
    dict(fft=6, ecut=5.0),
    dict(lmax=2, dfull=True, natom=3),
])
def test_fft_route_equals_explicit_matrix(kw):
    p = tiny(**kw)
    h = oracle.dense_h(p, 0, direct=True)
    y = oracle.apply_h(p, p.psi).reshape(p.nb, -1)
    ref = (h @ p.psi.reshape(p.nb, -1).T).T
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_non_orthogonal_cell_fft_equals_explicit_matrix():
    lat = np.array([[6.0, 0.0, 0.0], [1.5, 5.5, 0.0], [0.7, -0.4, 6.2]])
    p = W.make_problem(W.tiny_config(ecut=7.0, fft=8, kfrac=((0.2, 0.0, 0.1),)), lattice=lat)
    h = oracle.dense_h(p, 0, direct=True)
    y = oracle.apply_h(p, p.psi).reshape(p.nb, -1)
    ref = (h @ p.psi.reshape(p.nb, -1).T).T
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_local_matrix_elements_against_numpy_fft():
    """H[G][G'] - kinetic - nonlocal = numpy-fftn(V)[(m-m') mod N] / N (third-party transform)."""
    p = tiny(kfrac=((0.1, 0.2, 0.0),))
    h = oracle.dense_h(zeroed(p, v=False, d=True), 0, direct=False)
    kin = kinetic_closed_form(p, 0)
    vt = np.fft.fftn(p.vloc) / p.vloc.size
    m = p.miller_k(0)
    dm = (m[:, None, :] - m[None, :, :]) % np.array(p.fft)
    ref = vt[dm[..., 0], dm[..., 1], dm[..., 2]] + np.diag(kin)
    assert np.max(np.abs(h - ref)) < 1e-14


def test_c1_fft_route_equals_explicit_matrix():
    p = W.make_problem("C1")
    h = oracle.dense_h(p, 0)
    y = oracle.apply_h(p, p.psi).reshape(p.nb, -1)
    ref = (h @ p.psi.reshape(p.nb, -1).T).T
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_hermiticity():
    p = tiny(lmax=2, dfull=True, natom=3, kfrac=((0.3, 0.1, 0.2),), nb=6)
    x = p.psi.reshape(p.nb, -1)
    y = oracle.apply_h(p, p.psi).reshape(p.nb, -1)
    m = x.conj() @ y.T          # <x_i | H x_j>
    scale = np.max(np.abs(np.linalg.eigvalsh(oracle.dense_h(p, 0))))
    assert np.max(np.abs(m - m.conj().T)) <= 1e-13 * scale


def test_translation_covariance():
    """Shift V by a grid vector t and every atom by t: H' psi' = (H psi)' with psi'(G) = psi(G) e^{-i(k+G).t}."""
    cfg = W.tiny_config(fft=8, kfrac=((0.2, -0.1, 0.3),), lmax=2, natom=2, nb=3)
    p = W.make_problem(cfg)
    shift = np.array([3, 1, 6])
    t = (shift / np.array(p.fft)) @ p.lattice
    q = dataclasses.replace(p)
    q.vloc = np.roll(p.vloc, tuple(shift), axis=(0, 1, 2))
    q.beta = W.projectors(p.lattice, p.kpts[0], p.miller_k(0), p.tau + t, cfg.lmax).reshape(-1)
    b = 2 * np.pi * np.linalg.inv(p.lattice).T
    kg = p.kpts[0][None, :] + p.miller_k(0) @ b
    ph = np.exp(-1j * (kg @ t))
    x = p.psi.reshape(p.nb, -1)
    y = oracle.apply_h(p, p.psi).reshape(p.nb, -1)
    yq = oracle.apply_h(q, (x * ph).reshape(-1)).reshape(p.nb, -1)
    assert np.max(np.abs(yq - y * ph)) < 1e-13 * np.max(np.abs(y))


def test_time_reversal_spectrum():
    """Real V and real-space-real projectors: spec H(k) = spec H(-k)."""
    kf = (0.2, -0.15, 0.35)
    p = W.make_problem(W.tiny_config(kfrac=(kf,), lmax=2, dfull=True, natom=2))
    m = W.make_problem(W.tiny_config(kfrac=(tuple(-x for x in kf),), lmax=2, dfull=True, natom=2))
    e1 = np.linalg.eigvalsh(oracle.dense_h(p, 0))
    e2 = np.linalg.eigvalsh(oracle.dense_h(m, 0))
    assert np.max(np.abs(e1 - e2)) < 1e-12


def _secular_roots(kappa, w, d, count):
    """Lowest eigenvalues of diag(kappa) + d beta beta^H (d > 0) by bisection on
    1 = d sum_s w_s / (lam - kappa_s), shells s of equal kappa (w_s = sum |beta|^2)."""
    order = np.argsort(kappa)
    kappa, w = kappa[order], w[order]
    shells, sw, mult = [], [], []
    for kv, wv in zip(kappa, w):
        if shells and abs(kv - shells[-1]) < 1e-9:
            sw[-1] += wv
            mult[-1] += 1
        else:
            shells.append(kv)
            sw.append(wv)
            mult.append(1)
    shells, sw = np.array(shells), np.array(sw)

    def f(lam):
        return 1.0 - d * np.sum(sw / (lam - shells))

    out = []
    for s in range(len(shells)):
        out += [shells[s]] * (mult[s] - 1)       # directions orthogonal to beta inside the shell
        lo = shells[s]
        hi = shells[s + 1] if s + 1 < len(shells) else shells[s] + d * np.sum(sw) + 1.0
        a, b = lo + 1e-15 * max(1.0, abs(lo)), hi - 1e-15 * max(1.0, abs(hi))
        for _ in range(200):
            mid = 0.5 * (a + b)
            if f(mid) < 0.0:
                a = mid
            else:
                b = mid
        out.append(0.5 * (a + b))
        if len(out) > count + 40:
            break
    return np.sort(np.array(out))[:count]


def test_rank_one_nonlocal_secular_equation():
    p = W.make_problem(W.tiny_config(natom=1, lmax=0, kfrac=((0.1, 0.05, -0.2),), ecut=10.0))
    p = zeroed(p, v=True, d=False)
    d = float(p.dmat[0])
    h = oracle.dense_h(p, 0)
    kin = kinetic_closed_form(p, 0)
    w = np.abs(p.beta_k(0)[0]) ** 2
    ref = _secular_roots(kin, w, d, 30)
    ev = np.linalg.eigvalsh(h)[:30]
    np.testing.assert_allclose(ev, ref, atol=1e-11)


def test_davidson_matches_dense_eig_c1_within_residual_bounds():
    """C1, 20 iterations: Davidson eigenvalues vs dense eig, within Kato-Temple r^2/gap and r."""
    p = W.make_problem("C1")
    h = oracle.dense_h(p, 0)
    ev = np.linalg.eigvalsh(h)
    eig, psi, res, it = oracle.davidson(p, tol=1e-13, max_iter=20)
    assert it[0] == 20
    lam, r = eig[0], res[0]
    assert np.all(np.diff(lam) >= -1e-14)
    for n in range(p.nb):
        j = np.argmin(np.abs(ev - lam[n]))
        gap = np.min(np.abs(np.delete(ev, j) - lam[n]))
        err = abs(lam[n] - ev[j])
        assert err <= r[n] * (1 + 1e-9) + 1e-13                 # Krylov-Weinstein
        if gap > r[n]:
            assert err <= r[n] ** 2 / (gap - r[n]) + 1e-13      # Kato-Temple
    # converged bands agree with the dense spectrum tightly
    good = r < 1e-9
    assert np.sum(good) >= 7
    np.testing.assert_allclose(lam[good], ev[: p.nb][good], atol=1e-12)


def test_davidson_converges_to_dense_lowest_states_tiny():
    p = tiny(nb=5, ecut=10.0, kfrac=((0.1, 0.0, 0.2),), lmax=2, natom=2)
    ev = np.linalg.eigvalsh(oracle.dense_h(p, 0))[: p.nb]
    eig, psi, res, it = oracle.davidson(p, tol=1e-11, max_iter=300)
    assert np.max(res) < 1e-11
    np.testing.assert_allclose(eig[0], ev, atol=1e-12)
    x = psi.reshape(p.nb, -1)
    assert np.max(np.abs(x.conj() @ x.T - np.eye(p.nb))) < 1e-12


def test_davidson_free_electron_closed_form():
    p = zeroed(tiny(nb=7, ecut=10.0, fft=8))
    kin = np.sort(kinetic_closed_form(p, 0))
    eig, psi, res, it = oracle.davidson(p, tol=1e-12, max_iter=100)
    np.testing.assert_allclose(eig[0], kin[:7], atol=1e-12)


def test_davidson_locking_matches_dense():
    """Bands locked at restarts stay eigenpairs; the active ones converge in their complement.

    A projection of the corrections that missed the locked vectors would let active
    bands converge onto locked eigenpairs (repeated eigenvalues), and a wrong merge
    would break the ascending order: both fail the dense comparison.
    """
    p = tiny(nb=8, ecut=12.0, kfrac=((0.1, 0.0, 0.2),), lmax=2, natom=2, fft=16)
    h = oracle.dense_h(p, 0)
    ev = np.linalg.eigvalsh(h)[: p.nb]
    sub = oracle._single_k(p, 0)

    def hop(rows):
        return oracle.apply_h(sub, rows.reshape(-1), nb=rows.shape[0]).reshape(rows.shape)

    info = {}
    eig, x, res, it = oracle.davidson_k(hop, p.psi.reshape(p.nb, -1), oracle.kinetic(sub, 0), 1e-11, 300, 2,
                                        info=info)
    assert info["locked"] > 0 and info["restarts"] > 0
    np.testing.assert_allclose(eig, ev, atol=1e-12)
    assert np.max(np.abs(x.conj() @ x.T - np.eye(p.nb))) < 1e-12
    r = np.linalg.norm(x @ h.T - eig[:, None] * x, axis=1)
    assert np.max(r) < 1e-11
    np.testing.assert_allclose(r, res, atol=1e-13)
