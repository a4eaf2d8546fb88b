"""The seeded generator: sphere sizes per config, cutoff gaps, grid fit,
byte-for-byte reproducibility and the normalisations it promises."""
import hashlib

import numpy as np
import pytest

from paper_2501_08697_amd import workload as W

# Counts fixed by the strict rule |k+G|^2 < ecut (the configs' approximate
# "about N PWs" figures disagree with their own a and ecut; a and ecut win).
EXPECTED_NPW = {
    "C1": [1503],
    "C2": [23847],
    "C4": [161235],
    "C5": [48489, 48342, 48352, 48056],
    "C3": [115313, 115396, 115396, 115244, 115396, 115244, 115244, 115096],
}


@pytest.mark.parametrize("name", sorted(EXPECTED_NPW))
def test_sphere_sizes(name):
    cfg = W.CONFIGS[name]
    lat = np.eye(3) * cfg.a
    b = W.reciprocal(lat)
    got = [W.g_sphere(lat, np.asarray(kf) @ b, cfg.ecut).shape[0] for kf in cfg.kfrac]
    assert got == EXPECTED_NPW[name]


def test_sphere_order_and_fit():
    p = W.make_problem("C1")
    b = W.reciprocal(p.lattice)
    kg = p.miller @ b
    kg2 = np.sum(kg * kg, axis=1)
    assert np.all(np.diff(np.round(kg2, 9)) >= 0)
    assert np.all(kg2 < p.ecut)
    assert len({tuple(m) for m in p.miller}) == p.miller.shape[0]
    for i in range(3):
        assert 2 * np.max(np.abs(p.miller[:, i])) + 1 <= p.fft[i]


def _digest(p):
    h = hashlib.sha256()
    for a in (p.miller, p.vloc, p.beta, p.dmat, p.psi):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_reproducible_bytes():
    assert _digest(W.make_problem("C1")) == _digest(W.make_problem("C1"))
    assert _digest(W.make_problem("C1")) != _digest(W.make_problem("C1", seed=99))


def test_normalisations_c1():
    p = W.make_problem("C1")
    x = p.psi_k(0)
    assert np.max(np.abs(x.conj() @ x.T - np.eye(p.nb))) < 1e-14
    assert np.max(np.abs(np.linalg.norm(p.beta_k(0), axis=1) - 1.0)) < 1e-14
    for a in range(p.natom):
        d = p.dblock(a)
        assert np.all(d == d.T)
        assert np.all(np.diag(d) >= 0.1) and np.all(np.diag(d) <= 1.0)
    assert p.vloc.max() < 0.0 and p.vloc.min() > -2.0 * 8


def test_full_d_blocks_symmetric():
    cfg = W.tiny_config(lmax=2, dfull=True, natom=3)
    p = W.make_problem(cfg)
    assert p.nproj == 27
    for a in range(p.natom):
        d = p.dblock(a)
        assert d.shape == (9, 9)
        assert np.all(d == d.T) and np.all(np.abs(d) <= 1.0)


def test_projectors_real_in_real_space():
    """(-i)^l keeps beta(r) real: beta(-k-G) = conj(beta(k+G)) pointwise."""
    lat = np.eye(3) * 7.0
    b = W.reciprocal(lat)
    k = np.array([0.1, -0.2, 0.05]) @ b
    m = W.g_sphere(lat, k, 9.0)
    tau = np.array([[1.0, 2.0, 3.0]])
    bp = W.projectors(lat, k, m, tau, 2)
    bm = W.projectors(lat, -k, -m, tau, 2)
    assert np.max(np.abs(bm - bp.conj())) < 1e-14


def test_vloc_matches_direct_image_sum():
    lat = np.eye(3) * 6.0
    tau = np.array([[1.0, 5.5, 3.0], [4.0, 0.2, 2.5]])
    d = np.array([-1.0, -0.7])
    sep = W.gaussian_vloc(lat, (8, 8, 8), tau, d)
    direct = W._gaussian_vloc_direct(lat, (8, 8, 8), tau, d, W.VLOC_WIDTH)
    assert np.max(np.abs(sep - direct)) < 1e-14
