"""Pins for the oracle's own FFT: closed forms, brute-force DFT, invariants,
and numpy.fft as a third-party cross-check."""
import numpy as np
import pytest

import oracle

LENGTHS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32, 36, 45, 60, 64, 72, 96, 120, 128]


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 12])
def test_dft_closed_forms(n):
    # A delta at j0 transforms to exp(sign 2 pi i j0 k / n); a pure exponential to n delta.
    for j0 in range(n):
        x = np.zeros(n, dtype=complex)
        x[j0] = 1.0
        k = np.arange(n)
        for sign in (+1, -1):
            np.testing.assert_allclose(oracle.dft1d(x, sign), np.exp(sign * 2j * np.pi * j0 * k / n), atol=1e-14)
        e = np.exp(2j * np.pi * j0 * np.arange(n) / n)
        y = oracle.dft1d(e, -1)
        want = np.zeros(n)
        want[j0] = n
        np.testing.assert_allclose(y, want, atol=1e-12)


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_direct_dft(n):
    x = _rand(n, n)
    for sign in (+1, -1):
        y = oracle.fft1d(x, sign)
        ref = oracle.dft1d(x, sign)
        assert np.max(np.abs(y - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_numpy(n):
    x = _rand(n, 100 + n)
    np.testing.assert_allclose(oracle.fft1d(x, -1), np.fft.fft(x), atol=1e-12 * n)
    np.testing.assert_allclose(oracle.fft1d(x, +1), np.fft.ifft(x) * n, atol=1e-12 * n)


@pytest.mark.parametrize("n", [8, 72, 120])
def test_fft_inverse_and_parseval(n):
    x = _rand(n, 7)
    X = oracle.fft1d(x, -1)
    assert abs(np.sum(np.abs(X) ** 2) - n * np.sum(np.abs(x) ** 2)) <= 1e-12 * n * np.sum(np.abs(x) ** 2)
    back = oracle.fft1d(X, +1) / n
    assert np.max(np.abs(back - x)) <= 1e-14 * n


def _brute_3d(g, sign):
    """Y[k] = sum_j g[j] exp(sign 2 pi i sum_l k_l j_l / N_l), one big explicit sum."""
    n1, n2, n3 = g.shape
    j = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 3)
    frac = j / np.array([n1, n2, n3], dtype=float)
    ph = np.exp(sign * 2j * np.pi * (j @ frac.T))   # [k][j]: k . (j / N)
    return (ph @ g.reshape(-1)).reshape(g.shape)


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 6, 6), (10, 10, 10), (12, 12, 12), (6, 10, 15), (15, 15, 15)])
def test_fft3d_matches_brute_force(shape):
    g = _rand(shape, 3)
    for sign in (+1, -1):
        got = oracle.fft3d(g, sign)
        ref = _brute_3d(g, sign)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_fft3d_roundtrip_and_numpy():
    g = _rand((32, 24, 20), 5)
    fwd = oracle.fft3d(g, -1)
    np.testing.assert_allclose(fwd, np.fft.fftn(g), atol=1e-10)
    back = oracle.fft3d(fwd, +1) / g.size
    assert np.max(np.abs(back - g)) < 1e-13
