"""The dense FP64 steps of the Davidson iteration on the GPU (abacus_pw_eigh_lowest,
abacus_pw_cholesky) against LAPACK through numpy, at orders on both sides of the
switch from the one-CU kernels to the multi-CU ones (256 for the eigensolver,
136 for Cholesky) and up to the 2048 x 2048 subspace of 1024 bands at ndim 2.

Eigenvalues are compared with numpy.linalg.eigvalsh to 1e-12 of ||A||;
eigenvectors (unique up to a phase) through their residuals ||A x - w x|| and
their orthonormality. Cholesky factors are unique (positive diagonal) and are
compared entry by entry with numpy.linalg.cholesky, and L^{-1} with the
identity L^{-1} L = I.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def B():
    from paper_2501_08697_amd import binding
    return binding


def hermitian(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return spread * 0.5 * (x + x.conj().T)


def clustered(n, seed):
    """Q diag(ev) Q^H with pairs of eigenvalues 1e-9 apart and a few exact repeats."""
    rng = np.random.default_rng(seed)
    ev = np.sort(rng.uniform(-3.0, 3.0, n))
    ev[1::7] = ev[0::7][: len(ev[1::7])] + 1e-9
    ev[2::11] = ev[1::11][: len(ev[2::11])]
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return (q * ev) @ q.conj().T


@pytest.mark.parametrize("n,nw", [(64, 64), (256, 128), (257, 200), (300, 150), (640, 320), (1030, 515),
                                  (2048, 1024), (3000, 64)])
def test_eigh_lowest_against_lapack(n, nw):
    a = hermitian(n, n)
    print(f"[dense] eigh n={n} nw={nw}", flush=True)
    w, v = B().eigh_lowest(torch.from_numpy(a.copy()).cuda(), nw)
    w, v = w.cpu().numpy(), v.cpu().numpy()
    ref = np.linalg.eigvalsh(a)[:nw]
    an = np.max(np.abs(ref)) if nw == n else np.linalg.norm(a, 2)
    assert np.max(np.abs(w - ref)) < 1e-12 * an
    r = np.linalg.norm(v @ a.T - w[:, None] * v, axis=1)      # rows: A x = w x  <=>  x^T A^T = w x^T
    assert np.max(r) < 1e-11 * an
    assert np.max(np.abs(v.conj() @ v.T - np.eye(nw))) < 1e-9


@pytest.mark.parametrize("n", [200, 700])
def test_eigh_lowest_clustered_spectrum(n):
    a = clustered(n, 3 * n)
    w, v = B().eigh_lowest(torch.from_numpy(a.copy()).cuda(), n // 2)
    w, v = w.cpu().numpy(), v.cpu().numpy()
    ref = np.linalg.eigvalsh(a)[: n // 2]
    assert np.max(np.abs(w - ref)) < 1e-12 * 3.0
    r = np.linalg.norm(v @ a.T - w[:, None] * v, axis=1)
    assert np.max(r) < 1e-11 * 3.0
    # clusters are orthogonalised together: the whole set stays orthonormal
    assert np.max(np.abs(v.conj() @ v.T - np.eye(n // 2))) < 1e-9


@pytest.mark.parametrize("n", [1, 40, 136, 137, 200, 513, 1024])
def test_cholesky_against_lapack(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n + 8)) + 1j * rng.standard_normal((n, n + 8))
    g = x @ x.conj().T
    t = torch.from_numpy(g.copy()).cuda()
    li = B().cholesky(t).cpu().numpy()
    L = np.tril(t.cpu().numpy())
    ref = np.linalg.cholesky(g)
    assert np.max(np.abs(L - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(li @ ref - np.eye(n))) < 1e-10
    assert np.max(np.abs(np.triu(li, 1))) == 0.0


@pytest.mark.parametrize("n", [100, 400])
def test_cholesky_reports_indefinite(n):
    g = hermitian(n, 5)
    with pytest.raises(B().AbacusPwError) as e:
        B().cholesky(torch.from_numpy(g).cuda())
    assert e.value.name == "ECHOLESKY"


def test_dense_rejects_bad_sizes():
    b = B()
    a = torch.zeros((8, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(b.AbacusPwError):
        b.eigh_lowest(a, 9)
    with pytest.raises(b.AbacusPwError):
        b.cholesky(torch.zeros((1025, 1025), dtype=torch.complex128, device="cuda"))
