"""FP64 CPU oracle for the plane-wave H psi, its adjoint, the band density, the
nonlocal force, the Chebyshev-filtered application, and block Davidson.

TEST INFRASTRUCTURE ONLY: this package is used by ``tests/``, by the smoke
check and by the benchmark's CPU-baseline leg. The GPU library never imports,
links or calls it, and it shares no code with the GPU library; both only read
the same seeded inputs.

The arithmetic lives in ``oracle.c`` (own mixed-radix FFT, H psi, explicit H
matrix, adjoint, band density); this module loads it with ctypes and holds the block
Davidson driver (``davidson``) and the band-by-band conjugate-gradient
eigensolver (``cg``), written with numpy's dense linear algebra as their
library steps.

Problems are duck-typed: any object with the attributes of the generator's
``Problem`` (lattice, fft, kpts, npw, miller, vloc, nproj, natom,
proj_atom_offset, beta, dmat) works.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("lattice", C.c_double * 9), ("fft", C.c_int * 3), ("nk", C.c_int),
        ("kpts", C.c_void_p), ("npw", C.c_void_p), ("miller", C.c_void_p),
        ("vloc", C.c_void_p), ("nproj", C.c_int), ("natom", C.c_int),
        ("proj_atom_offset", C.c_void_p), ("beta", C.c_void_p), ("dmat", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER(_Problem)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        _lib.oracle_dft1d.argtypes = [i, i, vp, C.c_long, vp]
        _lib.oracle_fft1d.argtypes = [i, i, vp, C.c_long, vp]
        _lib.oracle_fft3d.argtypes = [vp, i, vp]
        _lib.oracle_apply_h.argtypes = [P, i, vp, vp, i]
        _lib.oracle_kinetic.argtypes = [P, i, vp]
        _lib.oracle_dense_h.argtypes = [P, i, i, vp]
        _lib.oracle_apply_h_backward.argtypes = [P, i, vp, vp, vp, vp, vp]
        _lib.oracle_density.argtypes = [P, i, vp, vp, vp]
        _lib.oracle_num_threads.restype = i
        _lib.oracle_set_num_threads.argtypes = [i]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Bound:
    """A C view of a problem that keeps every array it points to alive."""

    def __init__(self, prob, vloc=None, dmat=None):
        self.keep = [
            np.ascontiguousarray(prob.kpts, dtype=np.float64),
            np.ascontiguousarray(prob.npw, dtype=np.int32),
            np.ascontiguousarray(prob.miller, dtype=np.int32),
            np.ascontiguousarray(prob.vloc if vloc is None else vloc, dtype=np.float64),
            np.ascontiguousarray(prob.proj_atom_offset, dtype=np.int32),
            np.ascontiguousarray(prob.beta, dtype=np.complex128),
            np.ascontiguousarray(prob.dmat if dmat is None else dmat, dtype=np.float64),
        ]
        s = _Problem()
        s.lattice[:] = [float(x) for x in np.asarray(prob.lattice, dtype=np.float64).reshape(-1)]
        s.fft[:] = [int(x) for x in prob.fft]
        s.nk = int(len(prob.npw))
        s.kpts, s.npw, s.miller, s.vloc, s.proj_atom_offset, s.beta, s.dmat = [_ptr(a) for a in self.keep]
        s.nproj, s.natom = int(prob.nproj), int(prob.natom)
        self.s = s


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for later oracle calls."""
    lib().oracle_set_num_threads(int(n))


def dft1d(x: np.ndarray, sign: int) -> np.ndarray:
    """Direct O(n^2) DFT: y[k] = sum_j x[j] exp(sign 2 pi i j k / n)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    lib().oracle_dft1d(x.size, sign, _ptr(x), 1, _ptr(y))
    return y


def fft1d(x: np.ndarray, sign: int) -> np.ndarray:
    """Mixed-radix FFT with the same definition as dft1d."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    lib().oracle_fft1d(x.size, sign, _ptr(x), 1, _ptr(y))
    return y


def fft3d(g: np.ndarray, sign: int) -> np.ndarray:
    """3-D transform (unnormalised) of a [n1][n2][n3] array; +1 inverse, -1 forward."""
    out = np.ascontiguousarray(g, dtype=np.complex128).copy()
    nn = np.array(out.shape, dtype=np.int32)
    lib().oracle_fft3d(_ptr(nn), sign, _ptr(out))
    return out


def apply_h(prob, psi: np.ndarray, nb: int | None = None, terms: int = 7, vloc=None, dmat=None) -> np.ndarray:
    """y = H psi on a packed psi (per k a [nb][npw_k] block). terms: 1 kin, 2 local, 4 nonlocal."""
    nb = prob.nb if nb is None else nb
    b = _Bound(prob, vloc, dmat)
    x = np.ascontiguousarray(psi, dtype=np.complex128)
    assert x.size == nb * int(np.sum(prob.npw))
    y = np.empty_like(x)
    lib().oracle_apply_h(C.byref(b.s), nb, _ptr(x), _ptr(y), terms)
    return y


def kinetic(prob, k: int) -> np.ndarray:
    b = _Bound(prob)
    out = np.empty(int(prob.npw[k]))
    lib().oracle_kinetic(C.byref(b.s), k, _ptr(out))
    return out


def dense_h(prob, k: int, direct: bool = False) -> np.ndarray:
    """Explicit H matrix at k-point k (no transform of psi); direct=True also avoids the FFT for V."""
    b = _Bound(prob)
    n = int(prob.npw[k])
    h = np.empty((n, n), dtype=np.complex128)
    lib().oracle_dense_h(C.byref(b.s), k, 1 if direct else 0, _ptr(h))
    return h


def apply_h_backward(prob, psi, dy, nb=None, vloc=None, dmat=None, want=("psi", "v", "d")):
    """Adjoint of y = H psi: returns (grad_psi, grad_v, grad_d), None where not requested."""
    nb = prob.nb if nb is None else nb
    b = _Bound(prob, vloc, dmat)
    x = np.ascontiguousarray(psi, dtype=np.complex128)
    g = np.ascontiguousarray(dy, dtype=np.complex128)
    gp = np.empty_like(x) if "psi" in want else None
    gv = np.empty(tuple(prob.fft)) if "v" in want else None
    gd = np.empty(np.asarray(prob.dmat).size) if "d" in want else None
    lib().oracle_apply_h_backward(C.byref(b.s), nb, _ptr(x), _ptr(g), _ptr(gp), _ptr(gv), _ptr(gd))
    return gp, gv, gd


def density(prob, psi, occ, nb=None):
    """rho(r_j) = sum_{k,n} occ[k][n] |psi_nk(r_j)|^2 on the [N1][N2][N3] grid, with psi_nk(r)
    the unnormalised inverse transform of the coefficients (the k-weighted orbital density of
    Sec. III.C; occ carries the k weight times the occupation)."""
    nb = prob.nb if nb is None else nb
    b = _Bound(prob)
    x = np.ascontiguousarray(psi, dtype=np.complex128)
    w = np.ascontiguousarray(occ, dtype=np.float64).reshape(-1)
    assert x.size == nb * int(np.sum(prob.npw)) and w.size == nb * len(prob.npw)
    rho = np.empty(tuple(prob.fft))
    lib().oracle_density(C.byref(b.s), nb, _ptr(x), _ptr(w), _ptr(rho))
    return rho


def density_g(rho: np.ndarray) -> np.ndarray:
    """rho(G) = (1/N) sum_j rho(r_j) exp(-i G.r_j): the density transform of Sec. III.A,
    rho(G) = (1/Omega) int rho(r) e^{-iG.r} dr, on the grid (the integral becomes the
    grid sum times Omega/N). Entry [i1][i2][i3] holds the G whose Miller indices satisfy
    m = i mod N. The oracle's own forward 3-D transform, then the 1/N."""
    r = np.ascontiguousarray(rho, dtype=np.float64)
    return fft3d(r.astype(np.complex128), -1) / float(r.size)


def grid_values_at(grid: np.ndarray, miller: np.ndarray) -> np.ndarray:
    """Values of a [N1][N2][N3] grid array at Miller triples (index m mod N)."""
    m = np.asarray(miller).reshape(-1, 3)
    n = grid.shape
    return grid[m[:, 0] % n[0], m[:, 1] % n[1], m[:, 2] % n[2]]


# --------------------------------------------------------------------------
# Nonlocal energy and force (Sec. III.A: the Kleinman-Bylander energy and its
# derivative with respect to the atomic positions).
# --------------------------------------------------------------------------

def _kplusg(prob, k):
    """Cartesian k + G of the sphere points of k-point k, [npw][3] (bohr^-1)."""
    a = np.asarray(prob.lattice, dtype=np.float64).reshape(3, 3)
    recip = 2.0 * np.pi * np.linalg.inv(a).T           # rows b_i with a_i . b_j = 2 pi delta_ij
    off = int(np.sum(prob.npw[:k]))
    m = np.asarray(prob.miller).reshape(-1, 3)[off: off + int(prob.npw[k])].astype(np.float64)
    return m @ recip + np.asarray(prob.kpts, dtype=np.float64).reshape(-1, 3)[k]


def _beta_k(prob, k):
    off = int(np.sum(prob.npw[:k]))
    return np.asarray(prob.beta).reshape(-1)[prob.nproj * off: prob.nproj * (off + int(prob.npw[k]))].reshape(
        prob.nproj, int(prob.npw[k]))


def _d_blocks(prob):
    out, o = [], 0
    d = np.asarray(prob.dmat, dtype=np.float64).reshape(-1)
    for a in range(prob.natom):
        lo, hi = int(prob.proj_atom_offset[a]), int(prob.proj_atom_offset[a + 1])
        out.append((lo, hi, d[o: o + (hi - lo) ** 2].reshape(hi - lo, hi - lo)))
        o += (hi - lo) ** 2
    return out


def nonlocal_energy(prob, psi, occ, nb=None, shift=None):
    """E_NL = sum_k sum_n occ[k][n] sum_a sum_{i,j in a} conj(P_in) D^a_ij P_jn, P = B^H psi.
    shift ([natom][3] bohr) moves the atoms: the projectors carry exp(-i (k+G).tau_a), so
    moving atom a by delta multiplies its projectors by exp(-i (k+G).delta)."""
    nb = prob.nb if nb is None else nb
    occ = np.asarray(occ, dtype=np.float64).reshape(len(prob.npw), nb)
    x = np.asarray(psi)
    e = 0.0
    off = 0
    for k in range(len(prob.npw)):
        npw = int(prob.npw[k])
        bk = _beta_k(prob, k).copy()
        if shift is not None:
            kg = _kplusg(prob, k)
            for a, (lo, hi, _) in enumerate(_d_blocks(prob)):
                bk[lo:hi] *= np.exp(-1j * (kg @ np.asarray(shift[a], dtype=np.float64)))[None, :]
        xk = x[nb * off: nb * (off + npw)].reshape(nb, npw)
        P = bk.conj() @ xk.T                                  # [nproj][nb]
        for lo, hi, d in _d_blocks(prob):
            q = P[lo:hi]
            e += float(np.real(np.sum(occ[k][None, :] * (q.conj() * (d @ q)))))
        off += npw
    return e


def force_nl(prob, psi, occ, nb=None):
    """F[a][alpha] = -dE_NL/dtau_{a,alpha} = -2 sum_k sum_n occ[k][n] sum_{i,j in a}
    D^a_ij Im(conj(P^alpha_in) P_jn), with P = B^H psi and P^alpha = B^H ((k+G)_alpha psi)
    (d beta / d tau_alpha = -i (k+G)_alpha beta). Ry / bohr."""
    nb = prob.nb if nb is None else nb
    occ = np.asarray(occ, dtype=np.float64).reshape(len(prob.npw), nb)
    x = np.asarray(psi)
    f = np.zeros((prob.natom, 3))
    off = 0
    for k in range(len(prob.npw)):
        npw = int(prob.npw[k])
        bk = _beta_k(prob, k)
        kg = _kplusg(prob, k)
        xk = x[nb * off: nb * (off + npw)].reshape(nb, npw)
        P = bk.conj() @ xk.T
        for al in range(3):
            Pa = bk.conj() @ (xk * kg[None, :, al]).T
            for a, (lo, hi, d) in enumerate(_d_blocks(prob)):
                z = Pa[lo:hi].conj() * (d @ P[lo:hi])            # [i][n]: conj(P^a_in) sum_j D_ij P_jn
                f[a, al] -= 2.0 * float(np.sum(occ[k][None, :] * np.imag(z)))
        off += npw
    return f


# --------------------------------------------------------------------------
# Chebyshev-filtered application (Sec. III.C: the stochastic orbitals are
# filtered by f_H^{1/2}, expanded in Chebyshev polynomials of the scaled H).
# --------------------------------------------------------------------------

def chebyshev(prob, chi, coef, emin, emax, nb=None):
    """out = sum_n coef[n] T_n(Hs) chi with Hs = (H - c) / h, c = (emax + emin) / 2,
    h = (emax - emin) / 2, by the three-term recurrence T_{n+1} = 2 Hs T_n - T_{n-1}
    (T_0 = 1, T_1 = Hs) on the packed block chi (per k a [nb][npw_k] block)."""
    nb = prob.nb if nb is None else nb
    coef = np.asarray(coef, dtype=np.float64)
    c, h = 0.5 * (emax + emin), 0.5 * (emax - emin)
    v0 = np.ascontiguousarray(chi, dtype=np.complex128)
    out = coef[0] * v0
    if coef.size == 1:
        return out
    v1 = (apply_h(prob, v0, nb=nb) - c * v0) / h
    out = out + coef[1] * v1
    for n in range(2, coef.size):
        v2 = 2.0 * (apply_h(prob, v1, nb=nb) - c * v1) / h - v0
        out = out + coef[n] * v2
        v0, v1 = v1, v2
    return out


def fermi_sqrt_coefficients(order, emin, emax, mu, kt, power=0.5):
    """Chebyshev interpolation coefficients (degree ``order``) of f(E)^power on [emin, emax],
    f the Fermi-Dirac function 1 / (1 + exp((E - mu) / kt)) of Sec. III.C, via numpy's
    Chebyshev interpolation at the Chebyshev points of the first kind."""
    c, h = 0.5 * (emax + emin), 0.5 * (emax - emin)

    def f(x):
        z = (c + h * x - mu) / kt
        ez = np.exp(-np.abs(z))                    # the tail without cancellation
        return np.where(z > 0, ez / (1.0 + ez), 1.0 / (1.0 + ez)) ** power

    return np.polynomial.chebyshev.chebinterpolate(f, order)


# --------------------------------------------------------------------------
# Block Davidson (Sec. III.B names Davidson as the default eigensolver but
# gives no steps; this is the block scheme the library implements, with the
# Teter-Payne-Allan preconditioner that the paper cites for its CG solver).
# --------------------------------------------------------------------------

def tpa_preconditioner(kin: np.ndarray, ekin: np.ndarray) -> np.ndarray:
    """K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4), x = |k+G|^2 / max(E_kin, 1e-3)."""
    x = kin[None, :] / np.maximum(ekin, 1e-3)[:, None]
    num = 27.0 + 18.0 * x + 12.0 * x * x + 8.0 * x ** 3
    return num / (num + 16.0 * x ** 4)


def _gram(a, b):
    """M[i, j] = <a_i | b_j> for row-stacked vectors."""
    return a.conj() @ b.T


def cholqr(x: np.ndarray) -> np.ndarray:
    """One Cholesky-QR pass on the rows of x; shifted Cholesky-QR if S is not positive definite."""
    s = _gram(x, x)
    s = 0.5 * (s + s.conj().T)
    try:
        l = np.linalg.cholesky(s.T)
    except np.linalg.LinAlgError:
        m, n = x.shape
        shift = 11.0 * (m * n + m * (m + 1)) * np.finfo(float).eps * np.trace(s).real
        l = np.linalg.cholesky(s.T + shift * np.eye(m))
    import scipy.linalg as sla
    return sla.solve_triangular(l, x, lower=True)


def davidson_k(hop, psi0: np.ndarray, kin: np.ndarray, tol: float, max_iter: int, ndim: int = 2,
               drop: float = 1e-10, info: dict | None = None):
    """Lowest nb eigenpairs of the Hermitian operator hop (rows in, rows out).

    1. Cholesky-QR psi0; W = H psi; Rayleigh-Ritz.
    2. Repeat: residuals R = W - psi Lambda and their 2-norms; stop when all < tol.
       Preconditioned corrections T = K (.) R for unconverged bands. When the
       basis would exceed ndim*nb vectors it is restarted to the current Ritz
       vectors, and at that restart every band whose residual is already below
       tol is locked: its Ritz pair is frozen and leaves the Rayleigh-Ritz
       problem. T is projected out of the locked vectors and the basis twice
       (classical Gram-Schmidt, twice), columns whose norm fell below ``drop`` of
       their pre-projection norm are dropped, Cholesky-QR twice; append T and HT;
       Rayleigh-Ritz on the whole basis keeping the lowest nb - (locked) pairs.
    The result merges locked and active pairs in ascending order of their Ritz
    values (a stable sort, locked pairs first on ties).
    Returns (eig, psi, resid, iters); ``info``, when given, receives the number
    of restarts and of locked bands.
    """
    nb = psi0.shape[0]
    restarts = 0
    x = cholqr(psi0)
    w = hop(x)
    hs = _gram(x, w)
    hs = 0.5 * (hs + hs.conj().T)
    lam, y = np.linalg.eigh(hs)
    x = y.T @ x
    w = y.T @ w
    vb, hvb = x.copy(), w.copy()
    hsub = np.diag(lam).astype(np.complex128)
    xl = np.zeros((0, x.shape[1]), dtype=np.complex128)   # locked Ritz vectors
    lam_l, rn_l = np.zeros(0), np.zeros(0)
    iters = 0
    while True:
        r = w - lam[:, None] * x
        rn = np.sqrt(np.sum(np.abs(r) ** 2, axis=1))
        if np.all(rn < tol) or iters >= max_iter:
            break
        act = np.nonzero(rn >= tol)[0]
        ekin = np.sum(kin[None, :] * np.abs(x[act]) ** 2, axis=1)
        t = tpa_preconditioner(kin, ekin) * r[act]
        if vb.shape[0] + t.shape[0] > ndim * nb:
            conv = np.nonzero(rn < tol)[0]
            if conv.size:
                xl = np.concatenate([xl, x[conv]])
                lam_l = np.concatenate([lam_l, lam[conv]])
                rn_l = np.concatenate([rn_l, rn[conv]])
                x, w, lam = x[act], w[act], lam[act]
            vb, hvb = x.copy(), w.copy()
            hsub = np.diag(lam).astype(np.complex128)
            restarts += 1
        q = np.concatenate([xl, vb])
        n0 = np.linalg.norm(t, axis=1)
        for _ in range(2):
            t = t - _gram(q, t).T @ q
        keep = np.linalg.norm(t, axis=1) >= drop * n0
        t = t[keep]
        if t.shape[0] == 0:
            break
        t = cholqr(cholqr(t))
        ht = hop(t)
        vb = np.concatenate([vb, t])
        hvb = np.concatenate([hvb, ht])
        c = _gram(vb, ht)                      # new columns of V^H H V
        nold = hsub.shape[0]
        hn = np.zeros((vb.shape[0], vb.shape[0]), dtype=np.complex128)
        hn[:nold, :nold] = hsub
        hn[:, nold:] = c
        hn[nold:, :nold] = c[:nold].conj().T
        blk = hn[nold:, nold:]
        hn[nold:, nold:] = 0.5 * (blk + blk.conj().T)
        hsub = hn
        na = x.shape[0]
        theta, y = np.linalg.eigh(hsub)
        y = y[:, :na]
        lam = theta[:na]
        x = y.T @ vb
        w = y.T @ hvb
        iters += 1
    if info is not None:
        info.update(restarts=restarts, locked=xl.shape[0])
    lam_all = np.concatenate([lam_l, lam])
    order = np.argsort(lam_all, kind="stable")
    return lam_all[order], np.concatenate([xl, x])[order], np.concatenate([rn_l, rn])[order], iters


def davidson(prob, psi0=None, tol=1e-8, max_iter=100, ndim=2, nb=None):
    """Oracle block Davidson over every k-point; returns (eig [nk][nb], psi packed, resid, iters)."""
    nb = prob.nb if nb is None else nb
    psi0 = prob.psi if psi0 is None else psi0
    off = np.concatenate([[0], np.cumsum(prob.npw)]).astype(np.int64)
    nk = len(prob.npw)
    eig = np.empty((nk, nb))
    res = np.empty((nk, nb))
    its = np.empty(nk, dtype=np.int64)
    out = np.empty(nb * int(off[-1]), dtype=np.complex128)
    for k in range(nk):
        sub = _single_k(prob, k)
        npw = int(prob.npw[k])
        x0 = np.asarray(psi0[nb * off[k]: nb * off[k + 1]]).reshape(nb, npw)

        def hop(rows, sub=sub):
            return apply_h(sub, rows.reshape(-1), nb=rows.shape[0]).reshape(rows.shape)

        e, x, r, it = davidson_k(hop, x0, kinetic(sub, 0), tol, max_iter, ndim)
        eig[k], res[k], its[k] = e, r, it
        out[nb * off[k]: nb * off[k + 1]] = x.reshape(-1)
    return eig, out, res, its


def cg_k(hop, psi0: np.ndarray, kin: np.ndarray, tol: float, max_iter: int, history: bool = False):
    """Band-by-band preconditioned conjugate gradient for the lowest nb eigenpairs
    (the CG figure of Sec. III.B), rows in, rows out. For band i:

    1. project out bands 0 .. i-1 and normalise; p = H psi_i, lambda = <psi_i|p>.
    2. Repeat until ||p - lambda psi_i|| < tol or max_iter steps:
       r = p - lambda psi_i; g = K r (Teter-Payne-Allan K of the band's kinetic
       energy); project out bands 0 .. i; Polak-Ribiere
       gamma = max(0, Re<g_k|r_k - r_{k-1}> / Re<g_{k-1}|r_{k-1}>) (0 at the first
       step); d = g + gamma d_prev; the step direction is d with psi_i projected
       out, normalised (d itself, unnormalised, carries the recurrence);
       h = H d_hat; theta minimises the Rayleigh quotient on span{psi_i, d_hat}:
       theta = atan2(-2b, c - a) / 2, a = lambda, b = Re<p|d_hat>, c = <d_hat|h>;
       psi_i = cos(theta) psi_i + sin(theta) d_hat, p likewise with h,
       lambda = <psi_i|p>.
    Returns (lambda [nb], psi [nb][npw], residual norms [nb], steps [nb]) and, with
    history, the Rayleigh quotients of every band after each step.
    """
    nb, npw = psi0.shape
    x = np.array(psi0, dtype=np.complex128, copy=True)
    lam = np.empty(nb)
    rn = np.empty(nb)
    its = np.zeros(nb, dtype=np.int64)
    hist = []
    for i in range(nb):
        if i > 0:
            x[i] -= x[:i].T @ (x[:i].conj() @ x[i])
        x[i] /= np.linalg.norm(x[i])
        p = hop(x[i:i + 1])[0]
        lv = float(np.vdot(x[i], p).real)
        d = None
        r_prev = None
        gr_prev = 0.0
        k = 0
        seq = [lv]
        while True:
            r = p - lv * x[i]
            rnorm = float(np.linalg.norm(r))
            if rnorm < tol or k >= max_iter:
                break
            ek = float(np.sum(kin * np.abs(x[i]) ** 2))
            g = tpa_preconditioner(kin, np.array([ek]))[0] * r
            g -= x[:i + 1].T @ (x[:i + 1].conj() @ g)
            gr = float(np.vdot(g, r).real)
            if k == 0:
                d = g
            else:
                gamma = max(0.0, (gr - float(np.vdot(g, r_prev).real)) / gr_prev)
                d = g + gamma * d
            dp = d - np.vdot(x[i], d) * x[i]
            dh = dp / np.linalg.norm(dp)
            h = hop(dh[None, :])[0]
            a = lv
            b = float(np.vdot(p, dh).real)
            c = float(np.vdot(dh, h).real)
            theta = 0.5 * np.arctan2(-2.0 * b, c - a)
            ct, st = np.cos(theta), np.sin(theta)
            x[i] = ct * x[i] + st * dh
            p = ct * p + st * h
            lv = float(np.vdot(x[i], p).real)
            r_prev, gr_prev = r, gr
            k += 1
            seq.append(lv)
        lam[i], rn[i], its[i] = lv, rnorm, k
        hist.append(seq)
    if history:
        return lam, x, rn, its, hist
    return lam, x, rn, its


def cg(prob, psi0=None, tol=1e-8, max_iter=200, nb=None):
    """Oracle band-by-band CG over every k-point; returns (eig [nk][nb], psi packed, resid, steps [nk][nb])."""
    nb = prob.nb if nb is None else nb
    psi0 = prob.psi if psi0 is None else psi0
    off = np.concatenate([[0], np.cumsum(prob.npw)]).astype(np.int64)
    nk = len(prob.npw)
    eig = np.empty((nk, nb))
    res = np.empty((nk, nb))
    its = np.empty((nk, nb), dtype=np.int64)
    out = np.empty(nb * int(off[-1]), dtype=np.complex128)
    for k in range(nk):
        sub = _single_k(prob, k)
        npw = int(prob.npw[k])
        x0 = np.asarray(psi0[nb * off[k]: nb * off[k + 1]]).reshape(nb, npw)

        def hop(rows, sub=sub):
            return apply_h(sub, rows.reshape(-1), nb=rows.shape[0]).reshape(rows.shape)

        e, x, r, it = cg_k(hop, x0, kinetic(sub, 0), tol, max_iter)
        eig[k], res[k], its[k] = e, r, it
        out[nb * off[k]: nb * off[k + 1]] = x.reshape(-1)
    return eig, out, res, its


class _SingleK:
    pass


def _single_k(prob, k):
    """The sub-problem made of k-point k alone (same cell, grid, V, D)."""
    off = np.concatenate([[0], np.cumsum(prob.npw)]).astype(np.int64)
    s = _SingleK()
    s.lattice, s.fft, s.vloc, s.nproj, s.natom = prob.lattice, prob.fft, prob.vloc, prob.nproj, prob.natom
    s.proj_atom_offset, s.dmat = prob.proj_atom_offset, prob.dmat
    s.kpts = np.asarray(prob.kpts)[k:k + 1]
    s.npw = np.asarray(prob.npw)[k:k + 1]
    s.miller = np.asarray(prob.miller)[off[k]:off[k + 1]]
    s.beta = np.asarray(prob.beta)[prob.nproj * off[k]: prob.nproj * off[k + 1]]
    return s
