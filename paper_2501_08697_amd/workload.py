"""Seeded synthetic plane-wave problems (inputs only; no Hamiltonian arithmetic).

This module builds the arrays that define one instance of the plane-wave
Kohn-Sham eigenproblem of Sec. III.A (plane-wave expansion of the orbitals and
the KS equation in that basis) with the norm-conserving local + Kleinman-Bylander
split of Sec. II.A ("Pseudopotentials"): the cell, the cutoff, the k-points, the
G-sphere of every k-point (its Miller indices, in a canonical order), the local
potential sampled on the real-space FFT grid, the projectors beta(k+G), the
per-atom coupling blocks D, and orthonormal random trial orbitals.

It is shared by the test-suite oracle and the GPU library's callers, so it holds
none of the method's arithmetic: no kinetic factors, no FFTs, no H application.
Everything is fp64 / complex128 numpy, drawn from ``numpy.random.default_rng``
(PCG64) in a fixed order, so a (config, seed) pair always yields the same bytes.

Units are Rydberg atomic units (energies in Ry, lengths in bohr), so the kinetic
operator is |k+G|^2; the paper writes the same operator in Hartree as
(1/2)|k+G|^2.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# Projector channels per angular momentum, in the order used everywhere:
# s; p(x, y, z); d(xy, yz, 3z^2-r^2, xz, x^2-y^2).
LM_ORDER = {0: ["s"], 1: ["px", "py", "pz"], 2: ["dxy", "dyz", "dz2", "dxz", "dx2y2"]}

BETA_SIGMA = 0.8      # bohr, Gaussian radial width of every projector
VLOC_WIDTH = 1.0      # bohr, standard deviation of every local-potential Gaussian


@dataclass(frozen=True)
class Config:
    """A named workload: cubic cell, cutoff, FFT grid, k-points, atoms, bands."""
    name: str
    a: float                 # cubic lattice constant (bohr)
    ecut: float              # ecutwfc (Ry): plane waves with |k+G|^2 < ecut
    fft: int                 # FFT points per axis
    kfrac: tuple             # k-points in units of the reciprocal vectors
    natom: int
    lmax: int                # 1: s+p (4 projectors/atom), 2: s+p+d (9)
    nb: int                  # bands
    seed: int
    dfull: bool = False      # full symmetric D blocks U(-1,1) instead of diagonal U(0.1,1)
    with_grad_inputs: bool = False   # also draw occupations f and an upstream dY


_GAMMA = ((0.0, 0.0, 0.0),)
_GRID222 = tuple(itertools.product((0.0, 0.5), repeat=3))
_GXMR = ((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.5, 0.5))

CONFIGS = {
    # Plain FP64, Gamma only, the small case.
    "C1": Config("C1", 10.0, 20.0, 32, _GAMMA, 8, 1, 16, 1),
    # FP64 vs FP32 H psi, one k-point, 128 bands.
    "C2": Config("C2", 20.5, 30.0, 72, _GAMMA, 64, 1, 128, 2),
    # Batched uneven k-points: Gamma-centred {0,1/2}^3 grid (8 spheres of unequal size).
    "C3": Config("C3", 30.0, 40.0, 120, _GRID222, 216, 1, 512, 3),
    # Mixed precision: s+p+d projectors with full symmetric D blocks.
    "C4": Config("C4", 30.0, 50.0, 128, _GAMMA, 256, 2, 1024, 4, dfull=True),
    # Differentiation: Gamma, X, M, R with occupations and an upstream gradient.
    "C5": Config("C5", 24.0, 35.0, 96, _GXMR, 128, 1, 256, 5, with_grad_inputs=True),
}


@dataclass
class Problem:
    """One problem instance. Packed arrays are k-major with per-k offsets."""
    lattice: np.ndarray          # (3,3) rows a1, a2, a3 (bohr)
    fft: tuple                   # (N1, N2, N3)
    ecut: float
    kpts: np.ndarray             # (nk, 3) cartesian (bohr^-1)
    npw: np.ndarray              # (nk,) int32
    miller: np.ndarray           # (sum npw, 3) int32, k-major, canonical order per k
    vloc: np.ndarray             # (N1, N2, N3) float64, C order (j3 fastest)
    nproj: int
    natom: int
    proj_atom_offset: np.ndarray  # (natom+1,) int32
    beta: np.ndarray             # flat complex128: per k a [nproj][npw_k] block
    dmat: np.ndarray             # flat float64: per atom a [np_a][np_a] block (row-major)
    nb: int
    psi: np.ndarray              # flat complex128: per k a [nb][npw_k] block, orthonormal rows
    occ: np.ndarray | None = None    # (nk, nb) occupations f_n
    dy: np.ndarray | None = None     # like psi: upstream gradient
    tau: np.ndarray | None = None    # (natom, 3) cartesian atom positions
    depth: np.ndarray | None = None  # (natom,) Gaussian depths of V_loc
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nk(self) -> int:
        return int(self.kpts.shape[0])

    @property
    def pw_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.npw)]).astype(np.int64)

    def psi_k(self, k: int, arr: np.ndarray | None = None) -> np.ndarray:
        """View of a [nb][npw_k] block of a packed psi-like array."""
        arr = self.psi if arr is None else arr
        off = self.pw_offsets
        return arr[self.nb * off[k]: self.nb * off[k + 1]].reshape(self.nb, int(self.npw[k]))

    def beta_k(self, k: int) -> np.ndarray:
        off = self.pw_offsets
        return self.beta[self.nproj * off[k]: self.nproj * off[k + 1]].reshape(self.nproj, int(self.npw[k]))

    def miller_k(self, k: int) -> np.ndarray:
        off = self.pw_offsets
        return self.miller[off[k]: off[k + 1]]

    def single_k(self, k: int) -> "Problem":
        """The problem restricted to k-point k (views of the same arrays)."""
        off = self.pw_offsets
        sl = slice(self.nb * off[k], self.nb * off[k + 1])
        return Problem(
            lattice=self.lattice, fft=self.fft, ecut=self.ecut, kpts=self.kpts[k:k + 1], npw=self.npw[k:k + 1],
            miller=self.miller[off[k]:off[k + 1]], vloc=self.vloc, nproj=self.nproj, natom=self.natom,
            proj_atom_offset=self.proj_atom_offset, beta=self.beta[self.nproj * off[k]: self.nproj * off[k + 1]],
            dmat=self.dmat, nb=self.nb, psi=self.psi[sl],
            occ=None if self.occ is None else self.occ[k:k + 1], dy=None if self.dy is None else self.dy[sl],
            tau=self.tau, depth=self.depth, name=f"{self.name}[k{k}]")

    def dblock(self, atom: int) -> np.ndarray:
        n = int(self.proj_atom_offset[atom + 1] - self.proj_atom_offset[atom])
        o = int(sum((self.proj_atom_offset[i + 1] - self.proj_atom_offset[i]) ** 2 for i in range(atom)))
        return self.dmat[o: o + n * n].reshape(n, n)


def reciprocal(lattice: np.ndarray) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def g_sphere(lattice: np.ndarray, kcart: np.ndarray, ecut: float, min_gap: float = 1e-9) -> np.ndarray:
    """Miller indices m with |k + sum_i m_i b_i|^2 < ecut (strict), canonical order.

    Canonical order: ascending |k+G|^2 (rounded to 1e-9 Ry so that rounding noise
    cannot split exact ties), ties broken by (m1, m2, m3) lexicographically.
    Raises if any lattice point sits within ``min_gap`` Ry of the cutoff, where
    membership would depend on rounding.
    """
    b = reciprocal(lattice)
    kmax = math.sqrt(ecut) + float(np.linalg.norm(kcart))
    a = np.asarray(lattice, dtype=np.float64)
    bound = [int(math.ceil(kmax * np.linalg.norm(a[i]) / (2 * np.pi))) + 1 for i in range(3)]
    r = [np.arange(-bi, bi + 1) for bi in bound]
    m = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    kg = kcart[None, :] + m.astype(np.float64) @ b
    kg2 = np.einsum("ij,ij->i", kg, kg)
    gap = np.min(np.abs(kg2 - ecut))
    if gap <= min_gap:
        raise ValueError(f"a lattice point lies within {gap:.3e} Ry of the cutoff")
    keep = kg2 < ecut
    m, kg2 = m[keep], kg2[keep]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], np.round(kg2, 9)))
    return m[order].astype(np.int32)


def _solid_harmonics(q: np.ndarray, lmax: int) -> list:
    """q^l Y_lm(q-hat) for real Y_lm, order of LM_ORDER; q is (npw, 3) cartesian."""
    x, y, z = q[:, 0], q[:, 1], q[:, 2]
    out = [np.full(q.shape[0], 0.5 / math.sqrt(math.pi))]
    if lmax >= 1:
        c1 = math.sqrt(3.0 / (4.0 * math.pi))
        out += [c1 * x, c1 * y, c1 * z]
    if lmax >= 2:
        c2 = math.sqrt(15.0 / (4.0 * math.pi))
        c20 = math.sqrt(5.0 / (16.0 * math.pi))
        c22 = math.sqrt(15.0 / (16.0 * math.pi))
        r2 = x * x + y * y + z * z
        out += [c2 * x * y, c2 * y * z, c20 * (3.0 * z * z - r2), c2 * x * z, c22 * (x * x - y * y)]
    return out


def projectors(lattice, kcart, miller_k, tau, lmax, sigma=BETA_SIGMA) -> np.ndarray:
    """beta_{I,lm}(k+G) = n (-i)^l sigma^l q^l Y_lm exp(-sigma^2 q^2 / 2) exp(-i (k+G).tau_I).

    n normalises every projector to sum_G |beta|^2 = 1 at this k-point. The
    (-i)^l factor makes the real-space projectors real. Returns [natom*nlm][npw].
    """
    b = reciprocal(lattice)
    q = kcart[None, :] + miller_k.astype(np.float64) @ b
    q2 = np.einsum("ij,ij->i", q, q)
    radial = np.exp(-0.5 * sigma * sigma * q2)
    sh = _solid_harmonics(q, lmax)
    ls = [0] + [1] * 3 * (lmax >= 1) + [2] * 5 * (lmax >= 2)
    ang = [((-1j) ** l) * (sigma ** l) * s * radial for l, s in zip(ls, sh)]
    nlm = len(ang)
    out = np.empty((tau.shape[0] * nlm, q.shape[0]), dtype=np.complex128)
    for ia in range(tau.shape[0]):
        phase = np.exp(-1j * (q @ tau[ia]))
        for c in range(nlm):
            v = ang[c] * phase
            out[ia * nlm + c] = v / math.sqrt(float(np.vdot(v, v).real))
    return out


def gaussian_vloc(lattice, fft, tau, depth, width=VLOC_WIDTH) -> np.ndarray:
    """V(r_j) = sum_I d_I sum_{n in {-1,0,1}^3} exp(-|r_j - tau_I - n.A|^2 / (2 w^2)).

    r_j = sum_i (j_i / N_i) a_i. For an orthogonal cell the Gaussian and the
    image sum both factor over the three axes, which is what is evaluated.
    """
    a = np.asarray(lattice, dtype=np.float64)
    n1, n2, n3 = fft
    off = a - np.diag(np.diag(a))
    if np.any(off != 0.0):
        return _gaussian_vloc_direct(a, fft, tau, depth, width)
    L = np.diag(a)
    axes = [np.arange(n) * (L[i] / n) for i, n in enumerate(fft)]
    v = np.zeros((n1, n2, n3))
    for ia in range(tau.shape[0]):
        f = []
        for i in range(3):
            d = axes[i][:, None] - tau[ia, i] - np.array([-1.0, 0.0, 1.0])[None, :] * L[i]
            f.append(np.exp(-(d * d) / (2.0 * width * width)).sum(axis=1))
        v += depth[ia] * (f[0][:, None, None] * f[1][None, :, None]) * f[2][None, None, :]
    return v


def _gaussian_vloc_direct(a, fft, tau, depth, width):
    n1, n2, n3 = fft
    j = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3, indexing="ij"), -1)
    r = j.reshape(-1, 3) @ a
    v = np.zeros(r.shape[0])
    imgs = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.float64) @ a
    for ia in range(tau.shape[0]):
        for s in imgs:
            d = r - tau[ia] - s
            v += depth[ia] * np.exp(-np.einsum("ij,ij->i", d, d) / (2.0 * width * width))
    return v.reshape(n1, n2, n3)


def cholqr_rows(x: np.ndarray) -> np.ndarray:
    """Orthonormalise the rows of x (bands x npw) by one Cholesky-QR pass."""
    s = x.conj() @ x.T                     # s[i,j] = <x_i | x_j>
    s = 0.5 * (s + s.conj().T)
    l = np.linalg.cholesky(s.T)            # s^T = conj(s) = L L^H
    # rows y = L^{-1} x  ->  <y_i|y_j> = (L^{-1} s^T ... ) = I
    import scipy.linalg as sla
    return sla.solve_triangular(l, x, lower=True)


def make_problem(cfg: Config | str, seed: int | None = None, nb: int | None = None,
                 lattice: np.ndarray | None = None) -> Problem:
    """Build a problem for a named config (or a custom Config)."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    seed = cfg.seed if seed is None else seed
    nb = cfg.nb if nb is None else nb
    lat = np.eye(3) * cfg.a if lattice is None else np.asarray(lattice, dtype=np.float64)
    fft = (cfg.fft, cfg.fft, cfg.fft)
    b = reciprocal(lat)
    kpts = np.array([np.asarray(kf) @ b for kf in cfg.kfrac], dtype=np.float64).reshape(-1, 3)
    mills = [g_sphere(lat, kpts[k], cfg.ecut) for k in range(kpts.shape[0])]
    for m in mills:
        for i in range(3):
            if 2 * int(np.max(np.abs(m[:, i]))) + 1 > fft[i]:
                raise ValueError("the G-sphere does not fit the FFT grid")
    npw = np.array([m.shape[0] for m in mills], dtype=np.int32)
    rng = np.random.default_rng(seed)
    # Draw order: tau, depths, D, psi (re then im), occupations, dY (re then im).
    tau = rng.random((cfg.natom, 3)) @ lat
    depth = rng.uniform(-2.0, -0.5, size=cfg.natom)
    nlm = (cfg.lmax + 1) ** 2
    ls = [0] + [1] * 3 * (cfg.lmax >= 1) + [2] * 5 * (cfg.lmax >= 2)
    blocks = []
    if cfg.dfull:
        tri = rng.uniform(-1.0, 1.0, size=(cfg.natom, nlm * (nlm + 1) // 2))
        iu = np.triu_indices(nlm)
        for ia in range(cfg.natom):
            d = np.zeros((nlm, nlm))
            d[iu] = tri[ia]
            d = d + np.triu(d, 1).T
            blocks.append(d)
    else:
        dl = rng.uniform(0.1, 1.0, size=(cfg.natom, cfg.lmax + 1))
        for ia in range(cfg.natom):
            blocks.append(np.diag([dl[ia, l] for l in ls]))
    dmat = np.concatenate([d.reshape(-1) for d in blocks])
    ntot = int(npw.sum()) * nb
    re = rng.standard_normal(ntot)
    im = rng.standard_normal(ntot)
    psi = (re + 1j * im) / math.sqrt(2.0)
    occ = dy = None
    if cfg.with_grad_inputs:
        occ = rng.uniform(0.0, 2.0, size=(kpts.shape[0], nb))
        re = rng.standard_normal(ntot)
        im = rng.standard_normal(ntot)
        dy = (re + 1j * im) / math.sqrt(2.0)
    off = np.concatenate([[0], np.cumsum(npw)])
    for k in range(kpts.shape[0]):
        blk = psi[nb * off[k]: nb * off[k + 1]].reshape(nb, int(npw[k]))
        blk[:] = cholqr_rows(cholqr_rows(blk))
    beta = np.concatenate([projectors(lat, kpts[k], mills[k], tau, cfg.lmax).reshape(-1)
                           for k in range(kpts.shape[0])])
    vloc = gaussian_vloc(lat, fft, tau, depth)
    return Problem(
        lattice=lat, fft=fft, ecut=cfg.ecut, kpts=kpts, npw=npw,
        miller=np.ascontiguousarray(np.concatenate(mills, axis=0), dtype=np.int32),
        vloc=np.ascontiguousarray(vloc), nproj=cfg.natom * nlm, natom=cfg.natom,
        proj_atom_offset=(np.arange(cfg.natom + 1) * nlm).astype(np.int32),
        beta=beta, dmat=dmat, nb=nb, psi=psi, occ=occ, dy=dy, tau=tau, depth=depth,
        name=cfg.name)


def tiny_config(a=6.0, ecut=8.0, fft=8, kfrac=_GAMMA, natom=2, lmax=1, nb=4, seed=11,
                dfull=False, with_grad_inputs=False) -> Config:
    """A small custom configuration for tests."""
    return Config("tiny", a, ecut, fft, tuple(kfrac), natom, lmax, nb, seed, dfull, with_grad_inputs)


def band_weights(prob, seed: int = 0) -> np.ndarray:
    """Weights of the density sum, [nk][nb] float64: k-point weight 1/nk times an
    occupation f_n ~ U(0, 2) drawn from its own stream (seed 1000 + seed), so the
    problem's other draws are unchanged."""
    rng = np.random.default_rng(1000 + seed)
    nk = len(prob.npw)
    return rng.uniform(0.0, 2.0, size=(nk, prob.nb)) / nk


def stochastic_orbitals(prob, nchi: int, seed: int = 0) -> np.ndarray:
    """Plane-wave stochastic orbitals of Sec. III.C: per k-point and orbital a,
    chi_a(G) = exp(2 pi i theta) / sqrt(nchi) with theta ~ U(0, 1) drawn
    independently for every (k, a, G) from the stream of seed 2000 + seed.
    Packed like psi: per k a [nchi][npw_k] block, complex128."""
    rng = np.random.default_rng(2000 + seed)
    blocks = [np.exp(2j * np.pi * rng.uniform(0.0, 1.0, size=(nchi, int(n)))) / np.sqrt(nchi)
              for n in prob.npw]
    return np.concatenate([b.reshape(-1) for b in blocks]).astype(np.complex128)
