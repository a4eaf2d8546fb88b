"""ctypes binding of libabacus_pw.so (include/abacus_pw.h).

Argument marshalling only: every step of H psi, its adjoint and Davidson runs
in the library's HIP kernels. torch supplies device memory and the stream.
The library must be built (``python -m paper_2501_08697_amd.build``); when it
is missing every call raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabacus_pw.so")

FP64, FP32, MIXED_BF16, MIXED_FP32 = 0, 1, 2, 3
STATIC_OPERATOR = 1

ERRORS = {
    -1: "ENULL_ARG", -2: "EBAD_SHAPE", -3: "EBAD_FFT_SIZE", -4: "EBAD_SPHERE", -5: "EBAD_D",
    -6: "ENONFINITE", -7: "EBAD_PRECISION", -8: "EHIP", -9: "ECHOLESKY", -10: "EINTERNAL",
}

EXPORTS = ["abacus_pw_apply_h", "abacus_pw_davidson", "abacus_pw_cg", "abacus_pw_apply_h_backward", "abacus_pw_density",
           "abacus_pw_chebyshev", "abacus_pw_chebyshev_coefficients", "abacus_pw_force_nl", "abacus_pw_density_g",
           "abacus_pw_eigh_lowest", "abacus_pw_cholesky",
           "abacus_pw_workspace_size", "abacus_pw_apply_h_ws", "abacus_pw_density_g_noalloc",
           "abacus_pw_last_error",
           "abacus_pw_fft_supported", "abacus_pw_plan_reset", "abacus_pw_profile_enable",
           "abacus_pw_profile_read", "abacus_pw_set_tuning"]


class AbacusPwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class CProblem(C.Structure):
    _fields_ = [
        ("lattice", C.c_double * 9), ("fft", C.c_int * 3), ("ecutwfc", C.c_double), ("nk", C.c_int),
        ("kpts", C.c_void_p), ("npw", C.c_void_p), ("miller", C.c_void_p), ("vloc", C.c_void_p),
        ("nproj", C.c_int), ("natom", C.c_int), ("proj_atom_offset", C.c_void_p), ("beta", C.c_void_p),
        ("dmat", C.c_void_p), ("flags", C.c_uint),
    ]


_lib = None


def lib():
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2501_08697_amd.build")
        L = C.CDLL(LIB_PATH)
        P, vp, i, d = C.POINTER(CProblem), C.c_void_p, C.c_int, C.c_double
        sigs = {
            "abacus_pw_apply_h": [P, i, i, vp, vp, vp],
            "abacus_pw_apply_h_backward": [P, i, i, vp, vp, vp, vp, vp, vp],
            "abacus_pw_davidson": [P, i, i, vp, vp, d, i, i, vp, vp, vp],
            "abacus_pw_density": [P, i, i, vp, vp, vp, vp],
            "abacus_pw_chebyshev": [P, i, i, vp, vp, vp, i, d, d, vp],
            "abacus_pw_force_nl": [P, i, i, vp, vp, vp, vp],
            "abacus_pw_density_g": [vp, vp, i, vp, vp, vp],
            "abacus_pw_density_g_noalloc": [vp, vp, i, vp, vp, vp],
            "abacus_pw_workspace_size": [P, i, i, C.POINTER(C.c_size_t), vp],
            "abacus_pw_apply_h_ws": [P, i, i, vp, vp, vp, C.c_size_t, vp],
            "abacus_pw_eigh_lowest": [i, vp, i, i, vp, vp, i, vp],
            "abacus_pw_cholesky": [i, vp, i, vp, i, vp],
            "abacus_pw_chebyshev_coefficients": [i, d, d, d, d, d, vp],
            "abacus_pw_cg": [P, i, vp, vp, d, i, vp, vp, vp],
            "abacus_pw_last_error": [C.c_char_p, i],
            "abacus_pw_fft_supported": [i],
            "abacus_pw_profile_enable": [i],
            "abacus_pw_profile_read": [C.c_char_p, i],
            "abacus_pw_set_tuning": [i, i, i, i, i, i, i],
        }
        for name, sig in sigs.items():
            # a symbol missing from an older build fails when called, not at load
            if hasattr(L, name):
                getattr(L, name).argtypes = sig
        _lib = L
    return _lib


def last_error() -> str:
    buf = C.create_string_buffer(1024)
    lib().abacus_pw_last_error(buf, 1024)
    return buf.value.decode()


def check(code: int) -> int:
    if code < 0:
        raise AbacusPwError(code, last_error())
    return code


def _dev_tensor(t, name: str, dtype, numel: int, device=None):
    """Checks a tensor argument before its pointer crosses the C ABI: a CUDA
    (HIP) tensor of the given dtype, contiguous, with exactly numel elements, on
    the expected device. Raises AbacusPwError(EBAD_SHAPE) otherwise; nothing is
    copied or converted (a silent copy of an in/out buffer would drop the update)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise AbacusPwError(-2, f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise AbacusPwError(-2, f"{name} must be a device tensor (got {t.device})")
    if device is not None and t.device != device:
        raise AbacusPwError(-2, f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise AbacusPwError(-2, f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise AbacusPwError(-2, f"{name} must be contiguous")
    if t.numel() != numel:
        raise AbacusPwError(-2, f"{name} must hold {numel} elements (got {t.numel()})")
    return t


def _psi_dtype(precision: int):
    import torch
    if precision not in (FP64, FP32, MIXED_BF16, MIXED_FP32):
        raise AbacusPwError(-7, f"unknown precision {precision}")
    return torch.complex64 if precision == FP32 else torch.complex128


def _weights(dp, occ, nb, device):
    import torch
    w = torch.as_tensor(occ, dtype=torch.float64).to(device).contiguous()
    if w.numel() != dp.nk * nb:
        raise AbacusPwError(-2, f"occ must hold nk * nb = {dp.nk * nb} weights, got {w.numel()}")
    return w


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class DeviceProblem:
    """A problem with its operator arrays in device memory, ready for the C ABI.

    Host arrays (lattice, kpts, npw, miller, proj_atom_offset) are kept as
    contiguous numpy buffers; vloc, beta and dmat as torch device tensors.

    static=True sets ABACUS_PW_STATIC_OPERATOR: the library may then keep its
    reduced-precision copies of V and beta between calls, keyed by pointer. Only
    use it while these tensors stay alive and unchanged: a freed tensor's address
    is soon reused by torch's allocator for different data.
    """

    def __init__(self, prob, device="cuda", vloc=None, dmat=None, beta=None, static=False):
        import torch
        self.prob = prob
        self.nk = int(len(prob.npw))
        self.fft = tuple(int(x) for x in prob.fft)
        self.npw = np.ascontiguousarray(prob.npw, dtype=np.int32)
        self.pw_off = np.concatenate([[0], np.cumsum(self.npw)]).astype(np.int64)
        self._kpts = np.ascontiguousarray(prob.kpts, dtype=np.float64)
        self._miller = np.ascontiguousarray(prob.miller, dtype=np.int32)
        self._offs = np.ascontiguousarray(prob.proj_atom_offset, dtype=np.int32)
        self.vloc = vloc if vloc is not None else torch.from_numpy(np.ascontiguousarray(prob.vloc)).to(device)
        self.beta = beta if beta is not None else torch.from_numpy(np.ascontiguousarray(prob.beta)).to(device)
        self.dmat = dmat if dmat is not None else torch.from_numpy(np.ascontiguousarray(prob.dmat)).to(device)
        self.nproj, self.natom = int(prob.nproj), int(prob.natom)
        self.static = static

    def c(self, vloc=None, dmat=None) -> CProblem:
        s = CProblem()
        s.lattice[:] = [float(x) for x in np.asarray(self.prob.lattice, dtype=np.float64).reshape(-1)]
        s.fft[:] = list(self.fft)
        s.ecutwfc = float(self.prob.ecut)
        s.nk = self.nk
        s.kpts = self._kpts.ctypes.data
        s.npw = self.npw.ctypes.data
        s.miller = self._miller.ctypes.data
        v = self.vloc if vloc is None else vloc
        dm = self.dmat if dmat is None else dmat
        s.vloc = v.data_ptr()
        s.nproj, s.natom = self.nproj, self.natom
        s.proj_atom_offset = self._offs.ctypes.data if self.nproj > 0 else None
        s.beta = self.beta.data_ptr() if self.nproj > 0 else None
        s.dmat = dm.data_ptr() if self.nproj > 0 else None
        s.flags = STATIC_OPERATOR if (self.static and vloc is None and dmat is None) else 0
        return s

    def psi_len(self, nb: int) -> int:
        return nb * int(self.pw_off[-1])

    def check_operator(self, device, vloc=None, dmat=None):
        """The operator tensors passed to the library: vloc float64 [N1 N2 N3], beta complex128
        [nproj sum npw], dmat float64 (the concatenated atom blocks), all contiguous on `device`."""
        import torch
        n = self.fft[0] * self.fft[1] * self.fft[2]
        _dev_tensor(self.vloc if vloc is None else vloc, "vloc", torch.float64, n, device)
        if self.nproj > 0:
            offs = self._offs.astype(np.int64)
            dlen = int(np.sum((offs[1:] - offs[:-1]) ** 2))
            _dev_tensor(self.beta, "beta", torch.complex128, self.nproj * int(self.pw_off[-1]), device)
            _dev_tensor(self.dmat if dmat is None else dmat, "dmat", torch.float64, dlen, device)


def apply_h(dp: DeviceProblem, psi, precision: int = FP64, nb: int | None = None, out=None, stream=None,
            vloc=None, dmat=None):
    """H psi for a packed psi tensor (complex128, or complex64 for FP32)."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    dt = _psi_dtype(precision)
    _dev_tensor(psi, "psi", dt, dp.psi_len(nb))
    y = torch.empty_like(psi) if out is None else _dev_tensor(out, "out", dt, dp.psi_len(nb), psi.device)
    if y.data_ptr() == psi.data_ptr():
        raise AbacusPwError(-2, "out must not alias psi")
    dp.check_operator(psi.device, vloc, dmat)
    cp = dp.c(vloc, dmat)
    check(lib().abacus_pw_apply_h(C.byref(cp), int(precision), int(nb), psi.data_ptr(), y.data_ptr(),
                                  _stream(stream)))
    return y


def workspace_size(dp: DeviceProblem, precision: int = FP64, nb: int | None = None, stream=None) -> int:
    """Bytes of work space apply_h_ws needs (builds the plan and the operator copies)."""
    nb = dp.prob.nb if nb is None else nb
    out = C.c_size_t(0)
    cp = dp.c()
    check(lib().abacus_pw_workspace_size(C.byref(cp), int(precision), int(nb), C.byref(out), _stream(stream)))
    return int(out.value)


def apply_h_ws(dp: DeviceProblem, psi, workspace, precision: int = FP64, nb: int | None = None, out=None,
               stream=None):
    """H psi with a caller work space (a uint8 device tensor of workspace_size bytes)."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    dt = _psi_dtype(precision)
    _dev_tensor(psi, "psi", dt, dp.psi_len(nb))
    y = torch.empty_like(psi) if out is None else _dev_tensor(out, "out", dt, dp.psi_len(nb), psi.device)
    if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or not workspace.is_contiguous():
        raise AbacusPwError(-2, "workspace must be a contiguous device tensor")
    dp.check_operator(psi.device)
    cp = dp.c()
    check(lib().abacus_pw_apply_h_ws(C.byref(cp), int(precision), int(nb), psi.data_ptr(), y.data_ptr(),
                                     workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                     _stream(stream)))
    return y


def apply_h_backward(dp: DeviceProblem, psi, dy, precision: int = FP64, nb: int | None = None, want=("psi", "v", "d"),
                     stream=None, vloc=None, dmat=None):
    """(grad_psi, grad_vloc, grad_dmat) of L with upstream dy = dL/d(H psi)."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    if precision not in (FP64, FP32):
        raise AbacusPwError(-7, "the adjoint runs in FP64 or FP32")
    dt = _psi_dtype(precision)
    _dev_tensor(psi, "psi", dt, dp.psi_len(nb))
    _dev_tensor(dy, "dy", dt, dp.psi_len(nb), psi.device)
    dp.check_operator(psi.device, vloc, dmat)
    gp = torch.empty_like(psi) if "psi" in want else None
    gv = torch.empty(dp.fft, dtype=torch.float64, device=psi.device) if "v" in want else None
    gd = torch.empty_like(dp.dmat) if "d" in want else None
    cp = dp.c(vloc, dmat)
    check(lib().abacus_pw_apply_h_backward(C.byref(cp), int(precision), int(nb), psi.data_ptr(), dy.data_ptr(),
                                           None if gp is None else gp.data_ptr(),
                                           None if gv is None else gv.data_ptr(),
                                           None if gd is None else gd.data_ptr(), _stream(stream)))
    return gp, gv, gd


def density(dp: DeviceProblem, psi, occ, precision: int = FP64, nb: int | None = None, stream=None, out=None):
    """rho [N1][N2][N3] float64 = sum_{k,n} occ[k][n] |psi_nk(r)|^2 (occ: [nk][nb], numpy or torch)."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    if precision not in (FP64, FP32):
        raise AbacusPwError(-7, "the density runs in FP64 or FP32")
    _dev_tensor(psi, "psi", _psi_dtype(precision), dp.psi_len(nb))
    dp.check_operator(psi.device)
    w = _weights(dp, occ, nb, psi.device)
    n = dp.fft[0] * dp.fft[1] * dp.fft[2]
    rho = (torch.empty(dp.fft, dtype=torch.float64, device=psi.device) if out is None
           else _dev_tensor(out, "out", torch.float64, n, psi.device))
    cp = dp.c()
    check(lib().abacus_pw_density(C.byref(cp), int(precision), int(nb), psi.data_ptr(), w.data_ptr(), rho.data_ptr(),
                                  _stream(stream)))
    return rho


def density_g(rho, miller=None, stream=None, out=None):
    """rho(G) = (1/N) sum_j rho(r_j) e^{-iG.r_j} (complex128): on the whole grid ([N1][N2][N3],
    index m mod N) when miller is None, else at the Miller triples miller [ng][3] (int32)."""
    import torch
    if not isinstance(rho, torch.Tensor) or rho.dim() != 3:
        raise AbacusPwError(-2, "rho must be a [N1][N2][N3] tensor")
    _dev_tensor(rho, "rho", torch.float64, rho.numel())
    fft = np.ascontiguousarray(rho.shape, dtype=np.int32)
    if miller is None:
        ng = rho.numel()
        m = None
        shape = tuple(rho.shape)
    else:
        m = torch.as_tensor(miller, dtype=torch.int32).to(rho.device).contiguous()
        if m.dim() != 2 or m.shape[1] != 3:
            raise AbacusPwError(-2, "miller must be [ng][3]")
        ng = int(m.shape[0])
        shape = (ng,)
        if ng == 0:
            return torch.empty(0, dtype=torch.complex128, device=rho.device)
    y = (torch.empty(shape, dtype=torch.complex128, device=rho.device) if out is None
         else _dev_tensor(out, "out", torch.complex128, ng, rho.device))
    check(lib().abacus_pw_density_g(fft.ctypes.data, rho.data_ptr(), int(ng), None if m is None else m.data_ptr(),
                                    y.data_ptr(), _stream(stream)))
    return y


def eigh_lowest(a, nw: int, stream=None):
    """Lowest nw eigenpairs of the Hermitian complex128 [n][n] device matrix a (destroyed):
    (w [nw] float64 ascending, vec [nw][n] complex128, rows = eigenvectors)."""
    import torch
    if not isinstance(a, torch.Tensor) or a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise AbacusPwError(-2, "a must be a square [n][n] tensor")
    n = int(a.shape[0])
    _dev_tensor(a, "a", torch.complex128, n * n)
    w = torch.empty(nw, dtype=torch.float64, device=a.device)
    v = torch.empty((nw, n), dtype=torch.complex128, device=a.device)
    check(lib().abacus_pw_eigh_lowest(n, a.data_ptr(), n, int(nw), w.data_ptr(), v.data_ptr(), n, _stream(stream)))
    return w, v


def cholesky(g, stream=None):
    """G = L L^H for a Hermitian positive definite complex128 [n][n] device matrix: the lower
    triangle of g becomes L (in place); returns Linv = L^{-1}."""
    import torch
    if not isinstance(g, torch.Tensor) or g.dim() != 2 or g.shape[0] != g.shape[1]:
        raise AbacusPwError(-2, "g must be a square [n][n] tensor")
    n = int(g.shape[0])
    _dev_tensor(g, "g", torch.complex128, n * n)
    li = torch.zeros((n, n), dtype=torch.complex128, device=g.device)
    check(lib().abacus_pw_cholesky(n, g.data_ptr(), n, li.data_ptr(), n, _stream(stream)))
    return li


def force_nl(dp: DeviceProblem, psi, occ, nb: int | None = None, stream=None):
    """Nonlocal force [natom][3] (Ry/bohr, device float64) for band weights occ [nk][nb]."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    _dev_tensor(psi, "psi", torch.complex128, dp.psi_len(nb))
    dp.check_operator(psi.device)
    w = _weights(dp, occ, nb, psi.device)
    f = torch.empty((dp.natom, 3), dtype=torch.float64, device=psi.device)
    cp = dp.c()
    check(lib().abacus_pw_force_nl(C.byref(cp), FP64, int(nb), psi.data_ptr(), w.data_ptr(), f.data_ptr(),
                                   _stream(stream)))
    return f


def chebyshev(dp: DeviceProblem, chi, coef, emin, emax, precision: int = FP64, nb: int | None = None, stream=None,
              out=None):
    """sum_n coef[n] T_n((H - c)/h) chi, c and h the centre and half width of [emin, emax]."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    dt = _psi_dtype(precision)
    _dev_tensor(chi, "chi", dt, dp.psi_len(nb))
    cf = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1)
    if cf.size < 1:
        raise AbacusPwError(-2, "need at least one coefficient")
    y = torch.empty_like(chi) if out is None else _dev_tensor(out, "out", dt, dp.psi_len(nb), chi.device)
    if y.data_ptr() == chi.data_ptr():
        raise AbacusPwError(-2, "out must not alias chi")
    dp.check_operator(chi.device)
    cp = dp.c()
    check(lib().abacus_pw_chebyshev(C.byref(cp), int(precision), int(nb), chi.data_ptr(), y.data_ptr(),
                                    cf.ctypes.data, int(cf.size - 1), float(emin), float(emax), _stream(stream)))
    return y


def fermi_coefficients(order: int, emin: float, emax: float, mu: float, kt: float, power: float = 0.5) -> np.ndarray:
    """Chebyshev interpolation coefficients [order + 1] of the Fermi-Dirac function to `power`."""
    cf = np.empty(int(order) + 1, dtype=np.float64)
    check(lib().abacus_pw_chebyshev_coefficients(int(order), float(emin), float(emax), float(mu), float(kt),
                                                 float(power), cf.ctypes.data))
    return cf


def davidson(dp: DeviceProblem, psi, tol=1e-8, max_iter=100, ndim=2, precision: int = FP64, nb: int | None = None,
             stream=None):
    """Block Davidson; psi (complex128) is updated in place. Returns (eig, resid, iters, status)."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    _dev_tensor(psi, "psi", torch.complex128, dp.psi_len(nb))
    dp.check_operator(psi.device)
    eig = np.zeros((dp.nk, nb))
    res = np.zeros((dp.nk, nb))
    its = np.zeros(dp.nk, dtype=np.int32)
    cp = dp.c()
    st = check(lib().abacus_pw_davidson(C.byref(cp), int(precision), int(nb), psi.data_ptr(), eig.ctypes.data,
                                        float(tol), int(max_iter), int(ndim), its.ctypes.data, res.ctypes.data,
                                        _stream(stream)))
    return eig, res, its, st


def cg(dp: DeviceProblem, psi, tol=1e-8, max_iter=200, nb: int | None = None, stream=None):
    """Band-by-band preconditioned CG; psi (complex128) is updated in place.
    Returns (eig [nk][nb], resid [nk][nb], steps [nk][nb], status)."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    _dev_tensor(psi, "psi", torch.complex128, dp.psi_len(nb))
    dp.check_operator(psi.device)
    eig = np.zeros((dp.nk, nb))
    res = np.zeros((dp.nk, nb))
    its = np.zeros((dp.nk, nb), dtype=np.int32)
    cp = dp.c()
    st = check(lib().abacus_pw_cg(C.byref(cp), int(nb), psi.data_ptr(), eig.ctypes.data, float(tol), int(max_iter),
                                  its.ctypes.data, res.ctypes.data, _stream(stream)))
    return eig, res, its, st


def fft_supported(n: int) -> bool:
    return bool(lib().abacus_pw_fft_supported(int(n)))


def plan_reset():
    check(lib().abacus_pw_plan_reset())


def set_tuning(band_batch: int = 0, splitk_chunk: int = 0, yz_bands: int = 0, x_bands: int = 0, yz_mode: int = 0,
               overlap: int = 0, yz_threads: int = 0):
    """Process-wide kernel tuning knobs (0 = library default)."""
    check(lib().abacus_pw_set_tuning(int(band_batch), int(splitk_chunk), int(yz_bands), int(x_bands), int(yz_mode),
                                     int(overlap), int(yz_threads)))


def profile_enable(on: bool = True):
    check(lib().abacus_pw_profile_enable(1 if on else 0))


def profile_read(flops: bool = False) -> dict:
    """{kernel name: (launches, total_ms)} accumulated since the last read, or with
    flops=True (launches, total_ms, flops), the flops counted for the record (the
    Davidson subspace products, "subspace:<kernel>"; 0 elsewhere)."""
    buf = C.create_string_buffer(1 << 16)
    check(lib().abacus_pw_profile_read(buf, 1 << 16))
    out = {}
    for line in buf.value.decode().splitlines():
        f = line.split("\t")
        n, ms = int(f[1]), float(f[2])
        fl = float(f[3]) if len(f) > 3 else 0.0
        out[f[0]] = (n, ms, fl) if flops else (n, ms)
    return out
