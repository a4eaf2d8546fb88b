"""The C-ABI library on a machine without a GPU: it loads, exports every
entry point declared in include/abacus_pw.h, and rejects invalid problems on
the host before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2501_08697_amd import binding as B
from paper_2501_08697_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x1000   # never dereferenced: validation fails before any device access


def header_functions():
    txt = open(os.path.join(ROOT, "include", "abacus_pw.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(abacus_pw_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = B.lib()
    names = header_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def test_fft_lengths():
    for n in (8, 12, 16, 32, 72, 96, 120, 128):
        assert B.fft_supported(n)
    for n in (7, 14, 11, 256, 0):
        assert not B.fft_supported(n)


class Fake:
    """A CProblem with host arrays from a generated problem and fake device pointers."""

    def __init__(self, prob):
        self.kpts = np.ascontiguousarray(prob.kpts)
        self.npw = np.ascontiguousarray(prob.npw, dtype=np.int32)
        self.miller = np.ascontiguousarray(prob.miller, dtype=np.int32)
        self.offs = np.ascontiguousarray(prob.proj_atom_offset, dtype=np.int32)
        s = B.CProblem()
        s.lattice[:] = list(np.asarray(prob.lattice).reshape(-1))
        s.fft[:] = list(prob.fft)
        s.ecutwfc = prob.ecut
        s.nk = prob.nk
        s.kpts, s.npw, s.miller = self.kpts.ctypes.data, self.npw.ctypes.data, self.miller.ctypes.data
        s.vloc = FAKE
        s.nproj, s.natom = prob.nproj, prob.natom
        s.proj_atom_offset = self.offs.ctypes.data
        s.beta, s.dmat = FAKE, FAKE
        self.s = s

    def apply(self, prec=0, nb=1):
        return B.lib().abacus_pw_apply_h(C.byref(self.s), prec, nb, FAKE, FAKE + 64, None)


@pytest.fixture()
def prob():
    return W.make_problem(W.tiny_config(fft=12, ecut=12.0, nb=2))


def code_name(code):
    return B.ERRORS.get(code, code)


def test_rejects_null_and_shape(prob):
    f = Fake(prob)
    assert code_name(B.lib().abacus_pw_apply_h(None, 0, 1, FAKE, FAKE + 64, None)) == "ENULL_ARG"
    assert code_name(B.lib().abacus_pw_apply_h(C.byref(f.s), 0, 1, None, FAKE, None)) == "ENULL_ARG"
    assert code_name(B.lib().abacus_pw_apply_h(C.byref(f.s), 0, 1, FAKE, FAKE, None)) == "EBAD_SHAPE"
    assert code_name(f.apply(nb=0)) == "EBAD_SHAPE"
    f.s.nk = 0
    assert code_name(f.apply()) == "EBAD_SHAPE"


def test_rejects_bad_precision(prob):
    assert code_name(Fake(prob).apply(prec=7)) == "EBAD_PRECISION"


def test_rejects_bad_offsets(prob):
    f = Fake(prob)
    f.offs[-1] += 1
    assert code_name(f.apply()) == "EBAD_SHAPE"


def test_rejects_unsupported_grid(prob):
    f = Fake(prob)
    f.s.fft[0] = 14
    assert code_name(f.apply()) == "EBAD_FFT_SIZE"


def test_rejects_sphere_not_fitting():
    prob = W.make_problem(W.tiny_config(fft=12, ecut=20.0, nb=1))   # |m| reaches 4: needs N >= 9
    f = Fake(prob)
    f.s.fft[:] = [8, 8, 8]
    assert code_name(f.apply()) == "EBAD_FFT_SIZE"


def test_rejects_duplicate_and_outside_sphere(prob):
    f = Fake(prob)
    f.miller[5] = f.miller[6]
    assert code_name(f.apply()) == "EBAD_SPHERE"
    g = Fake(prob)
    g.s.ecutwfc = prob.ecut * 0.5
    assert code_name(g.apply()) == "EBAD_SPHERE"


def test_error_message_is_set(prob):
    f = Fake(prob)
    f.miller[5] = f.miller[6]
    f.apply()
    assert "duplicate" in B.last_error()


def test_tuning_rejects_negative():
    assert code_name(B.lib().abacus_pw_set_tuning(-1, 0, 0, 0, 0, 0, 0)) == "EBAD_SHAPE"
    assert code_name(B.lib().abacus_pw_set_tuning(0, 0, 0, -2, 0, 0, 0)) == "EBAD_SHAPE"
    assert code_name(B.lib().abacus_pw_set_tuning(0, 0, 0, 0, 3, 0, 0)) == "EBAD_SHAPE"
    assert code_name(B.lib().abacus_pw_set_tuning(0, 0, 0, 0, 0, 3, 0)) == "EBAD_SHAPE"
    assert code_name(B.lib().abacus_pw_set_tuning(0, 0, 0, 0, 0, 0, 300)) == "EBAD_SHAPE"
    assert B.lib().abacus_pw_set_tuning(0, 0, 0, 0, 0, 0, 1024) == 0
    assert B.lib().abacus_pw_set_tuning(0, 0, 0, 0, 0, 0, 0) == 0


def test_density_rejects_before_device_access(prob):
    f = Fake(prob)
    lib = B.lib()
    assert code_name(lib.abacus_pw_density(C.byref(f.s), 0, 1, None, FAKE, FAKE, None)) == "ENULL_ARG"
    assert code_name(lib.abacus_pw_density(C.byref(f.s), 0, 1, FAKE, None, FAKE, None)) == "ENULL_ARG"
    assert code_name(lib.abacus_pw_density(C.byref(f.s), 0, 1, FAKE, FAKE, None, None)) == "ENULL_ARG"
    assert code_name(lib.abacus_pw_density(C.byref(f.s), 0, 0, FAKE, FAKE, FAKE, None)) == "EBAD_SHAPE"
    assert code_name(lib.abacus_pw_density(C.byref(f.s), 3, 1, FAKE, FAKE, FAKE, None)) == "EBAD_PRECISION"
    f.miller[5] = f.miller[6]
    assert code_name(lib.abacus_pw_density(C.byref(f.s), 0, 1, FAKE, FAKE, FAKE, None)) == "EBAD_SPHERE"


def test_chebyshev_rejects_before_device_access(prob):
    f = Fake(prob)
    lib = B.lib()
    cf = np.array([1.0, 0.5, 0.25])
    p = cf.ctypes.data

    def call(chi=FAKE, out=FAKE + 64, coef=p, order=2, emin=-1.0, emax=1.0, prec=0, nb=1):
        return code_name(lib.abacus_pw_chebyshev(C.byref(f.s), prec, nb, chi, out, coef, order, emin, emax, None))

    assert call(chi=None) == "ENULL_ARG"
    assert call(coef=None) == "ENULL_ARG"
    assert call(out=FAKE) == "EBAD_SHAPE"
    assert call(order=-1) == "EBAD_SHAPE"
    assert call(emin=1.0) == "EBAD_SHAPE"
    assert call(emax=float("nan")) == "EBAD_SHAPE"
    assert call(prec=9) == "EBAD_PRECISION"
    bad = np.array([1.0, float("inf")])
    assert code_name(lib.abacus_pw_chebyshev(C.byref(f.s), 0, 1, FAKE, FAKE + 64, bad.ctypes.data, 1, -1.0, 1.0,
                                             None)) == "ENONFINITE"


def test_fermi_coefficients_match_oracle_interpolation():
    """The library's host routine against numpy's Chebyshev interpolation (the oracle's route)."""
    import oracle
    for order, kt, power in ((0, 1.0, 0.5), (1, 0.7, 0.5), (60, 2.0, 0.5), (300, 0.5, 1.0), (1200, 0.2, 0.5)):
        ref = oracle.fermi_sqrt_coefficients(order, -2.0, 35.0, 1.3, kt, power)
        got = B.fermi_coefficients(order, -2.0, 35.0, 1.3, kt, power)
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) < 1e-13, (order, np.max(np.abs(got - ref)))


def test_fermi_coefficients_reject_bad_arguments():
    out = np.empty(4)
    lib = B.lib()
    assert code_name(lib.abacus_pw_chebyshev_coefficients(3, 0.0, 1.0, 0.0, 1.0, 0.5, None)) == "ENULL_ARG"
    assert code_name(lib.abacus_pw_chebyshev_coefficients(-1, 0.0, 1.0, 0.0, 1.0, 0.5, out.ctypes.data)) == "EBAD_SHAPE"
    assert code_name(lib.abacus_pw_chebyshev_coefficients(3, 1.0, 1.0, 0.0, 1.0, 0.5, out.ctypes.data)) == "EBAD_SHAPE"
    assert code_name(lib.abacus_pw_chebyshev_coefficients(3, 0.0, 1.0, 0.0, 0.0, 0.5, out.ctypes.data)) == "EBAD_SHAPE"
    assert code_name(lib.abacus_pw_chebyshev_coefficients(3, 0.0, 1.0, 0.0, 1.0, -1.0, out.ctypes.data)) == "EBAD_SHAPE"


def test_force_rejects_before_device_access(prob):
    f = Fake(prob)
    lib = B.lib()
    assert code_name(lib.abacus_pw_force_nl(C.byref(f.s), 0, 1, None, FAKE, FAKE, None)) == "ENULL_ARG"
    assert code_name(lib.abacus_pw_force_nl(C.byref(f.s), 0, 1, FAKE, None, FAKE, None)) == "ENULL_ARG"
    assert code_name(lib.abacus_pw_force_nl(C.byref(f.s), 0, 1, FAKE, FAKE, None, None)) == "ENULL_ARG"
    assert code_name(lib.abacus_pw_force_nl(C.byref(f.s), 0, 0, FAKE, FAKE, FAKE, None)) == "EBAD_SHAPE"
    assert code_name(lib.abacus_pw_force_nl(C.byref(f.s), 1, 1, FAKE, FAKE, FAKE, None)) == "EBAD_PRECISION"


def test_binding_checks_tensors_before_the_library(prob):
    """Every binding entry point refuses host tensors, wrong dtypes, wrong lengths and
    non-contiguous views before a pointer reaches the C ABI (here no GPU exists, so a
    pointer that got through would fail differently)."""
    import torch
    dp = B.DeviceProblem(prob, device="cpu")
    n = dp.psi_len(prob.nb)
    psi = torch.zeros(n, dtype=torch.complex128)
    calls = {
        "apply_h": lambda x: B.apply_h(dp, x),
        "apply_h_fp32": lambda x: B.apply_h(dp, x, B.FP32),
        "apply_h_backward": lambda x: B.apply_h_backward(dp, x, x),
        "density": lambda x: B.density(dp, x, np.ones((dp.nk, prob.nb))),
        "force_nl": lambda x: B.force_nl(dp, x, np.ones((dp.nk, prob.nb))),
        "chebyshev": lambda x: B.chebyshev(dp, x, [1.0, 0.5], -1.0, 1.0),
        "davidson": lambda x: B.davidson(dp, x),
        "cg": lambda x: B.cg(dp, x),
    }
    for name, call in calls.items():
        for bad in (psi, psi[:-1], psi.to(torch.complex64) if name != "apply_h_fp32" else psi,
                    torch.zeros(2 * n, dtype=torch.complex128)[::2]):
            with pytest.raises(B.AbacusPwError) as e:
                call(bad)
            assert e.value.code == -2, (name, str(e.value))
    with pytest.raises(B.AbacusPwError) as e:
        B.apply_h(dp, psi, precision=7)
    assert e.value.code == -7


def test_density_g_rejects_before_device_access():
    L = B.lib()
    ok = np.array([16, 16, 16], dtype=np.int32)
    bad = np.array([14, 16, 16], dtype=np.int32)
    assert code_name(L.abacus_pw_density_g(bad.ctypes.data, FAKE, 14 * 256, None, FAKE, None)) == "EBAD_FFT_SIZE"
    assert code_name(L.abacus_pw_density_g(ok.ctypes.data, FAKE, 100, None, FAKE, None)) == "EBAD_SHAPE"
    assert code_name(L.abacus_pw_density_g(ok.ctypes.data, FAKE, -1, FAKE, FAKE, None)) == "EBAD_SHAPE"
    assert code_name(L.abacus_pw_density_g(None, FAKE, 1, FAKE, FAKE, None)) == "ENULL_ARG"
    assert code_name(L.abacus_pw_density_g(ok.ctypes.data, None, 1, FAKE, FAKE, None)) == "ENULL_ARG"


def test_workspace_entry_points_reject_before_device_access(prob):
    f = Fake(prob)
    L = B.lib()
    out = C.c_size_t(0)
    assert code_name(L.abacus_pw_workspace_size(C.byref(f.s), 0, 1, None, None)) == "ENULL_ARG"
    assert code_name(L.abacus_pw_workspace_size(C.byref(f.s), 0, 0, C.byref(out), None)) == "EBAD_SHAPE"
    assert code_name(L.abacus_pw_workspace_size(C.byref(f.s), 9, 1, C.byref(out), None)) == "EBAD_PRECISION"
    assert code_name(L.abacus_pw_apply_h_ws(C.byref(f.s), 0, 1, FAKE, FAKE + 64, None, 0, None)) == "ENULL_ARG"
    assert code_name(L.abacus_pw_apply_h_ws(C.byref(f.s), 0, 1, FAKE, FAKE, FAKE, 1 << 20, None)) == "EBAD_SHAPE"
    assert code_name(L.abacus_pw_apply_h_ws(C.byref(f.s), 0, 1, FAKE, FAKE + 64, FAKE + 8, 1 << 20, None)) == "EBAD_SHAPE"
