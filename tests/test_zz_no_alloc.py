"""abacus_pw_density_g_noalloc (the entry point for callers that cannot
allocate) against abacus_pw_density_g, through the C ABI: two calls in a row
on a G list, the second on a smaller grid and a shorter list, so the fixed
work grid holds the first call's values when the second starts; each result
must equal the allocating entry point's bit for bit (same kernels, same
order). Also the whole-grid form and the empty list."""
import ctypes as C

import numpy as np
import pytest

from paper_2501_08697_amd import workload as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def B():
    from paper_2501_08697_amd import binding
    return binding


def call(name, rho, miller, ng):
    b = B()
    fft = np.ascontiguousarray(rho.shape, dtype=np.int32)
    out = torch.empty(max(ng, 1), dtype=torch.complex128, device=rho.device)
    fn = getattr(b.lib(), name)
    mp = None if miller is None else C.c_void_p(miller.data_ptr())
    code = fn(fft.ctypes.data, C.c_void_p(rho.data_ptr()), int(ng), mp, C.c_void_p(out.data_ptr()),
              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    b.check(code)
    torch.cuda.synchronize()
    return out[:ng].cpu().numpy()


def case(n, ecut_scale, seed):
    rng = np.random.default_rng(seed)
    rho = torch.from_numpy(rng.uniform(0.0, 2.0, (n, n, n))).cuda()
    m = W.g_sphere(np.eye(3) * 10.0, np.zeros(3), ecut_scale)
    m = m[np.all(2 * np.abs(m) + 1 <= n, axis=1)]
    return rho, torch.from_numpy(np.ascontiguousarray(m, dtype=np.int32)).cuda(), len(m)


def test_noalloc_matches_allocating_entry_point_twice():
    rho1, m1, ng1 = case(96, 80.0, 1)
    rho2, m2, ng2 = case(32, 20.0, 2)
    assert rho2.numel() < rho1.numel() and ng2 < ng1
    print(f"[noalloc] 96^3 with {ng1} G, then 32^3 with {ng2} G", flush=True)
    a1 = call("abacus_pw_density_g_noalloc", rho1, m1, ng1)
    r1 = call("abacus_pw_density_g", rho1, m1, ng1)
    a2 = call("abacus_pw_density_g_noalloc", rho2, m2, ng2)
    r2 = call("abacus_pw_density_g", rho2, m2, ng2)
    assert np.array_equal(a1, r1)
    assert np.array_equal(a2, r2)
    assert np.max(np.abs(a1)) > 0 and np.max(np.abs(a2)) > 0


def test_noalloc_whole_grid_and_empty_list():
    rho, m, ng = case(48, 40.0, 3)
    full_a = call("abacus_pw_density_g_noalloc", rho, None, rho.numel())
    full_r = call("abacus_pw_density_g", rho, None, rho.numel())
    assert np.array_equal(full_a, full_r)
    one = torch.zeros((1, 3), dtype=torch.int32, device="cuda")   # a valid pointer, no entries read
    out = call("abacus_pw_density_g_noalloc", rho, one, 0)
    assert out.size == 0
