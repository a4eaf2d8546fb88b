"""H psi at the full size of the three largest workloads, against the FP64 oracle.

Each case runs the whole launch (every k-point, every band, every projector) in
the configuration the benchmark times, and compares sampled output rows
element by element with the oracle's H psi of the same bands (H psi is
independent per band, so the oracle applies H to the sampled rows only):

  * a = 30 bohr, ecutwfc = 50 Ry, 128^3, Gamma: 1024 bands, 161,235 PW,
    2304 projectors with full 9 x 9 D blocks; the first, middle and last band
    of every 64-band batch.
  * a = 30 bohr, ecutwfc = 40 Ry, 120^3, the eight uneven k-points of the
    {0, 1/2}^3 grid: 8 x 512 bands, 864 projectors; the first and last band of
    every 64-band batch at every k-point, and the middle band of the first and
    last batch.
  * a = 24 bohr, ecutwfc = 35 Ry, 96^3, Gamma, X, M, R: 4 x 256 bands; the
    first, middle and last band of every batch at every k-point.

Bounds (relative max-norm over the sampled rows): FP64 1e-12, FP32 and
MIXED_FP32 1e-5, MIXED_BF16 2e-2.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2501_08697_amd import workload as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BOUND = {0: 1e-12, 1: 1e-5, 3: 1e-5, 2: 2e-2}
NAMES = {0: "FP64", 1: "FP32", 2: "MIXED_BF16", 3: "MIXED_FP32"}
BATCH = 64


def B():
    from paper_2501_08697_amd import binding
    return binding


def say(msg):
    print(f"[fullsize {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def batch_samples(nb, middle_batches=None):
    """First and last band of every batch, plus the middle band of the given batches
    (all batches when None)."""
    out = set()
    nbat = (nb + BATCH - 1) // BATCH
    for q in range(nbat):
        lo, hi = q * BATCH, min(nb, (q + 1) * BATCH) - 1
        out.update((lo, hi))
        if middle_batches is None or q in middle_batches:
            out.add((lo + hi) // 2)
    return sorted(out)


class Case:
    def __init__(self, name, samples_fn):
        say(f"generating {name}")
        t = time.time()
        self.p = W.make_problem(name)
        say(f"{name}: generated in {time.time() - t:.1f} s; npw {list(map(int, self.p.npw))}, "
            f"nproj {self.p.nproj}, nb {self.p.nb}")
        self.samples = [samples_fn(self.p.nb) for _ in range(self.p.nk)]
        self.ref = []
        for k in range(self.p.nk):
            sub = oracle._single_k(self.p, k)
            rows = self.p.psi_k(k)[self.samples[k]]
            t = time.time()
            y = oracle.apply_h(sub, np.ascontiguousarray(rows).reshape(-1), nb=len(self.samples[k]))
            self.ref.append(y.reshape(len(self.samples[k]), -1))
            say(f"{name}: oracle k={k}, {len(self.samples[k])} bands in {time.time() - t:.1f} s "
                f"({oracle.num_threads()} threads)")
        self.dp = None

    def check(self, prec):
        b = B()
        if self.dp is None:
            self.dp = b.DeviceProblem(self.p, static=True)
        x = torch.from_numpy(self.p.psi).cuda()
        if prec == b.FP32:
            x = x.to(torch.complex64)
        b.set_tuning()
        y = b.apply_h(self.dp, x, prec)
        torch.cuda.synchronize()
        off = self.p.pw_offsets
        num = den = 0.0
        for k in range(self.p.nk):
            yk = y[self.p.nb * off[k]: self.p.nb * off[k + 1]].view(self.p.nb, -1)
            got = yk[self.samples[k]].to(torch.complex128).cpu().numpy()
            num = max(num, float(np.max(np.abs(got - self.ref[k]))))
            den = max(den, float(np.max(np.abs(self.ref[k]))))
        del y, x
        e = num / den
        say(f"{self.p.name} {NAMES[prec]}: relative max error over the sampled rows {e:.3e}")
        return e


@pytest.fixture(scope="module")
def c4():
    return Case("C4", lambda nb: batch_samples(nb))


@pytest.fixture(scope="module")
def c3():
    return Case("C3", lambda nb: batch_samples(nb, middle_batches={0, (nb - 1) // BATCH}))


@pytest.fixture(scope="module")
def c5():
    return Case("C5", lambda nb: batch_samples(nb))


@pytest.mark.parametrize("prec", [0, 1, 3, 2])
def test_c4_full_launch(c4, prec):
    assert c4.check(prec) < BOUND[prec]


@pytest.mark.parametrize("prec", [0, 1, 3, 2])
def test_c3_full_launch(c3, prec):
    assert c3.check(prec) < BOUND[prec]


@pytest.mark.parametrize("prec", [0, 2])
def test_c5_full_launch(c5, prec):
    assert c5.check(prec) < BOUND[prec]
