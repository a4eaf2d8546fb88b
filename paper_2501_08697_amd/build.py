"""Builds the HIP library libabacus_pw.so in this folder (gfx950 only).

Every source under csrc/ is compiled by hipcc (device code for gfx950, with
packed-FP32 instructions disabled) into an object under _build/, in parallel,
and the objects are linked into one shared library with a C ABI
(include/abacus_pw.h).

The compiler's per-kernel resource report is read back: a kernel that keeps
anything in scratch (private) memory fails the build unless it is listed in
SCRATCH_ALLOWED (instances that are compiled but never launched, or run only
off the hot path). Scratch use turns register arrays into memory traffic and
has doubled kernel times here before.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "abacus_pw")
LIB = os.path.join(HERE, "libabacus_pw.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
          f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


# kernel symbol prefixes allowed to use scratch, with the reason
SCRATCH_ALLOWED = {
    # full-plane y-z forward pass at 120 and 128 in FP64: never launched (the plane
    # exceeds LDS at FP64, the compact-row kernel runs instead)
    "_ZN3apw8k_yz_fwdILi120EddE": 128,
    "_ZN3apw8k_yz_fwdILi128EddE": 256,
    # tridiagonal reduction with its panel in global memory (subspace above 256): 8 bytes
    "_ZN3apw7k_hetrdILb0EE": 16,
}


def _scratch_report(stderr: str):
    """(kernel, bytes per lane) for every kernel with scratch, from -Rpass-analysis remarks."""
    out, name = [], None
    for line in stderr.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:")[1].split()[0]
        elif "ScratchSize [bytes/lane]:" in line and name:
            n = int(line.split("ScratchSize [bytes/lane]:")[1].split()[0])
            if n > 0:
                out.append((name, n))
    return out


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + ["-c", src, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    bad = [(k, n) for k, n in _scratch_report(r.stderr)
           if not any(k.startswith(a) and n <= lim for a, lim in SCRATCH_ALLOWED.items())]
    if bad:
        raise RuntimeError(f"kernels in {os.path.basename(src)} use scratch memory: {bad}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
