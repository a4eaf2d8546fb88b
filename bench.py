"""Benchmark of the plane-wave H psi hot path on one MI355X.

Headline workload (the batched uneven-k case, the largest that runs on one
GPU): simple-cubic cell a = 30 bohr, ecutwfc = 40 Ry, 120^3 grid, the eight
k-points of the {0, 1/2}^3 grid (spheres of 115,096 - 115,396 plane waves),
216 atoms x 4 Kleinman-Bylander projectors (s + p), 512 bands per k-point,
complex128, seeded synthetic inputs.

One step = one H psi over all 8 x 512 bands in FP64 (local term: three LDS
transform passes on the grid, every k-point of a band batch in one launch per
pass; nonlocal term: projection GEMM, D blocks, accumulation GEMM per
k-point), issued as one abacus_pw_apply_h call captured in a HIP graph and
replayed, inputs resident in HBM. `value` = band-applies per second =
4096 * steps / time.

The same JSON line carries: the roofline of the dominant kernel (per-kernel
times from HIP events the library records on its stream in a profiled copy of
the timed region), the local term against the pruned 5-pass byte model, the
batched form against one call per k-point and the graph against eager calls,
the launch gaps, complex64 / mixed precision rates, the 128^3 mixed-precision
workload, the 72^3 FP64-vs-FP32 workload with its Davidson and CG legs, the
band density, force, Chebyshev and adjoint legs, and the FP64 CPU oracle on a
sample of the headline workload on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-davidson] [--no-cg]
                      [--no-batched] [--no-autotune] [--no-density] [--no-backward] [--no-chebyshev]
                      [--no-force] [--no-c4] [--no-c2] [--traffic-probe]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, datasheet
BF16_PEAK_TFLOPS = 2500.0       # MI355X dense BF16 MFMA
FP64_PEAK_TFLOPS = 78.6         # MI355X dense FP64 (vector = matrix)
FP32_PEAK_TFLOPS = 157.3
WORKLOAD = "C3"
WORKLOAD_DESC = ("cubic a=30 bohr, ecutwfc=40 Ry, 120^3 grid, 8 k-points of the {0,1/2}^3 grid (uneven spheres), "
                 "216 atoms x 4 KB projectors, 512 bands per k-point, complex128")


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-davidson", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-density", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-chebyshev", action="store_true")
    ap.add_argument("--no-force", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the 72^3 legs (H psi, density, force, Chebyshev, "
                                                          "Davidson, CG)")
    ap.add_argument("--c4-davidson", action="store_true",
                    help="also run Davidson to a 1e-8 residual on the 128^3, 1024-band workload in FP64 and "
                         "MIXED_BF16 (several minutes)")
    ap.add_argument("--cpu-extended", action="store_true",
                    help="also time the oracle on C1, C2, C4 and C5 (H psi samples, C1 Davidson, C2 and C5 "
                         "Davidson iterations; several minutes of host time)")
    ap.add_argument("--c3-davidson", action="store_true",
                    help="also run Davidson to a 1e-8 residual on the headline workload (8 k-points x 512 bands) "
                         "in FP64 and MIXED_BF16 (about two minutes)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run a plain 256 MiB copy and a few FP64 H psi steps only (for counter collection)")
    ap.add_argument("--probe-workload", default=WORKLOAD,
                    help="workload of --traffic-probe (default: the headline workload)")
    ap.add_argument("--probe-precision", type=int, default=0,
                    help="precision of --traffic-probe: 0 FP64, 1 FP32, 2 MIXED_BF16, 3 MIXED_FP32")
    return ap.parse_args()


def slab_points(prob):
    """S = nslab N2 N3: the grid planes (union over k-points) that hold sphere points."""
    n1, n2, n3 = prob.fft
    m1 = prob.miller[:, 0]
    return (int(m1.max()) - int(m1.min()) + 1) * n2 * n3


def kernel_model(name, prob, nb, launches):
    """Algorithmic (bytes, flops counted, flops executed) of ONE launch of a library kernel.

    Per step (one H psi over nb bands at every k-point), with cb = 16 bytes per
    complex128, S = nslab * N2 * N3 (the slab: grid planes that hold sphere
    points), npw_k the sphere sizes; a step's figures are divided by the
    kernel's launches per step.
      yz_inv : nb cb sum_k (npw_k + S)          read psi, write the slab planes
      xpass  : nb cb 2 S nk + launches 8 N      slab in and out, V once per launch
      yz_fwd : nb cb sum_k (S + 2 npw_k)        slab in, psi in (kinetic), H psi out
      gemm_cn: flops 8 nproj nb sum_k npw_k     counted complex flops; the kernel's 3M
                                                products execute 6 nproj nb sum npw_k
      gemm_nn: flops 8 nb sum_k npw_k nproj     likewise (6 executed)
    """
    cb = 16
    n1, n2, n3 = prob.fft
    N = n1 * n2 * n3
    npw = [int(x) for x in prob.npw]
    nk = len(npw)
    S = slab_points(prob)
    npj = prob.nproj
    tot = sum(npw)
    per_step = {
        "yz_inv": (nb * cb * sum(n + S for n in npw), 0, 0),
        "xpass": (nb * cb * 2 * S * nk + launches * 8 * N, 0, 0),
        "yz_fwd": (nb * cb * sum(S + 2 * n for n in npw), 0, 0),
        "gemm_cn": (cb * (npj + nb) * tot, 8 * npj * nb * tot, 6 * npj * nb * tot),
        "gemm_nn": (cb * (npj * tot + 2 * nb * tot), 8 * nb * tot * npj, 6 * nb * tot * npj),
    }
    if name not in per_step:
        return None, None, None
    by, fl, fe = per_step[name]
    return by / launches, fl / launches, fe / launches


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "yz_inv": ["paper_2501_08697_amd/csrc/local.hip", "paper_2501_08697_amd/csrc/fft_device.hpp"],
    "xpass": ["paper_2501_08697_amd/csrc/local.hip", "paper_2501_08697_amd/csrc/fft_device.hpp"],
    "yz_fwd": ["paper_2501_08697_amd/csrc/local.hip", "paper_2501_08697_amd/csrc/fft_device.hpp"],
    "gemm_cn": ["paper_2501_08697_amd/csrc/gemm.hip"],
    "gemm_nn": ["paper_2501_08697_amd/csrc/gemm.hip"],
}


def local_model_bytes(prob):
    """Per band, averaged over the k-points: the pruned 5-pass model's bytes for the
    local term (z on the disk of columns that hold sphere points, y on the slab, x on
    all; cb N 4 (f_disk + f_slab) + 2 cb npw) and the bytes the three fused plane
    passes here move (4 cb S + 3 cb npw, the disk staying in LDS)."""
    cb = 16
    n1, n2, n3 = prob.fft
    N = n1 * n2 * n3
    off = prob.pw_offsets
    model = ours = fd = fs = 0.0
    nk = len(prob.npw)
    for k in range(nk):
        m = prob.miller[off[k]:off[k + 1]]
        npw = int(prob.npw[k])
        cols = len({(int(a) % n1, int(b) % n2) for a, b in zip(m[:, 0], m[:, 1])})
        f_disk = cols / (n1 * n2)
        nslab_k = int(m[:, 0].max()) - int(m[:, 0].min()) + 1
        f_slab = nslab_k / n1
        model += cb * N * 4 * (f_disk + f_slab) + 2 * cb * npw
        ours += 4 * cb * slab_points(prob) + 3 * cb * npw
        fd += f_disk
        fs += f_slab
    return model / nk, ours / nk, fd / nk, fs / nk


def measured_traffic(kernel, bands_per_launch, workload=WORKLOAD):
    """HBM bytes per launch from the committed counter summary, if it matches the current source.

    The summary was taken at its own launch shape (`bands_per_launch:` in the file,
    bands of all k-points one launch covers); the bytes scale with the bands one
    launch processes, so they are rescaled to the launch shape timed here."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    nb = re.search(r"bands_per_launch:\s*([0-9]+)", txt)
    if not m or not b or not nb or m.group(1) != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return float(b.group(1)) * bands_per_launch / int(nb.group(1))


def host_cpu():
    """CPU model, sockets, physical cores and logical CPUs of this host (lscpu)."""
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = dict(line.split(":", 1) for line in txt.splitlines() if ":" in line)
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "1"))
        cps = int(kv.get("Core(s) per socket", "0"))
        info["sockets"] = sockets
        info["physical_cores"] = sockets * cps
        info["logical_cpus"] = int(kv.get("CPU(s)", "0"))
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except OSError:
        pass
    return info


def cpu_baseline(prob, one_thread_bands=1):
    """The FP64 oracle's H psi on a sample of the headline workload: as many bands as
    there are OpenMP threads (the oracle runs one band per thread) at the first and the
    last k-point, with all threads, and one band of the first k-point on one thread.
    Band-applies per second of each."""
    import oracle
    nthreads = oracle.num_threads()
    bands_per_k = min(prob.nb, nthreads)
    ks = sorted({0, prob.nk - 1})
    t_all, n_all = 0.0, 0
    for k in ks:
        sub = oracle._single_k(prob, k)
        rows = np.ascontiguousarray(prob.psi_k(k)[:bands_per_k]).reshape(-1)
        t0 = time.perf_counter()
        oracle.apply_h(sub, rows, nb=bands_per_k)
        t_all += time.perf_counter() - t0
        n_all += bands_per_k
    log(f"cpu baseline: {n_all} bands on {nthreads} threads in {t_all:.1f} s")
    oracle.set_num_threads(1)
    try:
        sub = oracle._single_k(prob, 0)
        rows = np.ascontiguousarray(prob.psi_k(0)[:one_thread_bands]).reshape(-1)
        t0 = time.perf_counter()
        oracle.apply_h(sub, rows, nb=one_thread_bands)
        t_one = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(nthreads)
    log(f"cpu baseline: {one_thread_bands} band on 1 thread in {t_one:.1f} s")
    return {"value": n_all / t_all, "unit": "band-applies/s", "cores": nthreads, "kind": "oracle",
            "sample": f"FP64 H psi of the first {bands_per_k} bands at k-points {ks} of the benchmark workload "
                      f"({n_all} band-applies, {t_all:.2f} s wall, {nthreads} OpenMP threads, one band each)",
            "one_thread": {"value": one_thread_bands / t_one, "unit": "band-applies/s",
                           "sample": f"{one_thread_bands} band of k-point 0 on 1 thread ({t_one:.2f} s wall)"},
            "host": host_cpu()}


def cpu_extended(W, max_iter_small=3):
    """The oracle on the other workloads (opt-in: several minutes of host time): FP64 H psi
    band-applies/s on a band sample of C1, C2, C4 and C5 (as many bands as OpenMP threads,
    at the first k-point), the full Davidson of C1 to 1e-8, and seconds per Davidson
    iteration at k-point 0 of C2 and C5 after a fixed number of iterations. C3 and C4
    Davidson iterations are not timed: one iteration applies H to 512 or 1024 bands,
    which the H psi rates above put at minutes per iteration."""
    import oracle
    nthreads = oracle.num_threads()
    out = {"cores": nthreads, "kind": "oracle", "hpsi": {}, "davidson": {}}
    for name in ("C1", "C2", "C4", "C5"):
        prob = W.make_problem(name)
        nbs = min(prob.nb, nthreads)
        sub = oracle._single_k(prob, 0)
        rows = np.ascontiguousarray(prob.psi_k(0)[:nbs]).reshape(-1)
        t0 = time.perf_counter()
        oracle.apply_h(sub, rows, nb=nbs)
        dt = time.perf_counter() - t0
        out["hpsi"][name] = {"band_applies_per_s": nbs / dt, "bands": nbs, "s": dt}
        log(f"cpu extended: {name} H psi, {nbs} bands in {dt:.2f} s")
        if name == "C1":
            t0 = time.perf_counter()
            eig, _, res, its = oracle.davidson(prob, tol=1e-8, max_iter=200)
            dt = time.perf_counter() - t0
            out["davidson"][name] = {"s_per_kpoint": dt / prob.nk, "iterations": [int(x) for x in its],
                                     "max_resid": float(res.max()), "tol": 1e-8}
            log(f"cpu extended: C1 Davidson {dt:.2f} s, {list(its)} iterations")
        elif name in ("C2", "C5"):
            x0 = np.asarray(prob.psi_k(0))

            def hop(r, sub=sub):
                return oracle.apply_h(sub, r.reshape(-1), nb=r.shape[0]).reshape(r.shape)

            t0 = time.perf_counter()
            oracle.davidson_k(hop, x0, oracle.kinetic(sub, 0), 1e-8, 0, 2)
            t_start = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, _, _, it = oracle.davidson_k(hop, x0, oracle.kinetic(sub, 0), 1e-8, max_iter_small, 2)
            dt = time.perf_counter() - t0
            per = (dt - t_start) / max(1, int(it))
            out["davidson"][name] = {"s_start": t_start, "iterations": int(it), "s_per_iteration": per,
                                     "k_point": 0}
            log(f"cpu extended: {name} Davidson start {t_start:.1f} s, {per:.1f} s per iteration")
        del prob
    return out


def measured_hbm_peak(dev, nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read + write), best of reps, in GB/s: the
    achievable HBM rate on this GPU, beside the datasheet peak."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2 * nbytes / (best * 1e-3) / 1e9


def kernel_rows(kern, prob, nb, steps, ms_step):
    rows = {}
    for name, (n, tot_ms) in kern.items():
        avg = tot_ms / n
        by, fl, fe = kernel_model(name, prob, nb, n / steps)
        r = {"launches_per_step": n / steps, "avg_ms": avg, "share": tot_ms / (ms_step * steps),
             "alg_bytes": by, "alg_flops": fl}
        if fl:
            r["tflops_counted"] = fl / (avg * 1e-3) / 1e12
            r["tflops_executed"] = fe / (avg * 1e-3) / 1e12
            r["frac_executed_fp64"] = r["tflops_executed"] / FP64_PEAK_TFLOPS
        elif by:
            r["gbs"] = by / (avg * 1e-3) / 1e9
        rows[name] = r
    return rows


def roofline_of(rows, prob, nb, workload, mp):
    """Roofline of the kernel with the largest share of the step. MFMA kernels are
    priced at the flops they execute (the 3M complex products: 6 M N K), the
    counted 8 M N K rate beside it as `achieved_counted`."""
    dom = max(rows, key=lambda k: rows[k]["avg_ms"] * rows[k]["launches_per_step"])
    d = rows[dom]
    if d["alg_flops"]:
        achieved = d["tflops_executed"]
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "achieved_counted": d["tflops_counted"]}
    else:
        achieved = d["alg_bytes"] / (d["avg_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    roof["kernel"] = dom
    roof["avg_launch_ms"] = d["avg_ms"]
    roof["alg_bytes_per_launch"] = d["alg_bytes"]
    roof["traffic"] = measured_traffic(dom, prob.nk * nb / d["launches_per_step"], workload) \
        if dom in KERNEL_SOURCES else None
    if roof["bound"] == "hbm":
        roof["measured_peak"] = mp             # 1 GiB device copy on this GPU
        roof["frac_of_measured_peak"] = achieved / mp
    return roof


def local_term_of(rows, prob, nb, mp):
    t_local = sum(rows[k]["avg_ms"] * rows[k]["launches_per_step"] for k in ("yz_inv", "xpass", "yz_fwd") if k in rows)
    model_b, ours_b, f_disk, f_slab = local_model_bytes(prob)
    nbt = nb * prob.nk
    lt = {"ms_per_step": t_local, "f_disk": f_disk, "f_slab": f_slab,
          "model_bytes_per_band": model_b, "fused_bytes_per_band": ours_b,
          "effective_GBs": model_b * nbt / (t_local * 1e-3) / 1e9,
          "physical_GBs": ours_b * nbt / (t_local * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "measured_peak": mp}
    lt["frac_effective"] = lt["effective_GBs"] / HBM_PEAK_GBS
    lt["frac_physical"] = lt["physical_GBs"] / HBM_PEAK_GBS
    return lt


def timed_calls(fn, steps, stream=None):
    """ms per call of fn over `steps` calls, bracketed by synchronisations."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream) if stream is not None else a.record()
    for _ in range(steps):
        fn()
    b.record(stream) if stream is not None else b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding is design-only.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2501_08697_amd import binding as B
    from paper_2501_08697_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = args.probe_workload if args.traffic_probe else WORKLOAD
    log(f"generating {wl}")
    t0 = time.time()
    prob = W.make_problem(wl)
    nb, nk = prob.nb, prob.nk
    log(f"{wl}: {time.time() - t0:.1f} s; npw {list(map(int, prob.npw))}")
    dp = B.DeviceProblem(prob, device=dev, static=True)   # operator data constant for the whole run
    x64 = torch.from_numpy(prob.psi).to(dev)
    y64 = torch.empty_like(x64)
    stream = torch.cuda.current_stream()

    def step():
        B.apply_h(dp, x64, B.FP64, out=y64)

    if args.traffic_probe:
        # calibration: one plain device copy of a known size, then H psi steps with default tuning
        n = 256 << 20
        src = torch.ones(n // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        xp = x64.to(torch.complex64) if args.probe_precision == B.FP32 else x64
        yp = torch.empty_like(xp)
        for _ in range(max(1, args.steps)):
            B.apply_h(dp, xp, args.probe_precision, out=yp)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "workload": wl, "precision": args.probe_precision, "copy_bytes": n,
                          "steps": max(1, args.steps)}), flush=True)
        return

    # warm-up (builds the plan, allocates work space); the timed region runs the library's
    # default launch shapes (the autotuner's search is reported after it)
    B.set_tuning()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warm-up done")

    # the timed region: the H psi call replayed from a HIP graph
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    g.replay()
    torch.cuda.synchronize()
    ms_graph = timed_calls(g.replay, args.steps, stream)
    log(f"timed: {ms_graph:.2f} ms per step (graph replay)")

    # profiled copy of the timed work: HIP events around every library launch, recorded on its stream
    B.profile_read()
    B.profile_enable(True)
    prof_steps = max(2, min(args.steps, 5))
    ms_prof = timed_calls(step, prof_steps, stream)
    B.profile_enable(False)
    kern = B.profile_read()
    ms_eager = timed_calls(step, max(3, args.steps // 4), stream)
    rows = kernel_rows(kern, prob, nb, prof_steps, ms_prof)
    sum_kernels = sum(r["avg_ms"] * r["launches_per_step"] for r in rows.values())
    launches = sum(r["launches_per_step"] for r in rows.values())
    mp = measured_hbm_peak(dev)
    roof = roofline_of(rows, prob, nb, WORKLOAD, mp)
    tuning = None
    if not args.no_autotune:
        # what a search of the launch knobs finds beyond the defaults timed above
        from paper_2501_08697_amd import autotune
        cfg64, ms_tuned = autotune.tune(dp, x64, precision=B.FP64, use_cache=False, reps=2, sweeps=1, trials=2)
        tuning = {"fp64": cfg64, "ms_tuned": ms_tuned, "ms_default_eager": ms_eager,
                  "speedup_tuned_vs_default": ms_eager / ms_tuned}
        log(f"autotune: {cfg64} {ms_tuned:.2f} ms (default {ms_eager:.2f} ms)")
        B.set_tuning()

    out = {
        "metric": "Hψ band-applies/s, Davidson time/k-point vs plain FP64; % HBM & MFMA peak",
        "value": nk * nb / (ms_graph * 1e-3),
        "unit": "band-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: {WORKLOAD_DESC}", "kpoints": nk, "bands_per_kpoint": nb,
                   "npw": [int(x) for x in prob.npw], "fft": list(prob.fft), "nproj": prob.nproj,
                   "issue": "one abacus_pw_apply_h call over all k-points, replayed from a HIP graph"},
        "roofline": roof,
        "local_term": local_term_of(rows, prob, nb, mp),
        "kernels": rows,
        "launches": {"per_step": launches, "eager_ms_per_step": ms_eager,
                     "profiled_ms_per_step": ms_prof, "sum_of_kernel_ms_per_step": sum_kernels,
                     "gap_ms_per_step": ms_eager - sum_kernels,
                     "gap_fraction": (ms_eager - sum_kernels) / ms_eager,
                     "graph_vs_eager": ms_eager / ms_graph},
        "tuning": tuning,
    }
    if not args.no_batched:
        log("batched vs per-k-point calls, precisions")
        out["batched_kpoints"] = batched_times(B, W, dev, 3, prob=prob, dp=dp, x=x64)
    del y64
    torch.cuda.synchronize()
    if not args.no_davidson:
        log("C3 Davidson iterations")
        out["davidson_c3"] = davidson_iteration_times(B, dev, prob, dp, iters=2)
    if not args.no_cpu:
        log("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(prob)
        if args.cpu_extended:
            log("CPU oracle on the other workloads")
            out["cpu_baseline"]["other_workloads"] = cpu_extended(W)
    del x64, dp, prob
    torch.cuda.empty_cache()
    B.plan_reset()
    B.set_tuning()

    if not args.no_c4:
        log("C4 mixed precision")
        out["mixed_precision_c4"] = c4_times(B, W, dev, davidson=not args.no_davidson)
    if not args.no_c2:
        log("C2 legs")
        c2 = W.make_problem("C2")
        dp2 = B.DeviceProblem(c2, device=dev, static=True)
        x2 = torch.from_numpy(c2.psi).to(dev)
        out["c2_h_psi"] = c2_times(B, dev, c2, dp2, x2, max(10, args.steps))
        ms_c2 = out["c2_h_psi"]["fp64"]["ms_per_step"]
        if not args.no_density:
            out["density"] = density_times(B, W, dev, c2, dp2, x2, max(10, args.steps))
        if not args.no_force:
            out["force_nl"] = force_times(B, W, dev, c2, dp2, x2, max(10, args.steps))
        if not args.no_chebyshev:
            out["chebyshev"] = chebyshev_times(B, W, dev, c2, dp2, ms_c2)
        del dp2, x2
        B.plan_reset()
        if not args.no_davidson:
            log("C2 Davidson")
            out["davidson"] = davidson_times(B, W, dev)
            log("C5 Davidson")
            out["davidson_c5"] = davidson_times(B, W, dev, "C5", modes=(("fp64", 0), ("mixed_bf16", 2)))
        if not args.no_cg:
            log("C2 CG")
            out["cg_vs_davidson"] = cg_times(B, W, dev, out.get("davidson"))
    if args.c3_davidson:
        log("C3 Davidson to 1e-8")
        out["davidson_c3_full"] = davidson_times(B, W, dev, "C3", max_iter=300, modes=(("fp64", 0), ("mixed_bf16", 2)))
    if args.c4_davidson:
        log("C4 Davidson to 1e-8")
        out["davidson_c4"] = davidson_times(B, W, dev, "C4", max_iter=300, modes=(("fp64", 0), ("mixed_bf16", 2)))
    if not args.no_backward:
        log("C5 adjoint")
        out["backward"] = backward_times(B, W, dev, max(5, args.steps // 4))
    if not args.no_batched:
        log("C5 batched")
        out["batched_kpoints_c5"] = batched_times(B, W, dev, max(5, args.steps // 4), "C5")
    print(json.dumps(out), flush=True)


def c2_times(B, dev, prob, dp, x64, steps):
    """The FP64-vs-FP32 H psi workload (cubic a = 20.5 bohr, ecutwfc = 30 Ry, 72^3,
    23,847 PW at Gamma, 64 atoms x 4 projectors, 128 bands): FP64 and FP32 per H psi
    after the autotuner, with per-kernel rates."""
    import torch
    from paper_2501_08697_amd import autotune
    nb = prob.nb
    x32 = x64.to(torch.complex64)
    y64, y32 = torch.empty_like(x64), torch.empty_like(x32)
    for _ in range(3):
        B.apply_h(dp, x64, B.FP64, out=y64)
        B.apply_h(dp, x32, B.FP32, out=y32)
    cfg32, _ = autotune.tune(dp, x32, precision=B.FP32, use_cache=False)
    cfg64, _ = autotune.tune(dp, x64, precision=B.FP64, use_cache=False)
    B.profile_read()
    B.profile_enable(True)
    ms_prof = timed_calls(lambda: B.apply_h(dp, x64, B.FP64, out=y64), steps)
    B.profile_enable(False)
    kern = B.profile_read()
    ms64 = timed_calls(lambda: B.apply_h(dp, x64, B.FP64, out=y64), steps)
    B.set_tuning(**cfg32)
    ms32 = timed_calls(lambda: B.apply_h(dp, x32, B.FP32, out=y32), steps)
    B.set_tuning()
    rows = kernel_rows(kern, prob, nb, steps, ms_prof)
    res = {"workload": "C2: cubic a=20.5 bohr, ecutwfc=30 Ry, 72^3, 23847 PW, Gamma, 64 atoms x 4 projectors, "
                       "128 bands",
           "fp64": {"ms_per_step": ms64, "band_applies_per_s": nb / (ms64 * 1e-3)},
           "fp32": {"ms_per_step": ms32, "band_applies_per_s": nb / (ms32 * 1e-3), "speedup_vs_fp64": ms64 / ms32},
           "kernels": rows, "tuning": {"fp64": cfg64, "fp32": cfg32}}
    dom = max(rows, key=lambda k: rows[k]["avg_ms"] * rows[k]["launches_per_step"])
    res["dominant"] = {"kernel": dom, **rows[dom]}
    if dom in KERNEL_SOURCES:
        res["dominant"]["traffic"] = measured_traffic(dom, nb / rows[dom]["launches_per_step"], "C2")
    return res


def density_times(B, W, dev, prob, dp, x, steps):
    """Band density rho(r) = sum_n w_n |psi_n(r)|^2 of the benchmark's 128 bands on its 72^3 grid, FP64.

    Per call: the y-z inverse passes (sphere -> slab planes) and one x pass that
    transforms and accumulates (k_density_x), then the fixed-order sum of the
    partial grids. The model bytes are the inverse half of the pruned 5-pass
    local-term model plus rho written once: nb (cb N 2 (f_disk + f_slab) + cb npw) + 8 N.
    k_density_x moves nb cb S (slab in) plus its partial grids (G = 8 of N doubles,
    read and written once per band batch).
    """
    import torch
    nb = prob.nb
    occ = torch.from_numpy(W.band_weights(prob, 0)).to(dev)
    rho = torch.empty(tuple(prob.fft), dtype=torch.float64, device=dev)
    for _ in range(3):
        B.density(dp, x, occ, out=rho)
    torch.cuda.synchronize()
    B.profile_read()
    B.profile_enable(True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        B.density(dp, x, occ, out=rho)
    b.record()
    torch.cuda.synchronize()
    B.profile_enable(False)
    kern = B.profile_read()
    ms_ev = a.elapsed_time(b) / steps
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        B.density(dp, x, occ, out=rho)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    cb = 16
    n1, n2, n3 = prob.fft
    N = n1 * n2 * n3
    model_b, _, f_disk, f_slab = local_model_bytes(prob)
    npw = int(prob.npw[0])
    model = nb * (cb * N * 2 * (f_disk + f_slab) + cb * npw) + 8 * N
    m1 = prob.miller[:, 0]
    S = (int(m1.max()) - int(m1.min()) + 1) * n2 * n3
    rows = {}
    for name, (n, tot) in kern.items():
        rows[name] = {"launches_per_call": n / steps, "avg_ms": tot / n}
    res = {"ms_per_call": ms, "ms_per_call_with_kernel_events": ms_ev, "band_densities_per_s": nb / (ms * 1e-3),
           "model_bytes": model, "effective_GBs": model / (ms * 1e-3) / 1e9,
           "frac_effective": model / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "kernels": rows}
    if "density_x" in rows:
        r = rows["density_x"]
        bands = nb / r["launches_per_call"]
        by = bands * cb * S + 2 * 8 * 8 * N
        r["alg_bytes"] = by
        r["gbs"] = by / (r["avg_ms"] * 1e-3) / 1e9
    return res


def c4_times(B, W, dev, davidson=True):
    """The mixed-precision workload (C4: cubic a=30 bohr, ecutwfc=50 Ry, 128^3, 161,235 PW,
    256 atoms x 9 projectors (s+p+d, full D blocks), 1024 bands): one H psi in FP64, FP32,
    MIXED_FP32 (FP32 transforms and GEMMs, complex128 psi) and MIXED_BF16 (FP32 transforms,
    bf16 projector GEMMs with FP32 accumulation). GEMM rates count 8 nproj nb npw flops per
    product (counted) and the flops the MFMA pipe executes (6 for the 3M FP64 / FP32 products,
    8 for bf16), the fraction taken on the executed flops against the peak of the product's own
    precision; errors are relative max-norm against the FP64 result of the same GPU run (the
    bounds against the oracle at this size are in the GPU tests)."""
    import torch
    prob = W.make_problem("C4")
    B.set_tuning()
    dp = B.DeviceProblem(prob, device=dev, static=True)
    x = torch.from_numpy(prob.psi).to(dev)
    nb, npw = prob.nb, int(prob.npw[0])
    flops = 8.0 * prob.nproj * nb * npw
    res = {"workload": "C4: cubic a=30 bohr, ecutwfc=50 Ry, 128^3, 161235 PW, Gamma, 256 atoms x 9 projectors, "
                       "1024 bands"}
    ref = None
    steps = 3
    for name, prec in (("fp64", B.FP64), ("fp32", B.FP32), ("mixed_fp32", B.MIXED_FP32), ("mixed_bf16", B.MIXED_BF16)):
        xx = x.to(torch.complex64) if prec == B.FP32 else x
        y = torch.empty_like(xx)
        B.apply_h(dp, xx, prec, out=y)
        torch.cuda.synchronize()
        B.profile_read()
        B.profile_enable(True)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            B.apply_h(dp, xx, prec, out=y)
        b.record()
        torch.cuda.synchronize()
        B.profile_enable(False)
        kern = B.profile_read()
        ms = a.elapsed_time(b) / steps
        row = {"ms_per_h_psi": ms, "band_applies_per_s": nb / (ms * 1e-3)}
        for kn, (n, tot) in kern.items():
            if kn.startswith("gemm_") and "reduce" not in kn:
                avg = tot / n
                bf = kn.endswith("bf16")
                pk = BF16_PEAK_TFLOPS if bf else (FP64_PEAK_TFLOPS if prec == B.FP64 else FP32_PEAK_TFLOPS)
                tf = flops / (avg * 1e-3) / 1e12
                # executed: the FP64 / FP32 kernels form complex products with three real
                # MFMA products (3M, 6 M N K flops); the bf16 kernel with four (8 M N K)
                tx = tf * (1.0 if bf else 0.75)
                row[kn] = {"ms": avg, "tflops_counted": tf, "tflops_executed": tx, "peak": pk, "frac": tx / pk,
                           "frac_counted": tf / pk}
        yc = y.to(torch.complex128)
        if ref is None:
            ref = yc
            res["fp64_max_abs"] = float(ref.abs().max())
        else:
            row["rel_err_vs_fp64"] = float((yc - ref).abs().max() / ref.abs().max())
            row["speedup_vs_fp64"] = res["fp64"]["ms_per_h_psi"] / ms
        res[name] = row
        del y, yc
    del ref
    torch.cuda.synchronize()
    if davidson:
        log("C4 Davidson iterations")
        res["davidson_iterations"] = davidson_iteration_times(B, dev, prob, dp, iters=2)
    return res


def force_times(B, W, dev, prob, dp, x, steps):
    """Nonlocal force on the 64 atoms of the benchmark cell from its 128 bands, FP64: one
    stacking pass over beta, one GEMM [B; (k+G)_x B; (k+G)_y B; (k+G)_z B]^H psi
    (8 (4 nproj) nb npw flops), one reduction per atom."""
    import torch
    occ = torch.from_numpy(W.band_weights(prob, 0)).to(dev)
    for _ in range(2):
        B.force_nl(dp, x, occ)
    torch.cuda.synchronize()
    B.profile_read()
    B.profile_enable(True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        B.force_nl(dp, x, occ)
    b.record()
    torch.cuda.synchronize()
    B.profile_enable(False)
    kern = B.profile_read()
    ms = a.elapsed_time(b) / steps
    npw = int(prob.npw[0])
    flops = 8.0 * 4 * prob.nproj * prob.nb * npw
    rows = {name: {"launches_per_call": n / steps, "avg_ms": tot / n} for name, (n, tot) in kern.items()}
    res = {"ms_per_call_with_kernel_events": ms, "gemm_flops": flops, "kernels": rows}
    if "gemm_cn" in rows:
        res["gemm_tflops"] = flops / (rows["gemm_cn"]["avg_ms"] * 1e-3) / 1e12
        res["gemm_frac_fp64_peak"] = res["gemm_tflops"] / FP64_PEAK_TFLOPS
    return res


def chebyshev_times(B, W, dev, prob, dp, ms_apply):
    """Chebyshev filter f_H^{1/2} (order 100, mu = 0.5 Ry, kT = 1 Ry) on 128 plane-wave
    stochastic orbitals of the benchmark cell, FP64. Spectrum bounds by Weyl's inequality
    (kinetic + local + nonlocal extremes), padded by 0.5 Ry.
    k_cheb_step moves six vectors per element (H T_n, T_n, T_{n-1} and out read, T_{n+1}
    and out written)."""
    import torch
    order, nb = 100, prob.nb
    rec = W.reciprocal(np.asarray(prob.lattice, dtype=float))
    kin = float(np.max(np.sum((prob.miller @ rec + np.asarray(prob.kpts)[0]) ** 2, axis=1)))
    # Weyl: lambda_max(H) <= max |k+G|^2 + max(V, 0) + lambda_max(B D B^H), the last equal to
    # lambda_max(G^1/2 D G^1/2) with G = B^H B the projector Gram matrix
    beta = np.asarray(prob.beta).reshape(prob.nproj, -1)
    gram = beta.conj() @ beta.T
    w, u = np.linalg.eigh(gram)
    gh = (u * np.sqrt(np.clip(w, 0, None))) @ u.conj().T
    dfull = np.zeros((prob.nproj, prob.nproj))
    o = 0
    for a_ in range(prob.natom):
        lo, hi = prob.proj_atom_offset[a_], prob.proj_atom_offset[a_ + 1]
        dfull[lo:hi, lo:hi] = np.asarray(prob.dmat)[o: o + (hi - lo) ** 2].reshape(hi - lo, hi - lo)
        o += (hi - lo) ** 2
    nl_max = float(np.max(np.linalg.eigvalsh(gh @ dfull @ gh)))
    emin = float(np.min(prob.vloc)) + min(0.0, float(np.min(np.linalg.eigvalsh(gh @ dfull @ gh)))) - 0.5
    emax = kin + max(0.0, float(np.max(prob.vloc))) + nl_max + 0.5
    coef = B.fermi_coefficients(order, emin, emax, 0.5, 1.0)
    chi = torch.from_numpy(W.stochastic_orbitals(prob, nb, 0)).to(dev)
    out = torch.empty_like(chi)
    B.chebyshev(dp, chi, coef, emin, emax, out=out)
    torch.cuda.synchronize()
    steps = 3
    B.profile_read()
    B.profile_enable(True)
    a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        B.chebyshev(dp, chi, coef, emin, emax, out=out)
    b2.record()
    torch.cuda.synchronize()
    B.profile_enable(False)
    kern = B.profile_read()
    ms_ev = a.elapsed_time(b2) / steps
    a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        B.chebyshev(dp, chi, coef, emin, emax, out=out)
    b2.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b2) / steps
    n = nb * int(np.sum(prob.npw))
    res = {"order": order, "orbitals": nb, "emin": emin, "emax": emax, "ms_per_call": ms,
           "ms_per_call_with_kernel_events": ms_ev, "filtered_orbitals_per_s": nb / (ms * 1e-3),
           "h_band_applies_per_s_inside": order * nb / (ms * 1e-3),
           "overhead_vs_plain_apply": ms / (order * ms_apply)}
    if "cheb_step" in kern:
        cnt, tot = kern["cheb_step"]
        avg = tot / cnt
        res["cheb_step"] = {"launches_per_call": cnt / steps, "avg_ms": avg, "alg_bytes": 6 * 16 * n,
                            "gbs": 6 * 16 * n / (avg * 1e-3) / 1e9}
    return res


def backward_times(B, W, dev, steps):
    """Adjoint of H psi on the differentiation workload (C5: 96^3, k = G, X, M, R, 256 bands
    each, 128 atoms x 4 projectors, complex128): grad_psi = H dY, grad_V from recomputed
    grids, grad_D from two projections, FP64. k_gradv_x reads the psi and dY slab planes
    (2 nb cb S per call) plus its partial grids (G = 8 of N doubles, read and written once
    per band batch)."""
    import torch
    prob = W.make_problem("C5")
    nb, nk = prob.nb, prob.nk
    B.set_tuning()
    dp = B.DeviceProblem(prob, device=dev, static=True)
    x = torch.from_numpy(prob.psi).to(dev)
    dy = torch.from_numpy(prob.dy).to(dev)
    for _ in range(2):
        B.apply_h_backward(dp, x, dy)
    torch.cuda.synchronize()

    def timed():
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            B.apply_h_backward(dp, x, dy)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    B.profile_read()
    B.profile_enable(True)
    ms_ev = timed()
    B.profile_enable(False)
    kern = B.profile_read()
    ms = timed()
    cb, (n1, n2, n3) = 16, prob.fft
    N = n1 * n2 * n3
    m1 = prob.miller[:, 0]
    S = (int(m1.max()) - int(m1.min()) + 1) * n2 * n3
    rows = {name: {"launches_per_call": n / steps, "avg_ms": tot / n} for name, (n, tot) in kern.items()}
    res = {"workload": "C5: cubic a=24 bohr, ecutwfc=35 Ry, 96^3, k = G, X, M, R (npw " +
                       "/".join(str(int(n)) for n in prob.npw) + "), 256 bands each, 128 atoms x 4 projectors",
           "ms_per_call": ms, "ms_per_call_with_kernel_events": ms_ev,
           "band_adjoints_per_s": nk * nb / (ms * 1e-3), "kernels": rows}
    if "gradv_x" in rows:
        r = rows["gradv_x"]
        bands = nk * nb / r["launches_per_call"]
        r["alg_bytes"] = 2 * bands * cb * S + 2 * 8 * 8 * N
        r["gbs"] = r["alg_bytes"] / (r["avg_ms"] * 1e-3) / 1e9
    return res


def batched_times(B, W, dev, steps, workload="C3", prob=None, dp=None, x=None):
    """H psi over uneven k-points: C3 (the {0,1/2}^3 grid, eight spheres of 115,096 - 115,396 PW;
    120^3; 512 bands each; 864 projectors) or C5 (Gamma, X, M, R; 96^3; 256 bands each; 512
    projectors).

    Plain FP64 with one call per k-point, against every k-point in one call
    (one launch per pass per band batch), that call replayed from a HIP graph,
    and the complex64 (FP32), MIXED_FP32 and MIXED_BF16 forms of the replayed
    call, each with its relative max-norm difference from the FP64 result of the
    same GPU (context: the bounds against the oracle are in the GPU tests).
    Rates are band-applies per second over all k-points.
    """
    import torch
    if prob is None:
        prob = W.make_problem(workload)
        B.set_tuning()
        dp = B.DeviceProblem(prob, device=dev, static=True)
        x = torch.from_numpy(prob.psi).to(dev)
    nb, nk = prob.nb, prob.nk
    off = prob.pw_offsets
    subs = []
    for k in range(nk):
        sub = prob.single_k(k)
        beta_k = dp.beta[prob.nproj * off[k]: prob.nproj * off[k + 1]]
        dk = B.DeviceProblem(sub, device=dev, vloc=dp.vloc, dmat=dp.dmat, beta=beta_k, static=True)
        subs.append((dk, x[nb * off[k]: nb * off[k + 1]], torch.empty(nb * (off[k + 1] - off[k]),
                                                                        dtype=x.dtype, device=dev)))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        return timed_calls(fn, steps)

    desc = {"C5": "C5: cubic a=24 bohr, ecutwfc=35 Ry, 96^3, k = G, X, M, R", "C3": "C3: cubic a=30 bohr, "
            "ecutwfc=40 Ry, 120^3, k on the {0,1/2}^3 grid"}[prob.name or workload]
    res = {"workload": desc + " (npw " + "/".join(str(int(n)) for n in prob.npw) + f"), {nb} bands each, "
                       f"{prob.natom} atoms x {prob.nproj // prob.natom} projectors"}
    t_perk = timed(lambda: [B.apply_h(dk, xk, out=yk) for dk, xk, yk in subs])
    del subs
    y = torch.empty_like(x)
    t_batch = timed(lambda: B.apply_h(dp, x, out=y))
    ref = y.clone()
    out = {}
    for name, prec in (("fp64", B.FP64), ("fp32", B.FP32), ("mixed_fp32", B.MIXED_FP32), ("mixed_bf16", B.MIXED_BF16)):
        xx = x.to(torch.complex64) if prec == B.FP32 else x
        yy = torch.empty_like(xx)
        B.apply_h(dp, xx, prec, out=yy)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            B.apply_h(dp, xx, prec, out=yy)
        ms = timed(g.replay)
        err = float(((yy.to(torch.complex128) - ref).abs().max() / ref.abs().max()).item())
        out[name] = (ms, err)
        del g, yy, xx
    tot = nk * nb
    res["fp64_per_kpoint_calls"] = {"ms": t_perk, "band_applies_per_s": tot / (t_perk * 1e-3)}
    res["fp64_batched"] = {"ms": t_batch, "band_applies_per_s": tot / (t_batch * 1e-3),
                           "speedup_vs_per_kpoint": t_perk / t_batch}
    for name, (ms, err) in out.items():
        res[name + "_batched_graph"] = {"ms": ms, "band_applies_per_s": tot / (ms * 1e-3),
                                        "speedup_vs_fp64_per_kpoint": t_perk / ms,
                                        "speedup_vs_fp64_graph": out["fp64"][0] / ms,
                                        "rel_diff_vs_fp64_gpu": err}
    del y, ref
    return res


def cg_times(B, W, dev, dav):
    """Band-by-band preconditioned CG on the benchmark workload to the same 1e-8
    residual, FP64, beside the Davidson time of the same run."""
    import torch
    prob = W.make_problem("C2")
    dp = B.DeviceProblem(prob, device=dev)
    x = torch.from_numpy(prob.psi).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eig, r, its, st = B.cg(dp, x, tol=1e-8, max_iter=400)
    dt = time.perf_counter() - t0
    res = {"s_per_kpoint": dt / prob.nk, "steps_per_band_mean": float(its.mean()), "steps_per_band_max": int(its.max()),
           "max_resid": float(r.max()), "converged": st == 0, "lowest": float(eig.min())}
    if dav and "fp64" in dav and "s_per_kpoint" in dav["fp64"]:
        res["davidson_speedup_over_cg"] = dt / prob.nk / dav["fp64"]["s_per_kpoint"]
    return res


def davidson_times(B, W, dev, workload="C2", tol=1e-8, max_iter=200,
                   modes=(("fp64", 0), ("mixed_fp32", 3), ("mixed_bf16", 2))):
    """Block Davidson to a `tol` residual: FP64, and the mixed modes (reduced-precision
    phase with FP32 or bf16 products, then FP64 refinement); eigenvalue differences of
    each mixed run from the FP64 run of the same GPU (the FP64 Davidson itself is checked
    against the oracle in the GPU tests)."""
    import torch
    res = {"workload": workload, "tol": tol}
    prob = W.make_problem(workload)
    dp = B.DeviceProblem(prob, device=dev, static=True)
    x = torch.from_numpy(prob.psi).to(dev)
    B.apply_h(dp, x)   # plan and work space built outside the timed solves
    torch.cuda.synchronize()
    eigs = {}
    for name, prec in modes:
        x = torch.from_numpy(prob.psi).to(dev)
        torch.cuda.synchronize()
        log(f"Davidson {workload} {name}")
        t0 = time.perf_counter()
        try:
            eig, r, its, st = B.davidson(dp, x, tol=tol, max_iter=max_iter, precision=prec)
        except B.AbacusPwError as e:
            res[name] = {"error": str(e)}
            continue
        dt = time.perf_counter() - t0
        res[name] = {"s_per_kpoint": dt / prob.nk, "iterations": [int(v) for v in its], "max_resid": float(r.max()),
                     "converged": st == 0, "lowest": float(eig.min()), "highest": float(eig.max())}
        eigs[name] = eig
    if "fp64" in eigs:
        for name in eigs:
            if name != "fp64":
                res[name]["max_eig_diff_vs_fp64"] = float(np.max(np.abs(eigs[name] - eigs["fp64"])))
                res[name]["speedup_vs_fp64"] = res["fp64"]["s_per_kpoint"] / res[name]["s_per_kpoint"]
    del dp, x
    B.plan_reset()
    return res


def davidson_iteration_times(B, dev, prob, dp, iters=3):
    """Seconds per Davidson iteration on a large workload, FP64 and MIXED_BF16: the solve is
    run with max_iter = 0 (Cholesky-QR, H psi and Rayleigh-Ritz of the start) and with
    max_iter = iters (tol 1e-30, so exactly that many correction steps), and the difference
    is divided by iters * nk."""
    import torch
    out = {"iterations": iters}
    for name, prec in (("fp64", B.FP64), ("mixed_bf16", B.MIXED_BF16)):
        t = []
        for n in (0, iters):
            x = torch.from_numpy(prob.psi).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.davidson(dp, x, tol=1e-30, max_iter=n, precision=prec)
            t.append(time.perf_counter() - t0)
            del x
        out[name] = {"s_per_iteration_per_kpoint": (t[1] - t[0]) / (iters * prob.nk),
                     "s_start_per_kpoint": t[0] / prob.nk}
        log(f"Davidson iterations {name}: {out[name]}")
    # the subspace products of the FP64 iterations (projections, orthogonalisation, Ritz
    # updates, Cholesky-QR and Rayleigh-Ritz GEMMs, "subspace:" records of the library's
    # profile with their counted flops), from two profiled solves differenced like the times
    recs = []
    for n in (0, iters):
        x = torch.from_numpy(prob.psi).to(dev)
        B.profile_read()
        B.profile_enable(True)
        B.davidson(dp, x, tol=1e-30, max_iter=n, precision=B.FP64)
        B.profile_enable(False)
        recs.append(B.profile_read(flops=True))
        del x
    per = float(iters * prob.nk)
    sub = {}
    for lab in sorted(set(recs[0]) | set(recs[1])):
        a, b_ = recs[0].get(lab, (0, 0.0, 0.0)), recs[1].get(lab, (0, 0.0, 0.0))
        ms, fl = (b_[1] - a[1]) / per, (b_[2] - a[2]) / per
        sub[lab] = {"ms_per_iteration_per_kpoint": ms}
        if fl > 0 and ms > 0:
            tf = fl / (ms * 1e-3) / 1e12
            sub[lab].update({"tflops_counted": tf, "tflops_executed": 0.75 * tf, "frac_executed_fp64": 0.75 * tf / 78.6})
    gemm = [sub[k] for k in ("subspace:gemm_cn", "subspace:gemm_nn") if k in sub and "tflops_counted" in sub[k]]
    if gemm:
        tot_ms = sum(g["ms_per_iteration_per_kpoint"] for g in gemm)
        tot_tf = sum(g["tflops_counted"] * g["ms_per_iteration_per_kpoint"] for g in gemm) / tot_ms
        out["fp64_subspace_gemm"] = {"ms_per_iteration_per_kpoint": tot_ms, "tflops_counted": tot_tf,
                                     "tflops_executed": 0.75 * tot_tf, "frac_executed_fp64": 0.75 * tot_tf / 78.6}
    out["fp64_profile_per_iteration"] = sub
    return out

if __name__ == "__main__":
    main()
