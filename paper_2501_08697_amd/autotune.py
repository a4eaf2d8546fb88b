"""Autotuner for the H psi kernels' launch shapes.

Searches the library's tuning knobs (abacus_pw_set_tuning) for one problem and
precision by coordinate descent: starting from the defaults, each knob in turn
is swept over its candidate values with the others fixed, keeping the fastest;
two sweeps. Each candidate is timed with HIP events as the best of three
repetitions of `reps` H psi calls, after one warm-up call. The winner is cached in a JSON file keyed by the
problem's shape (grid, sphere sizes, projectors, bands, precision); the cache
path is ABACUS_PW_AUTOTUNE_CACHE or ~/.cache/abacus_pw/autotune.json.

The knobs change launch shapes, work-group band counts and whether the
projector GEMMs run on a second stream beside the local term; the split-K
chunk changes the grouping of the projection sums, so results move at the
rounding level (checked by the GPU tests).
"""
from __future__ import annotations

import json
import os

from . import binding as B

CANDIDATES = {
    "yz_mode": [1, 2],
    "band_batch": [32, 64, 128],
    "yz_bands": [1, 2, 4],
    "x_bands": [2, 4, 8],
    "splitk_chunk": [256, 512, 1024],
    "overlap": [1, 2],
    "yz_threads": [256, 512, 1024],
}
DEFAULT = {"band_batch": 0, "splitk_chunk": 0, "yz_bands": 0, "x_bands": 0, "yz_mode": 0, "overlap": 0,
           "yz_threads": 0}


def cache_path() -> str:
    return os.environ.get("ABACUS_PW_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "abacus_pw", "autotune.json"))


def key(dp: B.DeviceProblem, nb: int, precision: int) -> str:
    return f"fft={dp.fft};npw={list(map(int, dp.npw))};nproj={dp.nproj};nb={nb};prec={precision}"


def _apply(cfg):
    B.set_tuning(cfg["band_batch"], cfg["splitk_chunk"], cfg["yz_bands"], cfg["x_bands"], cfg.get("yz_mode", 0),
                 cfg.get("overlap", 0), cfg.get("yz_threads", 0))


def _time(dp, x, y, nb, precision, reps, trials=3):
    """Best over `trials` of the mean time of `reps` calls (the minimum filters out
    interference, so that near-equal candidates are not ranked by noise)."""
    import torch
    B.apply_h(dp, x, precision, nb=nb, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(trials):
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            B.apply_h(dp, x, precision, nb=nb, out=y)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / reps)
    return best


def tune(dp: B.DeviceProblem, x, nb: int | None = None, precision: int = B.FP64, reps: int = 10,
         use_cache: bool = True, sweeps: int = 2, log=None, trials: int = 3):
    """Returns (best config dict, best ms per H psi) and leaves the library set to it."""
    import torch
    nb = dp.prob.nb if nb is None else nb
    k = key(dp, nb, precision)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and k in cache:
        cfg = cache[k]["config"]
        _apply(cfg)
        return cfg, cache[k]["ms"]
    y = torch.empty_like(x)
    best = dict(DEFAULT)
    _apply(best)
    best_ms = _time(dp, x, y, nb, precision, reps, trials)
    for _ in range(sweeps):
        for name, values in CANDIDATES.items():
            for v in values:
                cand = dict(best)
                cand[name] = v
                _apply(cand)
                ms = _time(dp, x, y, nb, precision, reps, trials)
                if log:
                    log(f"autotune {cand} {ms:.4f} ms")
                if ms < best_ms:
                    best, best_ms = cand, ms
    _apply(best)
    if use_cache:
        cache[k] = {"config": best, "ms": best_ms}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best, best_ms
