"""Execution-option autotuner for the kappa-cycle library.

The library's results do not depend on its execution options (every kernel
variant rounds each operation the same way), so the options can be chosen by
measurement alone: for a hierarchy, a cycle (kappa, nu1, nu2) and a driver,
each candidate runs a fixed number of iterations and the fastest is kept.  The
search is coordinate descent over two groups of options, each searched with
the best of the other fixed: the shapes of the fused grid kernels (the
largest level sizes run in 8 x 8, 16 x 16 and 32 x 32 tiles, the smallest
level size streamed through registers), then the persistent-kernel options (coarse cutover,
threads, single-wave level size), then the grid shapes again (the best
cutover depends on how cheap the grid launches below it are).  The last group
re-tries only the few fastest grid shapes of the first.  Results are
cached per (device, instance sizes, precision, driver, kappa, nu1, nu2) in
memory and, when KC_AUTOTUNE_CACHE names a file, in that JSON file.
"""
from __future__ import annotations

import json
import os
import time

from . import kcycle

COARSE_CANDIDATES = tuple(
    dict(coarse_cutover=c, coarse_threads=t, coarse_wave_n=w)
    for c in (15, 31, 63) for t in (256, 512, 1024) for w in (7, 15)
    if not (c == 63 and t == 256)       # 63 rows need at least 8 waves
)   # 1024 threads: FP32 cycles only (set_exec rejects it otherwise and the candidate is skipped)
TILE_CANDIDATES = tuple(dict(tiny_tile_n=y, small_tile_n=s, mid_tile_n=t, stream_n=m) for y in (0, 63, 127, 255, 511)
                        for s in (0, 127, 255, 511, 1023) for t in (0, 1023, 2047, 4095) for m in (0, 1023, 2047, 4095))
# the third stage re-tries only the RETRY fastest tile shapes of the first under the chosen persistent-kernel options
RETRY = 4
DEFAULT_STAGES = (tuple(dict(coarse_cutover=31, coarse_threads=512, coarse_wave_n=15, **t) for t in TILE_CANDIDATES),
                  COARSE_CANDIDATES, "retry")


def _shapes(cand: dict, sizes) -> tuple:
    """Kernel shape of every level above the coarse cutover of a hierarchy with
    the given fine sizes (largest n per depth), as the library picks it: two
    candidates with the same shapes give the same schedule."""
    cut = cand.get("coarse_cutover", 31)
    small, mid, stream = cand.get("small_tile_n", 511), cand.get("mid_tile_n", 2047), cand.get("stream_n", 2047)
    tiny = cand.get("tiny_tile_n", 0)
    out = []
    n = max(sizes)
    while n > cut:
        if stream > 0 and n >= stream:
            out.append("stream")
        elif n <= tiny:
            out.append("8")
        elif n <= small:
            out.append("16")
        elif n <= mid:
            out.append("32")
        else:
            out.append("64x32")
        n = (n - 1) // 2
    return tuple(out)


def _relevant(cand: dict, seen: set, sizes) -> bool:
    """Skip a candidate whose per-level kernel shapes (and persistent-kernel
    options) equal those of one already tried."""
    key = (_shapes(cand, sizes), cand.get("coarse_cutover", 31), cand.get("coarse_threads", 512),
           cand.get("coarse_wave_n", 15))
    if key in seen:
        return False
    seen.add(key)
    return True

_memory: dict = {}


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _key(H, driver, kappa, nu1, nu2) -> str:
    return json.dumps([_device_name(), H.sizes, H.precision, driver, int(kappa), int(nu1), int(nu2)])


def _load_file() -> dict:
    path = os.environ.get("KC_AUTOTUNE_CACHE")
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_file(key: str, value: dict) -> None:
    path = os.environ.get("KC_AUTOTUNE_CACHE")
    if not path:
        return
    data = _load_file()
    data[key] = value
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1)
    os.replace(tmp, path)


def tune(H: "kcycle.Hierarchy", u, f, kappa: int, nu1: int = 2, nu2: int = 2, omega: float = 0.8,
         driver: str = "solve", iters: int = 12, stages=DEFAULT_STAGES, force: bool = False) -> dict:
    """Pick the fastest execution options for `driver` ("solve" or "pcg") on
    hierarchy H, apply them to H and return {"exec": ..., "ms_per_iter": ...,
    "trials": [...]}; u is used as scratch (zeroed before every trial)."""
    key = _key(H, driver, kappa, nu1, nu2)
    if not force:
        hit = _memory.get(key) or _load_file().get(key)
        if hit:
            H.set_exec(**hit["exec"])
            _memory[key] = hit
            return hit
    run = H.solve if driver == "solve" else H.pcg
    us = u if isinstance(u, (list, tuple)) else [u]
    trials = []
    seen: set = set()
    best = None
    tile_keys = ("tiny_tile_n", "small_tile_n", "mid_tile_n", "stream_n")
    for si, stage in enumerate(stages):
        base = dict(best["exec"]) if best else {}
        if stage == "retry":   # the fastest tile shapes of the first stage, under the current options
            first = sorted((t for t in trials if t.get("stage") == 0), key=lambda r: r["ms_per_iter"])[:RETRY]
            stage = tuple({k: t["exec"][k] for k in tile_keys if k in t["exec"]} for t in first)
        for part in stage:
            cand = dict(base, **part)
            if not _relevant(cand, seen, H.sizes):
                continue
            try:
                H.set_exec(**dict(cand, poll_every=iters + 2))
            except kcycle.KCycleError:
                continue                      # e.g. the levels do not fit the LDS
            for x in us:
                x.zero_()
            run(u, f, kappa=kappa, nu1=nu1, nu2=nu2, omega=omega, tol=0.0, maxit=2)   # capture
            for x in us:
                x.zero_()
            t0 = time.perf_counter()
            run(u, f, kappa=kappa, nu1=nu1, nu2=nu2, omega=omega, tol=0.0, maxit=iters)
            wall = time.perf_counter() - t0
            dev_ms = H.stats()["last_ms"]
            trials.append({"exec": cand, "ms_per_iter": dev_ms / (iters + 1), "wall_ms": wall * 1e3, "stage": si})
        if not trials:
            raise RuntimeError("no execution candidate is valid for this hierarchy")
        best = min(trials, key=lambda r: r["ms_per_iter"])
    H.set_exec(**best["exec"])
    for x in us:
        x.zero_()
    result = {"exec": best["exec"], "ms_per_iter": best["ms_per_iter"], "trials": trials}
    _memory[key] = result
    _store_file(key, result)
    return result
