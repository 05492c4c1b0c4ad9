"""Fit the run-time model of Section 3 on this GPU and report the quantities
of Tables 1 and 2 for it.

For each execution mode ("paper": one kernel per operation of Algorithm 4;
"fused": the library's default schedule) and each kappa in {1, 2, 3, 4, W},
n = 4..13 levels (N = (2^n - 1)^2), it times back-to-back cycles, then solves
the least-squares problem for (alpha, beta) in T = alpha * N_calls +
beta * N_ops, with N_ops = N * 2(1 - 3^-kappa) and N_calls the serialised
steps per cycle of that mode: grid launches plus persistent-kernel stages
(for "paper" exactly the paper's (5+nu) totalCalls(n-1) + totalCalls(n) -
totalCalls(n-1) launches).  As the paper cautions (Section 3.5), the work
term's cost depends on where the data live: the fit is made over all sizes
and separately for hierarchies inside the 256 MB Infinity Cache (up to 11
levels in FP64) and beyond it.  Prints one JSON object.

Usage: python -m paper_2010_00626_amd.fit_model [--nmax 13] [--modes paper,fused]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import kcycle, model


def measure(mode: str, kappa: int, n_levels: int, nu: int = 2, theta: float = math.pi / 4, eps: float = 1e-4,
            budget_ms: float = 60.0):
    import torch
    n = 2 ** n_levels - 1
    H = kcycle.Hierarchy([(n, theta, eps)], "f64", exec=dict(mode=mode))
    rng = np.random.default_rng(n_levels)
    f = torch.from_numpy(rng.uniform(-1, 1, (n, n))).to("cuda")
    v = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ms1 = H.time_cycles(v, f, kappa=kappa, nu1=nu // 2, nu2=nu - nu // 2, reps=1)
    reps = int(max(3, min(200, budget_ms / max(ms1, 1e-3))))
    ms = H.time_cycles(v, f, kappa=kappa, nu1=nu // 2, nu2=nu - nu // 2, reps=reps)
    st = H.stats()
    H.close()
    return ms, st["grid_launches_per_iteration"], st["subtree_stages_per_iteration"], reps


def n_calls(grid_launches: int, persistent_stages: int) -> int:
    """N_gpuCalls of a schedule: every grid launch and every stage (pre, post or
    coarsest-solve operation) of the persistent kernel is one serialised step;
    in the one-kernel-per-operation mode there are no persistent stages and
    this is the paper's launch count."""
    return grid_launches + persistent_stages


CACHE_LEVELS = 11   # FP64 hierarchies up to 2047^2 (about 134 MB) stay in the 256 MB Infinity Cache


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nmin", type=int, default=4)
    ap.add_argument("--nmax", type=int, default=13)
    ap.add_argument("--modes", default="paper,fused")
    ap.add_argument("--nu", type=int, default=4)
    ap.add_argument("--from-json", default="", help="refit the measurements of an earlier run's output (no GPU)")
    args = ap.parse_args(argv)
    kappas = [1, 2, 3, 4, kcycle.KAPPA_W]
    stored = None
    if args.from_json:
        with open(args.from_json) as fh:
            stored = json.load(fh)
    out = {"units": "alpha in us per call, beta in ns per operation unit", "nu": args.nu,
           "calls": "grid launches + persistent-kernel stages (the paper's launch count in the paper mode)",
           "regimes": {"cache": f"n <= {CACHE_LEVELS} levels (FP64 hierarchy inside the 256 MB Infinity Cache)",
                       "hbm": f"n > {CACHE_LEVELS} levels"}, "modes": {}}
    for mode in args.modes.split(","):
        rows, table = [], {}
        for k in kappas:
            key = "W" if k == kcycle.KAPPA_W else str(k)
            for nl in range(args.nmin, args.nmax + 1):
                t0 = time.perf_counter()
                if stored is not None:
                    m = stored["modes"][mode]["measurements"][f"{key},{nl}"]
                    ms, calls, stages, reps = m["ms"], m["calls"], m["persistent_stages"], m["reps"]
                    grid = calls - stages
                else:
                    ms, grid, stages, reps = measure(mode, k, nl, args.nu)
                calls = n_calls(grid, stages)
                if mode == "paper":
                    expect = model.n_gpu_calls_paper(k, nl, args.nu) + (args.nu % 2)
                    assert calls == expect, (calls, expect)
                ops = model.n_ops_2d(k, nl)
                rows.append(((key, nl), calls, ops, ms))
                table[f"{key},{nl}"] = {"ms": ms, "calls": calls, "persistent_stages": stages, "reps": reps}
                print(f"[fit] {mode} kappa={key} n={nl}: {ms:.4f} ms/cycle, {calls} calls "
                      f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
        res = {"measurements": table}
        for regime, sel in (("all", lambda nl: True), ("cache", lambda nl: nl <= CACHE_LEVELS),
                            ("hbm", lambda nl: nl > CACHE_LEVELS)):
            sub = [r for r in rows if sel(r[0][1])]
            if len(sub) < 3:
                continue
            for rel in (False, True):
                fit = model.fit(sub, relative=rel)
                errs = {f"{k[0]},{k[1]}": round(100.0 * e, 2) for k, e in fit.rel_errors.items() if k[1] >= 8}
                tps = {}
                if mode == "paper" and fit.alpha > 0 and fit.beta > 0:
                    for k in (1, 2, 3, 4, math.inf):
                        ntp = model.paper_turning_point(fit.alpha, fit.beta, k, 5 + args.nu)
                        tps["W" if math.isinf(k) else str(k)] = {"n_tp": round(ntp, 2),
                                                                 "N_tp": round((2 ** ntp - 1) ** 2)}
                res[regime + ("_relative" if rel else "")] = {
                    "alpha_us": fit.alpha * 1e3, "beta_ns": fit.beta * 1e6,
                    "alpha_over_beta": fit.alpha / fit.beta if fit.beta else None,
                    "rel_errors_percent_n8plus": errs,
                    "max_abs_err_percent_n8plus": max((abs(v) for v in errs.values()), default=None),
                    "turning_points": tps}
        out["modes"][mode] = res
    print(json.dumps(out))


if __name__ == "__main__":
    main()
