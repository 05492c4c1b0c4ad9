"""The paper's own solve protocol on this GPU (Section 4): f = 0, a random
initial guess, and the number of cycles (stand-alone) or CG iterations (MGCG)
until the L2 norm of the error has dropped by 1e8; FP64 throughout.

* Tables 3 and 4: 12 levels (4095^2), 45 degrees, eps = 1e-4, damped Jacobi
  (omega 0.8), nu = 2 + 2, kappa in {1, 2, 3, 4, W}.
* The solve-time figure: eps in {1e-5, ..., 1} at 9 and 13 levels, stand-alone.
* Tables 5 and 6 (alternating zebra line relaxation, Galerkin coarsening,
  one relaxation per direction before and after the coarse correction):
  eps = 1e-5 and angles 10, 30, 45, 60, 80 degrees, stand-alone and MGCG, at a
  chosen number of levels (the paper uses 14).
* Tables 7 and 8 (x-line zebra relaxation, two relaxations before and after
  the coarse correction, coarsening along y only, Galerkin operators): the
  same angles and eps, stand-alone and MGCG, at a chosen number of levels.

Stand-alone: with f = 0 the exact solution is 0, so the error after k cycles
is v_k itself.  Cycles run in chunks (one graph launch of `chunk` cycles, timed
with HIP events); when a chunk crosses the target, the iterate saved at its
start is stepped one cycle at a time to find the first k (the library's cycles
are deterministic, so the replay gives the same iterates).

MGCG: the library's CG starts from u = 0.  Running it on b = A v0 gives
iterates w_k whose error w_k - v0 is, in exact arithmetic, the negative of the
error of CG started at v0 with f = 0; k is found by bisection on the iteration
limit (error norms are checked on the device result of each run).

Times: stand-alone total = cycles x (median device time per cycle of the
chunks); MGCG total = wall time of one run of exactly k iterations (setup and
host polling included, as the paper's totals include theirs).

Timing only (`--solvers timing`): the device time per cycle (three back-to-back
cycles) and the wall time of CG runs of 2 and 6 iterations, without solving.
With `--counts FILE` (the JSON lines of an earlier full run of the same
tables) the totals are rebuilt from its counts: cycles x time per cycle, and
the 2-iteration run plus (iterations - 2) x time per iteration.  Iterates, and
so the counts, do not depend on the execution options, which only change the
time.

Usage: python -m paper_2010_00626_amd.protocol [--tables] [--sweep 9,13] [--zebra-levels 12] [--zebra-exec JSON]
       [--semi-levels 12] [--angles 10,30,45,60,80] [--solvers standalone,mgcg,timing] [--maxc 40000]
       [--counts FILE]
Prints one JSON object per result line and a summary object at the end.
"""
from __future__ import annotations

import argparse
import json
import math
import statistics
import sys
import time

import numpy as np

from . import inputs, kcycle

TARGET = 1e-8
KAPPAS = (1, 2, 3, 4, kcycle.KAPPA_W)


def _key(k: int) -> str:
    return "W" if k == kcycle.KAPPA_W else str(k)


def standalone(H, v0, kappa: int, nu: int = 2, omega: float = 0.8, chunk: int = 32, maxc: int = 40000,
               smoother: str = "jacobi") -> dict:
    import torch
    f = torch.zeros_like(v0)
    v = v0.clone()
    e0 = float(torch.linalg.vector_norm(v0))
    done, per_cycle = 0, []
    while done < maxc:
        start = v.clone()
        ms = H.time_cycles(v, f, kappa=kappa, nu1=nu, nu2=nu, omega=omega, reps=chunk - 1,
                           smoother=smoother)   # chunk cycles in all
        per_cycle.append(ms)
        err = float(torch.linalg.vector_norm(v)) / e0
        if (done // chunk) % 16 == 0:   # progress of long runs
            print(f"[protocol] kappa={_key(kappa)}: {done + chunk} cycles, error {err:.3e}, {ms:.3f} ms per cycle",
                  file=sys.stderr, flush=True)
        if err < TARGET:
            v.copy_(start)
            for j in range(chunk):
                H.cycle(v, f, kappa=kappa, nu1=nu, nu2=nu, omega=omega, smoother=smoother)
                if float(torch.linalg.vector_norm(v)) / e0 < TARGET:
                    cycles = done + j + 1
                    ms_c = statistics.median(per_cycle)
                    return {"cycles": cycles, "ms_per_cycle": ms_c, "total_ms": cycles * ms_c,
                            "final_error": float(torch.linalg.vector_norm(v)) / e0}
            raise RuntimeError("replay of a chunk did not reproduce its crossing")
        done += chunk
    return {"cycles": None, "cap": maxc, "ms_per_cycle": statistics.median(per_cycle),
            "final_error": float(torch.linalg.vector_norm(v)) / e0}


def mgcg(H, v0, kappa: int, nu: int = 2, omega: float = 0.8, kmax: int = 4000, smoother: str = "jacobi") -> dict:
    import torch
    b = torch.empty_like(v0)
    H.apply_A(b, v0)
    e0 = float(torch.linalg.vector_norm(v0))
    u = torch.zeros_like(v0)
    cache = {}

    def err(k: int) -> float:
        if k not in cache:
            u.zero_()
            H.pcg(u, b, kappa=kappa, nu1=nu, nu2=nu, omega=omega, tol=0.0, maxit=k, smoother=smoother)
            cache[k] = float(torch.linalg.vector_norm(u - v0)) / e0
            print(f"[protocol] mgcg kappa={_key(kappa)}: {k} iterations, error {cache[k]:.3e}", file=sys.stderr,
                  flush=True)
        return cache[k]

    hi = 8
    while err(hi) >= TARGET:
        if hi >= kmax:
            return {"iterations": None, "cap": kmax, "final_error": err(hi)}
        hi = min(2 * hi, kmax)
    lo = 0   # err(0) = 1
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if err(mid) < TARGET:
            hi = mid
        else:
            lo = mid
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, rr, st = H.pcg(u, b, kappa=kappa, nu1=nu, nu2=nu, omega=omega, tol=0.0, maxit=hi, smoother=smoother)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) * 1e3
    return {"iterations": hi, "total_ms": dt, "ms_per_iteration": dt / hi, "final_error": err(hi)}


def timing(H, v0, kappa: int, nu: int = 2, omega: float = 0.8, smoother: str = "jacobi") -> dict:
    import torch
    f = torch.zeros_like(v0)
    v = v0.clone()
    ms_c = H.time_cycles(v, f, kappa=kappa, nu1=nu, nu2=nu, omega=omega, reps=3, smoother=smoother)
    b = torch.empty_like(v0)
    H.apply_A(b, v0)
    u = torch.zeros_like(v0)
    wall = {}
    for m in (2, 6):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.pcg(u, b, kappa=kappa, nu1=nu, nu2=nu, omega=omega, tol=0.0, maxit=m, smoother=smoother)
        torch.cuda.synchronize()
        wall[m] = (time.perf_counter() - t0) * 1e3
    return {"ms_per_cycle": ms_c, "pcg_ms_2": wall[2], "ms_per_iteration": (wall[6] - wall[2]) / 4}


def with_counts(r: dict, counts: list) -> dict:
    """Totals of a timing result from the counts of an earlier full run of the same problem."""
    def same(c):
        return all(c.get(k) == r[k] for k in ("levels", "theta", "eps", "kappa", "smoother", "coarsening"))
    for c in counts:
        if not same(c):
            continue
        if c.get("solver") == "standalone" and c.get("cycles"):
            r["cycles"] = c["cycles"]
            r["standalone_total_ms"] = c["cycles"] * r["ms_per_cycle"]
        elif c.get("solver") == "standalone":
            r["cycles_cap"] = c.get("cap")
        if c.get("solver") == "mgcg" and c.get("iterations"):
            r["iterations"] = c["iterations"]
            r["mgcg_total_ms"] = r["pcg_ms_2"] + (c["iterations"] - 2) * r["ms_per_iteration"]
    return r


def run(levels: int, theta: float, eps: float, kappas, which: str, seed: int, maxc: int,
        smoother: str = "jacobi", exec_opts: dict | None = None, coarsening: str = "full",
        counts: list | None = None) -> list:
    import torch
    n = 2 ** levels - 1
    v0 = torch.from_numpy(inputs.uniform_rhs(np.random.default_rng(seed), n)).to("cuda")
    H = kcycle.Hierarchy([(n, theta, eps)], "f64", exec=exec_opts, coarsening=coarsening)
    out = []
    for k in kappas:
        t0 = time.perf_counter()
        if which == "timing":
            r = timing(H, v0, k, smoother=smoother)
        elif which == "standalone":
            r = standalone(H, v0, k, maxc=maxc, smoother=smoother)
        else:
            r = mgcg(H, v0, k, smoother=smoother)
        r.update({"solver": which, "smoother": smoother, "coarsening": coarsening, "exec": exec_opts or {},
                  "levels": levels, "n": n,
                  "theta": theta, "eps": eps,
                  "kappa": _key(k),
                  "unknowns_per_s": (n * n / (r["total_ms"] * 1e-3)) if r.get("total_ms") else None,
                  "wall_s": round(time.perf_counter() - t0, 2)})
        if which == "timing" and counts:
            with_counts(r, counts)
        print(json.dumps(r), flush=True)
        out.append(r)
    H.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--tables", action="store_true", help="Tables 3 and 4 (12 levels)")
    ap.add_argument("--sweep", default="", help="comma-separated level counts for the eps sweep (e.g. 9,13)")
    ap.add_argument("--eps", default="1e-5,1e-4,1e-3,1e-2,1e-1,1")
    ap.add_argument("--maxc", type=int, default=40000, help="stand-alone cycle cap")
    ap.add_argument("--seed", type=int, default=8)
    ap.add_argument("--zebra-levels", type=int, default=0, help="Tables 5 and 6 (zebra) at this many levels")
    ap.add_argument("--angles", default="10,30,45,60,80", help="degrees, for the zebra tables")
    ap.add_argument("--zebra-kappas", default="1,2,3,4,W")
    ap.add_argument("--zebra-exec", default="{}",
                    help='execution options of the zebra runs as JSON, e.g. \'{"mode": "paper"}\' (default: fused)')
    ap.add_argument("--semi-levels", type=int, default=0,
                    help="Tables 7 and 8 (x-line zebra, coarsening along y) at this many levels")
    ap.add_argument("--solvers", default="standalone,mgcg",
                    help="solvers of the zebra and semi tables (timing: times per cycle and CG iteration only)")
    ap.add_argument("--counts", default="", help="JSON lines of an earlier full run: totals for --solvers timing")
    ap.add_argument("--standalone-kappas", default="", help="kappas of the stand-alone zebra/semi runs (default: --zebra-kappas)")
    ap.add_argument("--mgcg-kappas", default="", help="kappas of the MGCG zebra/semi runs (default: --zebra-kappas)")
    a = ap.parse_args(argv)
    res = {"tables": [], "sweep": [], "zebra": [], "semi": []}
    counts = []
    if a.counts:
        with open(a.counts) as fh:
            counts = [json.loads(line) for line in fh if line.strip() and '"summary"' not in line[:12]]
    if a.tables:
        for which in ("standalone", "mgcg"):
            res["tables"] += run(12, math.pi / 4, 1e-4, KAPPAS, which, a.seed, a.maxc)
    for lv in [int(x) for x in a.sweep.split(",") if x]:
        for e in [float(x) for x in a.eps.split(",")]:
            res["sweep"] += run(lv, math.pi / 4, e, KAPPAS, "standalone", a.seed, a.maxc)
    def kappas_of(which: str) -> list:
        spec = {"standalone": a.standalone_kappas, "mgcg": a.mgcg_kappas}.get(which, "") or a.zebra_kappas
        return [kcycle.KAPPA_W if x == "W" else int(x) for x in spec.split(",")]

    if a.zebra_levels:
        for deg in [float(x) for x in a.angles.split(",")]:
            for which in a.solvers.split(","):
                res["zebra"] += run(a.zebra_levels, math.radians(deg), 1e-5, kappas_of(which), which, a.seed, a.maxc,
                                    "zebra", json.loads(a.zebra_exec), counts=counts)
    if a.semi_levels:
        for deg in [float(x) for x in a.angles.split(",")]:
            for which in a.solvers.split(","):
                res["semi"] += run(a.semi_levels, math.radians(deg), 1e-5, kappas_of(which), which, a.seed, a.maxc,
                                   "zebra", None, "semi", counts=counts)
    print(json.dumps({"summary": res}))


if __name__ == "__main__":
    sys.exit(main())
