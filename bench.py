"""Benchmark: fine-grid unknowns solved per second to a relative residual of
1e-8, per cycle counter kappa, on one MI355X.

Workload (default): 1023 x 1023 interior grid (10 levels to 1 x 1), theta=pi/6,
eps=1e-4, damped Jacobi omega=0.8 with nu1=nu2=2, f i.i.d. U[-1,1] from seed 1,
zero initial guess, stop at ||f - A u|| / ||f|| < 1e-8.  Every kappa in
{1, 2, 3, 4, 6, W} is run with FP64 cycles and with FP32 cycles inside FP64
iterative refinement; the headline `value` is the fastest FP64 configuration
(the paper's arithmetic), timed over `--steps` complete solves (inputs
resident in HBM, setup excluded).  The FP32-cycle results are reported beside
it, and the last key of the line, `summary`, repeats the figures the extras
measure (batched speed-up, PCG true residuals, fine-level bandwidth, the
model's predicted best kappa).

Prints ONE JSON line.  `--gpus N` with N > 1 exits: every run is one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-grid unknowns/s to 1e-8 rel. residual per κ; batched+FP32 vs plain FP64"
HBM_PEAK_GBS = 8000.0
# MI355X vector peak: 256 CUs x 2.4 GHz x 64 lanes x 2 flops (FMA) = 78.6 TFLOP/s in FP64 and, without
# packed issue (the library is compiled with packed FP32 off), in FP32 as well
VECTOR_PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}
CUS = 256


def traffic_of(kernel: str):
    """HBM bytes per launch of `kernel` measured with rocprofv3 counters
    (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size), from the
    committed summary; None when there is none for this kernel or the kernel
    source changed since it was taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "traffic.json")
    src = os.path.join(here, "paper_2010_00626_amd", "csrc", "kc_kernels.hip")
    try:
        with open(path) as fh:
            data = json.load(fh)
        with open(src, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if data.get("kernels_source_sha256") != digest:
        return None
    v = data.get("bytes_per_launch", {}).get(kernel)
    return round(v, 1) if v is not None else None


def kernel_row(k, prec):
    """Roofline entry of one kernel from the library's per-launch profile."""
    avg_s = k["avg_ms"] * 1e-3
    if k["name"].startswith("k_subtree"):
        # one workgroup per instance on one CU: the chip-wide fraction is tiny by construction, so the
        # per-CU fraction (one instance here) is reported beside it
        peak = VECTOR_PEAK_TFLOPS[prec]
        ach = k["flops_per_launch"] / avg_s / 1e12 if avg_s > 0 else 0.0
        return {"bound": "alu", "achieved": round(ach, 4), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 6),
                "frac_of_one_cu": round(ach / (peak / CUS), 4)}
    ach = k["bytes_per_launch"] / avg_s / 1e9 if avg_s > 0 else 0.0
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweep-reps", type=int, default=5, help="timed solves per (kappa, precision) in the sweep (median)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=40, help="oracle cycles timed for the CPU baseline")
    ap.add_argument("--kappa", type=int, default=0, help="force the headline kappa (0 = fastest of the sweep)")
    ap.add_argument("--precision", default="f64", help="headline precision (f64, the paper's arithmetic, or f32)")
    ap.add_argument("--no-model", action="store_true", help="skip the run-time model's calibration sweep")
    ap.add_argument("--no-tune", action="store_true", help="skip the execution-option autotuner")
    ap.add_argument("--exec", default="", help="JSON execution options for the headline configuration "
                    "(instead of the autotuned ones)")
    ap.add_argument("--extras", default="c4,c3,c5,hbm,zebra,convection",
                    help="extra measurements: c4 (batched uneven), c3 (PCG 4095^2), c5 (adjoint), hbm (8191^2 and 16383^2 kernels), "
                         "zebra (the 1023^2 problem with alternating zebra line relaxation), "
                         "convection (1023^2 convection-diffusion per kappa)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (no multi-GPU path is built)"}))
        sys.exit(2)
    import torch
    from paper_2010_00626_amd import autotune, inputs, kcycle, model

    dev = torch.device("cuda:0")
    w = inputs.config2()
    inst = w.instances[0]
    n = inst.n
    N = n * n
    f = torch.from_numpy(inst.f).to(dev)
    probs = [(n, inst.theta, inst.eps, w.n_coarsest)]
    H = {"f64": kcycle.Hierarchy(probs, "f64", device=dev), "f32": kcycle.Hierarchy(probs, "f32", device=dev)}
    u = torch.zeros((n, n), dtype=torch.float64, device=dev)
    kw = dict(nu1=w.nu1, nu2=w.nu2, omega=w.omega, tol=w.tol, maxit=8000)
    levels = len(kcycle.level_stencils(n, inst.theta, inst.eps))

    def solve(prec, kappa):
        u.zero_()
        return H[prec].solve(u, f, kappa=kappa, **kw)

    tuned = {}

    def tune(prec, kappa):
        if args.no_tune:
            return None
        r = autotune.tune(H[prec], u, f, kappa, w.nu1, w.nu2, w.omega, driver="solve", iters=10)
        tuned[(prec, kappa)] = r["exec"]
        return r["exec"]

    kappas = [1, 2, 3, 4, 6, kcycle.KAPPA_W]
    per = {}
    u64 = {}   # FP64 solutions by kappa (bit-identical to the CPU oracle's), to state the FP32 path's error
    if not args.no_sweep:
        for prec in ("f64", "f32"):
            for k in kappas:
                cfg = tune(prec, k)
                solve(prec, k)                       # warm-up (graph capture)
                times, its = [], None
                for _ in range(args.sweep_reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    its, rr, st = solve(prec, k)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                    assert st == [0], (prec, k, st)
                med = statistics.median(times)
                stats = H[prec].stats()
                key = "W" if k == kcycle.KAPPA_W else str(k)
                err = None
                if prec == "f64":
                    u64[key] = u.clone()
                elif key in u64:   # max-norm error of the FP32-cycle solution against the FP64 one
                    err = float((u - u64[key]).abs().max() / u64[key].abs().max())
                per.setdefault(key, {})[prec] = {
                    "cycles": its[0], "relres": rr[0], "ms": round(med * 1e3, 3),
                    "ms_per_cycle": round(med * 1e3 / max(its[0], 1), 4),
                    "unknowns_per_s": round(N / med),
                    "grid_launches_per_cycle": stats["grid_launches_per_iteration"],
                    "persistent_launches_per_cycle": stats["subtree_launches_per_iteration"],
                    "persistent_stages_per_cycle": stats["subtree_stages_per_iteration"],
                }
                if err is not None:
                    # the FP64 solutions equal the CPU oracle's bit for bit (full-size GPU test)
                    per[key][prec]["err_vs_f64_oracle"] = err
                print(f"[bench] {prec} kappa={key}: {its[0]} cycles, {med * 1e3:.2f} ms", file=sys.stderr, flush=True)

    # headline configuration: the fastest kappa in the headline precision
    best_p = args.precision
    if args.kappa:
        best_k = args.kappa
    elif per:
        best_k, best_t = None, math.inf
        for key, d in per.items():
            r = d.get(best_p)
            if r and r["ms"] < best_t:
                best_t, best_k = r["ms"], (kcycle.KAPPA_W if key == "W" else int(key))
    else:
        best_k = 2

    if args.exec:
        tuned[(best_p, best_k)] = json.loads(args.exec)
    elif (best_p, best_k) not in tuned and not args.no_tune:
        tune(best_p, best_k)
    if (best_p, best_k) in tuned:
        H[best_p].set_exec(**tuned[(best_p, best_k)])
    for _ in range(args.warmup):
        solve(best_p, best_k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        its, rr, st = solve(best_p, best_k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert st == [0]
    ms_step = elapsed * 1e3 / args.steps
    value = N * args.steps / elapsed

    # per-kernel profile of one iteration of the headline configuration; the
    # roofline object describes the kernel with the largest share of it
    Hb = H[best_p]
    solve(best_p, best_k)
    prof = Hb.profile_iteration("solve", kappa=best_k, nu1=w.nu1, nu2=w.nu2, omega=w.omega, reps=20)
    ms_pre, bytes_pre = Hb.time_stage(0, kappa=best_k, nu1=w.nu1, nu2=w.nu2, omega=w.omega, reps=200)
    solve(best_p, best_k)   # leave the hierarchy in a solved state
    it_ms = prof["iteration_ms"]
    kernels = {}
    for k in sorted(prof["kernels"], key=lambda r: -r["ms"]):
        row = {"launches_per_iteration": k["launches"], "avg_us": round(k["avg_ms"] * 1e3, 2),
               "share": round(k["ms"] / it_ms, 4)}
        if k["bytes_per_launch"] > 0 or k["flops_per_launch"] > 0:
            row.update(kernel_row(k, best_p))
        kernels[k["name"]] = row
    dom = max(prof["kernels"], key=lambda r: r["ms"])
    roofline = dict(kernel_row(dom, best_p), traffic=traffic_of(dom["name"]), kernel=dom["name"],
                    share_of_iteration=round(dom["ms"] / it_ms, 4), avg_launch_ms=round(dom["avg_ms"], 5),
                    launches_per_iteration=dom["launches"], bytes_per_launch=dom["bytes_per_launch"],
                    flops_per_launch=dom["flops_per_launch"],
                    note="1023^2 levels stay in the 256 MB Infinity Cache; coarse levels are latency-bound on one CU "
                         "per instance (the persistent kernel)")
    # per level (depth 0 = 1023^2): launches, time and algorithmic GB/s of one iteration
    per_level = {}
    for nm, depth, ms, nbytes in prof["sequence"]:
        e = per_level.setdefault(str(depth), {"launches": 0, "ms": 0.0, "bytes": 0.0})
        e["launches"] += 1
        e["ms"] += ms
        e["bytes"] += nbytes
    for e in per_level.values():
        e["GB_s"] = round(e["bytes"] / (e["ms"] * 1e-3) / 1e9, 1) if e["ms"] > 0 else None
        e["ms"] = round(e["ms"], 4)
        del e["bytes"]
    fine = {"kernel": "fine-level pre-smoothing", "avg_us": round(ms_pre * 1e3, 2),
            "GB_s": round(bytes_pre / (ms_pre * 1e-3) / 1e9, 1), "bytes_per_launch": bytes_pre}

    # run-time model (Section 3): alpha and beta fitted on a calibration sweep of other sizes (6-9 and 11
    # levels, kappa in {1, 2, 3, 4, W}, the default execution options), then used to predict the time per
    # cycle of the 1023^2 problem (10 levels) and, with the measured cycle counts, its best kappa
    model_info = None
    if per and not args.no_model:
        model_info = model_prediction(kcycle, model, torch, inst, w, per, f)
    extras = {}
    ex = set(x for x in args.extras.split(",") if x)
    del H, u64
    torch.cuda.empty_cache()
    if "hbm" in ex:
        extras["fine_kernels_hbm"] = hbm_kernel(kcycle, torch)
    if "c4" in ex:
        extras["c4_batched"] = c4_batched(inputs, kcycle, autotune, torch)
    if "c3" in ex:
        extras["c3_pcg"] = c3_pcg(inputs, kcycle, torch)
    if "c5" in ex:
        extras["c5_adjoint"] = c5_adjoint(inputs, torch)
    if "zebra" in ex:
        extras["zebra_c2"] = zebra_c2(inputs, kcycle, torch)
    if "convection" in ex:
        extras["convection_c2"] = convection_c2(inputs, kcycle, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst, w, best_k, per, args.cpu_cycles)

    f32_best = None
    if per:
        ks = [(d["f32"]["ms"], key) for key, d in per.items() if "f32" in d]
        if ks:
            key = min(ks)[1]
            f32_best = {"kappa": key, "ms": per[key]["f32"]["ms"], "cycles": per[key]["f32"]["cycles"],
                        "unknowns_per_s": per[key]["f32"]["unknowns_per_s"],
                        "err_vs_f64_oracle": per[key]["f32"].get("err_vs_f64_oracle")}
    out = {
        "metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-cycle+f64-refinement" if best_p == "f32" else "f64",
        "data": "synthetic (seeded, f ~ U[-1,1], seed 1)",
        "config": {"workload": "1023x1023 rotated anisotropic diffusion, theta=pi/6, eps=1e-4, 10 levels, "
                               "damped Jacobi 0.8, nu=2+2, tol 1e-8",
                   "kappa": "W" if best_k == kcycle.KAPPA_W else best_k, "precision": best_p,
                   "exec": tuned.get((best_p, best_k)),
                   "cycles": its[0], "unknowns": N},
        "roofline": roofline, "iteration_ms": round(it_ms, 4), "fine_level": fine, "per_level": per_level,
        "kernels": dict(list(kernels.items())[:8]),
        "per_kappa": per, "model": model_info,
        "extras": extras, "cpu_baseline": cpu,
    }
    out["summary"] = summary(out, f32_best)
    print(json.dumps(out))


def summary(out, f32_best):
    """The figures a reader wants first, repeated as the line's last key."""
    ex = out.get("extras", {})
    sm = {"headline": {"dtype": out["dtype"], "kappa": out["config"]["kappa"], "unknowns_per_s": round(out["value"]),
                       "ms_per_solve": round(out["ms_per_step"], 3), "cycles": out["config"]["cycles"]},
          "best_f32_cycles_f64_refinement": f32_best}
    if "c4_batched" in ex:
        c4 = ex["c4_batched"]
        sm["c4"] = {k: c4.get(k) for k in ("batched_f32_ms", "per_instance_f64_loop_ms",
                                           "speedup_batched_f32_vs_loop_f64", "batched_zebra_f32_ms",
                                           "per_instance_zebra_f64_loop_ms",
                                           "speedup_batched_zebra_f32_vs_zebra_loop_f64",
                                           "max_err_batched_f32_vs_f64")}
    if "c3_pcg" in ex:
        sm["c3_true_relres_f64"] = {k: v["true_relres_f64"] for k, v in ex["c3_pcg"].items()}
        sm["c3_ms"] = {k: v["ms"] for k, v in ex["c3_pcg"].items()}
    if "fine_kernels_hbm" in ex:
        hb = ex["fine_kernels_hbm"]
        sm["fine_TB_s_nu2"] = {f"{name}_{n}": round(hb[f"by_nu_{n}"][f"{name}_nu2"]["GB_s"] / 1e3, 3)
                               for n in (8191, 16383) for name in ("pre", "post") if f"by_nu_{n}" in hb}
        if "torch_streaming_8191" in hb:
            sm["fine_TB_s_nu2"]["torch_axpy_8191"] = hb["torch_streaming_8191"]["axpy"]
    if "c5_adjoint" in ex:
        sm["c5_forward_backward_ms"] = ex["c5_adjoint"]["forward_backward_ms"]
    if "convection_c2" in ex:
        sm["convection_ms"] = {k: v["ms"] for k, v in ex["convection_c2"].items()}
    if out.get("model"):
        m = out["model"]
        sm["model"] = {"predicted_best_kappa": m["predicted_best_kappa"],
                       "measured_best_kappa": str(out["config"]["kappa"]),
                       "max_rel_err": max(abs(v) for v in m["rel_err"].values())}
    sm["roofline"] = {k: out["roofline"].get(k) for k in ("kernel", "bound", "frac", "share_of_iteration")}
    return sm


def model_prediction(kcycle, model, torch, inst, w, per, f):
    """Calibrate T = alpha N_calls + beta N_ops (N_calls = grid launches +
    persistent-kernel stages, one serialised step each; N_ops = N 2(1 - 3^-kappa))
    on problems of 6-9 and 11 levels, predict the 1023^2 problem's time per cycle
    for every kappa (default execution options, checked against a measurement
    of the same), and its best kappa as argmin predicted time per cycle x
    measured cycles."""
    from paper_2010_00626_amd import fit_model
    kappas = [1, 2, 3, 4, kcycle.KAPPA_W]
    rows = []
    for k in kappas:
        for nl in (6, 7, 8, 9, 11):
            ms, launches, stages, _ = fit_model.measure("fused", k, nl, nu=w.nu1 + w.nu2, theta=inst.theta,
                                                        eps=inst.eps, budget_ms=40.0)
            rows.append(((k, nl), fit_model.n_calls(launches, stages), model.n_ops_2d(k, nl), ms))
    fitted = model.fit(rows)
    n = inst.n
    levels = int(round(math.log2(n + 1)))
    Hd = kcycle.Hierarchy([(n, inst.theta, inst.eps, w.n_coarsest)], "f64")
    v = torch.zeros_like(f)
    pred, meas, pred_total, meas_total = {}, {}, {}, {}
    for k in kappas:
        key = "W" if k == kcycle.KAPPA_W else str(k)
        ms = Hd.time_cycles(v, f, kappa=k, nu1=w.nu1, nu2=w.nu2, omega=w.omega, reps=40)
        st = Hd.stats()
        calls = fit_model.n_calls(st["grid_launches_per_iteration"], st["subtree_stages_per_iteration"])
        pred[key] = fitted.predict(calls, model.n_ops_2d(k, levels))
        meas[key] = ms
        cyc = per[key]["f64"]["cycles"]
        pred_total[key] = pred[key] * cyc
        meas_total[key] = ms * cyc
    Hd.close()
    return {"alpha_us": round(fitted.alpha * 1e3, 4), "beta_ns_per_op": round(fitted.beta * 1e6, 6),
            "calls": "grid launches + persistent-kernel stages", "calibration": "6-9 and 11 levels, kappa 1-4 and W",
            "calibration_rel_err_max": round(max(abs(e) for e in fitted.rel_errors.values()), 4),
            "predicted_ms_per_cycle": {k: round(v, 4) for k, v in pred.items()},
            "measured_ms_per_cycle": {k: round(v, 4) for k, v in meas.items()},
            "rel_err": {k: round((pred[k] - meas[k]) / meas[k], 4) for k in pred},
            "predicted_best_kappa": min(pred_total, key=pred_total.get),
            "measured_best_kappa_default_exec": min(meas_total, key=meas_total.get)}


def hbm_kernel(kcycle, torch):
    """Fine-level fused kernels on 8191^2 and 16383^2 FP64 grids (537 MB and 2.1 GB per
    array, far beyond the 256 MB Infinity Cache): achieved HBM bandwidth of one launch,
    for the benchmark's nu = 2 (pre, post) and per nu = 0, 1, 2 (by_nu: the pre-part is
    residual + full weighting after nu sweeps, the post-part prolong-add before nu sweeps)."""
    res = {}
    for n in (8191, 16383):
        Hh = kcycle.Hierarchy([(n, math.pi / 4, 1e-4)], "f64")
        fh = torch.zeros((n, n), dtype=torch.float64, device="cuda").uniform_(-1, 1)
        uh = torch.zeros_like(fh)
        Hh.solve(uh, fh, kappa=1, tol=0.0, maxit=1)      # binds the arrays
        by_nu = {}
        for nu in (0, 1, 2):
            for name, which in (("pre", 0), ("post", 1)):
                ms, b = Hh.time_stage(which, kappa=1, nu1=nu, nu2=nu, reps=20)
                gbs = b / (ms * 1e-3) / 1e9
                entry = {"ms": round(ms, 4), "bytes": b, "GB_s": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4)}
                by_nu[f"{name}_nu{nu}"] = entry
                if n == 8191 and nu == 2:
                    res[name] = entry
        res[f"by_nu_{n}"] = by_nu
        Hh.close()
        del Hh, fh, uh
        torch.cuda.empty_cache()
    res["torch_streaming_8191"] = torch_streaming(torch, 8191)
    return res


def torch_streaming(torch, n):
    """What PyTorch's own elementwise kernels reach on n x n FP64 arrays of the same size
    (copy: 1 read + 1 write, add and a + 0.5 b: 2 reads + 1 write), in TB/s: the practical
    streaming rate of this GPU next to which the fused kernels' rates can be read."""
    a = torch.zeros((n, n), dtype=torch.float64, device="cuda").uniform_(-1, 1)
    b = torch.zeros_like(a).uniform_(-1, 1)
    c = torch.zeros_like(a).uniform_(-1, 1)
    nb = a.numel() * 8

    def rate(fn, nbytes, reps=20):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return round(nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e12, 3)

    out = {"copy": rate(lambda: a.copy_(b), 2 * nb), "add": rate(lambda: torch.add(b, c, out=a), 3 * nb),
           "axpy": rate(lambda: torch.add(b, c, alpha=0.5, out=a), 3 * nb)}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def c4_batched(inputs, kcycle, autotune, torch):
    """64 uneven instances (255^2..2047^2), kappa=3 stand-alone to 1e-8:
    one batched FP32-cycle/FP64-refinement solve against a loop of plain
    per-instance FP64 solves."""
    wl = inputs.config4()
    probs = [(i.n, i.theta, i.eps) for i in wl.instances]
    fs = [torch.from_numpy(i.f).to("cuda") for i in wl.instances]
    us = [torch.zeros_like(x) for x in fs]
    N = wl.unknowns
    # two instances have grid-aligned anisotropy (theta within 0.03 rad of an axis, eps ~ 1e-4): the
    # pointwise smoother leaves a contraction factor near 0.997 there, so they need ~5000 cycles
    kw = dict(kappa=3, nu1=wl.nu1, nu2=wl.nu2, omega=wl.omega, tol=wl.tol, maxit=12000)
    Hb = kcycle.Hierarchy(probs, "f32")
    cfg = autotune.tune(Hb, us, fs, 3, wl.nu1, wl.nu2, wl.omega, driver="solve", iters=6)["exec"]
    for x in us:
        x.zero_()
    Hb.solve(us, fs, **dict(kw, maxit=3))
    times = []
    for _ in range(2):
        for x in us:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, rr, st = Hb.solve(us, fs, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    assert all(x == 0 for x in st), st
    tb = statistics.median(times)
    grid_b = Hb.stats()["grid_launches_per_iteration"]
    ub = [x.clone() for x in us]   # batched FP32-cycle solutions, compared with the FP64 loop's below
    Hb.close()
    del Hb
    # plain per-instance FP64 loop
    Hs = [kcycle.Hierarchy([p], "f64") for p in probs]
    for h_, x, fx in zip(Hs, us, fs):
        x.zero_()
        h_.solve(x, fx, **dict(kw, maxit=3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its64 = []
    for h_, x, fx in zip(Hs, us, fs):
        x.zero_()
        i64, _, s64 = h_.solve(x, fx, **kw)
        its64.append(i64[0])
        assert s64 == [0]
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    for h_ in Hs:
        h_.close()
    errs = [float((a - b).abs().max() / b.abs().max()) for a, b in zip(ub, us)]
    del ub
    # the same batch with alternating zebra line relaxation (the paper's smoother for any angle; fused
    # mode, calls at 63^2 in the persistent kernel): the grid-aligned instances no longer set the time
    Hz = kcycle.Hierarchy(probs, "f32", exec=dict(coarse_cutover=63))
    uz = [torch.zeros_like(x) for x in fs]
    Hz.solve(uz, fs, **dict(kw, maxit=3), smoother="zebra")
    tzs = []
    for _ in range(2):
        for x in uz:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        itz, rrz, stz = Hz.solve(uz, fs, **kw, smoother="zebra")
        torch.cuda.synchronize()
        tzs.append(time.perf_counter() - t0)
    assert all(x == 0 for x in stz), stz
    tz = statistics.median(tzs)
    az = [torch.empty_like(x) for x in uz]
    Hz.apply_A(az, uz)   # FP64 operator
    true_z = [float(torch.linalg.vector_norm(fx - a) / torch.linalg.vector_norm(fx)) for fx, a in zip(fs, az)]
    Hz.close()
    del Hz, uz, az
    # like for like: the per-instance FP64 loop with the same zebra smoother (fused mode, cutover 63)
    Hzs = [kcycle.Hierarchy([p], "f64", exec=dict(coarse_cutover=63)) for p in probs]
    for h_, x, fx in zip(Hzs, us, fs):
        x.zero_()
        h_.solve(x, fx, **dict(kw, maxit=3), smoother="zebra")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    itsz64 = []
    for h_, x, fx in zip(Hzs, us, fs):
        x.zero_()
        iz, _, sz = h_.solve(x, fx, **kw, smoother="zebra")
        itsz64.append(iz[0])
        assert sz == [0]
    torch.cuda.synchronize()
    tlz = time.perf_counter() - t0
    for h_ in Hzs:
        h_.close()
    sizes = sorted(set(p[0] for p in probs))
    return {"instances": len(probs), "sizes": {str(s): sum(1 for p in probs if p[0] == s) for s in sizes},
            "unknowns": N, "kappa": 3, "batched_f32_ms": round(tb * 1e3, 2),
            "batched_unknowns_per_s": N / tb, "batched_max_cycles": max(it),
            "batched_median_cycles": statistics.median(it), "batched_max_relres": max(rr), "batched_exec": cfg,
            "batched_grid_launches_per_cycle": grid_b,
            "per_instance_f64_loop_ms": round(tl * 1e3, 2), "per_instance_unknowns_per_s": N / tl,
            "per_instance_max_cycles": max(its64), "per_instance_median_cycles": statistics.median(its64),
            "max_err_batched_f32_vs_f64": max(errs),
            "speedup_batched_f32_vs_loop_f64": round(tl / tb, 3),
            "batched_zebra_f32_ms": round(tz * 1e3, 2), "batched_zebra_max_cycles": max(itz),
            "batched_zebra_median_cycles": statistics.median(itz), "batched_zebra_max_true_relres": max(true_z),
            "per_instance_zebra_f64_loop_ms": round(tlz * 1e3, 2), "per_instance_zebra_max_cycles": max(itsz64),
            "speedup_batched_zebra_f32_vs_zebra_loop_f64": round(tlz / tz, 3)}


def c3_pcg(inputs, kcycle, torch):
    """4095^2, theta=3pi/8, eps=1e-5: CG preconditioned by one kappa-cycle
    (nu=1+1), FP32 cycles with FP64 CG vectors, to 1e-8, per kappa; for each
    kappa the true FP64 relative residual of the result (the library confirms
    convergence on it) and its max-norm error against the FP64-preconditioned
    PCG solution (whose iterates equal the oracle's to 1e-11)."""
    wl = inputs.config3()
    inst = wl.instances[0]
    n = inst.n
    f = torch.from_numpy(inst.f).to("cuda")
    u = torch.zeros_like(f)
    u64 = torch.zeros_like(f)
    r = torch.empty_like(f)
    Hc = kcycle.Hierarchy([(n, inst.theta, inst.eps)], "f32")
    H64 = kcycle.Hierarchy([(n, inst.theta, inst.eps)], "f64")
    kw = dict(nu1=1, nu2=1, omega=wl.omega, tol=wl.tol, maxit=1000)
    nf = torch.linalg.vector_norm(f)
    out = {}
    for k in wl.kappas:
        u.zero_()
        Hc.pcg(u, f, kappa=k, **kw)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, rr, st = Hc.pcg(u, f, kappa=k, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        H64.apply_A(r, u)
        true_rel = float(torch.linalg.vector_norm(f - r) / nf)
        u64.zero_()
        it64, _, st64 = H64.pcg(u64, f, kappa=k, **kw)
        out[str(k)] = {"iterations": it[0], "relres": rr[0], "true_relres_f64": true_rel, "status": st[0],
                       "ms": round(dt * 1e3, 2), "ms_per_iteration": round(dt * 1e3 / max(it[0], 1), 4),
                       "unknowns_per_s": round(n * n / dt), "f64_precond_iterations": it64[0],
                       "err_vs_f64_precond": float((u - u64).abs().max() / u64.abs().max())}
        print(f"[bench] c3 pcg kappa={k}: {it[0]} iterations, {dt * 1e3:.1f} ms, true relres {true_rel:.2e}",
              file=sys.stderr, flush=True)
    Hc.close()
    H64.close()
    return out


def zebra_c2(inputs, kcycle, torch):
    """The 1023^2 workload with alternating zebra line Gauss-Seidel (FP64, nu = 2 + 2:
    one x- and one y-relaxation on each side), per kappa, to the same 1e-8 relative
    residual: in the fused mode (levels above 63^2 one kernel per operation, every
    call at 63^2 in one persistent launch) and in the paper-structured mode (one
    kernel per operation on every level)."""
    w = inputs.config2()
    inst = w.instances[0]
    n = inst.n
    f = torch.from_numpy(inst.f).to("cuda")
    u = torch.zeros_like(f)
    out = {}
    for mode in ("fused", "paper"):
        # fused: calls at 63^2 and below in the persistent kernel (the line solves of 63^2 fit its LDS)
        ex = dict(mode=mode, coarse_cutover=63) if mode == "fused" else dict(mode=mode)
        H = kcycle.Hierarchy([(n, inst.theta, inst.eps, w.n_coarsest)], "f64", exec=ex)
        res = {}
        for k in (1, 2, 3, 4, kcycle.KAPPA_W):
            u.zero_()
            H.solve(u, f, kappa=k, nu1=2, nu2=2, tol=w.tol, maxit=2000, smoother="zebra")   # warm-up + capture
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, rr, st = H.solve(u, f, kappa=k, nu1=2, nu2=2, tol=w.tol, maxit=2000, smoother="zebra")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            key = "W" if k == kcycle.KAPPA_W else str(k)
            res[key] = {"cycles": it[0], "status": st[0], "ms": round(dt * 1e3, 2),
                        "ms_per_cycle": round(dt * 1e3 / max(it[0], 1), 3), "unknowns_per_s": n * n / dt}
            print(f"[bench] zebra {mode} kappa={key}: {it[0]} cycles, {dt * 1e3:.2f} ms", file=sys.stderr, flush=True)
        H.close()
        out[mode] = res
    out["cycle_4095"] = zebra_4095(inst, kcycle, torch)
    return out


def zebra_4095(inst, kcycle, torch):
    """One zebra cycle on a 4095^2 grid (the same theta and eps, fused mode with the calls
    at 63^2 and below in the persistent kernel), ms per cycle per kappa, and the fine
    level's line-kernel launches (one colour of one relaxation each) from the launch
    profile of a kappa = 1 iteration: average time and algorithmic rate."""
    n = 4095
    H = kcycle.Hierarchy([(n, inst.theta, inst.eps)], "f64", exec=dict(mode="fused", coarse_cutover=63))
    f = torch.zeros((n, n), dtype=torch.float64, device="cuda").uniform_(-1, 1)
    u = torch.zeros_like(f)
    res = {"ms_per_cycle": {}}
    for k in (1, 2, 3, 4, kcycle.KAPPA_W):
        key = "W" if k == kcycle.KAPPA_W else str(k)
        res["ms_per_cycle"][key] = round(H.time_cycles(u, f, kappa=k, reps=5, smoother="zebra"), 3)
    u.zero_()
    H.solve(u, f, kappa=1, tol=0.0, maxit=2, smoother="zebra")
    prof = H.profile_iteration("solve", kappa=1, reps=5, smoother="zebra")
    fine = [e for e in prof["sequence"] if e[0].startswith("k_zebra") and e[1] == 0]
    if fine:
        ms = sum(e[2] for e in fine) / len(fine)
        b = sum(e[3] for e in fine) / len(fine)
        res["fine_colour"] = {"launches_per_cycle": len(fine), "avg_ms": round(ms, 4), "bytes": b,
                              "GB_s": round(b / (ms * 1e-3) / 1e9, 1)}
    print(f"[bench] zebra 4095^2: {res}", file=sys.stderr, flush=True)
    H.close()
    del f, u
    torch.cuda.empty_cache()
    return res


def convection_c2(inputs, kcycle, torch):
    """Convection-diffusion (the nonsymmetric problem of the conclusions) on the
    1023^2 grid: -div(D grad u) + b . grad u with theta = pi/6, eps = 1e-2,
    b = (20, 10), upwind convection, rediscretised levels, damped Jacobi
    nu = 2+2, f ~ U[-1,1] (seed 1), stand-alone FP64 to 1e-8, per kappa."""
    w = inputs.config2()
    n = w.instances[0].n
    f = torch.from_numpy(w.instances[0].f).to("cuda")
    u = torch.zeros_like(f)
    H = kcycle.Hierarchy([(n, math.pi / 6, 1e-2)], "f64")
    H.set_convection(20.0, 10.0)
    out = {}
    for k in (1, 2, 3, 4, kcycle.KAPPA_W):
        u.zero_()
        H.solve(u, f, kappa=k, nu1=2, nu2=2, tol=w.tol, maxit=3000)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, rr, st = H.solve(u, f, kappa=k, nu1=2, nu2=2, tol=w.tol, maxit=3000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = "W" if k == kcycle.KAPPA_W else str(k)
        out[key] = {"cycles": it[0], "status": st[0], "ms": round(dt * 1e3, 2), "unknowns_per_s": round(n * n / dt)}
        print(f"[bench] convection kappa={key}: {it[0]} cycles, {dt * 1e3:.2f} ms", file=sys.stderr, flush=True)
    H.close()
    return out


def c5_adjoint(inputs, torch):
    """16 x 1023^2 instances, kappa=3 PCG forward and adjoint to 1e-8:
    loss 1/2 ||u - u*||^2, u* for (theta + 0.1, 2 eps); forward + backward."""
    from paper_2010_00626_amd import autograd as ag
    wl = inputs.config5()
    th = torch.tensor([i.theta for i in wl.instances], dtype=torch.float64)
    ep = torch.tensor([i.eps for i in wl.instances], dtype=torch.float64)
    f = torch.from_numpy(np.stack([i.f for i in wl.instances])).to("cuda")
    cfg = ag.SolveConfig(kappa=3, nu1=1, nu2=1, tol=wl.tol, tol_adjoint=wl.tol)
    with torch.no_grad():
        target = ag.solve(f, th + 0.1, 2 * ep, cfg)
    times = []
    for _ in range(2):
        tht = th.clone().requires_grad_(True)
        ept = ep.clone().requires_grad_(True)
        fr = f.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = 0.5 * ((ag.solve(fr, tht, ept, cfg) - target) ** 2).sum()
        L.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = min(times)
    N = wl.unknowns
    return {"instances": len(wl.instances), "unknowns": N, "forward_backward_ms": round(dt * 1e3, 2),
            "unknowns_per_s": N / dt, "solves": 3, "loss": float(L.detach())}


def cpu_baseline(inst, w, kappa, per, cycles):
    """The oracle (single-threaded C, FP64) timed on this host: `cycles`
    kappa-cycles of the same 1023^2 solve, scaled by the cycle count the solve
    needs (the oracle's own count equals the GPU FP64 count)."""
    from oracle import oracle
    k = min(kappa, 64)
    H = oracle.Hierarchy(inst.n, inst.theta, inst.eps, n_coarsest=w.n_coarsest, omega=w.omega)
    key = "W" if kappa == 2 ** 31 - 1 else str(kappa)
    need = per.get(key, {}).get("f64", {}).get("cycles") if per else None
    v = np.zeros((inst.n, inst.n))
    t0 = time.perf_counter()
    for _ in range(cycles):
        v, _ = H.cycle(v, inst.f, kappa=k, nu1=w.nu1, nu2=w.nu2)
    dt = time.perf_counter() - t0
    per_cycle = dt / cycles
    if need is None:
        return {"value": None, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
                "sample": f"{cycles} cycles, s/cycle={per_cycle:.4f}"}
    total = per_cycle * (need + 1)   # cycles plus the final residual test (about one cycle's cost or less)
    return {"value": inst.n * inst.n / total, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"{cycles} FP64 kappa={key} cycles on the full 1023^2 problem ({dt:.1f} s), "
                      f"scaled to the {need} cycles the solve needs",
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_model() -> str:
    """The host CPU's model name (the lscpu 'Model name' field, read from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
