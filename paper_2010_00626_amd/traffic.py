"""HBM traffic per kernel launch from rocprofv3 counters.

Run mode (the program rocprofv3 profiles): a device copy of a known size,
then a fixed number of iterations of the 1023^2 stand-alone solve with the
given precision, kappa and execution options.  Profile it once per counter, e.g.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR_F -- python3 -m paper_2010_00626_amd.traffic run ...
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR_W -- python3 -m paper_2010_00626_amd.traffic run ...

Summarise mode reads both counter tables, scales each counter by the value
the copy reads for its known byte count (the calibration factor), and writes
a JSON file with the average HBM bytes per launch of every kernel (names as
the library's per-launch profile gives them) and the SHA-256 of the kernel
source the counters were taken on:

    python3 -m paper_2010_00626_amd.traffic summarise DIR_F DIR_W OUT.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import re
import sys
from collections import defaultdict

COPY_BYTES = 1 << 30          # bytes read (and written) by the calibration kernel
HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_digest() -> str:
    with open(os.path.join(HERE, "csrc", "kc_kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def short_name(name: str) -> str:
    """'void kc::k_pre<float, 2, 16, 16>(kc::StageArgs)' -> 'k_pre<float, 2, 16, 16>'."""
    name = name.strip().replace("void ", "")
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):   # cut the parameter list: first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    name = name[:cut]
    return re.sub(r"^kc::", "", name)


def run(args) -> None:
    import numpy as np
    import torch
    from . import inputs, kcycle

    # calibration: an elementwise kernel that reads COPY_BYTES and writes COPY_BYTES (a same-type
    # copy_ would go to the DMA engines, which the counters do not see)
    x = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(x, 1.5, out=y)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()

    if args.size:
        # the fine-level fused kernels alone on an n x n FP64 problem far beyond the Infinity
        # Cache: `cycles` launches each of the pre-part and the post-part at nu = 2
        n = args.size
        H = kcycle.Hierarchy([(n, math.pi / 4, 1e-4)], "f64", exec=json.loads(args.exec) if args.exec else None)
        f = torch.zeros((n, n), dtype=torch.float64, device="cuda").uniform_(-1, 1)
        u = torch.zeros_like(f)
        H.solve(u, f, kappa=1, tol=0.0, maxit=1)   # binds the arrays
        out = {}
        for name, which in (("pre", 0), ("post", 1)):
            ms, b = H.time_stage(which, kappa=1, nu1=2, nu2=2, reps=args.cycles)
            out[name] = {"ms": ms, "algorithmic_bytes": b}
        torch.cuda.synchronize()
        print(json.dumps(out), flush=True)
        return
    w = inputs.config2()
    inst = w.instances[0]
    n = inst.n
    ex = json.loads(args.exec) if args.exec else {}
    H = kcycle.Hierarchy([(n, inst.theta, inst.eps, w.n_coarsest)], args.precision, exec=ex or None)
    f = torch.from_numpy(inst.f).to("cuda")
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    kappa = kcycle.KAPPA_W if args.kappa == "W" else int(args.kappa)
    # a fixed number of iterations: counter collection serialises every dispatch
    it, rr, st = H.solve(u, f, kappa=kappa, nu1=w.nu1, nu2=w.nu2, omega=w.omega, tol=0.0, maxit=args.cycles)
    torch.cuda.synchronize()
    print(json.dumps({"iterations": it[0], "relres": rr[0], "status": st[0]}), flush=True)


def _counter_rows(root: str):
    files = sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {root}")
    for path in files:
        with open(path, newline="") as fh:
            yield from csv.DictReader(fh)


def per_kernel(root: str, counter: str) -> dict:
    """average counter value (KiB) per dispatch, by kernel"""
    acc = defaultdict(list)
    for r in _counter_rows(root):
        if r.get("Counter_Name") != counter:
            continue
        acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def calibration(table: dict, name_hint: str = "Mul") -> tuple:
    """bytes per counter unit: the calibration kernel is the elementwise
    multiply (by name), else the kernel whose average is closest to the
    calibration byte count in KiB (within a factor of 2)"""
    for k, (avg, cnt) in table.items():
        if name_hint in k and avg > 0 and 0.5 < avg / (COPY_BYTES / 1024.0) < 2.0:
            return COPY_BYTES / avg, k
    want = COPY_BYTES / 1024.0
    best = None
    for k, (avg, cnt) in table.items():
        if avg <= 0:
            continue
        ratio = avg / want
        if 0.5 < ratio < 2.0 and (best is None or abs(math.log(ratio)) < abs(math.log(best[1] / want))):
            best = (k, avg)
    if best is None:
        top = sorted(table.items(), key=lambda kv: -kv[1][0])[:8]
        raise SystemExit("calibration kernel not found in the counters; largest averages (KiB): " +
                         "; ".join(f"{k}: {v[0]:.0f} x{v[1]}" for k, v in top))
    return COPY_BYTES / best[1], best[0]


def summarise(dir_fetch: str, dir_write: str, out: str) -> None:
    fetch = per_kernel(dir_fetch, "FETCH_SIZE")
    write = per_kernel(dir_write, "WRITE_SIZE")
    cf, copy_k = calibration(fetch)
    cw, copy_w = calibration(write)
    res = {}
    for k in sorted(set(fetch) | set(write)):
        if k in (copy_k, copy_w):
            continue
        fb = fetch.get(k, (0.0, 0))[0] * cf
        wb = write.get(k, (0.0, 0))[0] * cw
        res[k] = fb + wb
    data = {"kernels_source_sha256": kernel_source_digest(), "calibration_kernel": copy_k,
            "bytes_per_kib_fetch": cf, "bytes_per_kib_write": cw,
            "fetch_bytes_per_launch": {k: fetch[k][0] * cf for k in fetch if k not in (copy_k, copy_w)},
            "write_bytes_per_launch": {k: write[k][0] * cw for k in write if k not in (copy_k, copy_w)},
            "bytes_per_launch": res}
    with open(out, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(f"calibration: {cf:.1f} B per FETCH_SIZE unit, {cw:.1f} B per WRITE_SIZE unit (kernel {copy_k}, "
          f"{COPY_BYTES} B read and written)")
    print(f"{'kernel':60s} {'launches':>8s} {'fetch MB':>10s} {'write MB':>10s} {'total MB':>10s}")
    for k, v in sorted(res.items(), key=lambda kv: -kv[1])[:20]:
        print(f"{k:60s} {fetch.get(k, (0, 0))[1]:8d} {fetch.get(k, (0.0, 0))[0] * cf / 1e6:10.3f} "
              f"{write.get(k, (0.0, 0))[0] * cw / 1e6:10.3f} {v / 1e6:10.3f}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--precision", default="f32")
    r.add_argument("--kappa", default="2")
    r.add_argument("--exec", default="", help="JSON execution options")
    r.add_argument("--cycles", type=int, default=20)
    r.add_argument("--size", type=int, default=0, help="fine-level kernels alone on an n x n FP64 grid (e.g. 8191)")
    s = sub.add_parser("summarise")
    s.add_argument("dir_fetch")
    s.add_argument("dir_write")
    s.add_argument("out")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run(a)
    else:
        summarise(a.dir_fetch, a.dir_write, a.out)


if __name__ == "__main__":
    main()
