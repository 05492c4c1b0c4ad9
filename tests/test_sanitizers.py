"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code
(host only; no GPU): the oracle, and the host runtime of the library, whose
host-only entry points (workspace sizing, level stencils of every problem
kind, the launch schedule) run under the sanitizers on this machine.  The
device code is not instrumented (the sanitizers apply to the host pass only).
A sanitizer finding aborts the child process, which fails the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def runtime_libs():
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"{name} not available")
        libs.append(p)
    return libs


def run_child(code, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = ":".join(runtime_libs())
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", *SAN,
                           "-o", lib, os.path.join(ROOT, "oracle", "kc_oracle.c"), "-lm"])
    out = run_child("""
        import math, numpy as np
        from oracle import oracle as O
        rng = np.random.default_rng(0)
        for n, nc in ((15, 1), (31, 3), (63, 7)):
            f = rng.uniform(-1, 1, (n, n))
            H = O.Hierarchy(n, 0.7, 1e-3, n_coarsest=nc)
            for k in (1, 2, 3, 64):
                H.cycle(np.zeros((n, n)), f, kappa=k)
            H.solve(f, kappa=2, tol=1e-8, maxit=200)
            H.pcg(f, kappa=2, tol=1e-8, maxit=100)
            H.pcg(f, kappa=1, tol=1e-8, maxit=100, precond_f32=True)
            H.ir_solve(f, kappa=2, tol=1e-8, maxit=200)
            H.grad_params(f, f)
            Z = O.Hierarchy(n, 0.7, 1e-3, n_coarsest=nc, smoother="zebra")
            Z.solve(f, kappa=3, tol=1e-8, maxit=100)
            S = O.Hierarchy(n, 0.7, 1e-3, coarsening="semi")
            S.solve(f, kappa=2, tol=1e-8, maxit=100)
            S.pcg(f, kappa=2, tol=1e-8, maxit=100)
            C = O.Hierarchy(n, 0.7, 1e-2, convection=(20.0, -10.0))
            C.solve(f, kappa=2, tol=1e-8, maxit=200)
        print("oracle ok")
    """, {"KC_ORACLE_LIB": lib})
    assert "oracle ok" in out


def test_host_runtime_under_asan_ubsan(tmp_path):
    """The library's host code built with the sanitizers on its host pass,
    linked with the ordinary device-code object."""
    hipcc = "/opt/rocm/bin/hipcc"
    kobj = os.path.join(ROOT, "paper_2010_00626_amd", "_build", "kc_kernels.o")
    if not os.path.exists(hipcc) or not os.path.exists(kobj):
        pytest.skip("hipcc or the built kernel object is missing")
    robj = str(tmp_path / "kc_runtime_san.o")
    lib = str(tmp_path / "libkcycle_san.so")
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san, "-x", "hip", "-c",
                           os.path.join(ROOT, "paper_2010_00626_amd", "csrc", "kc_runtime.cpp"), "-o", robj],
                          stderr=subprocess.DEVNULL)
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *host_san, "-o", lib, robj, kobj])
    out = run_child("""
        import math
        from paper_2010_00626_amd import kcycle as K
        probs = [(1023, math.pi / 6, 1e-4), (255, 0.3, 1e-3, 3), (63, 1.0, 1.0, 7), (1, 0.2, 0.5)]
        K.workspace_bytes(probs, "f64"); K.workspace_bytes(probs, "f32")
        K.workspace_bytes([(4095, 0.3, 1e-5)] * 2, "f64", coarsening="semi")
        for p in probs:
            K.level_stencils(*p)
        K.convection_stencils(511, 0.4, 1e-2, 20.0, -10.0)
        K.semi_stencils(16383, 0.4, 1e-5)
        for kappa in (1, 2, 3, 2 ** 31 - 1):
            for mode in ("fused", "paper"):
                for sm in ("jacobi", "zebra"):
                    K.schedule_counts(probs, kappa, mode=mode, smoother=sm)
                K.schedule_counts(probs, kappa, mode=mode, smoother="zebra", zebra_wave_n=1, zebra_quad_n=63)
        for bad in ([(1000, 0.3, 1e-3)], [(63, 0.3, -1.0)], [(63, 0.3, 1e-3, 5)]):
            try:
                K.workspace_bytes(bad)
            except K.KCycleError:
                pass
            else:
                raise SystemExit("bad problem accepted")
        print("runtime ok")
    """, {"KC_LIBRARY": lib})
    assert "runtime ok" in out
