"""Python view of the C oracle (``oracle/kc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain single-threaded FP64 CPU
implementation of the kappa-cycle method of Avnat & Yavneh, written from the
paper, used to check the GPU library.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product never does.
It shares no code with the GPU library.

Arrays are numpy float64 (float32 for the FP32 cycle), shape (n, n), row j
along +y, column i along +x, interior points only (zero Dirichlet outside).
The operator on a level is A = S / h^2 with h = 1/(n+1) (Section 4).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# a separately built copy (e.g. with sanitizers) may be named by KC_ORACLE_LIB
_LIB_PATH = os.environ.get("KC_ORACLE_LIB") or _LIB_PATH

OP_CALL, OP_SOLVE, OP_RELAX, OP_RESID, OP_RESTR, OP_ZERO, OP_PROL, OP_ADD = range(1, 9)
OK, NOT_CONVERGED, DIVERGED, BREAKDOWN = 0, 1, 2, 3
ERR_ARG, ERR_NONFINITE = -1, -4

KIND_KAPPA, KIND_GAMMA, KIND_F = 0, 1, 2


def _host_has_fma() -> bool:
    try:
        with open("/proc/cpuinfo") as fh:
            return any(line.startswith("flags") and " fma " in line + " " for line in fh)
    except OSError:
        return False


def build(force: bool = False) -> str:
    """Compile the oracle with gcc.  The compiler contracts nothing
    (-ffp-contract=off); the explicit fma() calls are inlined as the FMA
    instruction when the host has it (same result as the libm call, which is
    exact too, only faster)."""
    src = os.path.join(_HERE, "kc_oracle.c")
    deps = [src, os.path.join(_HERE, "kc_oracle.h"), os.path.join(_HERE, "kc_oracle_levels.inc"),
            os.path.join(_HERE, "kc_oracle_semi.inc")]
    if os.environ.get("KC_ORACLE_LIB"):
        return _LIB_PATH
    if not force and os.path.exists(_LIB_PATH):
        if os.path.getmtime(_LIB_PATH) >= max(os.path.getmtime(d) for d in deps):
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    arch = ["-mfma"] if _host_has_fma() else []
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", *arch, "-fPIC", "-shared",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        ip = C.POINTER(C.c_int)
        i32p = C.POINTER(C.c_int32)
        hp = C.c_void_p
        L.or_fine_stencil.argtypes = [C.c_double, C.c_double, dp]
        L.or_fine_stencil_derivs.argtypes = [C.c_double, C.c_double, dp, dp]
        L.or_apply_stencil.argtypes = [C.c_int, dp, dp, dp]
        L.or_restrict_fw.argtypes = [C.c_int, dp, dp]
        L.or_prolong.argtypes = [C.c_int, dp, dp]
        L.or_galerkin_stencil.argtypes = [dp, dp]
        L.or_hier_new.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, C.POINTER(hp)]
        L.or_hier_new.restype = C.c_int
        L.or_hier_new_semi.argtypes = [C.c_int, C.c_double, C.c_double, C.POINTER(hp)]
        L.or_hier_new_semi.restype = C.c_int
        L.or_hier_free.argtypes = [hp]
        L.or_hier_info.argtypes = [hp, ip, ip, dp]
        L.or_hier_apply.argtypes = [hp, dp, dp]
        L.or_set_smoother.argtypes = [hp, C.c_int]
        L.or_set_smoother.restype = C.c_int
        L.or_convection_stencil.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.or_set_convection.argtypes = [hp, C.c_double, C.c_double]
        L.or_set_convection.restype = C.c_int
        L.or_zebra_relax.argtypes = [hp, C.c_int, dp, dp]
        L.or_cycle.argtypes = [hp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, i32p, C.c_int64]
        L.or_cycle.restype = C.c_int64
        L.or_kcycle_f32.argtypes = [hp, C.c_int, C.c_int, C.c_int, fp, fp]
        L.or_solve.argtypes = [hp, C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.c_int, C.c_int, ip, dp]
        L.or_solve.restype = C.c_int
        L.or_pcg.argtypes = [hp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.c_int, ip, dp]
        L.or_pcg.restype = C.c_int
        L.or_ir_solve.argtypes = [hp, C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.c_int, ip, dp]
        L.or_ir_solve.restype = C.c_int
        L.or_ir_scale.argtypes = [C.c_double, C.c_int64]
        L.or_ir_scale.restype = C.c_double
        L.or_grad_params.argtypes = [hp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.or_zebra_tables.argtypes = [hp, C.c_int, C.c_int, dp, dp]
        L.or_zebra_tables.restype = C.c_int
        L.or_dot2.argtypes = [dp, dp, C.c_int64]
        L.or_dot2.restype = C.c_double
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fp(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_float))


def fine_stencil(theta: float, eps: float) -> np.ndarray:
    """Section 4 nine-point stencil as a 3x3 array s[b+1, a+1] (b along +y)."""
    s = np.zeros(9)
    lib().or_fine_stencil(theta, eps, _dp(s))
    return s.reshape(3, 3)


def convection_stencil(n: int, theta: float, eps: float, bx: float, by: float) -> np.ndarray:
    """h^2-scaled fine stencil of -div(D grad u) + b . grad u (upwind convection), 3 x 3."""
    s = np.zeros(9)
    lib().or_convection_stencil(n, theta, eps, bx, by, _dp(s))
    return s.reshape(3, 3)


def fine_stencil_derivs(theta: float, eps: float):
    dth, de = np.zeros(9), np.zeros(9)
    lib().or_fine_stencil_derivs(theta, eps, _dp(dth), _dp(de))
    return dth.reshape(3, 3), de.reshape(3, 3)


def apply_stencil(s: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = S x (no 1/h^2 factor) with zero values outside the grid."""
    s = np.ascontiguousarray(s, dtype=np.float64).reshape(9)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().or_apply_stencil(x.shape[0], _dp(s), _dp(x), _dp(y))
    return y


def restrict_fw(r: np.ndarray) -> np.ndarray:
    r = np.ascontiguousarray(r, dtype=np.float64)
    nc = (r.shape[0] - 1) // 2
    fc = np.empty((nc, nc))
    lib().or_restrict_fw(r.shape[0], _dp(r), _dp(fc))
    return fc


def prolong(vc: np.ndarray) -> np.ndarray:
    vc = np.ascontiguousarray(vc, dtype=np.float64)
    n = 2 * vc.shape[0] + 1
    e = np.empty((n, n))
    lib().or_prolong(vc.shape[0], _dp(vc), _dp(e))
    return e


def galerkin_stencil(s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float64).reshape(9)
    sc = np.zeros(9)
    lib().or_galerkin_stencil(_dp(s), _dp(sc))
    return sc.reshape(3, 3)


def dot2(x: np.ndarray, y: np.ndarray) -> float:
    """Dot2 dot product (Ogita, Rump and Oishi) as every driver computes it."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.ascontiguousarray(y, dtype=np.float64).ravel()
    assert x.size == y.size
    return lib().or_dot2(_dp(x), _dp(y), x.size)


def ir_scale(sumsq: float, npoints: int) -> float:
    return lib().or_ir_scale(sumsq, npoints)


def decode_trace(tr: np.ndarray):
    """[(op, level, counter), ...] from packed trace records."""
    t = tr.astype(np.int64) & 0xFFFFFFFF
    return list(zip((t >> 24).tolist(), ((t >> 16) & 0xFF).tolist(), (t & 0xFFFF).tolist()))


class Hierarchy:
    """Levels of the rotated anisotropic diffusion problem, Galerkin coarsened."""

    def __init__(self, n: int, theta: float, eps: float, n_coarsest: int = 1, omega: float = 0.8,
                 smoother: str = "jacobi", coarsening: str = "full", convection=None):
        """smoother: "jacobi" (damped, omega) or "zebra" (alternating line Gauss-Seidel);
        coarsening "semi": x-line zebra with coarsening along y only (the smoother is then
        always x-line zebra, and `sizes` lists lines per level); convection (bx, by): the
        convection-diffusion operator -div(D grad u) + b . grad u (upwind), damped Jacobi
        and a 1 x 1 coarsest level only."""
        self.n, self.theta, self.eps, self.omega = n, theta, eps, omega
        self.coarsening = coarsening
        h = C.c_void_p()
        if coarsening == "semi":
            rc = lib().or_hier_new_semi(n, theta, eps, C.byref(h))
            smoother = "zebra"
        else:
            rc = lib().or_hier_new(n, theta, eps, n_coarsest, omega, C.byref(h))
        if rc != OK:
            raise ValueError(f"hierarchy construction failed ({rc}) for n={n}, n_coarsest={n_coarsest}")
        self._h = h
        self.smoother = smoother
        if lib().or_set_smoother(h, {"jacobi": 0, "zebra": 1}[smoother]) != OK:
            raise ValueError(f"unknown smoother {smoother}")
        self.convection = None
        if convection is not None:
            bx, by = (float(c) for c in convection)
            if lib().or_set_convection(h, bx, by) != OK:
                raise ValueError("convection needs damped Jacobi, full coarsening and a 1 x 1 coarsest level")
            self.convection = (bx, by)
        nl = C.c_int()
        sizes = (C.c_int * 16)()
        st = np.zeros(16 * 9)
        lib().or_hier_info(h, C.byref(nl), sizes, _dp(st))
        self.levels = nl.value
        self.sizes = [sizes[k] for k in range(self.levels)]
        self.stencils = st[: 9 * self.levels].reshape(self.levels, 3, 3).copy()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().or_hier_free(h)
            self._h = None

    # ---- operators ----
    def apply(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        lib().or_hier_apply(self._h, _dp(x), _dp(y))
        return y

    def zebra_tables(self, level: int, direction: int):
        """(reciprocal pivots, upper multipliers) of level `level` (1-based) for
        x-lines (direction 0) or y-lines (1)."""
        n = self.n if self.coarsening == "semi" else self.sizes[level - 1]
        rp, um = np.zeros(n), np.zeros(n)
        if lib().or_zebra_tables(self._h, level, direction, _dp(rp), _dp(um)) != OK:
            raise ValueError("bad level or direction")
        return rp, um

    def zebra_relax(self, v, f, direction: int):
        """One zebra line relaxation of the fine level (0: x-lines, 1: y-lines); returns the new v."""
        v = np.array(v, dtype=np.float64, order="C", copy=True)
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().or_zebra_relax(self._h, int(direction), _dp(v), _dp(f))
        return v

    # ---- cycles ----
    def cycle(self, v, f, kappa=1, nu1=2, nu2=2, kind=KIND_KAPPA, trace_cap=0):
        """One cycle (Algorithm 3, 1 or 2 by `kind`); returns (v, trace-or-count)."""
        v = np.array(v, dtype=np.float64, order="C", copy=True)
        f = np.ascontiguousarray(f, dtype=np.float64)
        tr = np.zeros(max(trace_cap, 1), dtype=np.int32)
        cnt = lib().or_cycle(self._h, kind, kappa, nu1, nu2, _dp(v), _dp(f),
                             tr.ctypes.data_as(C.POINTER(C.c_int32)), trace_cap)
        if trace_cap:
            if cnt > trace_cap:
                raise RuntimeError("trace buffer too small")
            return v, decode_trace(tr[:cnt])
        return v, cnt

    def trace(self, kappa=1, kind=KIND_KAPPA, nu1=1, nu2=1):
        n = self.n
        cnt = self.cycle(np.zeros((n, n)), np.zeros((n, n)), kappa, nu1, nu2, kind)[1]
        return self.cycle(np.zeros((n, n)), np.zeros((n, n)), kappa, nu1, nu2, kind, trace_cap=cnt)[1]

    def cycle_f32(self, v, f, kappa=1, nu1=2, nu2=2):
        v = np.array(v, dtype=np.float32, order="C", copy=True)
        f = np.ascontiguousarray(f, dtype=np.float32)
        lib().or_kcycle_f32(self._h, kappa, nu1, nu2, _fp(v), _fp(f))
        return v

    # ---- drivers ----
    def solve(self, f, kappa=1, nu1=2, nu2=2, tol=1e-8, maxit=1000, u0=None, mode=0):
        n = self.n
        u = np.zeros((n, n)) if u0 is None else np.array(u0, dtype=np.float64, order="C", copy=True)
        f = np.ascontiguousarray(f, dtype=np.float64)
        hist = np.zeros(maxit + 1)
        it = C.c_int()
        rc = lib().or_solve(self._h, kappa, nu1, nu2, _dp(u), _dp(f), tol, maxit, mode, C.byref(it), _dp(hist))
        return u, rc, it.value, hist[: it.value + 1].copy()

    def ir_solve(self, f, kappa=1, nu1=2, nu2=2, tol=1e-8, maxit=1000, u0=None):
        n = self.n
        u = np.zeros((n, n)) if u0 is None else np.array(u0, dtype=np.float64, order="C", copy=True)
        f = np.ascontiguousarray(f, dtype=np.float64)
        hist = np.zeros(maxit + 1)
        it = C.c_int()
        rc = lib().or_ir_solve(self._h, kappa, nu1, nu2, _dp(u), _dp(f), tol, maxit, C.byref(it), _dp(hist))
        return u, rc, it.value, hist[: it.value + 1].copy()

    def pcg(self, f, kappa=1, nu1=1, nu2=1, tol=1e-8, maxit=500, precond_f32=False):
        n = self.n
        u = np.zeros((n, n))
        f = np.ascontiguousarray(f, dtype=np.float64)
        hist = np.zeros(maxit + 1)
        it = C.c_int()
        rc = lib().or_pcg(self._h, kappa, nu1, nu2, int(bool(precond_f32)), _dp(u), _dp(f), tol, maxit,
                          C.byref(it), _dp(hist))
        return u, rc, it.value, hist[: it.value + 1].copy()

    def grad_params(self, lam, u):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        dth, de = C.c_double(), C.c_double()
        lib().or_grad_params(self._h, self.theta, self.eps, _dp(lam), _dp(u), C.byref(dth), C.byref(de))
        return dth.value, de.value
