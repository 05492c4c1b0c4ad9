"""ctypes binding of libkcycle.so (C-ABI declared in include/kcycle.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (the workspace and the user's tensors) and the
stream.  There is no CPU fallback: if the library is missing, or no GPU is
visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KC_LIBRARY") or os.path.join(_HERE, "libkcycle.so")   # KC_LIBRARY: another build of it

KC_OK, KC_NOT_CONVERGED, KC_DIVERGED, KC_BREAKDOWN = 0, 1, 2, 3
KC_ERR_ARG, KC_ERR_HIP, KC_ERR_WORKSPACE, KC_ERR_NONFINITE, KC_ERR_STATE = -1, -2, -3, -4, -5
KC_F64, KC_F32_CYCLE = 0, 1
KAPPA_W = 2 ** 31 - 1

STATUS_NAMES = {KC_OK: "ok", KC_NOT_CONVERGED: "not_converged", KC_DIVERGED: "diverged",
                KC_BREAKDOWN: "breakdown", KC_ERR_ARG: "err_arg", KC_ERR_HIP: "err_hip",
                KC_ERR_WORKSPACE: "err_workspace", KC_ERR_NONFINITE: "err_nonfinite",
                KC_ERR_STATE: "err_state"}


class KCycleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_coarsest", C.c_int32), ("theta", C.c_double), ("eps", C.c_double)]


SMOOTHERS = {"jacobi": 0, "zebra": 1}   # damped Jacobi; alternating zebra line Gauss-Seidel


class CycleParams(C.Structure):
    _fields_ = [("kappa", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32), ("smoother", C.c_int32),
                ("omega", C.c_double)]


class Exec(C.Structure):
    _fields_ = [("mode", C.c_int32), ("use_graph", C.c_int32), ("coarse_cutover", C.c_int32),
                ("coarse_threads", C.c_int32), ("poll_every", C.c_int32), ("coarse_wave_n", C.c_int32),
                ("small_tile_n", C.c_int32), ("stream_n", C.c_int32),
                ("wave_regs", C.c_int32), ("fuse_junctions", C.c_int32), ("mid_tile_n", C.c_int32),
                ("tiny_tile_n", C.c_int32),
                ("zebra_wave_n", C.c_int32), ("zebra_quad_n", C.c_int32)]


_lib = None


def lib():
    """Load libkcycle.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2010_00626_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
        P = C.POINTER
        L.kc_exec_default.argtypes = [P(Exec)]
        L.kc_exec_default.restype = None
        L.kc_workspace_bytes.argtypes = [P(Problem), i32, i32, P(sz)]
        L.kc_create.argtypes = [P(Problem), i32, i32, P(Exec), vp, sz, vp, P(vp)]
        L.kc_workspace_bytes_semi.argtypes = [P(Problem), i32, i32, P(sz)]
        L.kc_create_semi.argtypes = [P(Problem), i32, i32, P(Exec), vp, sz, vp, P(vp)]
        L.kc_semi_stencils.argtypes = [P(Problem), i32, P(i32), P(dbl)]
        L.kc_destroy.argtypes = [vp]
        L.kc_set_exec.argtypes = [vp, P(Exec)]
        arr = [vp, P(vp), P(i64), P(vp), P(i64)]
        L.kc_cycle.argtypes = arr + [P(CycleParams)]
        L.kc_solve.argtypes = arr + [P(CycleParams), dbl, i32, P(i32), P(dbl), P(i32)]
        L.kc_pcg.argtypes = arr + [P(CycleParams), dbl, i32, P(i32), P(dbl), P(i32)]
        L.kc_apply_A.argtypes = arr
        L.kc_residual_history.argtypes = [vp, i32, P(dbl), i32, P(i32)]
        L.kc_grad_params.argtypes = arr + [P(dbl), P(dbl)]
        L.kc_grad_params_noalloc.argtypes = [P(Problem), i32, P(vp), P(i64), P(vp), P(i64), vp, P(dbl), P(dbl)]
        L.kc_level_stencils.argtypes = [P(Problem), i32, P(i32), P(dbl)]
        L.kc_convection_stencils.argtypes = [P(Problem), dbl, dbl, i32, P(i32), P(dbl)]
        L.kc_set_convection.argtypes = [vp, P(dbl), P(dbl)]
        L.kc_schedule_counts.argtypes = [P(Problem), i32, P(Exec), P(CycleParams), P(i64), P(i64), P(i64)]
        L.kc_stats.argtypes = [vp, C.c_char_p, sz]
        L.kc_profile_iteration.argtypes = [vp, i32, P(CycleParams), i32, C.c_char_p, sz]
        L.kc_time_stage.argtypes = [vp, i32, P(CycleParams), i32, P(dbl), P(dbl)]
        L.kc_time_cycles.argtypes = arr + [P(CycleParams), i32, P(dbl)]
        L.kc_status_string.argtypes = [i32]
        L.kc_status_string.restype = C.c_char_p
        L.kc_last_error.argtypes = []
        L.kc_last_error.restype = C.c_char_p
        for name in ("kc_workspace_bytes", "kc_create", "kc_destroy", "kc_set_exec", "kc_cycle", "kc_solve",
                     "kc_pcg", "kc_apply_A", "kc_residual_history", "kc_grad_params", "kc_level_stencils", "kc_schedule_counts",
                     "kc_stats", "kc_time_stage", "kc_time_cycles", "kc_profile_iteration", "kc_grad_params_noalloc",
                     "kc_convection_stencils", "kc_set_convection", "kc_workspace_bytes_semi", "kc_create_semi",
                     "kc_semi_stencils"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(status: int, allow_positive: bool = False) -> int:
    if status < 0 or (status > 0 and not allow_positive):
        raise KCycleError(status, lib().kc_last_error().decode())
    return status


def exec_options(mode: int | str = 0, use_graph: bool = True, coarse_cutover: int = 31,
                 coarse_threads: int = 512, poll_every: int = 0, coarse_wave_n: int = 15,
                 small_tile_n: int = 511, stream_n: int = 2047, wave_regs: int = 1,
                 fuse_junctions: int = 1, mid_tile_n: int = 2047, tiny_tile_n: int = 255,
                 zebra_wave_n: int = 63, zebra_quad_n: int = 8191) -> Exec:
    e = Exec()
    lib().kc_exec_default(C.byref(e))
    e.mode = {"fused": 0, "paper": 1}.get(mode, mode) if isinstance(mode, str) else int(mode)
    e.use_graph = int(bool(use_graph))
    e.coarse_cutover = int(coarse_cutover)
    e.coarse_threads = int(coarse_threads)
    e.poll_every = int(poll_every)
    e.coarse_wave_n = int(coarse_wave_n)
    e.small_tile_n = int(small_tile_n)
    e.stream_n = int(stream_n)
    e.wave_regs = int(wave_regs)
    e.fuse_junctions = int(fuse_junctions)
    e.mid_tile_n = int(mid_tile_n)
    e.tiny_tile_n = int(tiny_tile_n)
    e.zebra_wave_n = int(zebra_wave_n)
    e.zebra_quad_n = int(zebra_quad_n)
    return e


def _problems(problems) -> tuple:
    items = []
    for p in problems:
        if isinstance(p, Problem):
            items.append(p)
            continue
        if isinstance(p, dict):
            n, th, ep, nc = p["n"], p["theta"], p["eps"], p.get("n_coarsest", 1)
        else:
            n, th, ep = p[0], p[1], p[2]
            nc = p[3] if len(p) > 3 else 1
        items.append(Problem(int(n), int(nc), float(th), float(ep)))
    arr = (Problem * len(items))(*items)
    return arr, len(items)


def _precision(p) -> int:
    return {"f64": KC_F64, "f32": KC_F32_CYCLE, "f32_cycle": KC_F32_CYCLE}.get(p, p) if isinstance(p, str) else int(p)


def workspace_bytes(problems, precision="f64", coarsening="full") -> int:
    arr, n = _problems(problems)
    out = C.c_size_t()
    fn = lib().kc_workspace_bytes_semi if coarsening == "semi" else lib().kc_workspace_bytes
    _check(fn(arr, n, _precision(precision), C.byref(out)))
    return out.value


def semi_stencils(n: int, theta: float, eps: float) -> np.ndarray:
    """Stencils of every semi-coarsened level (units of the fine h^2; host computation, no GPU)."""
    p = Problem(n, 1, theta, eps)
    nl = C.c_int32()
    buf = np.zeros(16 * 9)
    _check(lib().kc_semi_stencils(C.byref(p), 16, C.byref(nl), buf.ctypes.data_as(C.POINTER(C.c_double))))
    return buf[: 9 * nl.value].reshape(nl.value, 3, 3).copy()


def level_stencils(n: int, theta: float, eps: float, n_coarsest: int = 1) -> np.ndarray:
    """h^2-scaled 3x3 stencils of every level (host computation, no GPU)."""
    p = Problem(n, n_coarsest, theta, eps)
    nl = C.c_int32()
    buf = np.zeros(16 * 9)
    _check(lib().kc_level_stencils(C.byref(p), 16, C.byref(nl), buf.ctypes.data_as(C.POINTER(C.c_double))))
    return buf[: 9 * nl.value].reshape(nl.value, 3, 3).copy()


def convection_stencils(n: int, theta: float, eps: float, bx: float, by: float) -> np.ndarray:
    """h^2-scaled stencils of every level of the convection-diffusion problem (host, no GPU)."""
    p = Problem(n, 1, theta, eps)
    nl = C.c_int32()
    buf = np.zeros(16 * 9)
    _check(lib().kc_convection_stencils(C.byref(p), float(bx), float(by), 16, C.byref(nl),
                                        buf.ctypes.data_as(C.POINTER(C.c_double))))
    return buf[: 9 * nl.value].reshape(nl.value, 3, 3).copy()


def schedule_counts(problems, kappa: int, nu1: int = 2, nu2: int = 2, omega: float = 0.8, smoother: str = "jacobi",
                    **exec_kw) -> dict:
    """Launches per cycle of the flattened schedule (host computation, no GPU)."""
    arr, n = _problems(problems)
    e = exec_options(**exec_kw)
    sm = SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
    c = CycleParams(int(kappa), int(nu1), int(nu2), sm, float(omega))
    g, s, st = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().kc_schedule_counts(arr, n, C.byref(e), C.byref(c), C.byref(g), C.byref(s), C.byref(st)))
    return {"grid_launches": g.value, "subtree_launches": s.value, "subtree_stages": st.value}


def _device_arrays(xs, sizes, what: str):
    """host arrays of device pointers and leading dimensions of FP64 tensors"""
    import torch
    if isinstance(xs, torch.Tensor):
        xs = [xs]
    xs = list(xs)
    if len(xs) != len(sizes):
        raise ValueError(f"{what}: expected {len(sizes)} tensors, got {len(xs)}")
    ptrs = (C.c_void_p * len(xs))()
    lds = (C.c_int64 * len(xs))()
    for i, (t, n) in enumerate(zip(xs, sizes)):
        if t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{what}[{i}] must be a float64 GPU tensor")
        if t.dim() != 2 or t.shape[0] != n or t.shape[1] != n or t.stride(1) != 1 or t.stride(0) < n:
            raise ValueError(f"{what}[{i}] must be a row-major ({n}, {n}) tensor")
        ptrs[i] = t.data_ptr()
        lds[i] = t.stride(0)
    return ptrs, lds


def grad_params_noalloc(problems, lam, u, stream=None):
    """kc_grad_params_noalloc: the gradient inner products of
    Hierarchy.grad_params without a hierarchy or workspace (the library keeps
    its tables and partial sums in a static device array).  Runs on the
    current device and stream unless `stream` is given."""
    import torch
    arr, count = _problems(problems)
    sizes = [arr[i].n for i in range(count)]
    pl, ll = _device_arrays(lam, sizes, "lam")
    pu, lu = _device_arrays(u, sizes, "u")
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    dth = (C.c_double * count)()
    de = (C.c_double * count)()
    _check(lib().kc_grad_params_noalloc(arr, count, pl, ll, pu, lu, handle, dth, de))
    return list(dth), list(de)


class Hierarchy:
    """A batch of problem instances resident on one GPU.

    problems: iterable of (n, theta, eps[, n_coarsest]) or dicts.
    precision: "f64" or "f32" (FP32 cycles, FP64 refinement / CG).
    """

    def __init__(self, problems: Iterable, precision="f64", exec=None, device=None, stream=None, coarsening="full"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the kappa-cycle library runs on the GPU only")
        self._torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._probs, self.count = _problems(problems)
        self.sizes = [self._probs[i].n for i in range(self.count)]
        self.precision = _precision(precision)
        if coarsening not in ("full", "semi"):
            raise ValueError("coarsening must be 'full' or 'semi' (x-line zebra, coarsening along y)")
        self.coarsening = coarsening
        nbytes = workspace_bytes(list(self._probs), self.precision, coarsening)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        handle = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._e = exec if isinstance(exec, Exec) else exec_options(**(exec or {}))
        h = C.c_void_p()
        create = lib().kc_create_semi if coarsening == "semi" else lib().kc_create
        _check(create(self._probs, self.count, self.precision, C.byref(self._e), C.c_void_p(aligned),
                      nbytes, handle, C.byref(h)))
        self._h = h

    # ---- helpers ----
    def _arrays(self, xs, what: str):
        torch = self._torch
        if isinstance(xs, torch.Tensor):
            xs = [xs]
        xs = list(xs)
        if len(xs) != self.count:
            raise ValueError(f"{what}: expected {self.count} tensors, got {len(xs)}")
        ptrs = (C.c_void_p * self.count)()
        lds = (C.c_int64 * self.count)()
        for i, t in enumerate(xs):
            n = self.sizes[i]
            if t.dtype != torch.float64:
                raise TypeError(f"{what}[{i}] must be float64")
            if t.device != self.device:
                raise ValueError(f"{what}[{i}] must live on {self.device}")
            if t.dim() != 2 or t.shape[0] != n or t.shape[1] != n or t.stride(1) != 1 or t.stride(0) < n:
                raise ValueError(f"{what}[{i}] must be a row-major ({n}, {n}) tensor")
            ptrs[i] = t.data_ptr()
            lds[i] = t.stride(0)
        return ptrs, lds

    def _params(self, kappa, nu1, nu2, omega, smoother="jacobi"):
        sm = SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
        return CycleParams(int(kappa), int(nu1), int(nu2), sm, float(omega))

    # ---- entry points ----
    def cycle(self, v, f, kappa=1, nu1=2, nu2=2, omega=0.8, smoother="jacobi"):
        """One kappa-cycle in place on v (FP64 hierarchies)."""
        pv, lv = self._arrays(v, "v")
        pf, lf = self._arrays(f, "f")
        c = self._params(kappa, nu1, nu2, omega, smoother)
        _check(lib().kc_cycle(self._h, pv, lv, pf, lf, C.byref(c)))

    def _solver(self, fn, u, f, kappa, nu1, nu2, omega, tol, maxit, smoother="jacobi"):
        pu, lu = self._arrays(u, "u")
        pf, lf = self._arrays(f, "f")
        c = self._params(kappa, nu1, nu2, omega, smoother)
        it = (C.c_int32 * self.count)()
        rr = (C.c_double * self.count)()
        st = (C.c_int32 * self.count)()
        rc = fn(self._h, pu, lu, pf, lf, C.byref(c), float(tol), int(maxit), it, rr, st)
        if rc < 0 and all(st[i] >= 0 for i in range(self.count)):
            _check(rc)
        return list(it), list(rr), list(st)

    def solve(self, u, f, kappa=1, nu1=2, nu2=2, omega=0.8, tol=1e-8, maxit=1000, smoother="jacobi"):
        """Stand-alone kappa-cycles until ||f - A u|| / ||f|| < tol; returns (iters, relres, status)."""
        return self._solver(lib().kc_solve, u, f, kappa, nu1, nu2, omega, tol, maxit, smoother)

    def pcg(self, u, f, kappa=1, nu1=1, nu2=1, omega=0.8, tol=1e-8, maxit=500, smoother="jacobi"):
        """CG preconditioned by one kappa-cycle per iteration; returns (iters, relres, status)."""
        return self._solver(lib().kc_pcg, u, f, kappa, nu1, nu2, omega, tol, maxit, smoother)

    def residual_history(self, instance: int = 0) -> list:
        """Relative residuals of the last solve / pcg of one instance, entry k
        after k cycles or CG iterations (the first 8192 are kept)."""
        n = C.c_int32()
        _check(lib().kc_residual_history(self._h, int(instance), None, 0, C.byref(n)))
        buf = (C.c_double * max(n.value, 1))()
        _check(lib().kc_residual_history(self._h, int(instance), buf, n.value, C.byref(n)))
        return list(buf[: n.value])

    def apply_A(self, y, x):
        py, ly = self._arrays(y, "y")
        px, lx = self._arrays(x, "x")
        _check(lib().kc_apply_A(self._h, py, ly, px, lx))

    def grad_params(self, lam, u):
        pl, ll = self._arrays(lam, "lam")
        pu, lu = self._arrays(u, "u")
        dth = (C.c_double * self.count)()
        de = (C.c_double * self.count)()
        _check(lib().kc_grad_params(self._h, pl, ll, pu, lu, dth, de))
        return list(dth), list(de)

    def set_convection(self, bx, by):
        """Switch every instance to -div(D grad u) + b . grad u (upwind convection,
        rediscretised levels); bx, by: one value for all instances or one per instance."""
        bxs = [float(bx)] * self.count if np.isscalar(bx) else [float(x) for x in bx]
        bys = [float(by)] * self.count if np.isscalar(by) else [float(x) for x in by]
        if len(bxs) != self.count or len(bys) != self.count:
            raise ValueError(f"expected {self.count} velocities")
        _check(lib().kc_set_convection(self._h, (C.c_double * self.count)(*bxs), (C.c_double * self.count)(*bys)))

    def set_exec(self, **kw):
        e = exec_options(**kw)
        _check(lib().kc_set_exec(self._h, C.byref(e)))
        self._e = e

    def time_stage(self, which: int, kappa=3, nu1=2, nu2=2, omega=0.8, reps=50, smoother="jacobi"):
        """Average ms of one launch of a schedule stage and its algorithmic bytes."""
        c = self._params(kappa, nu1, nu2, omega, smoother)
        ms, b = C.c_double(), C.c_double()
        _check(lib().kc_time_stage(self._h, int(which), C.byref(c), int(reps), C.byref(ms), C.byref(b)))
        return ms.value, b.value

    def time_cycles(self, v, f, kappa=1, nu1=2, nu2=2, omega=0.8, reps=10, smoother="jacobi"):
        """Milliseconds per kappa-cycle over `reps` back-to-back cycles (FP64)."""
        pv, lv = self._arrays(v, "v")
        pf, lf = self._arrays(f, "f")
        c = self._params(kappa, nu1, nu2, omega, smoother)
        ms = C.c_double()
        _check(lib().kc_time_cycles(self._h, pv, lv, pf, lf, C.byref(c), int(reps), C.byref(ms)))
        return ms.value

    def profile_iteration(self, driver: str = "solve", kappa=1, nu1=2, nu2=2, omega=0.8, reps=5,
                          smoother="jacobi") -> dict:
        """Per-kernel times of one solver iteration ("solve" or "pcg"; that
        driver must have run last on this hierarchy, whose arrays keep iterating)."""
        c = self._params(kappa, nu1, nu2, omega, smoother)
        buf = C.create_string_buffer(1 << 20)
        _check(lib().kc_profile_iteration(self._h, 1 if driver == "pcg" else 0, C.byref(c), int(reps), buf, len(buf)))
        return json.loads(buf.value.decode())

    def stats(self) -> dict:
        buf = C.create_string_buffer(1 << 16)
        _check(lib().kc_stats(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().kc_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
