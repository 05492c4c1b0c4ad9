"""Run-time model of the kappa-cycle (Section 3) and kappa selection.

Host-side analysis only; it does no multigrid arithmetic.

* ``level_calls`` / ``total_calls``: Proposition 2 and Proposition 3.
* ``f_ops``: the constant of Proposition 5 / Lemma 1, f(kappa, c).
* ``n_ops_2d``: the operation measure of equation (n_ops_2D), N * 2(1 - 3^-kappa).
* ``n_gpu_calls_paper``: launches of the paper's one-kernel-per-operation
  structure (Algorithm 4; the formula row of the notation table).
* ``fit``: least squares for (alpha, beta) in T = alpha * N_gpuCalls + beta * N_ops
  (equations LinearCombination and MinProblem).
* ``turning_point``: the fixed-point iteration of the Appendix for the level
  count where alpha * N_gpuCalls = beta * N_ops (equation equalCosts).
* ``best_kappa``: argmin over kappa of predicted time per cycle times the
  number of cycles (Section 4 shows the trade-off; Section 3 the use of the
  model for choosing kappa).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Iterable, Sequence

import numpy as np

KAPPA_W = 2 ** 31 - 1   # a counter at least the number of levels gives the W-cycle


def level_calls(kappa: int, level: int) -> int:
    """Calls to the cycle routine on level `level` (1 = finest) per cycle."""
    if kappa <= 0:
        return 0
    return sum(math.comb(level - 1, j) for j in range(0, min(kappa - 1, level - 1) + 1))


def total_calls(kappa: int, n: int) -> int:
    """Calls to the cycle routine in one cycle of n levels."""
    if n <= 0:
        return 0
    return sum(math.comb(n, j) for j in range(1, min(kappa, n) + 1))


def f_ops(kappa: float, c: float) -> float:
    """f(kappa, c) of Proposition 5; kappa = inf gives the W-cycle limit."""
    if math.isinf(kappa):
        if c >= 0.5:
            return math.inf
        return 1.0 / (1.0 - 2.0 * c)
    if c == 0.5:
        return 2.0 * kappa
    return (1.0 - (c / (1.0 - c)) ** kappa) / (1.0 - 2.0 * c)


def c_kappa(kappa: float) -> float:
    """C(kappa) = 2 (1 - 3^-kappa), i.e. f(kappa, 1/4)."""
    if math.isinf(kappa) or kappa >= 10 ** 6:
        return 2.0
    return 2.0 * (1.0 - 3.0 ** (-kappa))


def unknowns(n_levels: int) -> int:
    return (2 ** n_levels - 1) ** 2


def n_ops_2d(kappa: float, n_levels: int) -> float:
    return unknowns(n_levels) * c_kappa(kappa)


def n_gpu_calls_paper(kappa: int, n_levels: int, nu: int) -> int:
    """(5 + nu) launches per non-coarsest call and one per coarsest call."""
    k = kappa if kappa < 10 ** 6 else n_levels
    return (5 + nu) * total_calls(k, n_levels - 1) + total_calls(k, n_levels) - total_calls(k, n_levels - 1)


def predict(alpha: float, beta: float, calls: float, ops: float) -> float:
    return alpha * calls + beta * ops


@dataclass
class Fit:
    alpha: float
    beta: float
    rel_errors: dict

    def predict(self, calls: float, ops: float) -> float:
        return predict(self.alpha, self.beta, calls, ops)


def fit(samples: Iterable[tuple], relative: bool = False) -> Fit:
    """Least squares for (alpha, beta) over samples (key, calls, ops, time),
    both constrained to be non-negative (a per-call cost and a per-operation
    cost cannot be negative; with few samples the unconstrained fit can be).
    relative=True minimises the relative errors (each row divided by its
    time), the quantity Table 2 reports, instead of the absolute ones, which
    the largest runs dominate."""
    rows = list(samples)
    M = np.array([[r[1], r[2]] for r in rows], dtype=np.float64)
    t = np.array([r[3] for r in rows], dtype=np.float64)
    if relative:
        M = M / t[:, None]
        t = np.ones_like(t)
    (alpha, beta), *_ = np.linalg.lstsq(M, t, rcond=None)
    if alpha < 0 or beta < 0:
        from scipy.optimize import nnls
        (alpha, beta), _ = nnls(M, t)
    rows_t = np.array([r[3] for r in rows], dtype=np.float64)
    if relative:
        M = M * rows_t[:, None]
    errs = {r[0]: (predict(alpha, beta, r[1], r[2]) - r[3]) / r[3] for r in rows}
    return Fit(float(alpha), float(beta), errs)


def turning_point(alpha: float, beta: float, kappa: float, calls_fn: Callable[[float], float],
                  iterations: int = 20, n0: float = 2.0) -> float:
    """Appendix: iterate n <- log2(1 + sqrt((alpha/beta) * N_gpuCalls(n) / C(kappa)))
    from n = 2; calls_fn gives N_gpuCalls at the current (real) n."""
    n = n0
    for _ in range(iterations):
        calls = calls_fn(n)
        n = math.log2(1.0 + math.sqrt((alpha / beta) * calls / c_kappa(kappa)))
    return n


def total_calls_real(kappa: float, x: float) -> float:
    """totalCalls continued to a real level count x: the degree-kappa
    polynomial sum_{j=1..kappa} C(x, j) of Corollary 2 for finite kappa, and
    2^x - 1 for the W-cycle."""
    if math.isinf(kappa) or kappa >= 10 ** 6:
        return 2.0 ** x - 1.0
    acc = 0.0
    for j in range(1, int(kappa) + 1):
        p = 1.0
        for i in range(j):
            p *= (x - i)
        acc += p / math.factorial(j)
    return acc


def paper_turning_point(alpha: float, beta: float, kappa: float, launches_per_call: int) -> float:
    """Unrounded turning point (Table 1) with the paper's launch count:
    N_gpuCalls(x) = (5+nu) totalCalls(x-1) + totalCalls(x) - totalCalls(x-1),
    launches_per_call = 5 + nu, totalCalls continued to real x."""
    def calls(x: float) -> float:
        a, b = total_calls_real(kappa, x - 1.0), total_calls_real(kappa, x)
        return launches_per_call * a + b - a
    return turning_point(alpha, beta, kappa, calls)


def best_kappa(kappas: Sequence[int], time_per_cycle: Callable[[int], float],
               cycles: Callable[[int], float]) -> tuple:
    """argmin over kappa of time_per_cycle(kappa) * cycles(kappa)."""
    totals = {k: time_per_cycle(k) * cycles(k) for k in kappas}
    k = min(totals, key=totals.get)
    return k, totals


def cycles_from_rate(rate: float, tol: float) -> float:
    """Cycles to reduce the residual by `tol` at asymptotic factor `rate`."""
    if rate <= 0.0:
        return 1.0
    if rate >= 1.0:
        return math.inf
    return math.log(tol) / math.log(rate)
