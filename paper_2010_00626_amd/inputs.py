"""Seeded synthetic inputs for the five workloads of the kappa-cycle solver.

This module only draws random numbers and samples right-hand sides; it holds
none of the method's arithmetic.  Both the GPU library's callers (tests,
benchmark) and the oracle-side tests take their inputs from here.

Grid convention: an (n, n) array, row j along +y, column i along +x, interior
points x = (i+1) h, y = (j+1) h with h = 1/(n+1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Instance:
    n: int
    theta: float
    eps: float
    f: np.ndarray


@dataclass
class Workload:
    name: str
    instances: list
    kappas: tuple
    nu1: int
    nu2: int
    omega: float
    tol: float
    n_coarsest: int = 1
    solver: str = "standalone"          # "standalone" or "pcg"
    precision: str = "f64"              # "f64" or "f32" (FP32 cycle, FP64 refinement)
    notes: dict = field(default_factory=dict)

    @property
    def unknowns(self) -> int:
        return int(sum(inst.n * inst.n for inst in self.instances))


def uniform_rhs(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, (n, n))


def gaussian_sum_rhs(seed: int, n: int, count: int = 32, width: float = 0.05) -> np.ndarray:
    """Sum of `count` Gaussians exp(-|x-c|^2 / (2 width^2)) with centres
    U[0,1]^2 and amplitudes U[-1,1], drawn in that order."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (count, 2))
    amps = rng.uniform(-1.0, 1.0, count)
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    f = np.zeros((n, n))
    for (cx, cy), a in zip(centres, amps):
        gx = np.exp(-((x - cx) ** 2) / (2 * width * width))
        gy = np.exp(-((x - cy) ** 2) / (2 * width * width))
        f += a * np.outer(gy, gx)
    return f


def config1() -> Workload:
    """63x63, theta=pi/4, eps=1e-3, 5 levels down to 3x3, V-cycle, tol 1e-10."""
    rng = np.random.default_rng(0)
    f = uniform_rhs(rng, 63)
    return Workload("c1_63_v", [Instance(63, math.pi / 4, 1e-3, f)], (1,), 2, 2, 0.8, 1e-10,
                    n_coarsest=3)


def config2(n: int = 1023) -> Workload:
    """1023x1023, theta=pi/6, eps=1e-4, 10 levels to 1x1, kappa sweep, tol 1e-8."""
    rng = np.random.default_rng(1)
    f = uniform_rhs(rng, n)
    return Workload(f"c2_{n}_sweep", [Instance(n, math.pi / 6, 1e-4, f)], (1, 2, 3, 4, 6, 10), 2, 2, 0.8, 1e-8)


def config3(n: int = 4095) -> Workload:
    """4095x4095, theta=3pi/8, eps=1e-5, PCG with nu=1+1, Gaussian-sum f (seed 5)."""
    f = gaussian_sum_rhs(5, n)
    return Workload(f"c3_{n}_pcg", [Instance(n, 3 * math.pi / 8, 1e-5, f)], (1, 2, 3, 4), 1, 1, 0.8, 1e-8,
                    solver="pcg", precision="f32")


def config4(count: int = 64, sizes=(255, 511, 1023, 2047), weights=(8, 4, 2, 1)) -> Workload:
    """64 instances of uneven size, theta~U[0,pi), eps~logU[1e-5,1e-1], kappa=3."""
    rng = np.random.default_rng(2)
    p = np.asarray(weights, dtype=np.float64)
    p = p / p.sum()
    ns = rng.choice(np.asarray(sizes), count, p=p)
    thetas = rng.uniform(0.0, math.pi, count)
    epss = 10.0 ** rng.uniform(-5.0, -1.0, count)
    inst = [Instance(int(n), float(t), float(e), uniform_rhs(rng, int(n))) for n, t, e in zip(ns, thetas, epss)]
    return Workload(f"c4_batched_{count}", inst, (3,), 2, 2, 0.8, 1e-8, precision="f32")


def config5(count: int = 16, n: int = 1023) -> Workload:
    """16 instances of 1023x1023, theta~U[0,pi), eps~logU[1e-4,1e-1], kappa=3 PCG."""
    rng = np.random.default_rng(3)
    thetas = rng.uniform(0.0, math.pi, count)
    epss = 10.0 ** rng.uniform(-4.0, -1.0, count)
    inst = [Instance(n, float(t), float(e), uniform_rhs(rng, n)) for t, e in zip(thetas, epss)]
    return Workload(f"c5_adjoint_{count}", inst, (3,), 1, 1, 0.8, 1e-8, solver="pcg")


def small_instance(n: int, seed: int, theta: float | None = None, eps: float | None = None) -> Instance:
    """A reduced instance of the same recipe for tests that must finish quickly."""
    rng = np.random.default_rng(seed)
    if theta is None:
        theta = float(rng.uniform(0.0, math.pi))
    if eps is None:
        eps = float(10.0 ** rng.uniform(-5.0, 0.0))
    return Instance(n, theta, eps, uniform_rhs(rng, n))
