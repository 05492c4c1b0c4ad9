"""Differentiable kappa-cycle solves: u = A(theta, eps)^{-1} f as a
torch.autograd.Function.

Forward solves A u = f with CG preconditioned by one kappa-cycle per
iteration.  Backward recomputes u (no iterate is stored), solves the adjoint
system A lam = dL/du with the same preconditioned CG (A is symmetric, so the
adjoint is A itself) and returns

    dL/df = lam,   dL/dtheta = -lam^T (dA/dtheta) u,   dL/deps = -lam^T (dA/deps) u,

the last two from one fused GPU reduction over lam and u (derivative stencils
of the Section 4 nine-point operator).  This is the gradient of the exact
solution map; the coarse levels only accelerate the solves and do not enter.
All arithmetic runs in the HIP library; this module only marshals tensors.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import kcycle


@dataclass
class SolveConfig:
    kappa: int = 3
    nu1: int = 1
    nu2: int = 1
    omega: float = 0.8
    tol: float = 1e-8            # forward relative residual
    tol_adjoint: float = 1e-8    # adjoint relative residual
    maxit: int = 2000
    precision: str = "f64"
    n_coarsest: int = 1
    cache: dict = field(default_factory=dict, repr=False)

    def hierarchy(self, n: int, thetas, epss) -> "kcycle.Hierarchy":
        key = (n, tuple(float(t) for t in thetas), tuple(float(e) for e in epss), self.precision)
        H = self.cache.get(key)
        if H is None:
            if len(self.cache) > 8:
                self.cache.clear()
            H = kcycle.Hierarchy([(n, t, e, self.n_coarsest) for t, e in zip(key[1], key[2])], self.precision)
            self.cache[key] = H
        return H

    def solve(self, H, rhs: torch.Tensor, tol: float) -> torch.Tensor:
        u = torch.zeros_like(rhs)
        it, rr, st = H.pcg(list(u), list(rhs), kappa=self.kappa, nu1=self.nu1, nu2=self.nu2, omega=self.omega,
                           tol=tol, maxit=self.maxit)
        bad = [(i, s) for i, s in enumerate(st) if s != kcycle.KC_OK]
        if bad:
            raise kcycle.KCycleError(bad[0][1], f"instance {bad[0][0]} did not reach tol={tol}: "
                                     f"relres={rr[bad[0][0]]:.3e} after {it[bad[0][0]]} iterations")
        return u


def _params(x, B, device):
    t = torch.as_tensor(x, dtype=torch.float64)
    if t.dim() == 0:
        t = t.expand(B)
    return t.detach().to("cpu"), t


class KCycleSolve(torch.autograd.Function):
    """u = KCycleSolve.apply(f, theta, eps, cfg) for f of shape (B, n, n)
    (float64, on the GPU) and theta, eps of shape (B,)."""

    @staticmethod
    def forward(ctx, f, theta, eps, cfg: SolveConfig):
        if f.dim() != 3 or f.shape[1] != f.shape[2] or f.dtype != torch.float64 or not f.is_cuda:
            raise ValueError("f must be a float64 CUDA tensor of shape (B, n, n)")
        B, n = f.shape[0], f.shape[1]
        th, _ = _params(theta, B, f.device)
        ep, _ = _params(eps, B, f.device)
        H = cfg.hierarchy(n, th.tolist(), ep.tolist())
        u = cfg.solve(H, f.contiguous(), cfg.tol)
        ctx.save_for_backward(f, th, ep)      # recompute u in backward: no iterate is kept
        ctx.cfg = cfg
        ctx.theta_shape = torch.as_tensor(theta).shape
        ctx.eps_shape = torch.as_tensor(eps).shape
        ctx.theta_device = theta.device if torch.is_tensor(theta) else torch.device("cpu")
        ctx.eps_device = eps.device if torch.is_tensor(eps) else torch.device("cpu")
        ctx.param_is_tensor = (torch.is_tensor(theta), torch.is_tensor(eps))
        return u

    @staticmethod
    def backward(ctx, gu):
        f, th, ep = ctx.saved_tensors
        cfg = ctx.cfg
        want_f, want_th, want_ep = wanted_grads(ctx)
        if not (want_f or want_th or want_ep):
            return None, None, None, None
        n = f.shape[1]
        H = cfg.hierarchy(n, th.tolist(), ep.tolist())
        lam = cfg.solve(H, gu.contiguous(), cfg.tol_adjoint)
        dth = de = None
        if want_th or want_ep:
            u = cfg.solve(H, f.contiguous(), cfg.tol)   # recomputed: no forward iterate is kept
            dth, de = H.grad_params(list(lam), list(u))
        return assemble_grads(ctx, lam, dth, de)


def wanted_grads(ctx):
    """(dL/df, dL/dtheta, dL/deps) wanted: a parameter given as a Python
    number is not a graph input and takes no gradient."""
    th_t, ep_t = ctx.param_is_tensor
    return (bool(ctx.needs_input_grad[0]), bool(ctx.needs_input_grad[1]) and th_t,
            bool(ctx.needs_input_grad[2]) and ep_t)


def assemble_grads(ctx, lam, dth, de):
    """backward's return tuple: None for every input that takes no gradient,
    parameter gradients summed for a scalar parameter and placed on its device."""
    want_f, want_th, want_ep = wanted_grads(ctx)
    gth = gep = None
    if want_th:
        gth = torch.tensor(dth, dtype=torch.float64)
        if len(ctx.theta_shape) == 0:
            gth = gth.sum()
        gth = gth.to(ctx.theta_device)
    if want_ep:
        gep = torch.tensor(de, dtype=torch.float64)
        if len(ctx.eps_shape) == 0:
            gep = gep.sum()
        gep = gep.to(ctx.eps_device)
    return (lam if want_f else None), gth, gep, None


def solve(f, theta, eps, cfg: SolveConfig | None = None):
    """Differentiable batched solve (see KCycleSolve)."""
    return KCycleSolve.apply(f, theta, eps, cfg or SolveConfig())
