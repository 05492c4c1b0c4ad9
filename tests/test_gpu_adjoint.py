"""GPU checks of the adjoint backward (torch.autograd) against the oracle's
gradient and against central finite differences.

Loss L = 1/2 ||u - u*||^2 with u = A(theta, eps)^{-1} f and u* the solution
for (theta + 0.1, 2 eps) and the same f (held constant).  Finite differences
use step 1e-6 for theta and a relative step 1e-4 for eps, with forward and
adjoint solves converged to 1e-12 on the true FP64 residual (PCG confirms
convergence on f - A u; the attainable floor of these problems is 5e-13 to
9e-13 at 127^2 and up to 2.4e-12 at 255^2): with eps near 1e-4 a relative
step of 1e-6 makes the difference quotient carry the solver tolerance (about
1e-12 / 1e-10 relative), while the central-difference truncation error at
1e-4 is ~1e-8."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2010_00626_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def batch(n, count, seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, math.pi, count)
    ep = 10.0 ** rng.uniform(-4.0, -1.0, count)
    fs = np.stack([inputs.uniform_rhs(rng, n) for _ in range(count)])
    return th, ep, fs


def loss_fn(ag, cfg, f, th, ep, target):
    u = ag.solve(f, th, ep, cfg)
    return 0.5 * ((u - target) ** 2).sum()


def test_adjoint_matches_oracle_and_fd():
    from paper_2010_00626_amd import autograd as ag
    n, count = 127, 3
    print("[gpu-adjoint] n=127 batch=3", flush=True)
    th, ep, fs = batch(n, count, 3)
    cfg = ag.SolveConfig(kappa=3, nu1=1, nu2=1, tol=1e-12, tol_adjoint=1e-12, maxit=500)
    f = torch.from_numpy(fs).cuda()
    with torch.no_grad():
        target = ag.solve(f, torch.tensor(th + 0.1), torch.tensor(2 * ep), cfg)
    tht = torch.tensor(th, requires_grad=True)
    ept = torch.tensor(ep, requires_grad=True)
    fr = f.clone().requires_grad_(True)
    L = loss_fn(ag, cfg, fr, tht, ept, target)
    L.backward()
    gth, gep, gf = tht.grad.numpy(), ept.grad.numpy(), fr.grad.cpu().numpy()

    # oracle gradient: u, u*, lam by the oracle's PCG at 1e-12, then its inner products
    for k in range(count):
        H = O.Hierarchy(n, th[k], ep[k])
        Hs = O.Hierarchy(n, th[k] + 0.1, 2 * ep[k])
        u, rc, _, _ = H.pcg(fs[k], kappa=3, tol=1e-12, maxit=500)
        us, rc2, _, _ = Hs.pcg(fs[k], kappa=3, tol=1e-12, maxit=500)
        lam, rc3, _, _ = H.pcg(u - us, kappa=3, tol=1e-12, maxit=500)
        assert rc == rc2 == rc3 == O.OK
        ot, oe = H.grad_params(lam, u)
        assert abs(gth[k] - ot) <= 1e-8 * abs(ot) + 1e-14, (k, gth[k], ot)
        assert abs(gep[k] - oe) <= 1e-8 * abs(oe) + 1e-14, (k, gep[k], oe)
        assert np.abs(gf[k] - lam).max() <= 1e-8 * np.abs(lam).max()

    # central finite differences of the GPU loss
    with torch.no_grad():
        for k in range(count):
            d = 1e-6
            tp, tm = th.copy(), th.copy()
            tp[k] += d
            tm[k] -= d
            fd = (loss_fn(ag, cfg, f, torch.tensor(tp), torch.tensor(ep), target)
                  - loss_fn(ag, cfg, f, torch.tensor(tm), torch.tensor(ep), target)).item() / (2 * d)
            assert abs(fd - gth[k]) <= 1e-5 * abs(gth[k]) + 1e-12, (k, fd, gth[k])
            de = 1e-4 * ep[k]
            ep_p, ep_m = ep.copy(), ep.copy()
            ep_p[k] += de
            ep_m[k] -= de
            fd = (loss_fn(ag, cfg, f, torch.tensor(th), torch.tensor(ep_p), target)
                  - loss_fn(ag, cfg, f, torch.tensor(th), torch.tensor(ep_m), target)).item() / (2 * de)
            assert abs(fd - gep[k]) <= 1e-5 * abs(gep[k]) + 1e-12, (k, fd, gep[k])
        # dL/df along a random direction
        w = torch.from_numpy(np.random.default_rng(9).uniform(-1, 1, fs.shape)).cuda()
        dlt = 1e-4
        fd = (loss_fn(ag, cfg, f + dlt * w, torch.tensor(th), torch.tensor(ep), target)
              - loss_fn(ag, cfg, f - dlt * w, torch.tensor(th), torch.tensor(ep), target)).item() / (2 * dlt)
        an = float((torch.from_numpy(gf).cuda() * w).sum())
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_adjoint_tolerance_1e8_error_is_reported_small():
    """At the workload tolerance 1e-8 the gradient stays close to the one at
    5e-12 (near the FP64 floor of these problems)."""
    from paper_2010_00626_amd import autograd as ag
    n, count = 255, 2
    print("[gpu-adjoint] n=255 batch=2 tol 1e-8 vs 5e-12", flush=True)
    th, ep, fs = batch(n, count, 4)
    f = torch.from_numpy(fs).cuda()
    grads = []
    for tol in (1e-8, 5e-12):
        cfg = ag.SolveConfig(kappa=3, nu1=1, nu2=1, tol=tol, tol_adjoint=tol, maxit=800)
        with torch.no_grad():
            target = ag.solve(f, torch.tensor(th + 0.1), torch.tensor(2 * ep), cfg)
        tht = torch.tensor(th, requires_grad=True)
        ept = torch.tensor(ep, requires_grad=True)
        loss_fn(ag, cfg, f, tht, ept, target).backward()
        grads.append((tht.grad.numpy(), ept.grad.numpy()))
    for a, b in zip(grads[0], grads[1]):
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()
