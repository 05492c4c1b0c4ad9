"""Parity at the full sizes of the batched workload (64 uneven instances up to
2047^2, FP32 cycles with FP64 refinement) and of the gradient workload
(16 x 1023^2, PCG forward and adjoint), in the launch configuration the
benchmark times.  The oracle computes sampled instances one by one (the whole
batches would take it hours); properties that hold at any size cover the rest:
every instance's true FP64 residual, and each sampled instance's batched
result equal to its own solve bit for bit."""
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


def K():
    from paper_2010_00626_amd import kcycle
    return kcycle


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def banner(msg):
    print(f"[gpu-fullsize] {msg}", flush=True)


# the execution options the benchmark's autotuner chooses for this batch
C4_EXEC = dict(coarse_cutover=15, coarse_threads=256, coarse_wave_n=15, tiny_tile_n=63, small_tile_n=255,
               mid_tile_n=1023, stream_n=1023)


def test_full_size_batched_fp32_refinement():
    w = inputs.config4()
    probs = [(i.n, i.theta, i.eps) for i in w.instances]
    banner(f"batched full size: {len(probs)} instances, {w.unknowns} unknowns, kappa=3")
    Hb = K().Hierarchy(probs, "f32", exec=C4_EXEC)
    us = [torch.zeros((i.n, i.n), dtype=torch.float64, device="cuda") for i in w.instances]
    fs = [dev(i.f) for i in w.instances]
    iters, relres, status = Hb.solve(us, fs, kappa=3, nu1=w.nu1, nu2=w.nu2, omega=w.omega, tol=w.tol, maxit=20000)
    assert status == [0] * len(probs)
    # every instance: the true FP64 residual of its result is below the tolerance
    H64 = K().Hierarchy(probs, "f64")
    rs = [torch.empty_like(u) for u in us]
    H64.apply_A(rs, us)
    for k, (f, r) in enumerate(zip(fs, rs)):
        rel = float(torch.linalg.vector_norm(f - r) / torch.linalg.vector_norm(f))
        assert rel < w.tol, (k, rel)
    # sampled instances: the batched result is the instance's own solve, bit for bit
    nmin = min(p[0] for p in probs)
    few = min((k for k in range(len(probs)) if probs[k][0] == nmin), key=lambda k: iters[k])
    big = max(range(len(probs)), key=lambda k: (probs[k][0], -iters[k]))
    slow = max(range(len(probs)), key=lambda k: iters[k])
    for k in sorted({few, big, slow}):
        banner(f"  instance {k}: n={probs[k][0]}, {iters[k]} iterations, solved alone")
        Hs = K().Hierarchy([probs[k]], "f32", exec=C4_EXEC)
        u1 = torch.zeros_like(us[k])
        it1, _, st1 = Hs.solve(u1, fs[k], kappa=3, nu1=w.nu1, nu2=w.nu2, omega=w.omega, tol=w.tol, maxit=20000)
        assert st1 == [0] and it1[0] == iters[k] and torch.equal(u1, us[k]), k
        Hs.close()
    # the smallest instance needing the fewest iterations against the oracle's FP32-cycle refinement
    i = w.instances[few]
    u_ir, rc, it_ir, _ = O.Hierarchy(i.n, i.theta, i.eps).ir_solve(i.f, kappa=3, nu1=w.nu1, nu2=w.nu2, tol=w.tol,
                                                                       maxit=20000)
    assert rc == O.OK and abs(iters[few] - it_ir) <= 1
    assert relmax(host(us[few]), u_ir) <= 1e-6
    Hb.close()
    H64.close()


def test_full_size_gradients():
    """16 x 1023^2: loss 1/2 ||u - u*||^2 with u* for (theta + 0.1, 2 eps), PCG
    forward and adjoint at the workload's 1e-8; instance 0's gradients against
    the oracle's from PCG solves at 1e-10 (the rounding floor of the true
    residual at 1023^2 lies above 1e-12; the 1e-8 solves move a gradient by
    about 1e-6 of its size, see the adjoint tests)."""
    from paper_2010_00626_amd import autograd as ag
    wl = inputs.config5()
    banner(f"gradients full size: {len(wl.instances)} x {wl.instances[0].n}^2")
    th = torch.tensor([i.theta for i in wl.instances], dtype=torch.float64)
    ep = torch.tensor([i.eps for i in wl.instances], dtype=torch.float64)
    f = torch.from_numpy(np.stack([i.f for i in wl.instances])).to("cuda")
    cfg = ag.SolveConfig(kappa=3, nu1=1, nu2=1, tol=wl.tol, tol_adjoint=wl.tol)
    with torch.no_grad():
        target = ag.solve(f, th + 0.1, 2 * ep, cfg)
    tht = th.clone().requires_grad_(True)
    ept = ep.clone().requires_grad_(True)
    fr = f.clone().requires_grad_(True)
    L = 0.5 * ((ag.solve(fr, tht, ept, cfg) - target) ** 2).sum()
    L.backward()
    assert torch.isfinite(tht.grad).all() and torch.isfinite(ept.grad).all()
    k = 0
    i = wl.instances[k]
    banner("  oracle gradient of instance 0 (three PCG solves at 1e-10)")
    H = O.Hierarchy(i.n, i.theta, i.eps)
    Hs = O.Hierarchy(i.n, i.theta + 0.1, 2 * i.eps)
    u, rc1, _, _ = H.pcg(i.f, kappa=3, tol=1e-10, maxit=500)
    us, rc2, _, _ = Hs.pcg(i.f, kappa=3, tol=1e-10, maxit=500)
    lam, rc3, _, _ = H.pcg(u - us, kappa=3, tol=1e-10, maxit=500)
    assert rc1 == rc2 == rc3 == O.OK
    ot, oe = H.grad_params(lam, u)
    gth, gep = float(tht.grad[k]), float(ept.grad[k])
    assert abs(gth - ot) <= 1e-5 * abs(ot), (gth, ot)
    assert abs(gep - oe) <= 1e-5 * abs(oe), (gep, oe)
    gf = fr.grad[k].detach().cpu().numpy()
    assert np.abs(gf - lam).max() <= 1e-5 * np.abs(lam).max()
