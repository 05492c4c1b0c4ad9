"""GPU parity of the convection-diffusion problem (upwind convection over
the Section 4 diffusion, rediscretised levels) against the oracle: single
cycles and stand-alone solves bit for bit with identical cycle counts, in
both execution modes and for several kernel shapes, ragged batches with a
different velocity per instance, and FP32 cycles with FP64 refinement to the
FP64 tolerance; CG and the zebra smoother are refused."""
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


def K():
    from paper_2010_00626_amd import kcycle
    return kcycle


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def banner(msg):
    print(f"[gpu-convection] {msg}", flush=True)


@pytest.mark.parametrize("n,kappa,b,ex", [
    (63, 1, (10.0, 5.0), dict()),
    (127, 2, (-40.0, 15.0), dict()),
    (255, 3, (20.0, 10.0), dict(tiny_tile_n=255, coarse_cutover=63)),
    (511, 2 ** 31 - 1, (100.0, -50.0), dict(stream_n=511, coarse_cutover=15, coarse_wave_n=7)),
    (255, 2, (3.0, -8.0), dict(mode="paper")),
])
def test_convection_cycle_bitwise(n, kappa, b, ex):
    banner(f"cycle n={n} kappa={kappa} b={b} exec={ex}")
    rng = np.random.default_rng(n + kappa)
    th, ep = math.pi / 6, 1e-2
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep)], exec=ex)
    H.set_convection(*b)
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa, nu1=2, nu2=2)
    Ho = O.Hierarchy(n, th, ep, convection=b)
    ref = Ho.cycle(v0, f, kappa=min(kappa, 64), nu1=2, nu2=2)[0]
    assert np.array_equal(host(v), ref)
    H.cycle(v, dev(f), kappa=kappa, nu1=2, nu2=2)   # replay of the captured schedule
    assert np.array_equal(host(v), Ho.cycle(ref, f, kappa=min(kappa, 64), nu1=2, nu2=2)[0])
    H.close()


@pytest.mark.parametrize("kappa", [1, 2, 3, 2 ** 31 - 1])
def test_convection_solve_bitwise(kappa):
    n, th, ep, b = 511, math.pi / 6, 1e-2, (20.0, 10.0)
    banner(f"solve n={n} kappa={kappa}")
    f = inputs.uniform_rhs(np.random.default_rng(1), n)
    Ho = O.Hierarchy(n, th, ep, convection=b)
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=min(kappa, 64), tol=1e-8, maxit=2000)
    assert rc == O.OK
    assert np.all(np.abs(np.asarray(hist) - 1e-8) > 1e-12 * 1e-8)
    H = K().Hierarchy([(n, th, ep)])
    H.set_convection(*b)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    it, rr, st = H.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=2000)
    assert st == [0] and it[0] == it_ref
    assert np.allclose(H.residual_history(0), hist, rtol=1e-14, atol=0.0)
    assert np.array_equal(host(u), u_ref)
    H.close()


def test_convection_batched_ragged_and_fp32_refinement():
    """Instances of different sizes and velocities (one without convection)
    in one launch per stage; FP64 bit for bit, FP32 cycles with FP64
    refinement to the FP64 tolerance on the true residual."""
    banner("batched ragged, FP64 and FP32 refinement")
    specs = [(255, 0.3, 1e-2), (127, 1.2, 1.0), (511, 2.0, 1e-3), (63, 0.8, 0.1)]
    bs = [(20.0, 10.0), (-100.0, 40.0), (0.0, 0.0), (5.0, -5.0)]
    rng = np.random.default_rng(5)
    fs = [inputs.uniform_rhs(rng, s[0]) for s in specs]
    for prec in ("f64", "f32"):
        H = K().Hierarchy(specs, prec)
        H.set_convection([b[0] for b in bs], [b[1] for b in bs])
        us = [torch.zeros((s[0], s[0]), dtype=torch.float64, device="cuda") for s in specs]
        iters, relres, status = H.solve(us, [dev(f) for f in fs], kappa=2, tol=1e-8, maxit=3000)
        assert status == [0] * len(specs), prec
        for k, (s, b, f) in enumerate(zip(specs, bs, fs)):
            Ho = O.Hierarchy(*s, convection=b)
            got = host(us[k])
            if prec == "f64":
                u_ref, rc, it_ref, _ = Ho.solve(f, kappa=2, tol=1e-8, maxit=3000)
                assert iters[k] == it_ref and np.array_equal(got, u_ref), k
            else:
                u_ir, rc, it_ir, _ = Ho.ir_solve(f, kappa=2, tol=1e-8, maxit=3000)
                assert rc == O.OK and abs(iters[k] - it_ir) <= 1, (k, iters[k], it_ir)
                assert np.linalg.norm(f - Ho.apply(got)) / np.linalg.norm(f) < 1e-8, k
        H.close()


def test_convection_refusals():
    banner("refusals")
    KK = K()
    n = 63
    H = KK.Hierarchy([(n, 0.3, 1e-2)])
    H.set_convection(10.0, 5.0)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    f = dev(np.ones((n, n)))
    with pytest.raises(KK.KCycleError) as e:
        H.pcg(u, f, kappa=2)
    assert e.value.status == KK.KC_ERR_STATE
    with pytest.raises(KK.KCycleError) as e:
        H.solve(u, f, kappa=2, smoother="zebra")
    assert e.value.status == KK.KC_ERR_ARG
    with pytest.raises(KK.KCycleError):
        H.grad_params(u, u)
    H3 = KK.Hierarchy([(n, 0.3, 1e-2, 3)])
    with pytest.raises(KK.KCycleError) as e:
        H3.set_convection(1.0, 1.0)
    assert e.value.status == KK.KC_ERR_ARG
    H.close()
    H3.close()
