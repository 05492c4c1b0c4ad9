"""GPU parity: the HIP library against the oracle, element by element, on
seeded inputs (through the C-ABI via the ctypes binding).

FP64 paths use the same arithmetic order as the oracle (per-point stencil
sums, Jacobi update, full weighting, bilinear gather, Galerkin stencils,
Cholesky coarsest solve), so single cycles and stand-alone iterates are
compared bitwise; the bar stated by the workload is 1e-11 relative, which is
asserted everywhere.  Norms and dot products are Dot2 sums on both sides, in
different orders, so a relative residual may differ in the last bit only when
its exact value lies next to a rounding boundary: iteration counts must be
identical and the tests check that no stop decision lies within 1e-12 of the
tolerance.
"""
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


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def banner(msg):
    print(f"[gpu-parity] {msg}", flush=True)


@pytest.mark.parametrize("n", [7, 63, 127, 255, 1023])
def test_apply_A_bitwise(n):
    banner(f"apply_A n={n}")
    rng = np.random.default_rng(n)
    th, ep = 0.7, 3e-3
    x = rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep)])
    y = torch.empty((n, n), dtype=torch.float64, device="cuda")
    H.apply_A(y, dev(x))
    ref = O.Hierarchy(n, th, ep).apply(x)
    assert np.array_equal(host(y), ref)


CYCLE_CASES = [
    # n, n_coarsest, kappa, nu1, nu2, mode, graph
    (63, 3, 1, 2, 2, "fused", True),
    (63, 1, 3, 2, 2, "fused", False),
    (127, 1, 2, 2, 2, "fused", True),
    (255, 1, 3, 1, 1, "fused", True),
    (255, 1, 4, 2, 1, "fused", True),
    (511, 1, 2 ** 31 - 1, 2, 2, "fused", True),
    (1023, 1, 3, 2, 2, "fused", True),
    (127, 3, 2, 2, 2, "paper", True),
    (255, 1, 3, 1, 1, "paper", False),
    (63, 7, 1, 2, 2, "paper", True),
]


@pytest.mark.parametrize("n,nc,kappa,nu1,nu2,mode,graph", CYCLE_CASES)
def test_one_cycle_bitwise(n, nc, kappa, nu1, nu2, mode, graph):
    banner(f"one cycle n={n} nc={nc} kappa={kappa} nu={nu1}+{nu2} mode={mode} graph={graph}")
    rng = np.random.default_rng(n + kappa)
    th, ep = 0.9, 2e-3
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep, nc)], exec=dict(mode=mode, use_graph=graph))
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa, nu1=nu1, nu2=nu2)
    Ho = O.Hierarchy(n, th, ep, n_coarsest=nc)
    ref = Ho.cycle(v0, f, kappa=min(kappa, 64), nu1=nu1, nu2=nu2)[0]
    got = host(v)
    assert relmax(got, ref) <= 1e-11
    assert np.array_equal(got, ref)
    # a second cycle on the same handle reuses the captured schedule
    H.cycle(v, dev(f), kappa=kappa, nu1=nu1, nu2=nu2)
    ref2 = Ho.cycle(ref, f, kappa=min(kappa, 64), nu1=nu1, nu2=nu2)[0]
    assert np.array_equal(host(v), ref2)


@pytest.mark.parametrize("reps", [3, 4, 5, 9])
def test_multi_cycle_graphs_exact_count(reps):
    """Runs of cycles are replayed as graphs of four cycles plus single-cycle
    graphs for the remainder: time_cycles (one warm-up cycle, then reps timed
    ones) must leave exactly 1 + reps oracle cycles in v, bit for bit."""
    n, kappa = 127, 2
    banner(f"multi-cycle graphs n={n} kappa={kappa} reps={reps}")
    rng = np.random.default_rng(500 + reps)
    th, ep = 0.6, 4e-3
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep)])
    v = dev(v0)
    H.time_cycles(v, dev(f), kappa=kappa, reps=reps)
    Ho = O.Hierarchy(n, th, ep)
    ref = v0
    for _ in range(1 + reps):
        ref = Ho.cycle(ref, f, kappa=kappa)[0]
    assert np.array_equal(host(v), ref)
    H.close()


@pytest.mark.parametrize("n,kappa,small", [(255, 3, 4095), (1023, 2, 255), (1023, 2 ** 31 - 1, 511)])
def test_small_tile_option(n, kappa, small):
    """16 x 16 tiles on the small levels give the same bits as the oracle,
    for one cycle and for a solve whose stopping norm runs in those tiles."""
    banner(f"small tiles n={n} kappa={kappa} small_tile_n={small}")
    rng = np.random.default_rng(n + 7)
    th, ep = 2.1, 3e-4
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep)], exec=dict(small_tile_n=small, tiny_tile_n=0))
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa, nu1=2, nu2=2)
    Ho = O.Hierarchy(n, th, ep)
    assert np.array_equal(host(v), Ho.cycle(v0, f, kappa=min(kappa, 64), nu1=2, nu2=2)[0])
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=min(kappa, 64), tol=1e-6, maxit=500)
    check_stop_margin(hist, 1e-6)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.solve(u, dev(f), kappa=kappa, tol=1e-6, maxit=500)
    assert status == [0] and iters[0] == it_ref
    assert np.array_equal(host(u), u_ref)


TILE_SHAPE_CASES = [
    (255, 3, dict(tiny_tile_n=0, small_tile_n=0, mid_tile_n=4095)),      # 32 x 32 everywhere
    (1023, 2, dict(tiny_tile_n=0, small_tile_n=127, mid_tile_n=1023)),
    (511, 2 ** 31 - 1, dict(tiny_tile_n=0, small_tile_n=0, mid_tile_n=511)),
    (255, 2, dict(tiny_tile_n=255)),                                     # 8 x 8 everywhere
    (1023, 3, dict(tiny_tile_n=127, small_tile_n=255, mid_tile_n=1023)),  # 8, 16, 32 and 32 x 32 tiles
    (127, 2 ** 31 - 1, dict(tiny_tile_n=127)),
]


@pytest.mark.parametrize("n,kappa,shape", TILE_SHAPE_CASES)
def test_tile_shape_options(n, kappa, shape):
    """8 x 8 and 32 x 32 tiles give the oracle's bits (one cycle, and a solve
    whose stopping norm runs in them); FP32 cycles give the same bits in any shape."""
    banner(f"tile shapes n={n} kappa={kappa} {shape}")
    rng = np.random.default_rng(n + 11)
    th, ep = 0.7, 2e-3
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    ex = dict(shape, stream_n=0)
    H = K().Hierarchy([(n, th, ep)], exec=ex)
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa, nu1=2, nu2=2)
    Ho = O.Hierarchy(n, th, ep)
    assert np.array_equal(host(v), Ho.cycle(v0, f, kappa=min(kappa, 64), nu1=2, nu2=2)[0])
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=min(kappa, 64), tol=1e-6, maxit=500)
    check_stop_margin(hist, 1e-6)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.solve(u, dev(f), kappa=kappa, tol=1e-6, maxit=500)
    assert status == [0] and iters[0] == it_ref
    assert np.array_equal(host(u), u_ref)
    outs = []
    for e in (ex, dict(tiny_tile_n=0, small_tile_n=4095, stream_n=0)):
        H32 = K().Hierarchy([(n, th, ep)], "f32", exec=e)
        u.zero_()
        it32, _, st32 = H32.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=500)
        assert st32 == [0]
        outs.append((it32[0], host(u)))
        H32.close()
    assert outs[0][0] == outs[1][0] and np.array_equal(outs[0][1], outs[1][1])


STREAM_CASES = [
    # n, kappa, nu1, nu2, stream_n
    (255, 2, 2, 2, 63),
    (511, 3, 1, 1, 127),
    (255, 1, 3, 3, 31),
    (127, 2, 0, 2, 15),
    (511, 2 ** 31 - 1, 2, 1, 255),
]


@pytest.mark.parametrize("n,kappa,nu1,nu2,stream", STREAM_CASES)
def test_stream_kernels_one_cycle(n, kappa, nu1, nu2, stream):
    """Streaming strip kernels on every level >= stream_n give the oracle's bits."""
    banner(f"streaming n={n} kappa={kappa} nu={nu1}+{nu2} stream_n={stream}")
    rng = np.random.default_rng(n * 3 + kappa)
    th, ep = 0.35, 5e-3
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep)], exec=dict(stream_n=stream))
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa, nu1=nu1, nu2=nu2)
    ref = O.Hierarchy(n, th, ep).cycle(v0, f, kappa=min(kappa, 64), nu1=nu1, nu2=nu2)[0]
    assert np.array_equal(host(v), ref)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_stream_kernels_solve_and_batch(prec):
    """Stop-test norms from the streaming kernel, FP32 refinement and ragged batches."""
    banner(f"streaming solve + batch prec={prec}")
    specs = [(511, 0.3, 1e-3), (127, 1.2, 1e-2), (255, 2.0, 1e-4)]
    rng = np.random.default_rng(11)
    fs = [inputs.uniform_rhs(rng, s[0]) for s in specs]
    Hb = K().Hierarchy(specs, prec, exec=dict(stream_n=63))
    us = [torch.zeros((s[0], s[0]), dtype=torch.float64, device="cuda") for s in specs]
    iters, relres, status = Hb.solve(us, [dev(f) for f in fs], kappa=2, tol=1e-7, maxit=3000)
    assert status == [0] * len(specs)
    for k, (sp, f) in enumerate(zip(specs, fs)):
        Ho = O.Hierarchy(*sp)
        if prec == "f64":
            u_ref, rc, it_ref, hist = Ho.solve(f, kappa=2, tol=1e-7, maxit=3000)
            check_stop_margin(hist, 1e-7)
            assert iters[k] == it_ref, k
            assert np.array_equal(host(us[k]), u_ref), k
        else:
            Hs = K().Hierarchy([sp], prec, exec=dict(stream_n=0))
            u1 = torch.zeros_like(us[k])
            it1, rr1, st1 = Hs.solve(u1, dev(f), kappa=2, tol=1e-7, maxit=3000)
            assert st1 == [0] and it1[0] == iters[k] and torch.equal(u1, us[k]), k
            true_rel = np.linalg.norm(f - Ho.apply(host(us[k]))) / np.linalg.norm(f)
            assert true_rel < 1.01e-7


def check_stop_margin(hist, tol):
    """No relative residual of the run lies within 1e-12 (relative) of tol."""
    h = np.asarray(hist)
    assert np.all(np.abs(h - tol) > 1e-12 * tol)


@pytest.mark.parametrize("kappa", [1, 2, 3, 4, 5])
def test_config1_solve(kappa):
    w = inputs.config1()
    inst = w.instances[0]
    banner(f"config1 solve kappa={kappa}")
    Ho = O.Hierarchy(inst.n, inst.theta, inst.eps, n_coarsest=w.n_coarsest, omega=w.omega)
    u_ref, rc, it_ref, hist = Ho.solve(inst.f, kappa=kappa, nu1=w.nu1, nu2=w.nu2, tol=w.tol, maxit=1000)
    assert rc == O.OK
    check_stop_margin(hist, w.tol)
    H = K().Hierarchy([(inst.n, inst.theta, inst.eps, w.n_coarsest)])
    u = torch.zeros((inst.n, inst.n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.solve(u, dev(inst.f), kappa=kappa, nu1=w.nu1, nu2=w.nu2, omega=w.omega, tol=w.tol,
                                    maxit=1000)
    assert status == [0]
    assert iters[0] == it_ref
    assert abs(relres[0] - hist[-1]) <= 1e-12 * hist[-1]
    gh = H.residual_history(0)
    assert len(gh) == len(hist) == it_ref + 1
    assert np.allclose(gh, hist, rtol=1e-14, atol=0.0)
    got = host(u)
    assert relmax(got, u_ref) <= 1e-11
    assert np.array_equal(got, u_ref)


@pytest.mark.parametrize("n,kappa,mode", [(255, 1, "fused"), (255, 3, "fused"), (255, 2 ** 31 - 1, "fused"),
                                          (511, 2, "fused"), (255, 3, "paper")])
def test_standalone_solve_reduced_config2(n, kappa, mode):
    banner(f"stand-alone n={n} kappa={kappa} mode={mode}")
    rng = np.random.default_rng(1)
    f = inputs.uniform_rhs(rng, n)
    th, ep = math.pi / 6, 1e-4
    Ho = O.Hierarchy(n, th, ep)
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=min(kappa, 64), tol=1e-8, maxit=5000)
    assert rc == O.OK
    check_stop_margin(hist, 1e-8)
    H = K().Hierarchy([(n, th, ep)], exec=dict(mode=mode))
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=5000)
    assert status == [0] and iters[0] == it_ref
    got = host(u)
    assert relmax(got, u_ref) <= 1e-11
    assert np.array_equal(got, u_ref)


def test_batched_equals_per_instance():
    banner("batched ragged stand-alone")
    specs = [(255, 0.3, 1e-3), (63, 1.2, 1e-2), (511, 2.0, 1e-4), (127, 0.8, 0.05), (31, 2.7, 1e-5)]
    rng = np.random.default_rng(2)
    fs = [inputs.uniform_rhs(rng, s[0]) for s in specs]
    Hb = K().Hierarchy(specs)
    us = [torch.zeros((s[0], s[0]), dtype=torch.float64, device="cuda") for s in specs]
    iters, relres, status = Hb.solve(us, [dev(f) for f in fs], kappa=3, tol=1e-8, maxit=3000)
    assert status == [0] * len(specs)
    for k, (s, f) in enumerate(zip(specs, fs)):
        Ho = O.Hierarchy(*s)
        u_ref, rc, it_ref, hist = Ho.solve(f, kappa=3, tol=1e-8, maxit=3000)
        assert iters[k] == it_ref, k
        assert np.array_equal(host(us[k]), u_ref), k
        Hs = K().Hierarchy([s])
        u1 = torch.zeros_like(us[k])
        it1, _, st1 = Hs.solve(u1, dev(f), kappa=3, tol=1e-8, maxit=3000)
        assert it1[0] == iters[k] and torch.equal(u1, us[k])


@pytest.mark.parametrize("n,kappa", [(255, 1), (255, 3), (511, 4)])
def test_ir_fp32(n, kappa):
    banner(f"FP32 cycles + FP64 refinement n={n} kappa={kappa}")
    rng = np.random.default_rng(1)
    f = inputs.uniform_rhs(rng, n)
    th, ep = math.pi / 6, 1e-4
    Ho = O.Hierarchy(n, th, ep)
    u_ir, rc, it_ir, hist = Ho.ir_solve(f, kappa=kappa, tol=1e-8, maxit=5000)
    u64, rc64, it64, _ = Ho.solve(f, kappa=kappa, tol=1e-8, maxit=5000)
    assert rc == O.OK
    H = K().Hierarchy([(n, th, ep)], precision="f32")
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=5000)
    assert status == [0]
    got = host(u)
    true_rel = np.linalg.norm(f - Ho.apply(got)) / np.linalg.norm(f)
    assert true_rel < 1e-8
    assert abs(iters[0] - it_ir) <= 1
    assert iters[0] <= it64 + 2
    assert relmax(got, u_ir) <= 1e-6
    assert relmax(got, u64) <= 1e-6


@pytest.mark.parametrize("n,kappa,f32", [(127, 1, False), (255, 2, False), (255, 3, False), (255, 3, True),
                                         (511, 4, True)])
def test_pcg(n, kappa, f32):
    banner(f"PCG n={n} kappa={kappa} f32={f32}")
    f = inputs.gaussian_sum_rhs(5, n)
    th, ep = 3 * math.pi / 8, 1e-5
    Ho = O.Hierarchy(n, th, ep)
    u_ref, rc, it_ref, hist = Ho.pcg(f, kappa=kappa, nu1=1, nu2=1, tol=1e-8, maxit=500, precond_f32=f32)
    assert rc == O.OK
    H = K().Hierarchy([(n, th, ep)], precision="f32" if f32 else "f64")
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.pcg(u, dev(f), kappa=kappa, nu1=1, nu2=1, tol=1e-8, maxit=500)
    assert status == [0]
    assert abs(iters[0] - it_ref) <= (0 if not f32 else 1)
    gh = H.residual_history(0)
    assert len(gh) == iters[0] + 1 and gh[0] == 1.0 and gh[-1] == relres[0]
    if not f32:
        # Dot2 norms and dots on both sides: the histories agree to the last bits
        assert np.allclose(gh, hist[:len(gh)], rtol=1e-14, atol=0.0)
    got = host(u)
    assert relmax(got, u_ref) <= (1e-11 if not f32 else 1e-6)
    true_rel = np.linalg.norm(f - Ho.apply(got)) / np.linalg.norm(f)
    assert true_rel < 1e-8 and relres[0] < 1e-8


def test_pcg_residual_replacement():
    """At tol 1e-13 the recurrence residual of the FP64 PCG passes tol at
    iteration 57 while the true residual is 5e-13: both sides form the true
    residual, replace the recurrence residual by it and go on, with the same
    iterations, histories and iterates, and stop at maxit."""
    banner("PCG residual replacement")
    n, kappa, tol, maxit = 127, 2, 1e-13, 60
    f = inputs.gaussian_sum_rhs(5, n)
    th, ep = 3 * math.pi / 8, 1e-5
    Ho = O.Hierarchy(n, th, ep)
    u_ref, rc, it_ref, hist = Ho.pcg(f, kappa=kappa, nu1=1, nu2=1, tol=tol, maxit=maxit)
    assert rc == O.NOT_CONVERGED and it_ref == maxit
    H = K().Hierarchy([(n, th, ep)])
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.pcg(u, dev(f), kappa=kappa, nu1=1, nu2=1, tol=tol, maxit=maxit)
    assert status == [K().KC_NOT_CONVERGED] and iters == [maxit]
    gh = H.residual_history(0)
    assert np.allclose(gh, hist[:maxit + 1], rtol=1e-14, atol=0.0)
    assert gh[57] > tol   # the replaced (true) residual of iteration 57
    assert relmax(host(u), u_ref) <= 1e-11


def test_grad_params_match_oracle():
    banner("gradient inner products")
    n = 255
    rng = np.random.default_rng(3)
    specs = [(n, 0.4, 1e-3), (n, 2.2, 0.05)]
    lams = [rng.uniform(-1, 1, (n, n)) for _ in specs]
    us = [rng.uniform(-1, 1, (n, n)) for _ in specs]
    H = K().Hierarchy(specs)
    dth, de = H.grad_params([dev(x) for x in lams], [dev(x) for x in us])
    for k, s in enumerate(specs):
        rt, re = O.Hierarchy(*s).grad_params(lams[k], us[k])
        assert abs(dth[k] - rt) <= 1e-12 * abs(rt)
        assert abs(de[k] - re) <= 1e-12 * abs(re)


def test_failure_statuses():
    banner("failure statuses")
    n = 63
    f = inputs.uniform_rhs(np.random.default_rng(0), n)
    KK = K()
    H = KK.Hierarchy([(n, 0.4, 1e-3, 3)])
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    it, rr, st = H.solve(u, dev(f), kappa=2, tol=1e-10, maxit=1)
    assert st == [KK.KC_NOT_CONVERGED] and it == [1]
    u.zero_()
    it, rr, st = H.solve(u, dev(f), kappa=1, omega=2.5, tol=1e-10, maxit=500)
    assert st == [KK.KC_DIVERGED]
    bad = f.copy()
    bad[3, 4] = np.nan
    u.zero_()
    it, rr, st = H.solve(u, dev(bad), kappa=1, tol=1e-10, maxit=5)
    assert st == [KK.KC_ERR_NONFINITE]
    with pytest.raises(KK.KCycleError):
        H.cycle(u, dev(f), kappa=0)


def test_deterministic_rerun():
    banner("run-twice determinism")
    n = 511
    f = inputs.uniform_rhs(np.random.default_rng(7), n)
    H = K().Hierarchy([(n, 1.0, 1e-3)])
    outs = []
    for _ in range(2):
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        it, rr, st = H.solve(u, dev(f), kappa=3, tol=1e-9, maxit=2000)
        outs.append((it[0], rr[0], host(u)))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("prec,driver", [("f64", "solve"), ("f32", "solve"), ("f64", "pcg")])
def test_profile_iteration_covers_every_launch(prec, driver):
    """The per-launch profile lists every launch of one iteration once."""
    banner(f"profile iteration prec={prec} driver={driver}")
    n = 255
    f = inputs.uniform_rhs(np.random.default_rng(4), n)
    H = K().Hierarchy([(n, 0.5, 1e-3)], prec)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    run = H.pcg if driver == "pcg" else H.solve
    run(u, dev(f), kappa=2, nu1=1, nu2=1, tol=1e-6, maxit=200)
    st = H.stats()
    prof = H.profile_iteration(driver, kappa=2, nu1=1, nu2=1, reps=3)
    ks = prof["kernels"]
    launches = sum(k["launches"] for k in ks if k["name"] != "k_finalize")
    assert launches == st["grid_launches_per_iteration"] + st["subtree_launches_per_iteration"]
    assert abs(sum(k["ms"] for k in ks) - prof["iteration_ms"]) <= 1e-5 * (len(ks) + prof["iteration_ms"])
    assert all(k["avg_ms"] > 0 for k in ks)
    assert any(k["name"].startswith("k_subtree") for k in ks)
    assert all(k["bytes_per_launch"] > 0 for k in ks if k["name"].startswith(("k_pre", "k_post")))
    assert all(k["flops_per_launch"] > 0 for k in ks if k["name"].startswith("k_subtree"))
    seq = prof["sequence"]   # [kernel, depth, ms, algorithmic bytes] per launch
    assert len(seq) == launches and all(len(e) == 4 and e[2] > 0 and e[3] >= 0 for e in seq)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_compaction_keeps_results(prec):
    """Finished instances dropped from the launches mid-solve: every instance's
    iterate and count equal its stand-alone solve."""
    banner(f"batch compaction prec={prec}")
    specs = [(255, 0.7, 0.5), (255, 1.9, 0.4), (255, 2.5, 0.6), (127, 0.3, 2e-3), (255, 1.1, 1e-3)]
    rng = np.random.default_rng(12)
    fs = [inputs.uniform_rhs(rng, s[0]) for s in specs]
    Hb = K().Hierarchy(specs, prec)
    us = [torch.zeros((s[0], s[0]), dtype=torch.float64, device="cuda") for s in specs]
    iters, relres, status = Hb.solve(us, [dev(f) for f in fs], kappa=2, tol=1e-9, maxit=4000)
    assert status == [0] * len(specs)
    assert Hb.stats()["compactions"] >= 1
    assert max(iters) > 2 * min(iters)
    for k, (sp, f) in enumerate(zip(specs, fs)):
        Hs = K().Hierarchy([sp], prec)
        u1 = torch.zeros_like(us[k])
        it1, _, st1 = Hs.solve(u1, dev(f), kappa=2, tol=1e-9, maxit=4000)
        assert st1 == [0] and it1[0] == iters[k] and torch.equal(u1, us[k]), k
    # a second solve on the same handle starts from the full tables again
    for x in us:
        x.zero_()
    iters2, _, status2 = Hb.solve(us, [dev(f) for f in fs], kappa=2, tol=1e-9, maxit=4000)
    assert iters2 == iters and status2 == status


REG_CASES = [
    # n, kappa, nu1, nu2, cutover, wave_n, precision
    (255, 2, 2, 2, 15, 15, "f64"),
    (255, 3, 1, 1, 31, 7, "f64"),
    (127, 2 ** 31 - 1, 2, 1, 31, 3, "f64"),
    (255, 1, 0, 3, 63, 15, "f64"),
    (511, 4, 3, 0, 31, 15, "f64"),
    (255, 2, 2, 2, 15, 15, "f32"),
    (255, 3, 1, 2, 31, 7, "f32"),
]


@pytest.mark.parametrize("n,kappa,nu1,nu2,cut,wave_n,prec", REG_CASES)
def test_register_calls_match_lds_phases(n, kappa, nu1, nu2, cut, wave_n, prec):
    """Whole calls of the small levels in registers give the bits of the
    phase-by-phase LDS execution (and, in FP64, of the oracle)."""
    banner(f"register calls n={n} kappa={kappa} nu={nu1}+{nu2} cut={cut} wave_n={wave_n} {prec}")
    rng = np.random.default_rng(n + 17 * kappa)
    th, ep = 1.3, 2e-3
    f = rng.uniform(-1, 1, (n, n))
    res = []
    for regs in (1, 0):
        H = K().Hierarchy([(n, th, ep)], prec, exec=dict(coarse_cutover=cut, coarse_wave_n=wave_n, wave_regs=regs,
                                                         coarse_threads=512))
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        it, rr, st = H.solve(u, dev(f), kappa=kappa, nu1=nu1, nu2=nu2, tol=1e-6, maxit=400)
        assert st == [0]
        res.append((it[0], host(u)))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])
    if prec == "f64":
        u_ref, rc, it_ref, hist = O.Hierarchy(n, th, ep).solve(f, kappa=min(kappa, 64), nu1=nu1, nu2=nu2, tol=1e-6,
                                                                maxit=400)
        check_stop_margin(hist, 1e-6)
        assert res[0][0] == it_ref
        assert np.array_equal(res[0][1], u_ref)


@pytest.mark.parametrize("n,kappa,nu1,nu2,prec,tile", [(255, 2, 2, 2, "f64", 16), (511, 3, 1, 2, "f64", 16),
                                                       (255, 2 ** 31 - 1, 3, 0, "f64", 16), (255, 4, 0, 3, "f64", 16),
                                                       (511, 2, 2, 2, "f32", 16), (255, 2, 2, 2, "f64", 8),
                                                       (511, 3, 3, 3, "f64", 8), (511, 2, 2, 2, "f32", 8)])
def test_junction_fusion_bitwise(n, kappa, nu1, nu2, prec, tile):
    """Fused sibling junctions (16 x 16 or 8 x 8 tiles) give the bits of separate
    post / pre launches (and of the oracle in FP64)."""
    banner(f"junction fusion n={n} kappa={kappa} nu={nu1}+{nu2} {prec} tile {tile}")
    rng = np.random.default_rng(n + 31 * kappa + nu1)
    th, ep = 0.6, 4e-3
    f = rng.uniform(-1, 1, (n, n))
    res = []
    shape = dict(tiny_tile_n=0, small_tile_n=4095) if tile == 16 else dict(tiny_tile_n=4095)
    for fuse in (1, 0):
        H = K().Hierarchy([(n, th, ep)], prec, exec=dict(shape, coarse_cutover=15, fuse_junctions=fuse))
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        it, rr, st = H.solve(u, dev(f), kappa=kappa, nu1=nu1, nu2=nu2, tol=1e-6, maxit=400)
        assert st == [0]
        res.append((it[0], host(u), H.stats()["grid_launches_per_iteration"]))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])
    assert res[0][2] < res[1][2]   # the fused schedule has fewer launches
    if prec == "f64":
        u_ref, rc, it_ref, hist = O.Hierarchy(n, th, ep).solve(f, kappa=min(kappa, 64), nu1=nu1, nu2=nu2, tol=1e-6,
                                                                maxit=400)
        check_stop_margin(hist, 1e-6)
        assert res[0][0] == it_ref and np.array_equal(res[0][1], u_ref)


@pytest.mark.parametrize("n,kappa,cutover,wave_n", [(255, 2, 31, 15), (511, 3, 63, 15), (255, 2 ** 31 - 1, 63, 7),
                                                   (127, 2, 15, 0)])
def test_persistent_kernel_1024_threads(n, kappa, cutover, wave_n):
    """FP32 cycles with a 1024-thread persistent kernel give the bits of the
    512-thread one (same iterations and solution); FP64 rejects the option."""
    banner(f"persistent kernel 1024 threads n={n} kappa={kappa} cutover={cutover} wave_n={wave_n}")
    rng = np.random.default_rng(n + kappa % 97)
    th, ep = 1.1, 5e-3
    f = rng.uniform(-1, 1, (n, n))
    outs = []
    for threads in (1024, 512):
        H = K().Hierarchy([(n, th, ep)], "f32", exec=dict(coarse_cutover=cutover, coarse_threads=threads,
                                                          coarse_wave_n=wave_n))
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        it, rr, st = H.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=3000)
        assert st == [0]
        outs.append((it[0], host(u)))
        H.close()
    assert outs[0][0] == outs[1][0] and np.array_equal(outs[0][1], outs[1][1])
    with pytest.raises(K().KCycleError):
        K().Hierarchy([(n, th, ep)], "f64", exec=dict(coarse_cutover=cutover, coarse_threads=1024))


def test_autotuner_keeps_results():
    """The autotuner picks valid execution options; results under them are the default options' bits."""
    banner("autotuner")
    from paper_2010_00626_amd import autotune
    n = 255
    f = inputs.uniform_rhs(np.random.default_rng(21), n)
    H = K().Hierarchy([(n, 1.0, 1e-3)], "f64")
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    fd = dev(f)
    it0, _, st0 = H.solve(u, fd, kappa=3, tol=1e-7, maxit=500)
    ref = host(u)
    res = autotune.tune(H, u, fd, 3, iters=4, force=True)
    assert res["trials"] and res["exec"] in [t["exec"] for t in res["trials"]]
    assert H.stats()["coarse_cutover"] == res["exec"]["coarse_cutover"]
    u.zero_()
    it1, _, st1 = H.solve(u, fd, kappa=3, tol=1e-7, maxit=500)
    assert st1 == st0 == [0] and it1 == it0
    assert np.array_equal(host(u), ref)


def test_model_fit_paper_mode_counts():
    """The run-time model fit in the paper-structured mode launches exactly the
    paper's N_gpuCalls per cycle and finds positive alpha and beta."""
    banner("model fit (paper mode, small n)")
    from paper_2010_00626_amd import fit_model, model
    rows = []
    for kappa in (1, 2, K().KAPPA_W):
        for nl in (5, 6, 7, 8):
            ms, grid, stages, reps = fit_model.measure("paper", kappa, nl, nu=4, budget_ms=10.0)
            calls = fit_model.n_calls(grid, stages)
            assert stages == 0 and calls == model.n_gpu_calls_paper(kappa, nl, 4)
            rows.append(((kappa, nl), calls, model.n_ops_2d(kappa, nl), ms))
    fit = model.fit(rows)
    assert fit.alpha > 0 and fit.beta >= 0


@pytest.mark.parametrize("kappa", [1, 2])
def test_paper_protocol_counts(kappa):
    """The f = 0 error-reduction protocol counts the same cycles as the oracle's
    cycles from the same random start; its MGCG count is the first iteration
    count whose error is below the target."""
    banner(f"paper protocol kappa={kappa}")
    from paper_2010_00626_amd import protocol
    n, th, ep = 63, math.pi / 4, 1e-2
    v0 = inputs.uniform_rhs(np.random.default_rng(3), n)
    H = K().Hierarchy([(n, th, ep)], "f64")
    r = protocol.standalone(H, dev(v0), kappa, chunk=8, maxc=2000)
    Ho = O.Hierarchy(n, th, ep)
    v, f0, e0, k = v0.copy(), np.zeros((n, n)), np.linalg.norm(v0), 0
    while np.linalg.norm(v) / e0 >= protocol.TARGET:
        v = Ho.cycle(v, f0, kappa=kappa, nu1=2, nu2=2)[0]
        k += 1
    assert r["cycles"] == k
    m = protocol.mgcg(H, dev(v0), kappa, kmax=500)
    it = m["iterations"]
    assert it is not None and m["final_error"] < protocol.TARGET
    b = torch.empty((n, n), dtype=torch.float64, device="cuda")
    H.apply_A(b, dev(v0))
    u = torch.zeros_like(b)
    H.pcg(u, b, kappa=kappa, nu1=2, nu2=2, tol=0.0, maxit=it - 1)
    assert np.linalg.norm(host(u) - v0) / e0 >= protocol.TARGET
    H.close()


ZEBRA_CASES = [(63, 1, 2, 2, 1), (63, 3, 2, 2, 3), (255, 2, 2, 2, 1), (127, 2 ** 31 - 1, 1, 1, 1), (255, 4, 0, 3, 1),
               (127, 2, 3, 0, 7)]


@pytest.mark.parametrize("n,kappa,nu1,nu2,nc", ZEBRA_CASES)
def test_zebra_cycle_bitwise(n, kappa, nu1, nu2, nc):
    """Alternating zebra line relaxation (paper-structured mode) gives the oracle's bits."""
    banner(f"zebra cycle n={n} kappa={kappa} nu={nu1}+{nu2} n_coarsest={nc}")
    rng = np.random.default_rng(n + 3 * nu1 + nc)
    th, ep = 0.2, 1e-3
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep, nc)], "f64", exec=dict(mode="paper"))
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa, nu1=nu1, nu2=nu2, smoother="zebra")
    Ho = O.Hierarchy(n, th, ep, nc, smoother="zebra")
    ref = Ho.cycle(v0, f, kappa=min(kappa, 64), nu1=nu1, nu2=nu2)[0]
    assert np.array_equal(host(v), ref)
    H.cycle(v, dev(f), kappa=kappa, nu1=nu1, nu2=nu2, smoother="zebra")   # replay of the captured schedule
    assert np.array_equal(host(v), Ho.cycle(ref, f, kappa=min(kappa, 64), nu1=nu1, nu2=nu2)[0])
    H.close()


@pytest.mark.parametrize("n,kappa,theta", [(255, 2, 0.0), (255, 3, math.pi / 4), (511, 4, 1.4)])
def test_zebra_solve_bitwise(n, kappa, theta):
    """Stand-alone zebra solve: the oracle's iterations and bits; and the
    Jacobi hierarchy on the same handle is unaffected."""
    banner(f"zebra solve n={n} kappa={kappa} theta={theta}")
    f = inputs.uniform_rhs(np.random.default_rng(n + kappa), n)
    ep = 1e-4
    Ho = O.Hierarchy(n, theta, ep, smoother="zebra")
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=kappa, tol=1e-8, maxit=500)
    assert rc == O.OK
    check_stop_margin(hist, 1e-8)
    H = K().Hierarchy([(n, theta, ep)], "f64", exec=dict(mode="paper"))
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=500, smoother="zebra")
    assert status == [0] and iters[0] == it_ref
    assert np.array_equal(host(u), u_ref)
    v0 = np.random.default_rng(1).uniform(-1, 1, (n, n))   # a Jacobi cycle on the same handle (separate graph)
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa)
    assert np.array_equal(host(v), O.Hierarchy(n, theta, ep).cycle(v0, f, kappa=kappa)[0])
    H.close()


@pytest.mark.parametrize("n,kappa,f32", [(255, 2, False), (255, 4, True), (511, 3, False)])
def test_zebra_pcg(n, kappa, f32):
    banner(f"zebra PCG n={n} kappa={kappa} f32={f32}")
    f = inputs.gaussian_sum_rhs(5, n)
    th, ep = 3 * math.pi / 8, 1e-5
    Ho = O.Hierarchy(n, th, ep, smoother="zebra")
    u_ref, rc, it_ref, hist = Ho.pcg(f, kappa=kappa, nu1=2, nu2=2, tol=1e-8, maxit=300, precond_f32=f32)
    assert rc == O.OK
    H = K().Hierarchy([(n, th, ep)], precision="f32" if f32 else "f64", exec=dict(mode="paper"))
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.pcg(u, dev(f), kappa=kappa, nu1=2, nu2=2, tol=1e-8, maxit=300, smoother="zebra")
    assert status == [0]
    assert abs(iters[0] - it_ref) <= (0 if not f32 else 1)
    got = host(u)
    assert relmax(got, u_ref) <= (1e-11 if not f32 else 1e-6)
    assert np.linalg.norm(f - Ho.apply(got)) / np.linalg.norm(f) < 1e-8
    H.close()


@pytest.mark.parametrize("n,kappa", [(255, 2), (511, 3)])
def test_zebra_ir_fp32(n, kappa):
    banner(f"zebra FP32 cycles + FP64 refinement n={n} kappa={kappa}")
    f = inputs.uniform_rhs(np.random.default_rng(2), n)
    th, ep = 0.1, 1e-5
    Ho = O.Hierarchy(n, th, ep, smoother="zebra")
    u_ir, rc, it_ir, _ = Ho.ir_solve(f, kappa=kappa, tol=1e-8, maxit=500)
    assert rc == O.OK
    H = K().Hierarchy([(n, th, ep)], precision="f32", exec=dict(mode="paper"))
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    iters, relres, status = H.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=500, smoother="zebra")
    assert status == [0] and abs(iters[0] - it_ir) <= 1
    got = host(u)
    assert np.linalg.norm(f - Ho.apply(got)) / np.linalg.norm(f) < 1e-8
    assert relmax(got, u_ir) <= 1e-6
    H.close()


ZEBRA_WAVE_CASES = [(63, 2, 1, 1, 0), (127, 2 ** 31 - 1, 1, 1, 0), (255, 3, 3, 127, 0), (511, 2, 1, 511, 0),
                    (255, 1, 1, 0, 0),
                    # four lines per wave: every level (line lengths 1 to 127, chunk tails of every kind),
                    # the top levels only above two-line and one-thread levels, and the default thresholds
                    (127, 2 ** 31 - 1, 1, 1, 1), (255, 3, 3, 63, 127), (511, 2, 1, 127, 255), (63, 2, 1, 63, 63),
                    (255, 4, 1, 63, 8191)]


@pytest.mark.parametrize("n,kappa,nc,wave_n,quad_n", ZEBRA_WAVE_CASES)
def test_zebra_line_mappings_bitwise(n, kappa, nc, wave_n, quad_n):
    """Every line mapping of the zebra kernel (four lines per wave on levels
    with n >= zebra_quad_n, two lines per wave on levels with n >=
    zebra_wave_n, one thread per line below; 0 = never), with chunk tails of
    every kind, gives the oracle's bits."""
    banner(f"zebra mappings n={n} kappa={kappa} n_coarsest={nc} zebra_wave_n={wave_n} zebra_quad_n={quad_n}")
    rng = np.random.default_rng(7 * n + wave_n)
    th, ep = 2.3, 1e-4
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, th, ep, nc)], "f64", exec=dict(mode="paper", zebra_wave_n=wave_n, zebra_quad_n=quad_n))
    v = dev(v0)
    H.cycle(v, dev(f), kappa=kappa, nu1=2, nu2=2, smoother="zebra")
    Ho = O.Hierarchy(n, th, ep, nc, smoother="zebra")
    assert np.array_equal(host(v), Ho.cycle(v0, f, kappa=min(kappa, 64), nu1=2, nu2=2)[0])
    H.close()


@pytest.mark.parametrize("quad_n", [8191, 255])
def test_zebra_batched_ragged_mappings(quad_n):
    """A ragged batch whose instances take different line mappings in the
    same launches (with quad_n = 255: four lines per wave on 511^2 and
    255^2, two on 127^2, one thread per line below): each instance gets the
    oracle's iterations and bits."""
    banner(f"zebra batched ragged, zebra_quad_n={quad_n}")
    specs = [(255, 0.4, 1e-3), (63, 1.3, 1e-2), (127, 2.6, 1e-4), (511, 0.05, 1e-5)]
    rng = np.random.default_rng(12)
    fs = [inputs.uniform_rhs(rng, s[0]) for s in specs]
    H = K().Hierarchy(specs, "f64", exec=dict(mode="paper", zebra_wave_n=127, zebra_quad_n=quad_n))
    us = [torch.zeros((s[0], s[0]), dtype=torch.float64, device="cuda") for s in specs]
    iters, relres, status = H.solve(us, [dev(f) for f in fs], kappa=2, tol=1e-8, maxit=400, smoother="zebra")
    assert status == [0] * len(specs)
    for k, (s, f) in enumerate(zip(specs, fs)):
        u_ref, rc, it_ref, hist = O.Hierarchy(*s, smoother="zebra").solve(f, kappa=2, tol=1e-8, maxit=400)
        assert rc == O.OK and iters[k] == it_ref, k
        assert np.array_equal(host(us[k]), u_ref), k
    H.close()


ZEBRA_FUSED_CASES = [
    (63, 2, 1, dict(coarse_cutover=31)),                                   # top level in grid kernels, cut at 31
    (63, 2 ** 31 - 1, 1, dict(coarse_cutover=63)),                         # the whole instance in the persistent kernel
    (255, 3, 1, dict(coarse_cutover=63, coarse_threads=512)),
    (127, 4, 3, dict(coarse_cutover=15, coarse_threads=256)),              # 3 x 3 coarsest (Cholesky in LDS)
    (255, 1, 1, dict(coarse_cutover=31, coarse_threads=256, coarse_wave_n=0)),
    (511, 2, 1, dict(coarse_cutover=31, coarse_wave_n=7, wave_regs=0)),
    (511, 3, 1, dict(coarse_cutover=63, zebra_quad_n=127)),                # four lines per wave above the cut
]


@pytest.mark.parametrize("n,kappa,nc,ex", ZEBRA_FUSED_CASES)
def test_zebra_fused_cycle_bitwise(n, kappa, nc, ex):
    """Zebra relaxation in the fused mode (levels above the cutover one kernel
    per operation, every call at the cutover in one persistent launch with
    line solves in LDS): the oracle's bits, and the same bits as the
    paper-structured mode."""
    banner(f"zebra fused cycle n={n} kappa={kappa} n_coarsest={nc} exec={ex}")
    rng = np.random.default_rng(3 * n + nc)
    th, ep = 0.6, 1e-4
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    Ho = O.Hierarchy(n, th, ep, nc, smoother="zebra")
    ref = Ho.cycle(v0, f, kappa=min(kappa, 64), nu1=2, nu2=2)[0]
    for mode_ex in (dict(ex), dict(mode="paper")):
        H = K().Hierarchy([(n, th, ep, nc)], "f64", exec=mode_ex)
        v = dev(v0)
        H.cycle(v, dev(f), kappa=kappa, nu1=2, nu2=2, smoother="zebra")
        assert np.array_equal(host(v), ref), mode_ex
        H.cycle(v, dev(f), kappa=kappa, nu1=2, nu2=2, smoother="zebra")   # replay of the captured schedule
        assert np.array_equal(host(v), Ho.cycle(ref, f, kappa=min(kappa, 64), nu1=2, nu2=2)[0]), mode_ex
        H.close()


@pytest.mark.parametrize("n,kappa,theta", [(255, 3, 0.3), (511, 4, 1.2)])
def test_zebra_fused_solve_and_pcg(n, kappa, theta):
    """Fused-mode zebra: stand-alone solve with the oracle's iterations and
    bits (device stop test), PCG with FP64 and FP32 preconditioner cycles."""
    banner(f"zebra fused solve/pcg n={n} kappa={kappa}")
    ep = 1e-5
    f = inputs.uniform_rhs(np.random.default_rng(n + kappa), n)
    Ho = O.Hierarchy(n, theta, ep, smoother="zebra")
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=kappa, tol=1e-8, maxit=500)
    assert rc == O.OK
    check_stop_margin(hist, 1e-8)
    H = K().Hierarchy([(n, theta, ep)], "f64", exec=dict(coarse_cutover=63))
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    it, rr, st = H.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=500, smoother="zebra")
    assert st == [0] and it[0] == it_ref
    assert np.array_equal(host(u), u_ref)
    up_ref, rc, itp_ref, _ = Ho.pcg(f, kappa=kappa, nu1=2, nu2=2, tol=1e-8, maxit=300)
    assert rc == O.OK
    u.zero_()
    it, rr, st = H.pcg(u, dev(f), kappa=kappa, nu1=2, nu2=2, tol=1e-8, maxit=300, smoother="zebra")
    assert st == [0] and it[0] == itp_ref
    assert relmax(host(u), up_ref) <= 1e-11
    H.close()
    H32 = K().Hierarchy([(n, theta, ep)], "f32", exec=dict(coarse_cutover=31))
    u.zero_()
    it, rr, st = H32.pcg(u, dev(f), kappa=kappa, nu1=2, nu2=2, tol=1e-8, maxit=300, smoother="zebra")
    assert st == [0] and abs(it[0] - itp_ref) <= 1
    assert np.linalg.norm(f - Ho.apply(host(u))) / np.linalg.norm(f) < 1e-8
    u.zero_()
    it, rr, st = H32.solve(u, dev(f), kappa=kappa, tol=1e-8, maxit=500, smoother="zebra")
    assert st == [0]
    assert np.linalg.norm(f - Ho.apply(host(u))) / np.linalg.norm(f) < 1e-8
    H32.close()


def test_zebra_fused_batched_ragged():
    """A ragged batch in the fused mode whose instances reach the cutover at
    different depths (one lies below it altogether): each instance gets the
    oracle's iterations and bits."""
    banner("zebra fused batched ragged")
    specs = [(255, 0.4, 1e-3), (31, 1.3, 1e-2), (127, 2.6, 1e-4), (511, 0.05, 1e-5), (63, 2.2, 3e-3)]
    rng = np.random.default_rng(21)
    fs = [inputs.uniform_rhs(rng, s[0]) for s in specs]
    H = K().Hierarchy(specs, "f64", exec=dict(coarse_cutover=31))
    us = [torch.zeros((s[0], s[0]), dtype=torch.float64, device="cuda") for s in specs]
    iters, relres, status = H.solve(us, [dev(f) for f in fs], kappa=3, tol=1e-8, maxit=400, smoother="zebra")
    assert status == [0] * len(specs)
    for k, (s, f) in enumerate(zip(specs, fs)):
        u_ref, rc, it_ref, hist = O.Hierarchy(*s, smoother="zebra").solve(f, kappa=3, tol=1e-8, maxit=400)
        assert rc == O.OK and iters[k] == it_ref, k
        assert np.array_equal(host(us[k]), u_ref), k
    H.close()


@pytest.mark.parametrize("n,nc,mode", [(1, 1, "fused"), (1, 1, "paper"), (3, 1, "fused"), (3, 3, "paper"),
                                       (7, 7, "fused"), (7, 1, "paper"), (15, 3, "fused")])
def test_degenerate_sizes(n, nc, mode):
    """Problems with one point, no coarsening or a single coarse level: the
    solve gives the oracle's iterations and bits (FP64); FP32 refinement converges."""
    banner(f"degenerate size n={n} nc={nc} mode={mode}")
    th, ep = 0.7, 1e-2
    f = np.random.default_rng(n + nc).uniform(-1, 1, (n, n))
    Ho = O.Hierarchy(n, th, ep, n_coarsest=nc)
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=2, tol=1e-10, maxit=200)
    assert rc == O.OK
    check_stop_margin(hist, 1e-10)
    H = K().Hierarchy([(n, th, ep, nc)], "f64", exec=dict(mode=mode))
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    it, rr, st = H.solve(u, dev(f), kappa=2, tol=1e-10, maxit=200)
    assert st == [0] and it[0] == it_ref and np.array_equal(host(u), u_ref)
    H.close()
    H32 = K().Hierarchy([(n, th, ep, nc)], "f32", exec=dict(mode=mode))
    u.zero_()
    it, rr, st = H32.solve(u, dev(f), kappa=2, tol=1e-10, maxit=200)
    assert st == [0]
    assert np.linalg.norm(f - Ho.apply(host(u))) <= 1e-10 * np.linalg.norm(f)
    H32.close()


def test_zebra_fused_batched_fp32_refinement():
    """A ragged batch with FP32 zebra cycles and FP64 refinement in the fused
    mode (calls at 63^2 in the persistent kernel): every instance reaches the
    tolerance on its true FP64 residual within one cycle of the oracle's FP32
    emulation, including a grid-aligned instance that damped Jacobi barely
    reduces."""
    banner("zebra fused batched FP32 refinement")
    specs = [(511, 0.02, 1e-4), (255, 1.9, 1e-3), (127, 0.7, 1e-5), (1023, 3.1, 3e-5)]
    rng = np.random.default_rng(33)
    fs = [inputs.uniform_rhs(rng, s[0]) for s in specs]
    H = K().Hierarchy(specs, "f32", exec=dict(coarse_cutover=63))
    us = [torch.zeros((s[0], s[0]), dtype=torch.float64, device="cuda") for s in specs]
    iters, relres, status = H.solve(us, [dev(f) for f in fs], kappa=3, tol=1e-8, maxit=300, smoother="zebra")
    assert status == [0] * len(specs)
    for k, (s, f) in enumerate(zip(specs, fs)):
        Ho = O.Hierarchy(*s, smoother="zebra")
        u_ir, rc, it_ir, _ = Ho.ir_solve(f, kappa=3, tol=1e-8, maxit=300)
        assert rc == O.OK and abs(iters[k] - it_ir) <= 1, (k, iters[k], it_ir)
        got = host(us[k])
        assert np.linalg.norm(f - Ho.apply(got)) / np.linalg.norm(f) < 1e-8, k
        assert relmax(got, u_ir) <= 1e-6, k
    H.close()


def test_zebra_fp32_step_mapping_independent():
    """One FP32 zebra-cycle refinement step (maxit = 1) on 511^2 with every
    line mapping (four lines per wave from 255^2, from 63^2, two lines per
    wave only, one thread per line only): the four results are bitwise
    equal, and within FP32 rounding of the oracle's FP32 emulation."""
    banner("zebra FP32 step, line mappings")
    n, kappa, th, ep = 511, 2, 0.9, 1e-4
    f = inputs.uniform_rhs(np.random.default_rng(77), n)
    Ho = O.Hierarchy(n, th, ep, smoother="zebra")
    u_ref, rc, it_ref, _ = Ho.ir_solve(f, kappa=kappa, tol=1e-300, maxit=1)
    assert rc == O.NOT_CONVERGED and it_ref == 1
    outs = []
    for wave_n, quad_n in ((63, 255), (1, 63), (63, 0), (0, 0)):
        H = K().Hierarchy([(n, th, ep)], "f32", exec=dict(mode="paper", zebra_wave_n=wave_n, zebra_quad_n=quad_n))
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        it, rr, st = H.solve(u, dev(f), kappa=kappa, tol=1e-300, maxit=1, smoother="zebra")
        assert st == [K().KC_NOT_CONVERGED] and it == [1]
        outs.append(host(u))
        H.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    print(f"  bitwise equal to the oracle's FP32 emulation: {np.array_equal(outs[0], u_ref)}, "
          f"relmax {relmax(outs[0], u_ref):.2e}", flush=True)
    assert relmax(outs[0], u_ref) <= 1e-5


@pytest.mark.parametrize("n,nc,mode", [(1, 1, "fused"), (3, 1, "fused"), (3, 1, "paper"), (7, 7, "fused"),
                                       (7, 3, "paper"), (15, 1, "fused"), (15, 3, "paper")])
def test_zebra_degenerate_sizes(n, nc, mode):
    """Zebra relaxation on one-point problems, single coarse levels and
    problems below the cutover: the oracle's iterations and bits (FP64)."""
    banner(f"zebra degenerate size n={n} nc={nc} mode={mode}")
    th, ep = 1.1, 1e-3
    f = np.random.default_rng(5 * n + nc).uniform(-1, 1, (n, n))
    Ho = O.Hierarchy(n, th, ep, n_coarsest=nc, smoother="zebra")
    u_ref, rc, it_ref, hist = Ho.solve(f, kappa=2, tol=1e-10, maxit=200)
    assert rc == O.OK
    check_stop_margin(hist, 1e-10)
    H = K().Hierarchy([(n, th, ep, nc)], "f64", exec=dict(mode=mode))
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    it, rr, st = H.solve(u, dev(f), kappa=2, tol=1e-10, maxit=200, smoother="zebra")
    assert st == [0] and it[0] == it_ref and np.array_equal(host(u), u_ref)
    u.zero_()
    it, rr, st = H.solve(u, dev(np.zeros((n, n))), kappa=2, tol=1e-10, maxit=200, smoother="zebra")
    assert st == [0] and it[0] == 0 and not host(u).any()   # f = 0: stops before the first cycle
    H.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zero_right_hand_side(prec):
    """f = 0: the solvers stop before the first cycle with u = 0."""
    banner(f"zero right-hand side {prec}")
    n = 127
    H = K().Hierarchy([(n, 0.3, 1e-3)], prec)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    f = torch.zeros_like(u)
    it, rr, st = H.solve(u, f, kappa=2, tol=1e-8, maxit=50)
    assert st == [0] and it == [0] and rr == [0.0] and not bool(u.any())
    it, rr, st = H.pcg(u, f, kappa=2, tol=1e-8, maxit=50)
    assert st == [0] and it == [0] and not bool(u.any())
    H.close()


def test_full_size_c3_pcg_properties():
    """At the full 4095^2 size of the PCG workload: one FP64 cycle is the
    oracle's bits, and the FP32-preconditioned CG reaches the tolerance on
    the true residual (computed on the device in FP64) with an iteration
    count close to the FP64-preconditioned one."""
    banner("full-size 4095^2 PCG properties")
    w = inputs.config3()
    inst = w.instances[0]
    n = inst.n
    f = dev(inst.f)
    v0 = np.random.default_rng(12).uniform(-1, 1, (n, n))
    H64 = K().Hierarchy([(n, inst.theta, inst.eps)], "f64")
    v = dev(v0)
    H64.cycle(v, f, kappa=2, nu1=1, nu2=1)
    ref = O.Hierarchy(n, inst.theta, inst.eps).cycle(v0, inst.f, kappa=2, nu1=1, nu2=1)[0]
    assert np.array_equal(host(v), ref)
    u64 = torch.zeros_like(f)
    it64, _, st64 = H64.pcg(u64, f, kappa=2, nu1=1, nu2=1, tol=w.tol, maxit=1000)
    H32 = K().Hierarchy([(n, inst.theta, inst.eps)], "f32")
    u = torch.zeros_like(f)
    it, rr, st = H32.pcg(u, f, kappa=2, nu1=1, nu2=1, tol=w.tol, maxit=1000)
    assert st == [0] and st64 == [0] and abs(it[0] - it64[0]) <= 2
    r = torch.empty_like(f)
    H64.apply_A(r, u)
    rel = float(torch.linalg.vector_norm(f - r) / torch.linalg.vector_norm(f))
    assert rel < w.tol and rr[0] < w.tol
    assert float((u - u64).abs().max() / u64.abs().max()) < 1e-9
    H32.close()
    H64.close()


@pytest.mark.parametrize("kappa,execs", [
    (2, [dict(), dict(stream_n=1023), dict(tiny_tile_n=255, small_tile_n=511, coarse_cutover=63),
         dict(mode="paper")]),
    (2 ** 31 - 1, [dict(), dict(stream_n=1023, coarse_cutover=15, coarse_wave_n=7)]),
])
def test_full_size_c2_fp64_solve(kappa, execs):
    """The full 1023^2 stand-alone FP64 solve of the headline workload
    (theta = pi/6, eps = 1e-4, nu = 2+2, tol 1e-8): identical cycle counts and
    bit-for-bit iterates against the oracle, for the default execution options
    and for the kernel shapes the autotuner chooses between (streaming
    strips, 8 x 8 / 16 x 16 tiles, cutovers 15 and 63, the paper-structured
    schedule); every option set rounds each operation the same way."""
    w = inputs.config2()
    inst = w.instances[0]
    n = inst.n
    banner(f"full-size 1023^2 FP64 solve kappa={kappa}")
    Ho = O.Hierarchy(n, inst.theta, inst.eps, omega=w.omega)
    u_ref, rc, it_ref, hist = Ho.solve(inst.f, kappa=min(kappa, 64), nu1=w.nu1, nu2=w.nu2, tol=w.tol, maxit=5000)
    assert rc == O.OK
    check_stop_margin(hist, w.tol)
    f = dev(inst.f)
    for ex in execs:
        banner(f"  exec {ex}")
        H = K().Hierarchy([(n, inst.theta, inst.eps)], "f64", exec=ex)
        u = torch.zeros_like(f)
        it, rr, st = H.solve(u, f, kappa=kappa, nu1=w.nu1, nu2=w.nu2, omega=w.omega, tol=w.tol, maxit=5000)
        assert st == [0] and it[0] == it_ref, ex
        assert np.allclose(H.residual_history(0), hist, rtol=1e-14, atol=0.0), ex
        assert np.array_equal(host(u), u_ref), ex
        H.close()


FP32_STEP_CASES = [
    # n, kappa, execution options, kernels reached
    (1023, 2, dict(stream_n=1023), "streaming strips k_pre_s / k_post_s <float> on 1023^2"),
    (1023, 3, dict(stream_n=0, mid_tile_n=1023), "32 x 32 float tiles on 1023^2, 16 x 16 below"),
    (511, 3, dict(tiny_tile_n=255, small_tile_n=511, stream_n=0), "8 x 8 and 16 x 16 float tiles, junctions"),
    (511, 2, dict(coarse_cutover=31, coarse_threads=512, coarse_wave_n=15), "k_subtree<float, 512>, cutover 31"),
    (511, 4, dict(coarse_cutover=63, coarse_threads=1024, coarse_wave_n=15), "k_subtree<float, 1024>, cutover 63"),
    (255, 2, dict(coarse_cutover=63, coarse_threads=512, coarse_wave_n=7), "k_subtree<float, 512>, cutover 63"),
    (255, 3, dict(mode="paper"), "paper-structured FP32 kernels"),
]


@pytest.mark.parametrize("n,kappa,ex,what", FP32_STEP_CASES)
def test_fp32_refinement_step_elementwise(n, kappa, ex, what):
    """One FP32-cycle refinement step (maxit = 1) against the oracle's FP32
    emulation, element by element.  The FP32 right-hand side is the FP64
    residual times a power of two, rounded once on both sides, the FP32
    stencils and Jacobi weights are the FP64 ones rounded once, and the FP32
    kernels keep the FP64 kernels' operation order, so the step is expected
    bit for bit; the maximum difference in FP32 ulps is printed."""
    banner(f"FP32 refinement step n={n} kappa={kappa}: {what}")
    rng = np.random.default_rng(n + kappa)
    f = inputs.uniform_rhs(rng, n)
    th, ep = math.pi / 6, 1e-4
    Ho = O.Hierarchy(n, th, ep)
    u_ref, rc, it_ref, _ = Ho.ir_solve(f, kappa=kappa, tol=1e-300, maxit=1)
    assert rc == O.NOT_CONVERGED and it_ref == 1
    H = K().Hierarchy([(n, th, ep)], "f32", exec=ex)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    it, rr, st = H.solve(u, dev(f), kappa=kappa, tol=1e-300, maxit=1)
    assert st == [K().KC_NOT_CONVERGED] and it == [1]
    got = host(u)
    # u = e / scale with e the FP32 cycle result: compare e in FP32 ulps
    ulp = np.spacing(np.abs(u_ref).astype(np.float32)).astype(np.float64)
    diff = np.abs(got - u_ref)
    print(f"  max |diff| = {diff.max():.3e}, in FP32 ulps of u: {float((diff / np.maximum(ulp, 1e-300)).max()):.2f}",
          flush=True)
    assert np.array_equal(got, u_ref), what
    H.close()


def test_zebra_rejects_oversized_leading_dimension():
    """The zebra line kernels use 32-bit offsets: a caller's fine-level array
    whose (n - 1) * ld + n - 1 exceeds 2^31 - 1 is rejected with KC_ERR_ARG
    before anything is launched (the Jacobi kernels take it)."""
    import ctypes as C
    KK = K()
    n = 7
    H = KK.Hierarchy([(n, 0.3, 1e-3)])
    v = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    f = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    big = (2 ** 31 - 1) // (n - 1) + 1
    pv = (C.c_void_p * 1)(v.data_ptr())
    pf = (C.c_void_p * 1)(f.data_ptr())
    ok_ld = (C.c_int64 * 1)(n)
    big_ld = (C.c_int64 * 1)(big)
    cz = KK.CycleParams(1, 2, 2, 1, 0.8)
    rc = KK.lib().kc_cycle(H._h, pv, big_ld, pf, ok_ld, C.byref(cz))
    assert rc == KK.KC_ERR_ARG
    assert b"zebra" in KK.lib().kc_last_error()
    it = (C.c_int32 * 1)()
    rr = (C.c_double * 1)()
    st = (C.c_int32 * 1)()
    rc = KK.lib().kc_solve(H._h, pv, ok_ld, pf, big_ld, C.byref(cz), 1e-8, 5, it, rr, st)
    assert rc == KK.KC_ERR_ARG
    H.close()


def test_stream_kernels_8191_cycle_bitwise():
    """One FP64 V-cycle at 8191^2 (beyond the Infinity Cache): the streaming
    pre- and post-smoothing strips of 32 rows give the oracle's bits."""
    n = 8191
    banner(f"streaming kernels one cycle n={n}")
    rng = np.random.default_rng(81)
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = K().Hierarchy([(n, math.pi / 4, 1e-4)])
    v = dev(v0)
    H.cycle(v, dev(f), kappa=1, nu1=2, nu2=2)
    got = host(v)
    H.close()
    del v
    torch.cuda.empty_cache()
    ref = O.Hierarchy(n, math.pi / 4, 1e-4).cycle(v0, f, kappa=1, nu1=2, nu2=2)[0]
    assert np.array_equal(got, ref)
