"""CPU-only checks of the C-ABI library: it loads, exports every symbol that
include/kcycle.h declares, and its host-side logic (level stencils, workspace
sizing, argument validation, launch schedule) is right.  No GPU calls."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2010_00626_amd import kcycle as K
from paper_2010_00626_amd import model as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kcycle.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kc_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    lib = C.CDLL(K.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("n,theta,eps,nc", [(1023, math.pi / 6, 1e-4, 1), (63, math.pi / 4, 1e-3, 3),
                                            (4095, 3 * math.pi / 8, 1e-5, 1), (2047, 0.3, 0.1, 7),
                                            (255, 2.9, 1e-5, 1), (7, 1.0, 1.0, 7)])
def test_level_stencils_match_oracle_bitwise(n, theta, eps, nc):
    s = K.level_stencils(n, theta, eps, nc)
    H = O.Hierarchy(n, theta, eps, n_coarsest=nc)
    assert s.shape == H.stencils.shape
    assert np.array_equal(s, H.stencils)


def test_workspace_bytes_and_validation():
    b1 = K.workspace_bytes([(1023, 0.5, 1e-4)])
    b2 = K.workspace_bytes([(1023, 0.5, 1e-4), (255, 0.1, 1e-2)])
    assert b2 > b1 > 5 * 1023 * 1023 * 8
    assert K.workspace_bytes([(1023, 0.5, 1e-4)], "f32") > 0
    for bad in [(64, 0.5, 1e-4), (63, 0.5, 0.0), (63, 0.5, 1e-4, 5), (3, 0.5, 1e-4, 7), (63, float("nan"), 1e-4)]:
        with pytest.raises(K.KCycleError) as ei:
            K.workspace_bytes([bad])
        assert ei.value.status == K.KC_ERR_ARG


def test_create_rejects_bad_workspace_without_gpu():
    L = K.lib()
    probs, n = K._problems([(63, 0.5, 1e-3)])
    need = K.workspace_bytes([(63, 0.5, 1e-3)])
    h = C.c_void_p()
    e = K.exec_options()
    assert L.kc_create(probs, n, 0, C.byref(e), None, need, None, C.byref(h)) == K.KC_ERR_WORKSPACE
    assert L.kc_create(probs, n, 0, C.byref(e), C.c_void_p(4096), need - 1, None, C.byref(h)) == K.KC_ERR_WORKSPACE
    assert L.kc_create(probs, n, 0, C.byref(e), C.c_void_p(4096 + 8), need, None, C.byref(h)) == K.KC_ERR_WORKSPACE
    bad = K.exec_options(coarse_cutover=5)
    assert L.kc_create(probs, n, 0, C.byref(bad), C.c_void_p(4096), need, None, C.byref(h)) == K.KC_ERR_ARG
    assert h.value is None
    assert b"workspace" in L.kc_last_error() or b"cutover" in L.kc_last_error()
    assert L.kc_status_string(K.KC_DIVERGED) == b"KC_DIVERGED"


@pytest.mark.parametrize("L", [2, 3, 5, 8, 10, 12])
@pytest.mark.parametrize("nu", [(2, 2), (1, 1), (2, 1)])
def test_paper_mode_launch_count_is_algorithm4(L, nu):
    """One launch per operation: (5+nu) per non-coarsest call and one per
    coarsest call (Section 3.3), plus one copy when nu1+nu2 is odd."""
    n = 2 ** L - 1
    for kappa in (1, 2, 3, 4, K.KAPPA_W):
        c = K.schedule_counts([(n, 0.4, 1e-3)], kappa, nu[0], nu[1], mode="paper")
        expect = M.n_gpu_calls_paper(kappa, L, nu[0] + nu[1]) + ((nu[0] + nu[1]) % 2)
        assert c["grid_launches"] == expect
        assert c["subtree_launches"] == 0


@pytest.mark.parametrize("L,cutover", [(10, 63), (12, 63), (10, 31), (6, 63), (8, 15)])
def test_fused_mode_launch_count(L, cutover):
    """Fused mode: two grid launches (pre, post) per call above the cutover
    depth and one persistent launch per call at the depth above it."""
    n = 2 ** L - 1
    sizes = [2 ** (L - d) - 1 for d in range(L)]
    cut = next(d for d, s in enumerate(sizes) if s <= cutover)
    for kappa in (1, 2, 3, 4, K.KAPPA_W):
        c = K.schedule_counts([(n, 0.4, 1e-3)], kappa, coarse_cutover=cutover, fuse_junctions=0)
        kk = min(kappa, 10 ** 6)
        grid = 2 * sum(M.level_calls(kk, d + 1) for d in range(cut))
        subs = M.level_calls(kk, cut) if cut > 0 else 1
        assert c["grid_launches"] == grid
        assert c["subtree_launches"] == subs


@pytest.mark.parametrize("L,nu", [(6, (2, 2)), (9, (1, 1)), (12, (2, 0))])
def test_zebra_paper_mode_launch_count(L, nu):
    """Zebra relaxation, one launch per operation: a relaxation is two launches
    (one per colour) and relaxes in place, so a non-coarsest call costs
    5 + 2 (nu1 + nu2) launches and no final copy is needed."""
    n = 2 ** L - 1
    for kappa in (1, 2, 3, 4, K.KAPPA_W):
        c = K.schedule_counts([(n, 0.4, 1e-3)], kappa, nu[0], nu[1], smoother="zebra", mode="paper")
        assert c["grid_launches"] == M.n_gpu_calls_paper(kappa, L, 2 * (nu[0] + nu[1]))
        assert c["subtree_launches"] == 0


@pytest.mark.parametrize("L,cutover", [(10, 63), (12, 31), (6, 63), (8, 15), (5, 31)])
def test_zebra_fused_mode_launch_count(L, cutover):
    """Zebra relaxation in the fused mode: one launch per operation for every
    call above the cutover depth, one persistent launch per call at the depth
    above it (or one for the whole cycle when the fine grid is below the
    cutover), and the persistent op lists hold no register calls."""
    n = 2 ** L - 1
    sizes = [2 ** (L - d) - 1 for d in range(L)]
    cut = next(d for d, s in enumerate(sizes) if s <= cutover)
    for kappa in (1, 2, 3, 4, K.KAPPA_W):
        kk = min(kappa, 10 ** 6)
        c = K.schedule_counts([(n, 0.4, 1e-3)], kappa, 2, 2, smoother="zebra", coarse_cutover=cutover)
        assert c["grid_launches"] == (5 + 2 * 4) * sum(M.level_calls(kk, d + 1) for d in range(cut))
        assert c["subtree_launches"] == (M.level_calls(kk, cut) if cut > 0 else 1)
        j = K.schedule_counts([(n, 0.4, 1e-3)], kappa, 2, 2, coarse_cutover=cutover)
        assert j["subtree_launches"] == c["subtree_launches"]
        assert c["subtree_stages"] >= j["subtree_stages"]


def _grid_sequence(sizes, cut, kappa):
    """Grid-wide launches of one fused cycle, in order: ('pre' | 'post', depth, zero_guess),
    written from Algorithm 3's call structure (the persistent launches are left out)."""
    seq = []

    def call(d, k, zg):
        if d >= cut:
            return
        seq.append(("pre", d, zg))
        call(d + 1, k, True)
        if k > 1:
            call(d + 1, k - 1, False)
        seq.append(("post", d, False))
    call(0, kappa, False)
    return seq


@pytest.mark.parametrize("L,cutover,small,tiny", [(10, 31, 511, 0), (10, 15, 255, 0), (9, 31, 0, 0), (8, 15, 4095, 0),
                                                 (10, 31, 0, 255), (9, 15, 127, 63), (10, 31, 511, 255)])
def test_junction_fusion_launch_count(L, cutover, small, tiny):
    """With junction fusion, every post-smoothing launch followed by the next
    sibling's (non-zero-guess) pre-smoothing on a level run in 16 x 16 or 8 x 8
    tiles is one launch."""
    n = 2 ** L - 1
    sizes = [2 ** (L - d) - 1 for d in range(L)]
    cut = next(d for d, s in enumerate(sizes) if s <= cutover)
    for kappa in (1, 2, 3, 4, K.KAPPA_W):
        seq = _grid_sequence(sizes, cut, min(kappa, L + 1))
        fused = 0
        for a, b in zip(seq, seq[1:]):
            if a[0] == "post" and b[0] == "pre" and a[1] == b[1] and not b[2] and sizes[a[1]] <= max(small, tiny):
                fused += 1
        opts = dict(coarse_cutover=cutover, small_tile_n=small, tiny_tile_n=tiny)
        c0 = K.schedule_counts([(n, 0.4, 1e-3)], kappa, fuse_junctions=0, **opts)
        c1 = K.schedule_counts([(n, 0.4, 1e-3)], kappa, fuse_junctions=1, **opts)
        assert c0["grid_launches"] == len(seq)
        assert c1["grid_launches"] == len(seq) - fused
        if kappa > 1 and any(sizes[e] <= max(small, tiny) for e in range(1, cut)):
            assert fused > 0


def test_profsum_summaries(tmp_path):
    """The profile summaries group dispatches by kernel and grid size: mean
    durations from a kernel trace, mean counter values from a --pmc run."""
    from paper_2010_00626_amd import profsum
    (tmp_path / "t").mkdir()
    with open(tmp_path / "t" / "x_kernel_trace.csv", "w") as fh:
        fh.write("Kernel_Name,Start_Timestamp,End_Timestamp,Grid_Size_X,Grid_Size_Y,Grid_Size_Z\n")
        fh.write("void kc::k_a<float>(kc::StageArgs),0,2000,256,1,1\n")
        fh.write("void kc::k_a<float>(kc::StageArgs),5000,9000,256,1,1\n")
        fh.write("void kc::k_a<float>(kc::StageArgs),0,1000,512,1,1\n")
    out = profsum.summarise(str(tmp_path / "t"))
    assert "# dispatches: 3, kernel time 0.007 ms" in out
    line = [l for l in out.splitlines() if "k_a<float>" in l and " 256 " in l][0].split()
    assert line[-6:] == ["256", "2", "0.006", "3.00", "2.00", "4.00"]
    (tmp_path / "c").mkdir()
    with open(tmp_path / "c" / "x_counter_collection.csv", "w") as fh:
        fh.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        for v in (10.0, 30.0):
            fh.write(f"void kc::k_b<double>(kc::StageArgs),1024,VALUBusy,{v}\n")
        fh.write("void kc::k_b<double>(kc::StageArgs),1024,SQ_WAVES,16\n")
        fh.write("void kc::k_c(kc::StageArgs),64,VALUBusy,99\n")
    out = profsum.summarise_counters(str(tmp_path / "c"), match="k_b")
    rows = out.splitlines()
    assert rows[0].split()[-2:] == ["VALUBusy", "SQ_WAVES"] and len(rows) == 2
    assert rows[1].split()[-4:] == ["1024", "2", "20.0", "16.0"]


def test_exec_options_validated_without_gpu():
    """Execution options out of range are rejected by the host planner (the
    same check kc_create and kc_set_exec run), and the smoother must be 0 or 1."""
    ok = K.schedule_counts([(255, 0.4, 1e-3)], 2, smoother="zebra", zebra_wave_n=0)
    assert ok["grid_launches"] > 0
    ok = K.schedule_counts([(255, 0.4, 1e-3)], 2, smoother="zebra", zebra_quad_n=63)
    assert ok["grid_launches"] > 0
    for bad in (dict(zebra_wave_n=-1), dict(zebra_wave_n=16384), dict(zebra_quad_n=-1),
                dict(zebra_quad_n=16384), dict(coarse_threads=384),
                dict(tiny_tile_n=4096), dict(wave_regs=2)):
        with pytest.raises(K.KCycleError) as ei:
            K.schedule_counts([(255, 0.4, 1e-3)], 2, **bad)
        assert ei.value.status == K.KC_ERR_ARG, bad
    with pytest.raises(K.KCycleError):
        K.schedule_counts([(255, 0.4, 1e-3)], 2, smoother=2)


def test_autograd_gradient_return_for_number_parameters():
    """theta / eps given as Python numbers are no graph inputs: backward
    returns None for them (autograd rejects a tensor there), and tensor
    parameters get their (summed, for a scalar) gradient.  A CPU stand-in
    for the solve exercises the same return assembly as the GPU Function."""
    import torch
    from paper_2010_00626_amd import autograd as ag

    class Stub(torch.autograd.Function):
        @staticmethod
        def forward(ctx, f, theta, eps):
            ctx.theta_shape = torch.as_tensor(theta).shape
            ctx.eps_shape = torch.as_tensor(eps).shape
            ctx.theta_device = theta.device if torch.is_tensor(theta) else torch.device("cpu")
            ctx.eps_device = eps.device if torch.is_tensor(eps) else torch.device("cpu")
            ctx.param_is_tensor = (torch.is_tensor(theta), torch.is_tensor(eps))
            return 2.0 * f

        @staticmethod
        def backward(ctx, gu):
            B = gu.shape[0]
            return ag.assemble_grads(ctx, 2.0 * gu, [1.0] * B, [3.0] * B)[:3]

    f = torch.ones((2, 3, 3), dtype=torch.float64, requires_grad=True)
    Stub.apply(f, 0.3, 1e-3).sum().backward()           # numbers: no gradient for them, no error
    assert torch.equal(f.grad, torch.full_like(f, 2.0))
    th = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    ep = torch.tensor([1e-3, 2e-3], dtype=torch.float64, requires_grad=True)
    Stub.apply(f.detach(), th, ep).sum().backward()
    assert float(th.grad) == 2.0 and ep.grad.tolist() == [3.0, 3.0]
    ep2 = torch.tensor([1e-3, 2e-3], dtype=torch.float64)   # a tensor that needs no gradient
    Stub.apply(f, th.detach(), ep2).sum().backward()


@pytest.mark.parametrize("n,theta,eps,bx,by", [(1023, math.pi / 6, 1e-2, 20.0, 10.0), (63, 0.0, 1.0, -40.0, 15.0),
                                               (255, 2.0, 1e-4, 3.0, -8.0), (7, 1.1, 0.05, 0.0, 0.0)])
def test_convection_stencils_match_oracle_bitwise(n, theta, eps, bx, by):
    s = K.convection_stencils(n, theta, eps, bx, by)
    H = O.Hierarchy(n, theta, eps, convection=(bx, by))
    assert s.shape == H.stencils.shape
    assert np.array_equal(s, H.stencils)


@pytest.mark.parametrize("n,theta,eps", [(1023, math.pi / 4, 1e-5), (63, 0.0, 1e-3), (255, 1.3, 0.2), (1, 0.5, 1.0)])
def test_semi_stencils_match_oracle_bitwise(n, theta, eps):
    s = K.semi_stencils(n, theta, eps)
    H = O.Hierarchy(n, theta, eps, coarsening="semi")
    assert s.shape == H.stencils.shape
    assert np.array_equal(s, H.stencils)


def test_semi_workspace_and_arguments():
    """Semi-coarsened layouts hold n-point lines on every level (more bytes than
    full coarsening) and need one n for the whole batch and n_coarsest = 1."""
    full = K.workspace_bytes([(1023, 0.3, 1e-3)], "f64")
    semi = K.workspace_bytes([(1023, 0.3, 1e-3)], "f64", coarsening="semi")
    assert semi > full
    with pytest.raises(K.KCycleError):
        K.workspace_bytes([(255, 0.3, 1e-3), (127, 0.3, 1e-3)], "f64", coarsening="semi")
    with pytest.raises(K.KCycleError):
        K.workspace_bytes([(255, 0.3, 1e-3, 3)], "f64", coarsening="semi")
    with pytest.raises(K.KCycleError):
        K.workspace_bytes([(32767, 0.3, 1e-3)], "f64", coarsening="semi")


def test_protocol_totals_from_counts():
    """The timing-only protocol rebuilds its totals from an earlier run's
    counts of the same problem: cycles x time per cycle, and a 2-iteration
    CG run plus (iterations - 2) x time per iteration; other problems and
    uncapped runs contribute nothing."""
    from paper_2010_00626_amd import protocol
    key = dict(levels=14, theta=0.5, eps=1e-5, kappa="3", smoother="zebra", coarsening="full")
    counts = [dict(key, solver="standalone", cycles=100), dict(key, solver="mgcg", iterations=12),
              dict(key, solver="standalone", kappa="4", cycles=7), dict(key, solver="mgcg", eps=1e-4, iterations=3)]
    r = protocol.with_counts(dict(key, ms_per_cycle=2.5, pcg_ms_2=7.0, ms_per_iteration=3.0), counts)
    assert r["cycles"] == 100 and r["standalone_total_ms"] == 250.0
    assert r["iterations"] == 12 and r["mgcg_total_ms"] == 7.0 + 10 * 3.0
    capped = protocol.with_counts(dict(key, ms_per_cycle=1.0, pcg_ms_2=1.0, ms_per_iteration=1.0),
                                  [dict(key, solver="standalone", cycles=None, cap=8000)])
    assert capped["cycles_cap"] == 8000 and "standalone_total_ms" not in capped
