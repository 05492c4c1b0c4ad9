"""Pins of the oracle's cycles and drivers.

* Two- and three-level cycles equal a dense-matrix brute force of Algorithm 3.
* The cycle is an affine stationary iteration: cycle(u, f) = u + cycle(0, f - Au),
  and the exact solution is its fixed point.
* Cycle operator B (zero guess): symmetric and positive definite for V and W
  with nu1 = nu2, not symmetric for the F-cycle with four or more levels
  (Section 4, the discussion of MGCG); kappa = n-1 gives W's iterates.
* Poisson (eps=1) converges at a multigrid rate.
* PCG with an exact preconditioner (one level) converges in one iteration;
  PCG, FP32-refined and paper-protocol drivers reach their targets.
* Parameter gradients equal central differences of a dense brute force.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.test_oracle_operators import dense_bilinear, dense_stencil_matrix


def dense_levels(H):
    """Dense A_l (= S_l/h_l^2) and P_l for every level of an oracle hierarchy."""
    As, Ps = [], []
    for k in range(H.levels):
        n = H.sizes[k]
        As.append(dense_stencil_matrix(H.stencils[k], n) * (n + 1) ** 2)
        if k + 1 < H.levels:
            Ps.append(dense_bilinear(H.sizes[k + 1]))
    return As, Ps


def dense_kcycle(As, Ps, k, v, f, kappa, nu1, nu2, omega):
    A = As[k]
    if k == len(As) - 1:
        return np.linalg.solve(A, f)
    d = np.diag(A)
    for _ in range(nu1):
        v = v + omega * (f - A @ v) / d
    fc = (Ps[k].T / 4) @ (f - A @ v)
    vc = np.zeros(fc.shape)
    vc = dense_kcycle(As, Ps, k + 1, vc, fc, kappa, nu1, nu2, omega)
    if kappa > 1:
        vc = dense_kcycle(As, Ps, k + 1, vc, fc, kappa - 1, nu1, nu2, omega)
    v = v + Ps[k] @ vc
    for _ in range(nu2):
        v = v + omega * (f - A @ v) / d
    return v


@pytest.mark.parametrize("n,nc,kappa,nu", [(7, 3, 1, (2, 2)), (15, 3, 2, (1, 2)), (15, 1, 3, (2, 1)),
                                           (31, 7, 2, (2, 2)), (31, 1, 5, (1, 1))])
def test_cycle_equals_dense_bruteforce(n, nc, kappa, nu):
    H = O.Hierarchy(n, 0.5, 2e-3, n_coarsest=nc, omega=0.8)
    As, Ps = dense_levels(H)
    rng = np.random.default_rng(n + kappa)
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    v = H.cycle(v0, f, kappa=kappa, nu1=nu[0], nu2=nu[1])[0]
    vd = dense_kcycle(As, Ps, 0, v0.ravel(), f.ravel(), kappa, nu[0], nu[1], 0.8)
    assert np.abs(v.ravel() - vd).max() <= 1e-12 * np.abs(vd).max()


@pytest.mark.parametrize("kappa", [1, 2, 3, 9])
def test_affine_identity_and_fixed_point(kappa):
    n = 31
    H = O.Hierarchy(n, 1.1, 1e-2)
    rng = np.random.default_rng(kappa)
    u, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    a = H.cycle(u, f, kappa=kappa)[0]
    b = u + H.cycle(np.zeros((n, n)), f - H.apply(u), kappa=kappa)[0]
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    A = dense_stencil_matrix(H.stencils[0], n) * (n + 1) ** 2
    ustar = np.linalg.solve(A, f.ravel()).reshape(n, n)
    c = H.cycle(ustar, f, kappa=kappa)[0]
    assert np.abs(c - ustar).max() <= 1e-11 * np.abs(ustar).max()


def cycle_matrix(H, kappa, nu):
    n = H.n
    m = n * n
    B = np.zeros((m, m))
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        B[:, k] = H.cycle(np.zeros((n, n)), e.reshape(n, n), kappa=kappa, nu1=nu, nu2=nu)[0].ravel()
    return B


def asym(B):
    return np.abs(B - B.T).max() / np.abs(B).max()


@pytest.mark.parametrize("L", [3, 4, 5])
def test_cycle_operator_symmetry(L):
    H = O.Hierarchy(2 ** L - 1, math.pi / 4, 1e-3, omega=0.8)
    Bv = cycle_matrix(H, 1, 2)
    Bw = cycle_matrix(H, L, 2)
    Bw1 = cycle_matrix(H, L - 1, 2)
    assert asym(Bv) < 1e-13 and asym(Bw) < 1e-13
    assert np.array_equal(Bw, Bw1)                 # kappa = n-1 reproduces W
    for B in (Bv, Bw):                             # SPD preconditioners
        assert np.linalg.eigvalsh((B + B.T) / 2).min() > 0
    if L >= 4:
        assert asym(cycle_matrix(H, 2, 2)) > 1e-4   # the F-cycle is not symmetric
    if L == 5:
        assert asym(cycle_matrix(H, 3, 2)) > 1e-5


def test_poisson_multigrid_rate():
    """eps = 1 (Poisson): a V(2,2)-cycle with damped Jacobi reduces the error
    by a grid-independent factor well below 1."""
    rates = []
    for n in (63, 127, 255):
        H = O.Hierarchy(n, 0.0, 1.0)
        rng = np.random.default_rng(n)
        u0 = rng.uniform(-1, 1, (n, n))
        u, rc, it, hist = H.solve(np.zeros((n, n)), kappa=1, tol=1e-8, maxit=60, u0=u0, mode=1)
        assert rc == O.OK
        rates.append(hist[-1] ** (1.0 / it))
    assert max(rates) < 0.2
    assert max(rates) - min(rates) < 0.05


def test_paper_protocol_error_reduction():
    """f = 0, random initial guess, stop when the error norm drops by 1e8."""
    n = 127
    H = O.Hierarchy(n, math.pi / 4, 1e-2)
    u0 = np.random.default_rng(11).uniform(-1, 1, (n, n))
    counts = []
    for kappa in (1, 2, 3, 7):
        u, rc, it, hist = H.solve(np.zeros((n, n)), kappa=kappa, tol=1e-8, maxit=2000, u0=u0, mode=1)
        assert rc == O.OK
        assert np.linalg.norm(u) < 1e-8 * np.linalg.norm(u0)
        assert np.linalg.norm(u) >= 0.0
        counts.append(it)
    # stronger cycles converge in fewer (or as many) cycles
    assert counts == sorted(counts, reverse=True)


def test_standalone_stop_rule():
    n = 63
    H = O.Hierarchy(n, 0.4, 1e-3, n_coarsest=3)
    f = np.random.default_rng(0).uniform(-1, 1, (n, n))
    u, rc, it, hist = H.solve(f, kappa=2, tol=1e-10, maxit=500)
    assert rc == O.OK
    assert hist[-1] < 1e-10 and np.all(hist[:-1] >= 1e-10)
    r = f - H.apply(u)
    assert abs(np.linalg.norm(r) / np.linalg.norm(f) - hist[-1]) <= 1e-12 * hist[-1]
    # maxit reached: status "not converged", iterations = maxit
    u1, rc1, it1, h1 = H.solve(f, kappa=2, tol=1e-10, maxit=1)
    assert rc1 == O.NOT_CONVERGED and it1 == 1
    # a damping factor beyond the Jacobi stability bound diverges
    Hd = O.Hierarchy(n, 0.4, 1e-3, n_coarsest=3, omega=2.5)
    u2, rc2, it2, h2 = Hd.solve(f, kappa=1, tol=1e-10, maxit=500)
    assert rc2 == O.DIVERGED
    bad = f.copy()
    bad[3, 4] = np.nan
    assert H.solve(bad, kappa=1, tol=1e-10, maxit=5)[1] == O.ERR_NONFINITE
    assert H.ir_solve(bad, kappa=1, tol=1e-10, maxit=5)[1] == O.ERR_NONFINITE
    assert H.pcg(bad, kappa=1, tol=1e-10, maxit=5)[1] == O.ERR_NONFINITE


def test_restart_reproduces_iterates():
    """The stand-alone iteration is stationary: stopping after k cycles and
    restarting from the saved u gives the uninterrupted iterates bitwise."""
    n = 63
    H = O.Hierarchy(n, 0.7, 1e-3, n_coarsest=3)
    f = np.random.default_rng(4).uniform(-1, 1, (n, n))
    u10 = H.solve(f, kappa=3, tol=0.0, maxit=10)[0]
    u4 = H.solve(f, kappa=3, tol=0.0, maxit=4)[0]
    u10b = H.solve(f, kappa=3, tol=0.0, maxit=6, u0=u4)[0]
    assert np.array_equal(u10, u10b)


def test_pcg_exact_preconditioner_one_iteration():
    n = 7
    H = O.Hierarchy(n, 0.8, 1e-2, n_coarsest=7)
    f = np.random.default_rng(2).uniform(-1, 1, (n, n))
    u, rc, it, hist = H.pcg(f, kappa=1, tol=1e-12, maxit=10)
    assert rc == O.OK and it == 1


@pytest.mark.parametrize("kappa,f32", [(1, False), (2, False), (3, False), (3, True), (6, True)])
def test_pcg_converges_to_dense_solution(kappa, f32):
    n = 31
    H = O.Hierarchy(n, 3 * math.pi / 8, 1e-3, omega=0.8)
    f = np.random.default_rng(kappa).uniform(-1, 1, (n, n))
    u, rc, it, hist = H.pcg(f, kappa=kappa, nu1=1, nu2=1, tol=1e-10, maxit=300, precond_f32=f32)
    assert rc == O.OK and hist[-1] < 1e-10
    A = dense_stencil_matrix(H.stencils[0], n) * (n + 1) ** 2
    ustar = np.linalg.solve(A, f.ravel())
    # recurrence residual and true residual agree; error bounded by cond * tol
    true_rel = np.linalg.norm(f.ravel() - A @ u.ravel()) / np.linalg.norm(f)
    assert true_rel < 1e-9
    assert np.linalg.norm(u.ravel() - ustar) / np.linalg.norm(ustar) < 1e-6


@pytest.mark.parametrize("kappa", [1, 3])
def test_ir_reaches_fp64_tolerance(kappa):
    n = 127
    H = O.Hierarchy(n, math.pi / 6, 1e-4)
    f = np.random.default_rng(1).uniform(-1, 1, (n, n))
    u64, rc64, it64, _ = H.solve(f, kappa=kappa, tol=1e-8, maxit=3000)
    u32, rc32, it32, hist = H.ir_solve(f, kappa=kappa, tol=1e-8, maxit=3000)
    assert rc64 == O.OK and rc32 == O.OK
    assert hist[-1] < 1e-8
    true_rel = np.linalg.norm(f - H.apply(u32)) / np.linalg.norm(f)
    assert true_rel < 1e-8
    assert it32 <= it64 + 2
    assert np.abs(u32 - u64).max() <= 1e-5 * np.abs(u64).max()


def test_fp32_cycle_close_to_fp64():
    n = 63
    H = O.Hierarchy(n, 0.6, 1e-2)
    f = np.random.default_rng(9).uniform(-1, 1, (n, n))
    v64 = H.cycle(np.zeros((n, n)), f, kappa=3)[0]
    v32 = H.cycle_f32(np.zeros((n, n), np.float32), f.astype(np.float32), kappa=3)
    assert np.abs(v32 - v64).max() <= 1e-5 * np.abs(v64).max()


def test_ir_scale_power_of_two():
    for ss, N in [(1.0, 1), (3.7e-20, 1000), (5e10, 7), (1e-300, 10 ** 6)]:
        s = O.ir_scale(ss, N)
        m, e = math.frexp(s)
        assert m == 0.5
        rms = math.sqrt(ss / N)
        assert 1.0 <= s * rms < 2.0
    assert O.ir_scale(0.0, 10) == 1.0


def dense_loss_grad(n, theta, eps, f):
    h = 1.0 / (n + 1)

    def A(t, e):
        return dense_stencil_matrix(O.fine_stencil(t, e), n) / h ** 2

    def loss(t, e):
        u = np.linalg.solve(A(t, e), f.ravel())
        us = np.linalg.solve(A(theta + 0.1, 2 * eps), f.ravel())
        return 0.5 * np.dot(u - us, u - us)

    d = 1e-6
    g_th = (loss(theta + d, eps) - loss(theta - d, eps)) / (2 * d)
    de = 1e-6 * eps
    g_e = (loss(theta, eps + de) - loss(theta, eps - de)) / (2 * de)
    return g_th, g_e, A(theta, eps), np.linalg.solve(A(theta + 0.1, 2 * eps), f.ravel())


@pytest.mark.parametrize("theta,eps", [(0.4, 1e-2), (2.2, 0.07), (math.pi / 4, 1e-3)])
def test_grad_params_bruteforce(theta, eps):
    n = 15
    f = np.random.default_rng(5).uniform(-1, 1, (n, n))
    g_th, g_e, A, us = dense_loss_grad(n, theta, eps, f)
    u = np.linalg.solve(A, f.ravel())
    lam = np.linalg.solve(A.T, u - us)
    H = O.Hierarchy(n, theta, eps)
    dth, de = H.grad_params(lam.reshape(n, n), u.reshape(n, n))
    assert abs(dth - g_th) <= 1e-6 * abs(g_th) + 1e-12
    assert abs(de - g_e) <= 1e-6 * abs(g_e) + 1e-12
