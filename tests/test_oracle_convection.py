"""Pins of the oracle's convection-diffusion operator and cycles (the
nonsymmetric problem named in the conclusions): -div(D grad u) + b . grad u
with the Section 4 diffusion D = R(theta) diag(1, eps) R(theta)^T and upwind
convection, every level rediscretised at its own mesh width.

* The fine stencil applies the continuous diffusion and the one-sided
  (upwind) difference quotients exactly to every quadratic; it is the
  diffusion stencil when b = 0 and an M-matrix row for any b.
* Every coarse level carries the same operator at its own mesh width.
* Two- and three-level cycles equal a dense brute force built here from the
  definitions (dense stencil matrices, dense bilinear P, R = P^T / 4, dense
  Jacobi, a dense coarsest solve).
* The cycle operator is not symmetric; the method converges fast where
  Galerkin operators R A P of the same upwind operator diverge (the reason
  for rediscretisation); PCG refuses the nonsymmetric operator.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from test_oracle_operators import dense_bilinear, dense_stencil_matrix, diffusion_tensor, grid_xy

CASES = [(0.0, 1.0, 10.0, 5.0), (math.pi / 6, 1e-2, 20.0, 10.0), (2.0, 0.3, -40.0, 15.0), (0.7, 1e-4, 3.0, -8.0),
         (1.1, 0.05, -100.0, -50.0)]


@pytest.mark.parametrize("theta,eps,bx,by", CASES)
def test_convection_stencil_exact_on_quadratics(theta, eps, bx, by):
    n = 15
    X, Y, h = grid_xy(n)
    D = diffusion_tensor(theta, eps)
    s = O.convection_stencil(n, theta, eps, bx, by)
    rng = np.random.default_rng(3)
    for _ in range(3):
        a, b, c, d, e, g = rng.uniform(-1, 1, 6)
        q = lambda x, y: a * x * x + b * x * y + c * y * y + d * x + e * y + g
        Aq = O.apply_stencil(s, q(X, Y)) / (h * h)
        # upwind quotients: backward along a positive component, forward along a negative one
        qx = (q(X, Y) - q(X - h, Y)) / h if bx > 0 else (q(X + h, Y) - q(X, Y)) / h
        qy = (q(X, Y) - q(X, Y - h)) / h if by > 0 else (q(X, Y + h) - q(X, Y)) / h
        exact = -(2 * a * D[0, 0] + 2 * b * D[0, 1] + 2 * c * D[1, 1]) + bx * qx + by * qy
        assert np.allclose(Aq[1:-1, 1:-1], exact[1:-1, 1:-1], rtol=0, atol=1e-8 * (1 + np.abs(exact).max()))


@pytest.mark.parametrize("theta,eps,bx,by", CASES)
def test_convection_stencil_structure(theta, eps, bx, by):
    n = 31
    s = O.convection_stencil(n, theta, eps, bx, by)
    h = 1.0 / (n + 1)
    d = O.fine_stencil(theta, eps)
    assert np.array_equal(O.convection_stencil(n, theta, eps, 0.0, 0.0), d)
    diff = s - d      # the convection part only: row sum zero, weight h |b| on the upwind side
    assert abs(diff.sum()) < 1e-14
    assert diff[1, 1] == pytest.approx(h * (abs(bx) + abs(by)), rel=1e-15)
    assert diff[1, 0] == pytest.approx(-h * max(bx, 0.0), abs=1e-14)
    assert diff[1, 2] == pytest.approx(-h * max(-bx, 0.0), abs=1e-14)
    assert diff[0, 1] == pytest.approx(-h * max(by, 0.0), abs=1e-14)
    assert diff[2, 1] == pytest.approx(-h * max(-by, 0.0), abs=1e-14)
    assert np.count_nonzero(diff[[0, 0, 2, 2], [0, 2, 0, 2]]) == 0


@pytest.mark.parametrize("theta,eps,bx,by", CASES)
def test_coarse_levels_rediscretised(theta, eps, bx, by):
    n = 63
    H = O.Hierarchy(n, theta, eps, convection=(bx, by))
    assert H.sizes == [63, 31, 15, 7, 3, 1]
    for k, nk in enumerate(H.sizes):
        assert np.array_equal(H.stencils[k], O.convection_stencil(nk, theta, eps, bx, by))
    # the convection part doubles from level to level (h_l doubles)
    c0 = H.stencils[0] - O.fine_stencil(theta, eps)
    c1 = H.stencils[1] - O.fine_stencil(theta, eps)
    assert np.allclose(c1, 2 * c0, rtol=1e-14, atol=1e-17)


def dense_cycle(n, theta, eps, b, kappa, nu1, nu2, omega, v, f):
    """Algorithm 3 with dense matrices built from the definitions."""
    ns = [n]
    while ns[-1] > 1:
        ns.append((ns[-1] - 1) // 2)
    A = [dense_stencil_matrix(O.convection_stencil(m, theta, eps, *b), m) * (m + 1) ** 2 for m in ns]

    def kc(l, v, f, k):
        if l == len(ns) - 1:
            return np.linalg.solve(A[l], f)
        D = np.diag(A[l])
        for _ in range(nu1):
            v = v + omega * (f - A[l] @ v) / D
        P = dense_bilinear(ns[l + 1])
        fc = (P.T / 4) @ (f - A[l] @ v)
        vc = kc(l + 1, np.zeros(ns[l + 1] ** 2), fc, k)
        if k > 1:
            vc = kc(l + 1, vc, fc, k - 1)
        v = v + P @ vc
        for _ in range(nu2):
            v = v + omega * (f - A[l] @ v) / D
        return v

    return kc(0, v.ravel(), f.ravel(), kappa).reshape(n, n)


@pytest.mark.parametrize("n,kappa", [(3, 1), (7, 1), (7, 2), (15, 3), (15, 1)])
@pytest.mark.parametrize("case", CASES[:3])
def test_cycle_equals_dense_brute_force(n, kappa, case):
    theta, eps, bx, by = case
    rng = np.random.default_rng(n * 10 + kappa)
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    H = O.Hierarchy(n, theta, eps, convection=(bx, by))
    got = H.cycle(v0, f, kappa=kappa, nu1=2, nu2=1)[0]
    ref = dense_cycle(n, theta, eps, (bx, by), kappa, 2, 1, 0.8, v0, f)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def cycle_matrix(H, n, kappa, nu=2):
    M = np.zeros((n * n, n * n))
    z = np.zeros((n, n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1.0
        M[:, j] = H.cycle(e.reshape(n, n), z, kappa=kappa, nu1=nu, nu2=nu)[0].ravel()
    return M


def test_converges_where_galerkin_diverges():
    """Isotropic diffusion with b = (40, 20) on 15^2: the V-cycle with
    rediscretised levels contracts by about 0.27 per cycle; with the Galerkin
    coarse stencils S_c = 4 R S P of the same upwind operator (the coarse
    operators the symmetric problem uses, applied as constant stencils) the
    iteration diverges."""
    n, b = 15, (40.0, 20.0)
    H = O.Hierarchy(n, 0.0, 1.0, convection=b)
    rho = max(abs(np.linalg.eigvals(cycle_matrix(H, n, 1))))
    assert rho < 0.4
    # Galerkin stencil hierarchy of the same fine operator: dense cycle
    ns = [15, 7, 3, 1]
    s = O.convection_stencil(15, 0.0, 1.0, *b)
    A = [dense_stencil_matrix(s, 15) * 256.0]
    for m_c in ns[1:]:
        s = O.galerkin_stencil(s)
        A.append(dense_stencil_matrix(s, m_c) * (m_c + 1) ** 2)

    def kc(l, v, f):
        if l == len(ns) - 1:
            return np.linalg.solve(A[l], f)
        D = np.diag(A[l])
        for _ in range(2):
            v = v + 0.8 * (f - A[l] @ v) / D
        P = dense_bilinear(ns[l + 1])
        v = v + P @ kc(l + 1, np.zeros(ns[l + 1] ** 2), (P.T / 4) @ (f - A[l] @ v))
        for _ in range(2):
            v = v + 0.8 * (f - A[l] @ v) / D
        return v

    M = np.column_stack([kc(0, e, np.zeros(n * n)) for e in np.eye(n * n)])
    assert max(abs(np.linalg.eigvals(M))) > 1.0


def test_cycle_not_symmetric_and_solvers():
    n = 15
    H = O.Hierarchy(n, 0.3, 0.1, convection=(20.0, -10.0))
    # B = (I - M) A^{-1}: with f = e_j and v = 0 the cycle returns column j of B
    B = np.column_stack([H.cycle(np.zeros((n, n)), e.reshape(n, n), kappa=1, nu1=2, nu2=2)[0].ravel()
                         for e in np.eye(n * n)])
    assert np.abs(B - B.T).max() > 1e-3 * np.abs(B).max()
    f = np.random.default_rng(4).uniform(-1, 1, (127, 127))
    H2 = O.Hierarchy(127, math.pi / 6, 1e-2, convection=(20.0, 10.0))
    its = []
    for kappa in (1, 2, 64):
        u, rc, it, hist = H2.solve(f, kappa=kappa, tol=1e-10, maxit=500)
        assert rc == O.OK
        its.append(it)
        assert np.linalg.norm(f - H2.apply(u)) / np.linalg.norm(f) < 1e-10
    assert its[0] > its[1] >= its[2]
    u, rc, it, hist = H2.ir_solve(f, kappa=2, tol=1e-10, maxit=500)
    assert rc == O.OK
    assert H2.pcg(f, kappa=2)[1] == -1   # OR_ERR_ARG: CG needs a symmetric operator
    with pytest.raises(ValueError):
        O.Hierarchy(15, 0.3, 0.1, n_coarsest=3, convection=(1.0, 1.0))
    with pytest.raises(ValueError):
        O.Hierarchy(15, 0.3, 0.1, smoother="zebra", convection=(1.0, 1.0))
