"""Pins of the oracle's level operators against facts fixed by mathematics.

* Fine stencil (Section 4 table): it applies -div(D grad q) exactly to every
  quadratic q, with D = R(theta) diag(1, eps) R(theta)^T (rows of the table
  along +y); zero row sum; point symmetry.
* Derivative stencils: central differences of the stencil itself.
* Prolongation and restriction: equal to dense bilinear-interpolation matrices
  built here from the definition, R = P^T / 4.
* Galerkin coarse operators: equal to dense R A P on small grids at every row
  (boundary rows included), the textbook Poisson values, and consistency with
  the PDE on quadratics at every level.
* Coarsest solve: a dense direct solve.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

CASES = [(math.pi / 4, 1.0), (math.pi / 4, 1e-3), (math.pi / 6, 1e-4), (0.3, 0.05), (3 * math.pi / 8, 1e-5),
         (2.9, 0.7)]


def diffusion_tensor(theta, eps):
    c, s = math.cos(theta), math.sin(theta)
    R = np.array([[c, -s], [s, c]])
    return R @ np.diag([1.0, eps]) @ R.T


def grid_xy(n):
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(x, x)   # X[j, i] = x_i, Y[j, i] = y_j
    return X, Y, h


def dense_stencil_matrix(s, n):
    s = np.asarray(s).reshape(3, 3)
    A = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    jj, ii = j + b, i + a
                    if 0 <= jj < n and 0 <= ii < n:
                        A[j * n + i, jj * n + ii] = s[b + 1, a + 1]
    return A


def dense_bilinear(nc):
    """P: coarse (J,I) sits at fine (2J+1, 2I+1); weight 1 there, 1/2 at the
    four edge neighbours, 1/4 at the four diagonal neighbours."""
    n = 2 * nc + 1
    P = np.zeros((n * n, nc * nc))
    for J in range(nc):
        for I in range(nc):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    w = (1.0 if dx == 0 else 0.5) * (1.0 if dy == 0 else 0.5)
                    P[(2 * J + 1 + dy) * n + (2 * I + 1 + dx), J * nc + I] = w
    return P


@pytest.mark.parametrize("theta,eps", CASES)
def test_fine_stencil_exact_on_quadratics(theta, eps):
    n = 15
    X, Y, h = grid_xy(n)
    D = diffusion_tensor(theta, eps)
    s = O.fine_stencil(theta, eps)
    rng = np.random.default_rng(7)
    for _ in range(3):
        a, b, c, d, e, g = rng.uniform(-1, 1, 6)
        q = a * X * X + b * X * Y + c * Y * Y + d * X + e * Y + g
        Aq = O.apply_stencil(s, q) / (h * h)
        # -div(D grad q) = -(2a D11 + 2b D12 + 2c D22) for the quadratic part
        exact = -(2 * a * D[0, 0] + 2 * b * D[0, 1] + 2 * c * D[1, 1])
        inner = Aq[1:-1, 1:-1]   # away from the zero Dirichlet extension
        assert np.allclose(inner, exact, rtol=0, atol=1e-9 * (1 + abs(exact)))


@pytest.mark.parametrize("theta,eps", CASES)
def test_fine_stencil_structure(theta, eps):
    s = O.fine_stencil(theta, eps)
    assert abs(s.sum()) < 1e-15
    assert np.array_equal(s, s[::-1, ::-1])           # point symmetry
    assert s[1, 1] == 2 * (1 + eps)
    # theta=0: strong coupling along x, weak along y
    s0 = O.fine_stencil(0.0, eps)
    assert np.allclose(s0, [[0, -eps, 0], [-1, 2 + 2 * eps, -1], [0, -eps, 0]], atol=1e-16)


@pytest.mark.parametrize("theta,eps", CASES)
def test_derivative_stencils(theta, eps):
    dth, de = O.fine_stencil_derivs(theta, eps)
    d = 1e-6
    fd_th = (O.fine_stencil(theta + d, eps) - O.fine_stencil(theta - d, eps)) / (2 * d)
    fd_e = (O.fine_stencil(theta, eps + d) - O.fine_stencil(theta, eps - d)) / (2 * d)
    assert np.allclose(dth, fd_th, atol=1e-8)
    assert np.allclose(de, fd_e, atol=1e-8)
    assert abs(dth.sum()) < 1e-14 and abs(de.sum()) < 1e-14


@pytest.mark.parametrize("nc", [1, 3, 7])
def test_prolong_restrict_dense(nc):
    rng = np.random.default_rng(nc)
    P = dense_bilinear(nc)
    n = 2 * nc + 1
    vc = rng.uniform(-1, 1, (nc, nc))
    r = rng.uniform(-1, 1, (n, n))
    assert np.allclose(O.prolong(vc).ravel(), P @ vc.ravel(), atol=1e-15)
    assert np.allclose(O.restrict_fw(r).ravel(), (P.T / 4) @ r.ravel(), atol=1e-15)
    # adjointness <P x, y> = 4 <x, R y>
    assert abs(np.dot(O.prolong(vc).ravel(), r.ravel()) - 4 * np.dot(vc.ravel(), O.restrict_fw(r).ravel())) < 1e-12


@pytest.mark.parametrize("theta,eps", CASES)
@pytest.mark.parametrize("n", [7, 15, 31])
def test_galerkin_equals_dense_rap(theta, eps, n):
    """A_c = R A P with A = S/h^2, R = P^T/4; the oracle's coarse operator is
    a constant stencil S_c / (2h)^2 -- it must equal the dense product at
    every row, boundary rows included."""
    H = O.Hierarchy(n, theta, eps)
    h = 1.0 / (n + 1)
    A = dense_stencil_matrix(H.stencils[0], n) / h ** 2
    nc = (n - 1) // 2
    P = dense_bilinear(nc)
    Ac = (P.T / 4) @ A @ P
    Ac_or = dense_stencil_matrix(H.stencils[1], nc) / (2 * h) ** 2
    assert np.abs(Ac - Ac_or).max() <= 1e-13 * np.abs(Ac).max()
    # and one more level down
    if nc >= 3:
        P2 = dense_bilinear((nc - 1) // 2)
        Acc = (P2.T / 4) @ Ac_or @ P2
        Acc_or = dense_stencil_matrix(H.stencils[2], (nc - 1) // 2) / (4 * h) ** 2
        assert np.abs(Acc - Acc_or).max() <= 1e-13 * np.abs(Acc).max()


def test_galerkin_poisson_textbook():
    """eps = 1 is the 5-point Laplacian; its Galerkin operator with full
    weighting and bilinear interpolation is the 9-point stencil
    (1/H^2) [-1/4 -1/2 -1/4; -1/2 3 -1/2; -1/4 -1/2 -1/4]."""
    H = O.Hierarchy(63, 0.4, 1.0)
    assert np.allclose(H.stencils[0], [[0, -1, 0], [-1, 4, -1], [0, -1, 0]], atol=1e-15)
    assert np.allclose(H.stencils[1], [[-0.25, -0.5, -0.25], [-0.5, 3.0, -0.5], [-0.25, -0.5, -0.25]], atol=1e-15)
    assert np.allclose(H.stencils[2], [[-5 / 16, -3 / 8, -5 / 16], [-3 / 8, 11 / 4, -3 / 8], [-5 / 16, -3 / 8, -5 / 16]],
                       atol=1e-15)


@pytest.mark.parametrize("theta,eps", CASES)
def test_galerkin_levels_consistent_on_quadratics(theta, eps):
    """Every Galerkin level still applies -div(D grad q) to quadratics."""
    H = O.Hierarchy(255, theta, eps)
    D = diffusion_tensor(theta, eps)
    exact = -(2 * 0.3 * D[0, 0] + 2 * (-0.7) * D[0, 1] + 2 * 0.5 * D[1, 1])
    for k in range(1, 5):
        n = H.sizes[k]
        X, Y, h = grid_xy(n)
        q = 0.3 * X * X - 0.7 * X * Y + 0.5 * Y * Y
        Aq = O.apply_stencil(H.stencils[k], q) / (h * h)
        assert np.allclose(Aq[1:-1, 1:-1], exact, rtol=1e-9, atol=1e-9)
        assert abs(H.stencils[k].sum()) < 1e-12 * np.abs(H.stencils[k]).max()
        assert np.allclose(H.stencils[k], H.stencils[k][::-1, ::-1], atol=1e-15)


@pytest.mark.parametrize("nc", [1, 3, 7])
def test_coarsest_solve_dense(nc):
    """A one-level hierarchy is the coarsest solve alone (Algorithm 3, the coarsest grid)."""
    theta, eps = 0.9, 3e-3
    H = O.Hierarchy(nc, theta, eps, n_coarsest=nc)
    assert H.levels == 1
    h = 1.0 / (nc + 1)
    A = dense_stencil_matrix(O.fine_stencil(theta, eps), nc) / h ** 2
    f = np.random.default_rng(nc).uniform(-1, 1, (nc, nc))
    v = H.cycle(np.full((nc, nc), 123.0), f, kappa=3)[0]
    assert np.allclose(v.ravel(), np.linalg.solve(A, f.ravel()), rtol=1e-13, atol=1e-16)


def test_hierarchy_shapes():
    assert O.Hierarchy(1023, 0.1, 0.1).sizes == [1023, 511, 255, 127, 63, 31, 15, 7, 3, 1]
    assert O.Hierarchy(63, 0.1, 0.1, n_coarsest=3).sizes == [63, 31, 15, 7, 3]
    with pytest.raises(ValueError):
        O.Hierarchy(64, 0.1, 0.1)
    with pytest.raises(ValueError):
        O.Hierarchy(63, 0.1, 0.1, n_coarsest=5)
