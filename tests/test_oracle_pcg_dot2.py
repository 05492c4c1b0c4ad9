"""Pins of the oracle's norms, dot products, PCG recurrence and line-solve
tables, against what the mathematics fixes (no GPU).

* Dot2 (Ogita, Rump and Oishi 2005): equals the correctly rounded exact dot
  product (rational arithmetic) on random vectors; recovers cancellations that
  ordinary summation loses; captures a product's rounding error exactly; is
  independent of the summation order on random data.
* PCG with an SPD preconditioner (V- and W-cycles with nu1 = nu2, Section 4's
  symmetry discussion): the k-th iterate is the A-norm minimiser over the
  Krylov space K_k(BA, Bf), computed densely.
* PCG with the nonsymmetric F-cycle preconditioner: the residual history is
  that of the Fletcher-Reeves recurrence run densely with the cycle matrix B.
* Residual replacement: a converged run's reported residual is the true
  residual of the returned iterate and lies below the tolerance.
* Zebra line tables: reciprocal pivots and multipliers are those of the LU
  factorisation of the dense line matrix (pivots as ratios of leading
  principal minors).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from tests.test_oracle_cycle import cycle_matrix
from tests.test_oracle_operators import dense_stencil_matrix


def exact_dot(x, y):
    return float(sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0)))


@pytest.mark.parametrize("seed,signed", [(0, True), (1, False), (2, True), (3, True)])
def test_dot2_is_correctly_rounded(seed, signed):
    rng = np.random.default_rng(seed)
    m = 2000
    x = rng.uniform(-1 if signed else 0, 1, m) * 2.0 ** rng.integers(-30, 30, m)
    y = rng.uniform(-1, 1, m) if signed else x
    assert O.dot2(x, y) == exact_dot(x, y)


def test_dot2_recovers_cancellation():
    # ordinary summation loses the 1 under 1e16; Dot2 keeps it
    x = np.array([1e16, 1.0, -1e16])
    assert O.dot2(x, np.ones(3)) == 1.0
    assert (x[0] + x[1]) + x[2] == 0.0
    # a product's rounding error is kept exactly: a*a - fl(a*a) = 2^-60
    a = 1.0 + 2.0 ** -30
    p = a * a
    assert O.dot2(np.array([a, -p]), np.array([a, 1.0])) == 2.0 ** -60
    # an ill-conditioned sum with exact value 3
    x = np.array([2.0 ** 60, 1.0, -(2.0 ** 60), 2.0, 2.0 ** 55, -(2.0 ** 55)])
    assert O.dot2(x, np.ones(6)) == 3.0


def test_dot2_order_independent():
    rng = np.random.default_rng(7)
    x, y = rng.uniform(-1, 1, 10000), rng.uniform(-1, 1, 10000)
    ref = O.dot2(x, y)
    for s in range(3):
        p = np.random.default_rng(100 + s).permutation(x.size)
        assert O.dot2(x[p], y[p]) == ref
    # ordinary summation is not order independent on the same data (sanity
    # check that the test data can tell the difference)
    sums = {float(np.add.reduce((x * y)[np.random.default_rng(s).permutation(x.size)])) for s in range(8)}
    assert len(sums) > 1


def dense_A(H):
    n = H.n
    return dense_stencil_matrix(H.stencils[0], n) * (n + 1) ** 2


def krylov_minimiser(A, B, f, k):
    """argmin over u in span{Bf, (BA)Bf, ..., (BA)^{k-1}Bf} of ||u - A^{-1} f||_A,
    from an orthonormal basis (Gram-Schmidt, applied twice)."""
    V = []
    w = B @ f
    for _ in range(k):
        for _ in range(2):
            for q in V:
                w = w - (q @ w) * q
        w = w / np.linalg.norm(w)
        V.append(w)
        w = B @ (A @ w)
    V = np.array(V).T
    y = np.linalg.solve(V.T @ A @ V, V.T @ f)
    return V @ y


@pytest.mark.parametrize("L,kappa", [(4, 1), (4, 4), (3, 1)])
def test_pcg_iterates_are_krylov_minimisers(L, kappa):
    n = 2 ** L - 1
    H = O.Hierarchy(n, math.pi / 3, 1e-2, omega=0.8)
    B = cycle_matrix(H, kappa, 1)
    A = dense_A(H)
    f = np.random.default_rng(L + kappa).uniform(-1, 1, (n, n))
    for k in range(1, 6):
        u, rc, it, hist = H.pcg(f, kappa=kappa, nu1=1, nu2=1, tol=0.0, maxit=k)
        assert rc == O.NOT_CONVERGED and it == k
        ref = krylov_minimiser(A, B, f.ravel(), k)
        assert np.abs(u.ravel() - ref).max() <= 1e-10 * np.abs(ref).max()


def dense_fr_pcg(A, B, f, tol, maxit):
    """Fletcher-Reeves PCG from x0 = 0 with z = B r (B need not be symmetric)."""
    u = np.zeros_like(f)
    r = f.copy()
    nf = np.linalg.norm(f)
    hist = [np.linalg.norm(r) / nf]
    p = None
    rz = None
    for _ in range(maxit):
        z = B @ r
        rz_new = r @ z
        p = z if p is None else z + (rz_new / rz) * p
        rz = rz_new
        q = A @ p
        alpha = rz / (p @ q)
        u = u + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r) / nf)
        if hist[-1] < tol:
            break
    return u, hist


def test_pcg_fletcher_reeves_history_nonsymmetric_preconditioner():
    n = 15
    H = O.Hierarchy(n, 0.9, 1e-3, omega=0.8)
    B = cycle_matrix(H, 2, 1)
    assert np.abs(B - B.T).max() > 1e-6 * np.abs(B).max()   # the F-cycle is not symmetric
    A = dense_A(H)
    f = np.random.default_rng(5).uniform(-1, 1, (n, n))
    ud, hd = dense_fr_pcg(A, B, f.ravel(), 0.0, 12)
    u, rc, it, hist = H.pcg(f, kappa=2, nu1=1, nu2=1, tol=0.0, maxit=12)
    assert it == 12
    np.testing.assert_allclose(hist, hd, rtol=1e-9, atol=0)
    assert np.abs(u.ravel() - ud).max() <= 1e-9 * np.abs(ud).max()
    # with a tolerance: the same iteration count (no residual lies near tol)
    tol = 1e-7
    ud, hd = dense_fr_pcg(A, B, f.ravel(), tol, 100)
    assert all(abs(h / tol - 1) > 1e-3 for h in hd)
    u, rc, it, hist = H.pcg(f, kappa=2, nu1=1, nu2=1, tol=tol, maxit=100)
    assert rc == O.OK and it == len(hd) - 1


@pytest.mark.parametrize("kappa,f32", [(1, False), (2, False), (3, True)])
def test_pcg_reports_true_residual_below_tol(kappa, f32):
    n = 31
    H = O.Hierarchy(n, 3 * math.pi / 8, 1e-4, omega=0.8)
    A = dense_A(H)
    f = np.random.default_rng(11 + kappa).uniform(-1, 1, (n, n))
    tol = 1e-11
    u, rc, it, hist = H.pcg(f, kappa=kappa, nu1=1, nu2=1, tol=tol, maxit=400, precond_f32=f32)
    assert rc == O.OK
    true_rel = np.linalg.norm(f.ravel() - A @ u.ravel()) / np.linalg.norm(f)
    assert true_rel < tol
    # the reported value is the true residual, up to the cancellation noise of
    # forming f - Au in a different order (~1e-16 relative to ||f||)
    assert abs(hist[-1] - true_rel) <= 1e-14


def test_pcg_unattainable_tolerance_runs_to_maxit():
    """Below the attainable accuracy the recurrence residual keeps falling but
    the true residual cannot: every crossing is replaced by the true residual
    and the run ends at maxit, not with a false convergence."""
    n = 15
    H = O.Hierarchy(n, 0.4, 1e-2, omega=0.8)
    A = dense_A(H)
    f = np.random.default_rng(3).uniform(-1, 1, (n, n))
    u, rc, it, hist = H.pcg(f, kappa=1, nu1=1, nu2=1, tol=1e-19, maxit=60)
    assert rc == O.NOT_CONVERGED and it == 60
    true_rel = np.linalg.norm(f.ravel() - A @ u.ravel()) / np.linalg.norm(f)
    assert true_rel < 1e-13
    # once replaced, the carried residual is the true one: the history cannot
    # fall far below the attainable accuracy
    assert hist[-1] > 1e-19


@pytest.mark.parametrize("n,theta,eps", [(15, 0.3, 1e-2), (31, 2.0, 1e-5), (7, math.pi / 4, 1e-3)])
def test_zebra_tables_are_line_lu(n, theta, eps):
    H = O.Hierarchy(n, theta, eps, omega=0.8, smoother="zebra")
    for level in range(1, H.levels + 1):
        nl = H.sizes[level - 1]
        A = dense_stencil_matrix(H.stencils[level - 1], nl) * (nl + 1) ** 2
        for direction in (0, 1):
            # the line matrix: A restricted to the points of one line (row 0 for
            # x-lines, column 0 for y-lines); every line has the same matrix
            idx = np.arange(nl) if direction == 0 else np.arange(nl) * nl
            T = A[np.ix_(idx, idx)]
            rp, um = H.zebra_tables(level, direction)
            # pivots are ratios of leading principal minors
            piv = []
            prev = 0.0
            for q in range(nl):
                sgn, ld = np.linalg.slogdet(T[: q + 1, : q + 1])
                piv.append(sgn * math.exp(ld - prev))
                prev = ld
            piv = np.array(piv)
            np.testing.assert_allclose(1.0 / rp, piv, rtol=1e-12)
            if nl > 1:
                np.testing.assert_allclose(um[:-1], np.diag(T, 1) / piv[:-1], rtol=1e-12)
            # L U reproduces T: U = diag(piv) (I + diag(um, 1)), L unit lower
            # with multipliers lo / piv
            U = np.diag(1.0 / rp) @ (np.eye(nl) + np.diag(um[:-1], 1))
            Lm = np.eye(nl) + np.diag(np.diag(T, -1) * rp[:-1], -1)
            np.testing.assert_allclose(Lm @ U, T, rtol=0, atol=1e-12 * np.abs(T).max())
