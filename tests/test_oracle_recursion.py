"""Pins of the oracle's recursion against the facts Section 2 fixes.

* Proposition 1: kappa=1 is Algorithm 1 with gamma=1 (V), kappa=2 is
  Algorithm 2 (F), kappa >= n is Algorithm 1 with gamma=2 (W) -- compared as
  exact operation sequences and as bitwise-equal iterates.
* Proposition 2 / Corollary 1: calls per level.
* Proposition 3 / Corollary 2: total calls, a degree-kappa polynomial in n.
* Lemma 2: the coarsest level is called C(n-1, j) times with counter kappa-j.
* Section 1 worked example: a ten-level W-cycle makes 1023 calls against 10
  for the V-cycle, with about 50% more operations.
The closed forms are evaluated here with math.comb; the counts come from the
oracle's trace of its actual recursion.
"""
import math
from collections import Counter

import numpy as np
import pytest

from oracle import oracle as O


def level_calls(kappa, l):
    return sum(math.comb(l - 1, j) for j in range(0, min(kappa - 1, l - 1) + 1))


def total_calls(kappa, n):
    return sum(math.comb(n, j) for j in range(1, min(kappa, n) + 1))


def ops_levels(trace):
    return [(op, lev) for op, lev, _ in trace]


@pytest.fixture(scope="module")
def hiers():
    # L levels, coarsest 1x1: n = 2^L - 1
    return {L: O.Hierarchy(2 ** L - 1, 0.7, 0.01) for L in range(1, 9)}


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
def test_prop1_sequences(hiers, L):
    H = hiers[L]
    v_seq = ops_levels(H.trace(kappa=1))
    assert v_seq == ops_levels(H.trace(kappa=1, kind=O.KIND_GAMMA))
    f_seq = ops_levels(H.trace(kappa=2))
    assert f_seq == ops_levels(H.trace(kind=O.KIND_F))
    w_seq = ops_levels(H.trace(kappa=2, kind=O.KIND_GAMMA))
    for kappa in (L, L + 1, L + 5, 2 ** 31 - 1):
        assert ops_levels(H.trace(kappa=kappa)) == w_seq
    if L >= 3:
        # kappa = n-1 keeps W's iterates but drops one redundant coarsest call
        assert ops_levels(H.trace(kappa=L - 1)) != w_seq


@pytest.mark.parametrize("L", [3, 4, 5])
def test_prop1_iterates_bitwise(hiers, L):
    H = hiers[L]
    n = H.n
    rng = np.random.default_rng(L)
    v0, f = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    pairs = [((0, 1), (O.KIND_GAMMA, 1)), ((0, 2), (O.KIND_F, 0)), ((0, L), (O.KIND_GAMMA, 2)),
             ((0, L - 1), (O.KIND_GAMMA, 2))]
    for (k1, p1), (k2, p2) in pairs:
        a = H.cycle(v0, f, kappa=p1, kind=k1)[0]
        b = H.cycle(v0, f, kappa=p2, kind=k2)[0]
        assert np.array_equal(a, b)


@pytest.mark.parametrize("L", range(1, 9))
def test_prop2_prop3_counts(hiers, L):
    H = hiers[L]
    for kappa in range(1, L + 3):
        tr = H.trace(kappa=kappa)
        calls = Counter(lev for op, lev, _ in tr if op == O.OP_CALL)
        for l in range(1, L + 1):
            assert calls[l] == level_calls(kappa, l), (kappa, l)
        assert sum(calls.values()) == total_calls(kappa, L)
        # Corollary 1: levels at or above the counter see 2^(l-1) calls
        for l in range(1, min(kappa, L) + 1):
            assert calls[l] == 2 ** (l - 1)


def test_cor2_polynomial_degree(hiers):
    """For kappa < n, totalCalls is a degree-kappa polynomial in n: its
    kappa-th finite difference is the constant 1 and the next one vanishes."""
    for kappa in (1, 2, 3):
        ns = list(range(kappa + 1, kappa + 1 + kappa + 3))
        vals = []
        for n in ns:
            if n in hiers:
                tr = hiers[n].trace(kappa=kappa)
                vals.append(sum(1 for op, _, _ in tr if op == O.OP_CALL))
            else:
                vals.append(total_calls(kappa, n))
        d = np.array(vals, dtype=np.int64)
        for _ in range(kappa):
            d = np.diff(d)
        assert np.all(d == 1)
        assert np.all(np.diff(d) == 0)


@pytest.mark.parametrize("L,kappa", [(5, 3), (6, 2), (6, 4), (7, 3), (4, 9)])
def test_lemma2_coarsest_histogram(hiers, L, kappa):
    tr = hiers[L].trace(kappa=kappa)
    hist = Counter(c for op, lev, c in tr if op == O.OP_CALL and lev == L)
    expect = {kappa - j: math.comb(L - 1, j) for j in range(0, min(kappa - 1, L - 1) + 1)}
    assert dict(hist) == expect
    if (L, kappa) == (5, 3):
        assert dict(hist) == {3: 1, 2: 4, 1: 6}


def test_section1_worked_example():
    """Ten levels: W makes 2^10-1 = 1023 calls vs 10 for V; work ratio ~1.5."""
    H = O.Hierarchy(2 ** 10 - 1, 0.3, 0.1)
    w = H.trace(kappa=10)
    v = H.trace(kappa=1)
    calls_w = [lev for op, lev, _ in w if op == O.OP_CALL]
    calls_v = [lev for op, lev, _ in v if op == O.OP_CALL]
    assert len(calls_w) == 1023 and len(calls_v) == 10
    size = {l: (2 ** (10 - l + 1) - 1) ** 2 for l in range(1, 11)}
    work_w = sum(size[l] for l in calls_w)
    work_v = sum(size[l] for l in calls_v)
    assert abs(work_w / work_v - 1.5) < 0.015   # "only 50% more": (2^k-1)^2 sizes give 1.489


def test_paper_structured_launch_count(hiers):
    """Algorithm 4: 5+nu launches per non-coarsest call, one per coarsest call
    (relax nu1, residual, restrict, zero, prolong, add, relax nu2)."""
    for L in (4, 6, 8):
        H = hiers[L]
        for kappa in (1, 2, 3, 4, 2 ** 31 - 1):
            for nu1, nu2 in ((1, 1), (2, 2)):
                tr = H.trace(kappa=kappa, nu1=nu1, nu2=nu2)
                launches = sum(1 for op, _, _ in tr if op != O.OP_CALL)
                k = min(kappa, 10 ** 6)
                expect = (5 + nu1 + nu2) * total_calls(k, L - 1) + total_calls(k, L) - total_calls(k, L - 1)
                assert launches == expect
