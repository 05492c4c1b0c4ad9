"""Pins of the host-side run-time model (Section 3) against the paper's
printed numbers and against brute-force recursion counts."""
import json
import math
import os

import numpy as np
import pytest

from paper_2010_00626_amd import model as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def kap(x):
    return math.inf if x == "inf" else int(x)


def test_table1_turning_points():
    """Table 1 (Section 3.4) from alpha, beta (Section 3.2) and the Appendix
    iteration.  Reading: rows kappa=1..4 reproduce with 7 launches per call,
    the W row with 9 (= 5 + nu for nu = 2 + 2)."""
    g = gold("paper_section3_model.json")
    a, b = g["fit"]["alpha_ms"], g["fit"]["beta_ms"]
    t = g["table1_turning_points"]
    for k, ntp, Ntp in zip(t["kappa"], t["n_tp"], t["N_tp"]):
        k = kap(k)
        lpc = 9 if math.isinf(k) else 7
        n = M.paper_turning_point(a, b, k, lpc)
        assert abs(n - ntp) < 0.051, (k, n)
        N = (2 ** n - 1) ** 2
        assert abs(N - Ntp) / Ntp < 0.12, (k, N)


def test_table3_per_cycle_times_from_model():
    """alpha * N_gpuCalls + beta * N_ops at 12 levels, nu = 4 reproduces the
    per-cycle times of Table 3 within the model's stated accuracy."""
    g = gold("paper_section3_model.json")
    t3 = gold("paper_section4_tables.json")["table3_standalone"]
    a, b = g["fit"]["alpha_ms"], g["fit"]["beta_ms"]
    for k, ms in zip(t3["kappa"], t3["ms_per_cycle"]):
        k = M.KAPPA_W if k == "inf" else int(k)
        pred = M.predict(a, b, M.n_gpu_calls_paper(k, 12, 4), M.n_ops_2d(k, 12))
        assert abs(pred - ms) / ms < 0.025, (k, pred, ms)
    # total time = per-cycle time x cycles (Table 3's own arithmetic)
    for tot, ms, cyc in zip(t3["total_ms"], t3["ms_per_cycle"], t3["cycles"]):
        assert abs(ms * cyc - tot) / tot < 0.01


def test_launch_counts_section3():
    assert [M.n_gpu_calls_paper(k, 12, 4) for k in (1, 2, 3, 4, M.KAPPA_W)] == [100, 606, 2146, 5281, 20471]
    assert [M.total_calls(k, 12) for k in (1, 2, 3, 4, 12)] == [12, 78, 298, 793, 4095]
    assert [M.level_calls(3, l) for l in range(1, 13)] == [1, 2, 4, 7, 11, 16, 22, 29, 37, 46, 56, 67]


def brute_ops(kappa, n, c, C, Ct, modified):
    """Operations of a kappa-cycle with n levels (level 1 = coarsest here, as
    in Section 2.3): C * N_l per call on non-coarsest levels, coarsest cost
    Ct * N_1 (or f(kappa_call, c) C N_1 for Lemma 1)."""
    N1 = 1.0

    def N(l):
        return N1 * c ** (1 - l)

    def ops(k, l):
        if l == 1:
            return M.f_ops(k, c) * C * N1 if modified else Ct * N1
        s = C * N(l) + ops(k, l - 1)
        if k > 1:
            s += ops(k - 1, l - 1)
        return s
    return ops(kappa, n), N(n)


@pytest.mark.parametrize("c", [0.25, 0.3, 0.5, 0.1])
def test_lemma1_and_prop5(c):
    C, Ct = 3.0, 11.0
    for kappa in range(1, 6):
        for n in range(1, 9):
            tot, Nn = brute_ops(kappa, n, c, C, Ct, modified=True)
            assert abs(tot - M.f_ops(kappa, c) * C * Nn) <= 1e-9 * tot
            tot2, _ = brute_ops(kappa, n, c, C, Ct, modified=False)
            P = sum((Ct - M.f_ops(kappa - j, c) * C) * math.comb(n - 1, j) for j in range(0, min(kappa - 1, n - 1) + 1))
            assert abs(tot2 - (M.f_ops(kappa, c) * C * Nn + P)) <= 1e-9 * abs(tot2)


def test_f_ops_special_values():
    assert M.f_ops(1, 0.25) == pytest.approx(4 / 3)
    assert M.f_ops(math.inf, 0.25) == 2.0
    assert M.f_ops(3, 0.5) == 6.0
    for k in (1, 2, 3, 4, 7):
        assert M.c_kappa(k) == pytest.approx(M.f_ops(k, 0.25))
    # the measure is close to the actual per-level sums with (2^k-1)^2 points
    for k, expect in zip((1, 2, 3, 4, 12), (1.3330, 1.7767, 1.9240, 1.9725, 1.9947)):
        s = sum(M.level_calls(k, l) * (2 ** (12 - l + 1) - 1) ** 2 for l in range(1, 13)) / (2 ** 12 - 1) ** 2
        assert abs(s - expect) < 2e-4


def test_fit_recovers_parameters():
    rng = np.random.default_rng(0)
    a, b = 4.1e-3, 2.2e-7
    rows = []
    for k in (1, 2, 3, 4, M.KAPPA_W):
        for n in range(4, 14):
            calls, ops = M.n_gpu_calls_paper(k, n, 4), M.n_ops_2d(k, n)
            rows.append(((k, n), calls, ops, a * calls + b * ops))
    f = M.fit(rows)
    assert f.alpha == pytest.approx(a, rel=1e-10) and f.beta == pytest.approx(b, rel=1e-10)
    assert max(abs(e) for e in f.rel_errors.values()) < 1e-10
    noisy = [(r[0], r[1], r[2], r[3] * (1 + 0.01 * rng.standard_normal())) for r in rows]
    g = M.fit(noisy)
    assert g.alpha == pytest.approx(a, rel=0.05) and g.beta == pytest.approx(b, rel=0.05)


def test_best_kappa_tradeoff_table3():
    """With Table 3's cycle counts and the model's per-cycle times, kappa=4
    has the smallest predicted total, as measured."""
    g = gold("paper_section3_model.json")
    t3 = gold("paper_section4_tables.json")["table3_standalone"]
    a, b = g["fit"]["alpha_ms"], g["fit"]["beta_ms"]
    cyc = {(M.KAPPA_W if k == "inf" else int(k)): c for k, c in zip(t3["kappa"], t3["cycles"])}
    k, totals = M.best_kappa(list(cyc), lambda k: M.predict(a, b, M.n_gpu_calls_paper(k, 12, 4), M.n_ops_2d(k, 12)),
                             lambda k: cyc[k])
    assert k == 4


def test_cycles_from_rate():
    assert M.cycles_from_rate(0.1, 1e-8) == pytest.approx(8.0)
    assert math.isinf(M.cycles_from_rate(1.0, 1e-8))
