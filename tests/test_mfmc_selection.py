"""MFMC model selection and sample allocation (Sec. 3.1, 3.2, Sec. 4) -- CPU.

The FP64 reference (oracle.mfmc) is pinned to the paper's printed Table 2
(computed from Table 1's statistics) and to the closed forms it states; the
library's mfmc_select / mfmc_allocate are then compared with it.

Known properties of the printed tables (see the golden files): rows 4, 6, 8, 9
and 10 of Table 2 carry the f_7 / f_8 labels exchanged, and B_min of subsets
holding f_2 cannot be recovered from the seven printed digits of
rho_{1,2} = 0.9999999 (1 - rho^2 ~ 2e-7), so those B_min values are not
compared.
"""
import math
import os

import numpy as np
import pytest

from oracle import mfmc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C1_SECONDS = 63.089


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def _pool():
    rows = _rows("table1_models.txt")
    rho = [float(r[3]) for r in rows]
    cost = [float(r[4]) for r in rows]
    sigma = [float(r[5]) for r in rows]
    return cost, rho, sigma


def _sub(text, swap=False):
    s = [int(x) for x in text.split(",")]
    if swap:
        s = [7 if x == 8 else (8 if x == 7 else x) for x in s]
    return tuple(sorted(x - 1 for x in s))  # 0-based pool indices, pool order


def _canon(sub, rho):
    return tuple(sorted(sub, key=lambda k: -rho[k] ** 2))


def test_table2_feasible_count():
    cost, rho, _ = _pool()
    feas, ncand = mfmc.select(cost, rho)
    assert ncand == 255
    assert len(feas) == 131


def test_table2_rows_ranks_and_values():
    cost, rho, _ = _pool()
    feas, _ = mfmc.select(cost, rho)
    vrank = {s: i + 1 for i, (s, _, _) in enumerate(feas)}
    by_b = sorted(feas, key=lambda t: t[2])
    brank = {s: i + 1 for i, (s, _, _) in enumerate(by_b)}
    val = {s: (V, b) for s, V, b in feas}
    rows = _rows("table2_subsets.txt")
    printed_v = {int(r[0]): float(r[2]) for r in rows}
    for vi, sub, V, bm, bi, sw in rows:
        s = _canon(_sub(sub, swap=sw == "1"), rho)
        vi = int(vi)
        # printed neighbours closer than the 1e-4 that Table 1's rounding
        # moves V by may trade places
        near_tie = any(abs(printed_v.get(vi + d, 9.0) - float(V)) < 1e-4 for d in (-1, 1))
        assert abs(vrank[s] - vi) <= (1 if near_tie else 0), (sub, vrank[s])
        assert brank[s] == int(bi), sub
        # with f_2, the term sqrt(1 - rho_{1,2}^2) ~ 4e-4 carries the rounding
        # of rho_{1,2} into V at the 1e-4 level
        vtol = 2e-4 if 1 in s else 1e-4
        assert abs(val[s][0] - float(V)) <= vtol, (sub, val[s][0], V)
        if 1 not in s:  # f_2 absent: B_min is well conditioned
            assert abs(val[s][1] - float(bm)) <= 2.5e-3 * float(bm), (sub, val[s][1], bm)


def test_cases_minimum_budget_seconds():
    cost, rho, _ = _pool()
    for case, sub, V, bm, secs in _rows("mfmc_cases.txt"):
        assert abs(float(bm) * C1_SECONDS - float(secs)) <= 0.1
        s = _canon(_sub(sub), rho)
        assert abs(mfmc.variance_reduction_ratio(cost, rho, s) - float(V)) <= 1e-4
        if 1 not in s:
            b = mfmc.min_budget([c * C1_SECONDS for c in cost], rho, s)
            assert abs(b - float(secs)) <= 2.5e-3 * float(secs)


def test_paper_ratio_statements():
    """Sec. 4 text: Case 2's V is 0.50% above Case 1's, Case 3's 3.65% above."""
    rows = {r[0]: float(r[2]) for r in _rows("mfmc_cases.txt")}
    assert abs(rows["2"] / rows["1"] - 1 - 0.0050) < 0.0002
    assert abs(rows["3"] / rows["1"] - 1 - 0.0365) < 0.0002


def test_bmin_identity_and_mse_closed_form():
    """sum_j C_{i_j} r_j = C_1 sqrt(V / (1 - rho_{1,i_2}^2)) (eq. bmin) and the
    theoretical MSE sigma_1^2 (1 - rho^2) B / ((m_1*)^2 C_1) equals
    sigma_1^2 C_1 V / B."""
    cost, rho, sigma = _pool()
    feas, _ = mfmc.select(cost, rho)
    for s, V, b in feas:
        r = mfmc.oversampling(cost, rho, s)
        assert abs(r[0] - 1.0) < 1e-12
        assert abs(sum(cost[i] * rj for i, rj in zip(s, r)) - cost[0] * b) <= 1e-9 * cost[0] * b
        for B in (1e3, 10 ** (5 + 1 / 3)):
            mse = mfmc.mse_theory(sigma[0], rho, cost, s, B)
            assert abs(mse - sigma[0] ** 2 * cost[0] * V / B) <= 1e-9 * mse


BUDGETS = [10 ** (3 + i / 3) for i in range(8)]  # the MSE study's budgets


@pytest.mark.parametrize("case", ["1", "2", "3", "4", "5"])
def test_allocation_properties(case):
    cost, rho, _ = _pool()
    sub = {r[0]: r[1] for r in _rows("mfmc_cases.txt")}[case]
    s = _canon(_sub(sub), rho)
    C = [c * C1_SECONDS for c in cost]
    for B in BUDGETS:
        m, mi, m1 = mfmc.allocate(C, rho, s, B)
        if m1 >= 1:
            assert abs(sum(C[i] * v for i, v in zip(s, m)) - B) <= 1e-9 * B
            assert all(m[j] <= m[j + 1] for j in range(len(m) - 1))
        else:
            floor_cost = sum((l + 1) * C[i] for l, i in enumerate(s))
            if B < floor_cost:
                with pytest.raises(ValueError):
                    mfmc.allocate_below_min(C, rho, s, B)
                continue
            m, mi = mfmc.allocate_below_min(C, rho, s, B)
            assert all(m[l] >= l + 1 for l in range(len(s) - 1))
            assert abs(sum(C[i] * v for i, v in zip(s, m)) - B) <= 1e-9 * B
        assert sum(C[i] * v for i, v in zip(s, mi)) <= B + 1e-9


def test_allocation_minimises_estimator_variance():
    """Synthetic models with known statistics: the MFMC estimator with the
    allocation of eq. samples and alpha of eq. alpha has the variance
    sigma_1^2 C_1 V / B (replicated estimates)."""
    a = np.array([1.0, 1.0, 1.0])
    b = np.array([0.05, 0.15, 0.4])
    sig = np.sqrt(a * a + b * b)
    rho = [1.0] + [float(a[0] * a[j] / (sig[0] * sig[j])) for j in (1, 2)]
    cost = [1.0, 0.05, 0.004]
    s = (0, 1, 2)
    assert mfmc.condition_a(rho, s) and mfmc.condition_b(cost, rho, s)
    V = mfmc.variance_reduction_ratio(cost, rho, s)
    B = 60.0
    m, mi, _ = mfmc.allocate(cost, rho, s, B)
    alpha = [rho[j] * sig[0] / sig[j] for j in (1, 2)]
    rng = np.random.default_rng(21)
    R = 4000
    z = rng.normal(size=(R, mi[2]))
    est = np.empty(R)
    for k in range(R):
        ys = [a[j] * z[k] + b[j] * rng.normal(size=mi[2]) for j in range(3)]
        est[k] = mfmc.mfmc_estimate(ys, mi, alpha)["q_mfmc"]
    theory = sig[0] ** 2 * cost[0] * V / B
    assert abs(est.var(ddof=1) / theory - 1) < 0.12


# ------------------------------------------------------ library parity ----

def test_library_select_matches_oracle():
    from paper_2310_10750_amd import nlch
    cost, rho, _ = _pool()
    feas, _ = mfmc.select(cost, rho)
    got, ncand = nlch.mfmc_select(cost, rho)
    assert ncand == 255 and len(got) == len(feas) == 131
    for (s, V, b), (gs, gV, gb) in zip(feas, got):
        assert tuple(s) == gs
        assert abs(gV - V) <= 1e-13 * V
        assert abs(gb - b) <= 1e-11 * b
    # a shuffled pool (model 0 stays first) selects the same subsets
    perm = [0, 5, 2, 8, 1, 7, 3, 6, 4]
    got2, _ = nlch.mfmc_select([cost[p] for p in perm], [rho[p] for p in perm])
    back = {tuple(perm[i] for i in s) for s, _, _ in got2}
    assert back == {s for s, _, _ in feas}


@pytest.mark.parametrize("case", ["1", "2", "3", "4", "5"])
def test_library_allocate_matches_oracle(case):
    from paper_2310_10750_amd import nlch
    cost, rho, _ = _pool()
    C = [c * C1_SECONDS for c in cost]
    sub = {r[0]: r[1] for r in _rows("mfmc_cases.txt")}[case]
    s = _canon(_sub(sub), rho)
    for B in BUDGETS + [777.0, 5e6]:
        m, mi, m1 = mfmc.allocate(C, rho, s, B)
        if m1 < 1:
            floor_cost = sum((l + 1) * C[i] for l, i in enumerate(s))
            if B < floor_cost:
                with pytest.raises(nlch.NlchError):
                    nlch.mfmc_allocate(s, C, rho, B)
                continue
            m, mi = mfmc.allocate_below_min(C, rho, s, B)
        gm, gmi, gm1 = nlch.mfmc_allocate(s, C, rho, B)
        assert abs(gm1 - m1) <= 1e-12 * m1
        np.testing.assert_allclose(gm, m, rtol=1e-12)
        assert gmi == mi


def test_library_selection_argument_errors():
    from paper_2310_10750_amd import nlch
    with pytest.raises(nlch.NlchError):
        nlch.mfmc_select([1.0], [1.0])
    with pytest.raises(nlch.NlchError):
        nlch.mfmc_select([1.0, 0.0], [1.0, 0.9])
    with pytest.raises(nlch.NlchError):
        nlch.mfmc_select([1.0, 0.5], [0.9, 1.0])
    with pytest.raises(nlch.NlchError):
        nlch.mfmc_allocate((1, 0), [1.0, 0.5], [1.0, 0.9], 10.0)
    with pytest.raises(nlch.NlchError):
        nlch.mfmc_allocate((0, 1), [1.0, 0.5], [1.0, 0.9], -1.0)
    with pytest.raises(nlch.NlchError):
        nlch.mfmc_allocate((0, 1, 2), [1.0, 0.5, 0.1], [1.0, 0.8, 0.9], 10.0)
