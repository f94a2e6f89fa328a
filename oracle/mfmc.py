"""FP64 reference of the multifidelity Monte Carlo estimator (arXiv 2310.10750,
Sec. 3.2).  TEST INFRASTRUCTURE ONLY (see the package docstring).

Plain numpy, two-pass moments, written from the paper's formulas:

* Monte Carlo estimate of model j over its first k samples:
  ``Q^{(j)}_k = (1/k) sum_{i<k} y_j[i]``                       (eq. mc)
* telescoping estimator
  ``Q_MFMC = Q^{(1)}_{m_1} + sum_{j>=2} alpha_j (Q^{(j)}_{m_j} - Q^{(j)}_{m_{j-1}})``
                                                              (eq. MFMC_estimator)
* ``alpha_j = rho_{1,j} sigma_1 / sigma_j``                     (eq. alpha)

Sample nesting: every model evaluates the same parameter draws theta_1, theta_2,
..., so model j uses the first m_j of them and the first m_{j-1} are shared
with model j-1.  The statistics sigma_j and rho_{1,j} that enter alpha are
estimated from the first m_1 draws, the only ones every model has evaluated
(the paper estimates them from pilot samples; with alpha given by the caller
they are reported only).  A model with zero sample variance gets rho = 0 and
alpha = 0.
"""
from __future__ import annotations

import numpy as np


def _mean(a):
    return float(np.sum(np.asarray(a, dtype=np.float64)) / len(a))


def mfmc_estimate(ys, m, alpha=None):
    """Returns a dict with q_mfmc, q_mc, mean_mj, mean_mjm1, var, rho, alpha.

    ys: list of K 1-D arrays (model outputs, model 1 first); m: K sample
    counts, non-decreasing, m[0] >= 2 (m[0] >= 1 when alpha is given: the
    below-minimum-budget allocation of Sec. 4 sets m_1 = 1, and the estimator
    needs only means; var and rho are then NaN); alpha: None or K-1
    coefficients for models 2..K.
    """
    K = len(ys)
    m = [int(v) for v in m]
    if K < 1 or len(m) != K:
        raise ValueError("need one sample count per model")
    if m[0] < (1 if alpha is not None else 2) or any(m[j] < m[j - 1] for j in range(1, K)):
        raise ValueError("sample counts must be non-decreasing with m[0] >= 2 "
                         "(>= 1 with alpha given)")
    ys = [np.asarray(y, dtype=np.float64) for y in ys]
    for j in range(K):
        if ys[j].size < m[j]:
            raise ValueError("model %d has fewer than m_j outputs" % (j + 1))

    mean_mj = [_mean(ys[j][:m[j]]) for j in range(K)]
    mean_mjm1 = [float("nan")] + [_mean(ys[j][:m[j - 1]]) for j in range(1, K)]

    m0 = m[0]
    centred = []
    var = []
    for j in range(K):
        s = ys[j][:m0]
        c = s - _mean(s)
        centred.append(c)
        var.append(float(np.sum(c * c) / (m0 - 1)) if m0 > 1 else float("nan"))
    rho = []
    for j in range(K):
        if m0 < 2:
            rho.append(float("nan"))
        elif var[0] == 0.0 or var[j] == 0.0:
            rho.append(0.0)
        else:
            cov = float(np.sum(centred[0] * centred[j]) / (m0 - 1))
            rho.append(cov / np.sqrt(var[0] * var[j]))
    if alpha is None:
        al = [1.0]
        for j in range(1, K):
            al.append(0.0 if var[j] == 0.0
                      else rho[j] * np.sqrt(var[0]) / np.sqrt(var[j]))
    else:
        alpha = [float(a) for a in alpha]
        if len(alpha) != K - 1:
            raise ValueError("need K-1 alpha values")
        al = [1.0] + alpha
    q = mean_mj[0]
    for j in range(1, K):
        q += al[j] * (mean_mj[j] - mean_mjm1[j])
    return {
        "q_mfmc": q,
        "q_mc": mean_mj[0],
        "mean_mj": mean_mj,
        "mean_mjm1": mean_mjm1,
        "var": var,
        "rho": rho,
        "alpha": al,
    }


# ---------------------------------------------------------------------------
# Model selection and sample allocation (Sec. 3.1 and 3.2).  A model pool is
# given by cost[k] and rho[k] (= rho_{1,k}), k = 0..K-1, model 0 being the
# high-fidelity one; a subset is a tuple of pool indices starting with 0 and
# ordered by decreasing rho^2.  Throughout, rho_{i_{|S|+1}} = 0.
# ---------------------------------------------------------------------------

def _rho2_next(rho, subset, j):
    """rho^2 of the model after position j (0 past the end)."""
    return rho[subset[j + 1]] ** 2 if j + 1 < len(subset) else 0.0


def condition_a(rho, subset):
    """eq. conditiona: squared correlations strictly decrease along the subset
    (rho_{1,1} = 1 first)."""
    r2 = [rho[i] ** 2 for i in subset]
    return subset[0] == 0 and all(r2[j] > r2[j + 1] for j in range(len(r2) - 1))


def condition_b(cost, rho, subset):
    """eq. conditionb for j = 2..|S| (positions 1..|S|-1 here)."""
    for j in range(1, len(subset)):
        prev, cur = subset[j - 1], subset[j]
        lhs = cost[prev] / cost[cur]
        num = rho[prev] ** 2 - rho[cur] ** 2
        den = rho[cur] ** 2 - _rho2_next(rho, subset, j)
        if not lhs > num / den:
            return False
    return True


def variance_reduction_ratio(cost, rho, subset):
    """eq. variance_reduction_ratio."""
    s = 0.0
    for j, i in enumerate(subset):
        s += np.sqrt(cost[i] / cost[0] * (rho[i] ** 2 - _rho2_next(rho, subset, j)))
    return s * s


def min_budget(cost, rho, subset):
    """eq. bmin: C_1 sqrt(V / (1 - rho_{1,i_2}^2))."""
    V = variance_reduction_ratio(cost, rho, subset)
    return cost[0] * np.sqrt(V / (1.0 - rho[subset[1]] ** 2))


def candidate_subsets(K):
    """All 2^(K-1) - 1 subsets holding model 0 and at least one surrogate, in
    pool order."""
    out = []
    for mask in range(1, 1 << (K - 1)):
        out.append((0,) + tuple(k + 1 for k in range(K - 1) if mask >> k & 1))
    return out


def select(cost, rho):
    """Sec. 3.1: order the pool by decreasing rho^2, keep the subsets meeting
    conditions (a) and (b), sorted by increasing V.  Returns a list of
    (subset, V, B_min / C_1) and the number of candidates."""
    K = len(cost)
    order = sorted(range(K), key=lambda k: -rho[k] ** 2)
    if order[0] != 0:
        raise ValueError("model 0 must have the largest correlation (rho = 1)")
    cands = candidate_subsets(K)
    feas = []
    for c in cands:
        sub = tuple(sorted(c, key=lambda k: order.index(k)))
        if condition_a(rho, sub) and condition_b(cost, rho, sub):
            feas.append((sub, variance_reduction_ratio(cost, rho, sub),
                         min_budget(cost, rho, sub) / cost[0]))
    feas.sort(key=lambda t: t[1])
    return feas, len(cands)


def oversampling(cost, rho, subset):
    """eq. rk: r_j for every position of the subset (r_1 = 1)."""
    den = 1.0 - rho[subset[1]] ** 2
    return [np.sqrt(cost[0] * (rho[i] ** 2 - _rho2_next(rho, subset, j))
                    / (cost[i] * den)) for j, i in enumerate(subset)]


def allocate(cost, rho, subset, budget):
    """eq. samples: m_1* = B / sum C r, m_j = m_1* r_j (real), and their
    floors (Remark after eq. bmin).  Returns (m_real, m_int, m1_star)."""
    r = oversampling(cost, rho, subset)
    m1 = budget / sum(cost[i] * rj for i, rj in zip(subset, r))
    m = [m1 * rj for rj in r]
    return m, [int(np.floor(v)) for v in m], m1


def allocate_below_min(cost, rho, subset, budget):
    """Allocation for budgets below B_min (the modified Algorithm 2 of Sec. 4):
    while some model j < |S| has m_j < j, the smallest such j and every model
    before it take m = their position, and the remaining budget is shared by
    the later models with ratios relative to model j+1.  Requires
    B >= sum_l l C_{i_l} (the paper's stricter rule).  Returns (m_real, m_int)."""
    S = len(subset)
    floor_cost = sum((l + 1) * cost[i] for l, i in enumerate(subset))
    if budget < floor_cost:
        raise ValueError("budget below sum_l l C_{i_l}")
    m, _, _ = allocate(cost, rho, subset, budget)
    m = list(m)
    while True:
        viol = [j for j in range(S - 1) if m[j] < j + 1]
        if not viol:
            break
        j = viol[0]  # zero-based position; the paper's index is j + 1
        for l in range(j + 1):
            m[l] = float(l + 1)
        head = subset[j + 1]
        head_gap = rho[head] ** 2 - _rho2_next(rho, subset, j + 1)
        r = [np.sqrt(cost[head] * (rho[subset[l]] ** 2 - _rho2_next(rho, subset, l))
                     / (cost[subset[l]] * head_gap)) for l in range(j + 1, S)]
        rest = budget - sum((l + 1) * cost[subset[l]] for l in range(j + 1))
        mh = rest / sum(cost[subset[l]] * r[l - j - 1] for l in range(j + 1, S))
        for l in range(j + 1, S):
            m[l] = mh * r[l - j - 1]
    return m, [int(np.floor(v)) for v in m]


def mse_theory(sigma1, rho, cost, subset, budget):
    """eq. error_theory with m_1* of eq. samples."""
    _, _, m1 = allocate(cost, rho, subset, budget)
    return sigma1 ** 2 * (1.0 - rho[subset[1]] ** 2) * budget / (m1 * m1 * cost[0])
