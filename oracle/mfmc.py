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
    counts, non-decreasing, m[0] >= 2; alpha: None or K-1 coefficients for
    models 2..K.
    """
    K = len(ys)
    m = [int(v) for v in m]
    if K < 1 or len(m) != K:
        raise ValueError("need one sample count per model")
    if m[0] < 2 or any(m[j] < m[j - 1] for j in range(1, K)):
        raise ValueError("sample counts must be non-decreasing with m[0] >= 2")
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
        var.append(float(np.sum(c * c) / (m0 - 1)))
    rho = []
    for j in range(K):
        if var[0] == 0.0 or var[j] == 0.0:
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
