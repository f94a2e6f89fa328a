"""Pins of the FP64 MFMC estimator reference (oracle.mfmc) -- CPU only.

Pinned against: the Monte Carlo special case (alpha = 0), the telescoping
identity for identical models, numpy's own covariance routines for the alpha of
eq. alpha, and unbiasedness of eq. MFMC_estimator on synthetic outputs with a
known mean.
"""
import math

import numpy as np
import pytest

from oracle import mfmc


def _data(seed, m):
    rng = np.random.default_rng(seed)
    z = rng.normal(0.5, 1.0, m[-1])
    y1 = z + 0.05 * rng.normal(size=m[-1])
    y2 = 0.9 * z + 0.2 * rng.normal(size=m[-1]) + 0.1
    y3 = 0.7 * z + 0.5 * rng.normal(size=m[-1]) - 0.3
    return [y1, y2, y3]


def test_alpha_zero_is_monte_carlo():
    m = [10, 40, 200]
    ys = _data(1, m)
    r = mfmc.mfmc_estimate(ys, m, alpha=[0.0, 0.0])
    assert r["q_mfmc"] == r["q_mc"]
    assert abs(r["q_mc"] - math.fsum(ys[0][:10]) / 10) < 1e-15


def test_identical_models_telescope():
    """With y_j = y_1 and alpha_j = 1 the sum telescopes to the mean of y_1
    over the largest sample set."""
    m = [5, 17, 64, 300]
    y = np.random.default_rng(2).uniform(size=300)
    r = mfmc.mfmc_estimate([y, y, y, y], m, alpha=[1.0, 1.0, 1.0])
    assert abs(r["q_mfmc"] - math.fsum(y) / 300) < 1e-14


def test_alpha_matches_library_covariance():
    m = [50, 100, 400]
    ys = _data(3, m)
    r = mfmc.mfmc_estimate(ys, m)
    Y = np.stack([y[:50] for y in ys])
    C = np.cov(Y)
    R = np.corrcoef(Y)
    for j in (1, 2):
        assert abs(r["alpha"][j] - C[0, j] / C[j, j]) < 1e-12
        assert abs(r["rho"][j] - R[0, j]) < 1e-12
        assert abs(r["var"][j] - C[j, j]) < 1e-12
        assert abs(r["mean_mj"][j] - np.mean(ys[j][:m[j]])) < 1e-14
        assert abs(r["mean_mjm1"][j] - np.mean(ys[j][:m[j - 1]])) < 1e-14


def test_estimator_is_unbiased():
    """Fixed alpha: E[Q_MFMC] = E[y_1] exactly; check by replication."""
    m = [4, 16, 64]
    reps = 20000
    rng = np.random.default_rng(4)
    qs = np.empty(reps)
    for i in range(reps):
        z = rng.normal(0.5, 1.0, m[-1])
        y1 = z + 0.05 * rng.normal(size=m[-1])
        y2 = 0.9 * z + 0.2 * rng.normal(size=m[-1]) + 0.1
        y3 = 0.7 * z + 0.5 * rng.normal(size=m[-1]) - 0.3
        qs[i] = mfmc.mfmc_estimate([y1, y2, y3], m, alpha=[1.1, 0.8])["q_mfmc"]
    se = qs.std(ddof=1) / math.sqrt(reps)
    assert abs(qs.mean() - 0.5) < 4 * se


def test_mfmc_beats_mc_variance_on_correlated_models():
    """With well-correlated cheap models the estimator's spread is below the
    Monte Carlo spread at the same number of high-fidelity draws."""
    m = [8, 64, 512]
    rng = np.random.default_rng(5)
    q, qmc = [], []
    for _ in range(3000):
        z = rng.normal(0.0, 1.0, m[-1])
        y1 = z + 0.05 * rng.normal(size=m[-1])
        y2 = z + 0.1 * rng.normal(size=m[-1])
        y3 = z + 0.2 * rng.normal(size=m[-1])
        r = mfmc.mfmc_estimate([y1, y2, y3], m, alpha=[1.0, 1.0])
        q.append(r["q_mfmc"])
        qmc.append(r["q_mc"])
    assert np.var(q) < 0.2 * np.var(qmc)


def test_rejects_bad_sample_counts():
    y = np.zeros(10)
    with pytest.raises(ValueError):
        mfmc.mfmc_estimate([y, y], [1, 5])
    with pytest.raises(ValueError):
        mfmc.mfmc_estimate([y, y], [5, 4])
    with pytest.raises(ValueError):
        mfmc.mfmc_estimate([y, y], [5, 11])


def test_zero_variance_model_gets_zero_alpha():
    m = [4, 8]
    y1 = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8])
    y2 = np.full(8, 0.25)
    r = mfmc.mfmc_estimate([y1, y2], m)
    assert r["alpha"][1] == 0.0 and r["rho"][1] == 0.0
    assert r["q_mfmc"] == r["q_mc"]


def test_single_shared_draw_with_given_alpha():
    """The below-minimum-budget allocation of Sec. 4 can give m_1 = 1; with
    alpha given the estimator needs only means (variance and correlation are
    undefined)."""
    ys = [np.array([2.0]), np.array([1.0, 2.0, 3.0]), np.array([5.0, 1.0, 0.0, 4.0])]
    r = mfmc.mfmc_estimate(ys, [1, 3, 4], [0.5, 0.25])
    assert r["q_mfmc"] == 2.0 + 0.5 * (2.0 - 1.0) + 0.25 * (2.5 - 2.0)
    assert math.isnan(r["var"][0]) and math.isnan(r["rho"][1])
    with pytest.raises(ValueError):
        mfmc.mfmc_estimate(ys, [1, 3, 4])
