"""Pins of the FP64 beta2 > 0 step (oracle.b2) -- CPU only.

Pinned against: the beta2 = 0 limit (the projection step of the pinned base
oracle), the closed-form Fourier symbol of the linear step with the 5-point
Laplacian inside A = beta1 I - beta2 Delta_h, the KKT conditions of the
obstacle, and an independent solver of the same step written as a
box-constrained quadratic program in u.
"""
import math

import numpy as np
import pytest

from oracle import b2


def _amp_for(n, delta, kind, sigma, xi):
    """Kernel amplitude with c_gamma_h = 1 + xi (c_F = 1)."""
    from oracle import constants
    return (1.0 + xi) / constants(n, delta, kind, 1.0, sigma, 1.0)[0]


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return np.clip(rng.uniform(-1.5, 1.5, (n, n)), -1, 1)


def test_beta2_zero_is_the_projection_step(orc):
    n, delta = 16, 3 / 16
    sigma = delta / 3
    u = _rand(n, 1)
    for kind in (0, 1):
        a = _amp_for(n, delta, kind, sigma, 0.08)
        _, xi, _ = orc.constants(n, delta, kind, a, sigma, 1.0)
        assert xi > 0
        got, _, _ = b2.step_b2(u, n, delta, kind, a, sigma, 1.0, 1.0, 0.0, 0.05)
        ref = orc.step(u, n, delta, kind, a, sigma, 1.0, 1.0, 0.05)
        assert np.max(np.abs(got - ref)) <= 1e-13


@pytest.mark.parametrize("k", [(1, 0), (2, 3), (5, 1)])
def test_linear_step_fourier_symbol(k):
    """u = a cos(theta . x) with |u| small: one step multiplies the amplitude
    by (1 + tau a_k G_k) / (1 + tau a_k xi), a_k = beta1 + beta2 n^2 (4 - 2
    cos theta_x - 2 cos theta_y), G_k = h^2 amp sum_{d in D} cos(theta . d)."""
    n, r2 = 16, 5
    delta = math.sqrt(r2) / n
    N = sum(1 for dy in range(-3, 4) for dx in range(-3, 4) if dy * dy + dx * dx <= r2)
    amp = 1.05 * n * n / N          # c_gamma = 1.05, xi = 0.05
    beta1, beta2, tau = 1.0, 0.05, 0.01
    tx, ty = 2 * math.pi * k[0] / n, 2 * math.pi * k[1] / n
    y, x = np.mgrid[0:n, 0:n]
    a0 = 1e-3
    u = a0 * np.cos(tx * x + ty * y)
    got, _, _ = b2.step_b2(u, n, delta, 0, amp, 0.0, 1.0, beta1, beta2, tau)
    Gk = amp / (n * n) * sum(math.cos(tx * dx + ty * dy) for dy in range(-3, 4)
                             for dx in range(-3, 4) if dy * dy + dx * dx <= r2)
    ak = beta1 + beta2 * n * n * (4 - 2 * math.cos(tx) - 2 * math.cos(ty))
    factor = (1 + tau * ak * Gk) / (1 + tau * ak * 0.05)
    assert np.max(np.abs(got - factor * u)) <= 1e-13


def test_kkt_conditions():
    n, delta = 20, 3 / 20
    sigma = 0.05
    amp = _amp_for(n, delta, 1, sigma, 0.03)
    u0 = _rand(n, 3)
    from oracle import constants
    _, xi, _ = constants(n, delta, 1, amp, sigma, 1.0)
    assert xi > 0
    u, _, _ = b2.step_b2(u0, n, delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.05)
    mu = b2.multiplier(u, u0, n, delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.05)
    top, bot, inner = u == 1, u == -1, np.abs(u) < 1
    assert top.any() and bot.any() and inner.any()
    assert np.min(mu[top]) >= -1e-9
    assert np.max(mu[bot]) <= 1e-9
    assert np.max(np.abs(mu[inner])) <= 1e-9
    assert np.all(np.abs(u) <= 1)


@pytest.mark.parametrize("n", [10, 20, 32])
@pytest.mark.parametrize("kind", [0, 1])
def test_newton_and_projected_gradient_agree(kind, n):
    """The Newton step (z = xi u + mu) and accelerated projected gradient on
    the box QP in u (dense A^-1; no shared reformulation) reach the same
    point, up to 32^2 (1024 unknowns)."""
    delta = 2 / 10 if n == 10 else 3 / n
    sigma = delta / 2
    amp = _amp_for(n, delta, kind, sigma, 0.1)
    u0 = _rand(n, 4 + kind)
    a, _, _ = b2.step_b2(u0, n, delta, kind, amp, sigma, 1.0, 1.0, 0.05, 0.01)
    b = b2.step_b2_qp(u0, n, delta, kind, amp, sigma, 1.0, 1.0, 0.05, 0.01)
    assert np.max(np.abs(a - b)) <= 1e-9


def test_trajectory_stays_admissible():
    n, delta = 24, 3 / 24
    sigma = 0.05
    amp = _amp_for(n, delta, 1, sigma, 0.02)
    from paper_2310_10750_amd import synth
    u0 = synth.ic_nuclei(n, synth.draw_theta(synth.rng_for(4, 0)))
    u, mean, f1 = b2.solve_b2(u0, 5, n, delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.01)
    assert np.all(np.abs(u) <= 1) and abs(f1 - 0.5 * (1 + mean)) <= 1e-16


# ---------------- xi <= 0: the concave term xi u at the previous step ------

def _amp_xi(n, delta, kind, sigma, xi):
    return _amp_for(n, delta, kind, sigma, xi)


@pytest.mark.parametrize("n", [10, 20, 32])
@pytest.mark.parametrize("xi", [-0.085, -0.01, -1e-12])
@pytest.mark.parametrize("kind", [0, 1])
def test_split_step_active_set_and_projected_gradient_agree(kind, xi, n):
    """For xi <= 0 (including the non-convex regime of the literal step,
    xi < -1/(tau lambda_max(A))) the split step is a strictly convex box QP:
    the active-set iteration and accelerated projected gradient reach the
    same point, up to 32^2."""
    delta = 2 / 10 if n == 10 else 3 / n
    sigma = delta / 2
    amp = _amp_xi(n, delta, kind, sigma, xi)
    u0 = _rand(n, 11 + kind)
    a, mu, it = b2.step_b2_split(u0, n, delta, kind, amp, sigma, 1.0, 1.0, 0.05, 0.01)
    b = b2.step_b2_qp(u0, n, delta, kind, amp, sigma, 1.0, 1.0, 0.05, 0.01, split=True)
    assert np.max(np.abs(a - b)) <= 1e-9
    assert it < 50


@pytest.mark.parametrize("xi", [-0.085, 0.0])
def test_split_step_kkt(xi):
    n, delta = 20, 3 / 20
    sigma = 0.05
    amp = _amp_xi(n, delta, 1, sigma, xi)
    u0 = _rand(n, 21)
    u, mu_pdas, _ = b2.step_b2_split(u0, n, delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.05)
    mu = b2.multiplier(u, u0, n, delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.05)
    top, bot, inner = u == 1, u == -1, np.abs(u) < 1
    assert top.any() and bot.any() and inner.any()
    assert np.min(mu[top]) >= -1e-9
    assert np.max(mu[bot]) <= 1e-9
    assert np.max(np.abs(mu[inner])) <= 1e-9
    assert np.max(np.abs(mu - mu_pdas)) <= 1e-9
    assert np.all(np.abs(u) <= 1)


@pytest.mark.parametrize("k", [(1, 0), (3, 2)])
def test_split_linear_step_fourier_symbol(k):
    """Small cosine data (no site reaches the obstacle): the split step is
    u = u_old + tau A (g - xi u_old), amplitude factor 1 + tau a_k (G_k - xi)."""
    n, r2 = 16, 5
    delta = math.sqrt(r2) / n
    N = sum(1 for dy in range(-3, 4) for dx in range(-3, 4) if dy * dy + dx * dx <= r2)
    amp = 0.93 * n * n / N          # c_gamma = 0.93, xi = -0.07
    beta1, beta2, tau = 1.0, 0.05, 0.01
    tx, ty = 2 * math.pi * k[0] / n, 2 * math.pi * k[1] / n
    y, x = np.mgrid[0:n, 0:n]
    a0 = 1e-3
    u = a0 * np.cos(tx * x + ty * y)
    got, _, _ = b2.step_b2_split(u, n, delta, 0, amp, 0.0, 1.0, beta1, beta2, tau)
    Gk = amp / (n * n) * sum(math.cos(tx * dx + ty * dy) for dy in range(-3, 4)
                             for dx in range(-3, 4) if dy * dy + dx * dx <= r2)
    ak = beta1 + beta2 * n * n * (4 - 2 * math.cos(tx) - 2 * math.cos(ty))
    assert np.max(np.abs(got - (1 + tau * ak * (Gk + 0.07)) * u)) <= 1e-13


def test_split_and_implicit_steps_meet_at_xi_zero():
    """As xi -> 0+ the implicit step (Newton in z) tends to the split step
    at xi = 0 (both drop the xi u term)."""
    n, delta = 16, 3 / 16
    sigma = delta / 3
    u0 = _rand(n, 31)
    a0 = _amp_xi(n, delta, 1, sigma, 0.0)
    s0, _, _ = b2.step_b2_split(u0, n, delta, 1, a0, sigma, 1.0, 1.0, 0.05, 0.01)
    for eps in (1e-6, 1e-8):
        a = _amp_xi(n, delta, 1, sigma, eps)
        u, _, _ = b2.step_b2(u0, n, delta, 1, a, sigma, 1.0, 1.0, 0.05, 0.01)
        assert np.max(np.abs(u - s0)) <= 10 * eps


def test_split_constant_states_are_stationary():
    n, delta = 12, 2 / 12
    amp = _amp_xi(n, delta, 0, 0.0, -0.085)
    for c in (1.0, -1.0, 0.0):
        u, _, _ = b2.step_b2_split(np.full((n, n), c), n, delta, 0, amp, 0.0, 1.0, 1.0, 0.05,
                                   0.01)
        assert np.all(u == c)


def test_split_step_at_beta2_zero_is_a_pointwise_projection(orc):
    """With beta2 = 0, A = beta1 I and the split step is the pointwise
    projection of u_old + tau beta1 (gamma*u_old - xi u_old) onto [-1, 1]."""
    n, delta = 16, 3 / 16
    sigma = delta / 3
    for kind, xi in ((0, -0.085), (1, -0.03), (1, 0.0)):
        amp = _amp_xi(n, delta, kind, sigma, xi)
        _, xi_h, _ = orc.constants(n, delta, kind, amp, sigma, 1.0)
        u0 = _rand(n, 41 + kind)
        got, _, _ = b2.step_b2_split(u0, n, delta, kind, amp, sigma, 1.0, 1.0, 0.0, 0.05)
        g = orc.convolve(u0, n, delta, kind, amp, sigma)
        ref = np.clip(u0 + 0.05 * (g - xi_h * u0), -1, 1)
        assert np.max(np.abs(got - ref)) <= 1e-13


def test_split_trajectory_of_the_papers_delta_0125_model(orc):
    """The paper's delta = 0.125 model on 64^2 (Gaussian kernel of
    delta_hf = 0.25, xi ~ -0.09: the non-convex regime of the literal step)
    runs 8 steps with every step's KKT conditions met and the state
    admissible."""
    from paper_2310_10750_amd import synth
    n, delta = 64, 0.125
    amp, sigma, _ = synth.gaussian_params(0.25)
    _, xi, _ = orc.constants(n, delta, 1, amp, sigma, 1.0)
    # below -1/(tau lambda_max(A)), lambda_max(A) = beta1 + 8 beta2 n^2
    assert xi < -1.0 / (0.01 * (1.0 + 8 * 0.05 * n * n))
    u = np.clip(synth.ic_nuclei(n, synth.draw_theta(synth.rng_for(6, 0))), -1, 1)
    for _ in range(8):
        un, _, it = b2.step_b2_split(u, n, delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.01)
        mu = b2.multiplier(un, u, n, delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.01)
        assert np.min(mu[un == 1], initial=0.0) >= -1e-9
        assert np.max(mu[un == -1], initial=0.0) <= 1e-9
        assert np.max(np.abs(mu[np.abs(un) < 1]), initial=0.0) <= 1e-9
        assert it < 50
        u = un
    assert np.all(np.abs(u) <= 1)
    _, mean, f1 = b2.solve_b2(synth.ic_nuclei(n, synth.draw_theta(synth.rng_for(6, 0))), 8, n,
                              delta, 1, amp, sigma, 1.0, 1.0, 0.05, 0.01)
    assert abs(mean - np.mean(u)) <= 1e-14
