"""Pins of the volume-constrained oracle (bounded Omega, data on Omega_I;
arXiv 2310.10750 Sec. 2.1, eq. nonl_operator over Omega and Omega_I) against
facts that do not come from the oracle itself (CPU only): the torus step of
the pinned periodic oracle when the ring is the periodic image, a dense
operator built from Euclidean distances, a closed-form count of the disc
points that fall into Omega_I, the constancy of c_gamma over Omega, locality
of the ring's influence, stationary states and exact symmetries.
"""
import math

import numpy as np
import pytest

from oracle import volume as vol

TB = dict(beta1=1.0, tau=0.02)


def _model(n, R2, kind=0, amp=None, sigma=0.1):
    delta = math.sqrt(R2 + 0.25) / n
    if amp is None:
        amp = 1.0253 * n * n / _disc_count(R2) if kind == 0 else 30.0
    return dict(n=n, delta=delta, kind=kind, amp=amp, sigma=sigma)


def _disc_count(R2):
    r = math.isqrt(R2)
    return sum(2 * math.isqrt(R2 - dy * dy) + 1 for dy in range(-r, r + 1))


def _state(n, m, seed, amp=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(n + 2 * m, n + 2 * m))


@pytest.mark.parametrize("n,R2,kind", [(12, 4, 0), (16, 9, 1), (20, 16, 0), (24, 25, 1)])
def test_periodic_image_ring_gives_the_torus_step(orc, n, R2, kind):
    """With the ring holding the periodic image of Omega, one step on Omega
    equals the periodic oracle's step (pinned independently)."""
    md = _model(n, R2, kind)
    m = vol.ring_width(n, md["delta"])
    assert m == math.isqrt(R2)
    u = np.random.default_rng(7).uniform(-0.6, 0.6, size=(n, n))
    U = np.pad(u, m, mode="wrap")
    out = vol.step(U, c_F=1.0, **md, **TB)
    ref = orc.step(u, n, md["delta"], md["kind"], md["amp"], md["sigma"], 1.0,
                   TB["beta1"], TB["tau"])
    np.testing.assert_allclose(out[m:m + n, m:m + n], ref, rtol=0, atol=1e-15)
    ring = np.ones_like(U, dtype=bool)
    ring[m:m + n, m:m + n] = False
    assert np.array_equal(out[ring], U[ring])


@pytest.mark.parametrize("n,R2,kind", [(10, 4, 0), (12, 9, 1)])
def test_c_gamma_is_constant_over_omega(orc, n, R2, kind):
    """gamma * 1 over Omega and Omega_I is the same full-disc mass at every node
    of Omega (the constancy the paper states after eq. nonl_operator), equal
    to the torus value."""
    md = _model(n, R2, kind)
    m = vol.ring_width(n, md["delta"])
    g = vol.convolve_interior(np.ones((n + 2 * m, n + 2 * m)), **md)
    c, _, _ = orc.constants(n, md["delta"], md["kind"], md["amp"], md["sigma"], 1.0)
    np.testing.assert_allclose(g, c, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,R2", [(9, 4), (14, 10), (17, 16)])
def test_closed_form_ring_count(n, R2):
    """Omega at 0 and the ring at b: after one step (constant kernel) node i
    holds tau beta1 w b c_out(i) / (1 + tau beta1 xi), where c_out(i) is the
    number of disc points of i outside Omega, counted from the row half-widths
    isqrt(R2 - dy^2) clipped to the box."""
    md = _model(n, R2, 0)
    m = math.isqrt(R2)
    N = _disc_count(R2)
    b = 0.3
    U = np.full((n + 2 * m, n + 2 * m), b)
    U[m:m + n, m:m + n] = 0.0
    c_F = 1.0
    out = vol.step(U, c_F=c_F, **md, **TB)[m:m + n, m:m + n]
    w = md["amp"] / (n * n)
    xi = N * w - c_F
    den = 1.0 + TB["tau"] * TB["beta1"] * xi
    exp = np.zeros((n, n))
    for y in range(n):
        for x in range(n):
            inside = 0
            for dy in range(-m, m + 1):
                if 0 <= y + dy < n:
                    hw = math.isqrt(R2 - dy * dy)
                    inside += min(x + hw, n - 1) - max(x - hw, 0) + 1
            exp[y, x] = TB["tau"] * TB["beta1"] * w * b * (N - inside) / den
    np.testing.assert_allclose(out, np.clip(exp, -1, 1), rtol=1e-13, atol=1e-16)
    assert exp[n // 2, n // 2] == 0.0 or n <= 2 * m
    assert exp.max() > 0.0


@pytest.mark.parametrize("kind", [0, 1])
def test_dense_operator_from_distances(kind):
    """A dense operator over the extended lattice built from Euclidean node
    distances (|x_i - x_j| <= delta) and the kernel formula reproduces the
    step on Omega."""
    n, R2 = 7, 5
    md = _model(n, R2, kind, amp=20.0 if kind else None, sigma=0.2)
    m = math.isqrt(R2)
    ne = n + 2 * m
    h = 1.0 / n
    U = _state(n, m, 3, amp=0.8)
    c_F = 0.97
    ys, xs = np.meshgrid(np.arange(ne), np.arange(ne), indexing="ij")
    pos = np.stack([ys.ravel(), xs.ravel()], 1) * h
    G = np.zeros((n * n, ne * ne))
    for r in range(n):
        for c in range(n):
            i = (r + m) * ne + (c + m)
            d2 = np.sum((pos - pos[i]) ** 2, axis=1)
            inn = d2 <= md["delta"] ** 2 * (1 + 1e-12)
            gam = md["amp"] * (np.exp(-d2 / md["sigma"] ** 2) if kind else np.ones_like(d2))
            G[r * n + c] = np.where(inn, h * h * gam, 0.0)
    cg = G.sum(axis=1)
    np.testing.assert_allclose(cg, cg[0], rtol=1e-14)
    tb = TB["tau"] * TB["beta1"]
    den = 1.0 + tb * (cg[0] - c_F)
    inner = U[m:m + n, m:m + n].ravel()
    exp = np.clip((inner + tb * (G @ U.ravel())) / den, -1, 1).reshape(n, n)
    out = vol.step(U, c_F=c_F, **md, **TB)
    np.testing.assert_allclose(out[m:m + n, m:m + n], exp, rtol=1e-13, atol=1e-15)


def test_ring_influence_is_local():
    """Nodes of Omega more than m rows and columns from Omega_I do not see the
    ring within one step; nodes next to it do."""
    n, R2 = 24, 16
    md = _model(n, R2, 0)
    m = 4
    U1 = _state(n, m, 11)
    U2 = U1.copy()
    ring = np.ones_like(U1, dtype=bool)
    ring[m:m + n, m:m + n] = False
    U2[ring] = -U2[ring]
    a = vol.step(U1, c_F=1.0, **md, **TB)[m:m + n, m:m + n]
    b = vol.step(U2, c_F=1.0, **md, **TB)[m:m + n, m:m + n]
    deep = (slice(m, n - m), slice(m, n - m))
    assert np.array_equal(a[deep], b[deep])
    assert np.all(a[0] != b[0]) and np.all(a[:, -1] != b[:, -1])


@pytest.mark.parametrize("c", [-1.0, 0.0, 1.0])
def test_constant_states_are_stationary(c):
    n, R2 = 16, 9
    md = _model(n, R2, 0)
    U = np.full((n + 6, n + 6), c)
    assert np.array_equal(vol.step(U, c_F=1.0, **md, **TB), U)


def test_sign_and_lattice_symmetries():
    """step(-U) = -step(U) exactly; transposes and reflections of the extended
    state commute with the step to rounding."""
    n, R2 = 18, 10
    md = _model(n, R2, 1, amp=25.0, sigma=0.15)
    m = 3
    U = _state(n, m, 5, amp=0.9)
    s = vol.step(U, c_F=1.0, **md, **TB)
    assert np.array_equal(vol.step(-U, c_F=1.0, **md, **TB), -s)
    for f in (np.transpose, np.flipud, np.fliplr):
        np.testing.assert_allclose(vol.step(f(U), c_F=1.0, **md, **TB), f(s), rtol=0,
                                   atol=1e-15)


def test_solve_projects_and_reduces_over_omega():
    """The initial projection covers every node; the output of interest is the
    mean over Omega's n^2 nodes only; u stays in [-1, 1]."""
    n, R2 = 12, 4
    md = _model(n, R2, 0)
    m = 2
    U0 = _state(n, m, 9, amp=1.5)
    U, mean, f1 = vol.solve(U0, 5, c_F=1.0, **md, **TB)
    ring = np.ones_like(U0, dtype=bool)
    ring[m:m + n, m:m + n] = False
    assert np.array_equal(U[ring], np.clip(U0[ring], -1, 1))
    assert np.all(np.abs(U) <= 1.0)
    assert mean == pytest.approx(U[m:m + n, m:m + n].mean(), rel=1e-15)
    assert f1 == pytest.approx(0.5 * (1 + mean), rel=1e-15)


def test_site_evaluation_matches_the_full_step():
    """step_sites reproduces the full step at random nodes, including nodes
    next to the ring and the corners."""
    n, R2 = 40, 25
    md = _model(n, R2, 1, amp=40.0, sigma=0.1)
    m = 5
    U = _state(n, m, 21, amp=1.0)
    full = vol.step(U, c_F=1.0, **md, **TB)[m:m + n, m:m + n].ravel()
    sites = np.concatenate([[0, n - 1, n * n - 1, n * (n - 1)],
                            np.random.default_rng(2).choice(n * n, 200, replace=False)])
    got = vol.step_sites(U, sites, c_F=1.0, **md, **TB)
    np.testing.assert_allclose(got, full[sites], rtol=0, atol=1e-15)
