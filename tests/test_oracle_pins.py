"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics,
not by the oracle itself (CPU only).

Each test names what it pins: lattice counts (Gauss circle problem), a dense
brute-force operator built from minimum-image distances, the Fourier symbol of
the linear step in closed form (Dirichlet kernel), the implicit-Euler
optimality (KKT) conditions, exact symmetries, the energy decrease that the
scheme guarantees for tau*beta1*c_F <= 2, and the paper's printed kernel
normalisation (xi ~ 0.0253, Sec. 4).
"""
import math
import os

import numpy as np
import pytest

from paper_2310_10750_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_pairs(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


# ---------------------------------------------------------------- disc ----

def _count_brute(R2):
    r = int(math.isqrt(R2)) + 1
    return sum(1 for dy in range(-r, r + 1) for dx in range(-r, r + 1)
               if dy * dy + dx * dx <= R2)


def test_gauss_circle_counts_golden(orc):
    """N for integer radii equals the published Gauss-circle counts
    (tests/golden/gauss_circle.txt) and a brute-force enumeration."""
    for R2s, Ns in _golden_pairs("gauss_circle.txt"):
        R2, N = int(R2s), int(Ns)
        assert _count_brute(R2) == N
        # choose n and delta with (delta n)^2 = R2 (+ rounding of delta)
        n = 4 * math.isqrt(R2) + 8
        delta = math.sqrt(R2) / n
        gR2, m, gN, halfw = orc.disc(n, delta)
        assert gR2 == R2
        assert gN == N
        assert m == math.isqrt(R2)
        assert halfw.sum() * 2 + halfw.size == N


def test_disc_halfwidths_match_isqrt(orc):
    """Row half-widths equal isqrt(R2 - dy^2) (independent formula) and the
    count equals 1 + 4 floor(r) + 4 sum floor(sqrt(R2 - i^2))."""
    for n, delta in [(64, 4 / 64), (88, 0.1875), (128, 0.25), (64, 0.125),
                     (512, 16 / 512), (40, 0.1), (30, 0.1), (2048, 32 / 2048)]:
        R2, m, N, halfw = orc.disc(n, delta)
        assert R2 == math.floor((delta * n) ** 2 + 1e-9)
        for dy in range(-m, m + 1):
            assert halfw[dy + m] == math.isqrt(R2 - dy * dy)
        r = math.isqrt(R2)
        assert N == 1 + 4 * r + 4 * sum(math.isqrt(R2 - i * i)
                                        for i in range(1, r + 1))


def test_decimal_horizon_keeps_boundary_ring(orc):
    """delta = 0.1 on n = 40 is delta/h = 4 up to decimal rounding; the closed
    ball must keep the ring |d| = 4."""
    R2, m, N, _ = orc.disc(40, 0.1)
    assert (R2, m, N) == (16, 4, 49)
    R2, m, N, _ = orc.disc(30, 0.1)  # delta/h = 3 exactly in decimal
    assert (R2, m, N) == (9, 3, 29)


# ------------------------------------------------------------- weights ----

def test_constant_kernel_mass_is_lattice_count(orc):
    for n, r in [(64, 4), (128, 8), (512, 16)]:
        amp = 3.7
        c, xi, N = orc.constants(n, r / n, 0, amp, 0.0, 1.0)
        assert N == synth.GAUSS_CIRCLE[r]
        assert abs(c - amp * N / n ** 2) <= 1e-14 * c


def test_paper_kernel_normalisation_gives_printed_xi(orc):
    """Sec. 4: c_F = 1, eps^2 = 0.00178, delta_hf = 0.25, width delta_hf/3,
    xi ~ 0.0253.  The 2-D normalisation 4 eps^2/(pi sigma^4) reproduces it at
    h = 1/128 (the printed sigma^3 would give xi ~ -0.9)."""
    p = {k: float(v) for k, v in _golden_pairs("paper_parameters.txt")}
    sigma = p["delta_hf"] / 3
    amp = 4 * p["eps2"] / (math.pi * sigma ** 4)
    c, xi, _ = orc.constants(128, p["delta_hf"], 1, amp, sigma, p["c_F"])
    assert abs(xi - p["xi"]) < 3e-4
    # the continuum mass 4 eps^2/sigma^2 (1 - e^{-9}) is approached as h -> 0
    cont = 4 * p["eps2"] / sigma ** 2 * (1 - math.exp(-(p["delta_hf"] / sigma) ** 2))
    c512, _, _ = orc.constants(512, p["delta_hf"], 1, amp, sigma, p["c_F"])
    assert abs(c512 - cont) < abs(c - cont) + 1e-12
    assert abs(c512 - cont) < 2e-4 * cont
    amp3 = 4 * p["eps2"] / (math.pi * sigma ** 3)
    _, xi3, _ = orc.constants(128, p["delta_hf"], 1, amp3, sigma, p["c_F"])
    assert xi3 < -0.5


def test_weights_canonical_order_and_values(orc):
    n, delta, sigma, amp = 32, 3.5 / 32, 0.05, 2.0
    ddy, ddx, wd, c = orc.weights(n, delta, 1, amp, sigma)
    pairs = list(zip(ddy.tolist(), ddx.tolist()))
    assert pairs == sorted(pairs)
    h = 1.0 / n
    for (dy, dx), w in zip(pairs, wd):
        r2 = (dy * dy + dx * dx) * h * h
        assert abs(w - h * h * amp * math.exp(-r2 / sigma ** 2)) <= 1e-15 * w
    assert abs(c - math.fsum(wd)) <= 1e-14 * c


# ------------------------------------------------- brute-force operator ----

def _dense_operator(n, delta, kind, amp, sigma):
    """W[i, j] = h^2 gamma(h |x_i - x_j|) over minimum-image lattice
    displacements inside the closed disc; built from all node pairs."""
    R2 = math.floor((delta * n) ** 2 + 1e-9)
    h = 1.0 / n
    ys, xs = np.divmod(np.arange(n * n), n)
    dy = ys[None, :] - ys[:, None]
    dx = xs[None, :] - xs[:, None]
    dy = (dy + n // 2) % n - n // 2
    dx = (dx + n // 2) % n - n // 2
    d2 = dy * dy + dx * dx
    if kind == 0:
        g = np.full(d2.shape, amp, dtype=np.float64)
    else:
        g = amp * np.exp(-(d2 * h * h) / sigma ** 2)
    return np.where(d2 <= R2, h * h * g, 0.0)


@pytest.mark.parametrize("n,r2,kind", [(12, 4, 0), (13, 9, 0), (16, 10, 1),
                                       (11, 5, 1), (16, 16, 0)])
def test_convolution_matches_dense_brute_force(orc, n, r2, kind):
    delta = math.sqrt(r2) / n
    amp, sigma = 1.7, 0.11
    W = _dense_operator(n, delta, kind, amp, sigma)
    rng = np.random.default_rng(11)
    u = rng.uniform(-1, 1, (n, n))
    g = orc.convolve(u, n, delta, kind, amp, sigma)
    ref = (W @ u.reshape(-1)).reshape(n, n)
    assert np.max(np.abs(g - ref)) < 1e-13
    c, _, _ = orc.constants(n, delta, kind, amp, sigma, 1.0)
    assert abs(c - W[0].sum()) < 1e-13


def test_step_matches_dense_implicit_euler(orc):
    """Dense solve of the unconstrained implicit-Euler equation, then
    projection, agrees with the oracle step."""
    n, delta, kind, amp, sigma = 14, 2.3 / 14, 1, 60.0, 0.08
    c_F, beta1, tau = 0.9, 1.0, 0.05
    W = _dense_operator(n, delta, kind, amp, sigma)
    cg = W[0].sum()
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, (n, n))
    A = np.eye(n * n) * (1.0 / tau + beta1 * (cg - c_F))
    rhs = u.reshape(-1) / tau + beta1 * (W @ u.reshape(-1))
    v = np.linalg.solve(A, rhs)
    ref = np.clip(v, -1, 1).reshape(n, n)
    got = orc.step(u, n, delta, kind, amp, sigma, c_F, beta1, tau)
    assert np.max(np.abs(got - ref)) < 1e-13


# --------------------------------------------------- Fourier symbol -------

def _dirichlet(w, theta):
    if abs(math.sin(theta / 2)) < 1e-300:
        return 2 * w + 1
    return math.sin((w + 0.5) * theta) / math.sin(theta / 2)


@pytest.mark.parametrize("n,r,k", [(32, 4, (1, 0)), (32, 4, (3, 5)),
                                   (48, 6, (7, 2)), (40, 3, (0, 9))])
def test_linear_step_fourier_symbol(orc, n, r, k):
    """For a small cosine mode (no clamping) one step multiplies the amplitude
    by (1 + tau beta1 G(k)) / (1 + tau beta1 xi), G(k) the kernel's discrete
    Fourier symbol; for the constant kernel G(k) = h^2 amp sum_dy
    cos(2 pi k_y dy/n) D_{w(dy)}(2 pi k_x / n) with the Dirichlet kernel D."""
    delta = r / n
    amp, c_F, beta1, tau = 2.5, 1.0, 1.0, 0.07
    ky, kx = k
    y, x = np.mgrid[0:n, 0:n]
    a = 1e-3
    u = a * np.cos(2 * np.pi * (kx * x + ky * y) / n)
    R2 = r * r
    th = 2 * math.pi * kx / n
    G = sum(math.cos(2 * math.pi * ky * dy / n) * _dirichlet(math.isqrt(R2 - dy * dy), th)
            for dy in range(-r, r + 1)) * amp / n ** 2
    cg = amp * sum(2 * math.isqrt(R2 - dy * dy) + 1 for dy in range(-r, r + 1)) / n ** 2
    factor = (1 + tau * beta1 * G) / (1 + tau * beta1 * (cg - c_F))
    out = orc.step(u, n, delta, 0, amp, 0.0, c_F, beta1, tau)
    assert np.max(np.abs(out - factor * u)) < 1e-15


# ------------------------------------------------------- invariants -------

def _c1_params():
    return dict(n=24, delta=3 / 24, kind=0, amp=1.0253 * 24 * 24 / 29,
                sigma=0.0, c_F=1.0, beta1=1.0, tau=0.05)


def test_constant_states(orc):
    p = _c1_params()
    n = p["n"]
    args = (n, p["delta"], p["kind"], p["amp"], p["sigma"], p["c_F"], p["beta1"],
            p["tau"])
    for c in (1.0, -1.0, 0.0):
        out = orc.step(np.full((n, n), c), *args)
        assert np.all(out == c)
    cg, xi, _ = orc.constants(n, p["delta"], 0, p["amp"], 0.0, p["c_F"])
    tb = p["tau"] * p["beta1"]
    c = 0.3
    out = orc.step(np.full((n, n), c), *args)
    assert np.max(np.abs(out - c * (1 + tb * cg) / (1 + tb * xi))) < 1e-15


def test_exact_symmetries(orc):
    """Odd symmetry and lattice translations are exact in FP64 (same operation
    order at every site); transposition holds to rounding."""
    p = _c1_params()
    n = p["n"]
    args = (n, p["delta"], p["kind"], p["amp"], p["sigma"], p["c_F"], p["beta1"],
            p["tau"])
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, (n, n))
    s = orc.step(u, *args)
    assert np.array_equal(orc.step(-u, *args), -s)
    for sh in [(1, 0), (0, 5), (7, 11)]:
        assert np.array_equal(orc.step(np.roll(u, sh, (0, 1)), *args),
                              np.roll(s, sh, (0, 1)))
    assert np.max(np.abs(orc.step(u.T.copy(), *args) - s.T)) < 1e-15
    assert np.max(np.abs(orc.step(u[::-1].copy(), *args) - s[::-1])) < 1e-15


def test_kkt_conditions_of_implicit_step(orc):
    """u^k solves (u^k - u^{k-1})/tau + beta1 (c_gamma u^k - g - c_F u^k + mu) = 0
    with mu in the normal cone of [-1, 1] at u^k (Sec. 2 subdifferential)."""
    n, delta, kind, amp, sigma = 32, 5 / 32, 1, 4 * 0.00064 / (math.pi * 0.05 ** 4), 0.05
    c_F, beta1, tau = 1.0, 1.0, 0.02
    rng = np.random.default_rng(9)
    u = np.clip(rng.uniform(-1.3, 1.3, (n, n)), -1, 1)
    cg, _, _ = orc.constants(n, delta, kind, amp, sigma, c_F)
    g = orc.convolve(u, n, delta, kind, amp, sigma)
    uk = orc.step(u, n, delta, kind, amp, sigma, c_F, beta1, tau)
    mu = -(uk - u) / (tau * beta1) - (cg - c_F) * uk + g
    inner = np.abs(uk) < 1
    assert inner.any() and (uk == 1).any() and (uk == -1).any()
    assert np.max(np.abs(mu[inner])) < 1e-11
    assert np.min(mu[uk == 1]) > -1e-11
    assert np.max(mu[uk == -1]) < 1e-11
    assert np.all(np.abs(uk) <= 1)


def test_energy_two_forms_and_monotone_decrease(orc):
    """E_h via 1/2 <u, L u> equals the oracle's pairwise form, and E_h does not
    increase along the scheme when tau*beta1*c_F <= 2."""
    w = synth.workload("C1", n=32)
    m = w.models[0]
    s = w.samples[0]
    u0 = synth.initial_state(w, s)
    u, mean, f1, en = orc.solve(u0, 60, m.n, m.delta, m.kernel, s.amp, m.sigma,
                                s.c_F, m.beta1, m.tau, with_energy=True)
    assert m.tau * m.beta1 * s.c_F <= 2
    assert np.all(np.diff(en) <= 1e-13 * np.abs(en[:-1]))
    assert en[-1] < en[0]
    cg, _, _ = orc.constants(m.n, m.delta, m.kernel, s.amp, m.sigma, s.c_F)
    g = orc.convolve(u, m.n, m.delta, m.kernel, s.amp, m.sigma)
    Lu = cg * u - g
    e2 = (0.5 * np.sum(u * Lu) + 0.5 * s.c_F * np.sum(1 - u * u)) / m.n ** 2
    assert abs(e2 - en[-1]) < 1e-12 * max(1.0, abs(e2))


@pytest.mark.parametrize("n,r,kind", [(12, 3, 0), (13, 2.5, 1), (20, 4, 0)])
def test_energy_matches_exactly_rounded_pair_sum(orc, n, r, kind):
    """E_h against math.fsum over every lattice pair within the horizon
    (minimum-image distances, no disc tables), on random data."""
    rng = np.random.default_rng(n)
    u = rng.uniform(-1, 1, (n, n))
    delta = r / n
    sigma, amp, c_F = delta / 3, 3.7, 0.9
    h = 1.0 / n
    terms, pot = [], []
    for y in range(n):
        for x in range(n):
            pot.append(1.0 - u[y, x] ** 2)
            for yy in range(n):
                for xx in range(n):
                    dy = min(abs(y - yy), n - abs(y - yy))
                    dx = min(abs(x - xx), n - abs(x - xx))
                    if dy * dy + dx * dx > (delta * n) ** 2 + 1e-9:
                        continue
                    rr = h * math.sqrt(dy * dy + dx * dx)
                    g = amp * (math.exp(-rr * rr / sigma ** 2) if kind else 1.0)
                    terms.append(h * h * g * (u[y, x] - u[yy, xx]) ** 2)
    exact = h * h * (0.25 * math.fsum(terms) + 0.5 * c_F * math.fsum(pot))
    got = orc.energy(u, n, delta, kind, amp, sigma, c_F)
    assert abs(got - exact) <= 1e-14 * abs(exact)


def test_output_of_interest_is_fsum_mean(orc):
    w = synth.workload("C1", n=40, nsteps=30)
    m = w.models[0]
    s = w.samples[0]
    u, mean, f1 = orc.solve(synth.initial_state(w, s), w.nsteps, m.n, m.delta,
                            m.kernel, s.amp, m.sigma, s.c_F, m.beta1, m.tau)
    exact = math.fsum(u.reshape(-1)) / m.n ** 2
    assert abs(mean - exact) <= m.n ** 2 * 2.0 ** -53
    assert abs(f1 - 0.5 * (1 + mean)) <= 1e-16
    assert np.all(np.abs(u) <= 1)


def test_initial_projection_and_zero_steps(orc):
    n = 16
    u0 = np.linspace(-1.5, 1.5, n * n).reshape(n, n)
    u, mean, f1 = orc.solve(u0, 0, n, 2 / n, 0, 1.0, 0.0, 1.0, 1.0, 0.01)
    assert np.array_equal(u, np.clip(u0, -1, 1))


def test_solve_many_matches_solve(orc):
    w = synth.workload("C3", n_samples=3, nsteps=20, n=32)
    m = w.models[0]
    u0 = np.stack([synth.initial_state(w, s) for s in w.samples])
    cF = [s.c_F for s in w.samples]
    amp = [s.amp for s in w.samples]
    U, mean, f1 = orc.solve_many(u0, w.nsteps, m.n, m.delta, m.kernel, m.sigma,
                                 m.beta1, m.tau, cF, amp)
    for i, s in enumerate(w.samples):
        u, mm, ff = orc.solve(u0[i], w.nsteps, m.n, m.delta, m.kernel, s.amp,
                              m.sigma, s.c_F, m.beta1, m.tau)
        assert np.array_equal(u, U[i])
        assert mm == mean[i] and ff == f1[i]


def test_rejects_unstable_denominator(orc):
    n = 16
    with pytest.raises(Exception):
        orc.step(np.zeros((n, n)), n, 2 / n, 0, 1.0, 0.0, 500.0, 1.0, 1.0)
    with pytest.raises(Exception):
        orc.step(np.zeros((n, n)), n, 8 / n, 0, 1.0, 0.0, 1.0, 1.0, 0.01)


# ------------------------------------------------ per-site step -----------

def _edge_sites(n):
    """Flat indices of the four corners, a site on each edge, the sites next
    to the corners and the centre of an n x n lattice."""
    pts = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1),
           (0, n // 2), (n - 1, n // 3), (n // 2, 0), (n // 3, n - 1),
           (1, 1), (1, n - 2), (n - 2, 1), (n - 2, n - 2), (n // 2, n // 2)]
    return np.array([y * n + x for y, x in pts], dtype=np.int64)


@pytest.mark.parametrize("n,r2,kind", [(12, 4, 0), (16, 10, 1), (23, 16, 0),
                                       (24, 25, 1), (40, 64, 0), (41, 81, 1)])
def test_step_sites_matches_full_step_and_dense_step(orc, n, r2, kind):
    """One step evaluated at chosen sites equals the whole-lattice step there
    bit for bit, and equals the dense implicit-Euler step (the minimum-image
    operator built from all node pairs, then the projection) to rounding: at
    random interior sites, the four corners, every edge and the sites next to
    the corners, where the disc wraps around the torus."""
    delta = math.sqrt(r2) / n
    amp, sigma = (1.0253 * n * n / 49.0, 0.0) if kind == 0 else (2500.0, 0.04)
    c_F, beta1, tau = 0.95, 1.0, 0.05
    rng = np.random.default_rng(n * 100 + r2)
    u = np.clip(rng.uniform(-1.2, 1.2, (n, n)), -1, 1)
    sites = np.concatenate([_edge_sites(n),
                            rng.choice(n * n, size=min(40, n * n), replace=False)])
    got = orc.step_sites(u, sites, n, delta, kind, amp, sigma, c_F, beta1, tau)
    full = orc.step(u, n, delta, kind, amp, sigma, c_F, beta1, tau).reshape(-1)
    assert np.array_equal(got, full[sites])
    W = _dense_operator(n, delta, kind, amp, sigma)
    cg = W[0].sum()
    tb = tau * beta1
    dense = np.clip((u.reshape(-1) + tb * (W @ u.reshape(-1))) / (1 + tb * (cg - c_F)),
                    -1, 1)
    assert np.max(np.abs(got - dense[sites])) < 1e-13
    # the sites are evaluated independently: order and repeats do not matter
    perm = np.concatenate([sites[::-1], sites[:3]])
    got2 = orc.step_sites(u, perm, n, delta, kind, amp, sigma, c_F, beta1, tau)
    assert np.array_equal(got2, full[perm])


def test_step_sites_rejects_out_of_range_sites(orc):
    n = 16
    u = np.zeros((n, n))
    for bad in ([-1], [n * n], [0, n * n + 5]):
        with pytest.raises(Exception):
            orc.step_sites(u, np.array(bad, dtype=np.int64), n, 2 / n, 0, 1.0, 0.0,
                           1.0, 1.0, 0.01)


def test_trajectory_goldens_are_consistent():
    """The stored full-size oracle results parse, name the recipes' shapes,
    satisfy f_1 = (1 + mean)/2 (eq. ooi) and keep every stored value in
    [-1, 1]; the sites include the four corners."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_trajectory_goldens", os.path.join(GOLDEN, "make_trajectory_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    g = mod.read_goldens(os.path.join(GOLDEN, "trajectories.txt"))
    assert set(g) == set(mod.CASES)
    for name, v in g.items():
        recipe, idx, prec, nsteps = mod.CASES[name]
        assert (v["recipe"], v["sample"], v["precision"], v["nsteps"]) == (recipe, idx, prec,
                                                                            nsteps)
        w = synth.workload(recipe)
        assert v["n"] == w.models[w.samples[idx].model].n
        assert abs(v["f1"] - 0.5 * (1 + v["mean"])) <= 1e-16
        assert np.all(np.abs(v["values"]) <= 1.0)
        n = v["n"]
        assert {0, n - 1, (n - 1) * n, n * n - 1} <= set(v["sites"].tolist())
        assert np.array_equal(v["sites"], mod.case_sites(n, 1000 + idx))
