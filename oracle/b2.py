"""FP64 reference of the time step with beta2 > 0 (arXiv 2310.10750, eq.
nonl_CH_nm with beta1 > 0 and beta2 > 0: the non-mass-conserving nonlocal
model of the paper's experiments).  TEST INFRASTRUCTURE ONLY (see the package
docstring).

Model (Sec. 2.1):  du/dt + A w = 0 with A = beta1 I - beta2 Delta and
w = L u + dF_obs(u) = xi u - gamma*u + mu,  mu in N_K(u),  K = [-1, 1]^{n^2}
(eq. nonl_operator, eq. potential_obstacle and its subdifferential,
xi = c_gamma - c_F as in eq. xi_constant).

Discretisation (Sec. 4: implicit Euler with the convolution explicit; nodal
quadrature of the convolution; Delta_h the periodic 5-point Laplacian, which
is what lumped P1 elements give on the uniform right-triangle mesh):

    u + tau A (xi u + mu) = r,    r = u_old + tau A g,    g = gamma * u_old.

For xi > 0 put z = xi u + mu.  Then mu in N_K(u) is the same as
u = P_K(z / xi), and z is the root of

    F(z) = tau A z + P_K(z / xi) - r,

the gradient of the strictly convex function
Phi(z) = tau/2 z'Az + sum_i phi(z_i) - r'z with phi(s) = s^2/(2 xi) for
|s| <= xi and |s| - xi/2 otherwise.  The step is therefore unique.

* step_b2: semismooth Newton on F (Jacobian tau A + diag(1/xi on |z| < xi)),
  each Newton system solved by a sparse direct factorisation, backtracking on
  Phi; returns u = P_K(z / xi) and z.
* step_b2_qp: the same step as the box-constrained quadratic program in u,
  min 1/2 u'Mu - c'u over K with M = A^{-1}/tau + xi I and
  c = A^{-1} u_old / tau + g (the step equation multiplied by A^{-1}/tau),
  solved by accelerated projected gradient with a dense A^{-1}: an
  independent method for cross-checking on tiny lattices.
* multiplier: mu = A^{-1}(r - u)/tau - xi u, for the KKT checks.

For xi <= 0 the term xi u of the potential's derivative is concave, and the
literal step minimises a function that is not convex once
xi < -1/(tau lambda_max(A)), so it may have several solutions.  Reading used
(convex splitting applied to the paper's implicit/explicit split): xi u is
implicit where it is convex (xi > 0, above) and taken at the previous step
where it is concave (xi <= 0):

    u + tau A mu = r',   r' = u_old + tau A (g - xi u_old),   mu in N_K(u),

a strictly convex problem (u is the A^{-1}-weighted projection of r' onto K)
with a unique solution.

* step_b2_split: that step by a primal-dual active-set iteration on the
  complementarity problem in mu (matrix tau A, an M-matrix): with
  A+ = {mu + c (u - 1) > 0}, A- = {mu + c (u + 1) < 0}, u = +-1 there, mu = 0
  elsewhere, solve tau A_AA mu_A = r'_A - u_A and u_I = r'_I - tau A_IA mu_A;
  repeat until the active sets repeat (finite for M-matrices).
* step_b2_qp(..., split=True): the same step as the box QP
  min 1/2 u'(A^{-1}/tau)u - c'u, c = A^{-1} u_old/tau + g - xi u_old, by
  accelerated projected gradient (independent solver, tiny lattices).
* step_b2_any: the step for either sign of xi.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import constants, convolve


def laplacian(n: int) -> sp.csr_matrix:
    """Periodic 5-point Laplacian on the n x n lattice, h = 1/n, index y n + x."""
    N = n * n
    idx = np.arange(N).reshape(n, n)
    rows, cols, vals = [], [], []
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        rows.append(idx.ravel())
        cols.append(np.roll(np.roll(idx, -dy, axis=0), -dx, axis=1).ravel())
        vals.append(np.full(N, float(n * n)))
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(np.full(N, -4.0 * n * n))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def a_matrix(n, beta1, beta2):
    return (beta1 * sp.identity(n * n, format="csr") - beta2 * laplacian(n)).tocsr()


def _phi(z, xi):
    a = np.abs(z)
    return np.where(a <= xi, z * z / (2.0 * xi), a - 0.5 * xi)


def step_b2(u_old, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau, z0=None,
            tol=1e-13, max_newton=100):
    """One step from u_old (n x n, in K).  Returns (u, z, newton iterations)."""
    _, xi, _ = constants(n, delta, kind, amp, sigma, c_F)
    if not xi > 0:
        raise ValueError("the reformulation u = P_K(z/xi) needs xi > 0 (xi = %g)" % xi)
    A = a_matrix(n, beta1, beta2)
    u_old = np.asarray(u_old, dtype=np.float64).reshape(-1)
    g = convolve(u_old.reshape(n, n), n, delta, kind, amp, sigma).reshape(-1)
    r = u_old + tau * (A @ g)
    z = xi * u_old if z0 is None else np.asarray(z0, dtype=np.float64).reshape(-1).copy()

    def Phi(v):
        return 0.5 * tau * v @ (A @ v) + _phi(v, xi).sum() - r @ v

    scale = max(1.0, np.linalg.norm(r))
    for it in range(max_newton):
        F = tau * (A @ z) + np.clip(z / xi, -1.0, 1.0) - r
        if np.linalg.norm(F) <= tol * scale:
            return np.clip(z / xi, -1.0, 1.0).reshape(n, n), z.reshape(n, n), it
        D = np.where(np.abs(z) < xi, 1.0 / xi, 0.0)
        J = (tau * A + sp.diags(D)).tocsc()
        d = spla.spsolve(J, -F)
        f0, slope, a = Phi(z), F @ d, 1.0
        while Phi(z + a * d) > f0 + 1e-4 * a * slope and a > 1e-12:
            a *= 0.5
        z = z + a * d
    raise RuntimeError("semismooth Newton did not converge")


def step_b2_split(u_old, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau, c=1.0,
                  max_iter=200):
    """One step for xi <= 0 (xi u at the previous step; see the module
    docstring) by the primal-dual active-set iteration.  Returns
    (u, mu, iterations)."""
    _, xi, _ = constants(n, delta, kind, amp, sigma, c_F)
    if xi > 0:
        raise ValueError("the split step is the reading for xi <= 0 (xi = %g)" % xi)
    A = a_matrix(n, beta1, beta2)
    u_old = np.asarray(u_old, dtype=np.float64).reshape(-1)
    g = convolve(u_old.reshape(n, n), n, delta, kind, amp, sigma).reshape(-1)
    rp = u_old + tau * (A @ (g - xi * u_old))
    u, mu = rp.copy(), np.zeros_like(rp)
    prev = None
    for it in range(max_iter):
        up = mu + c * (u - 1.0) > 0
        dn = mu + c * (u + 1.0) < 0
        key = (up.tobytes(), dn.tobytes())
        if key == prev:
            return u.reshape(n, n), mu.reshape(n, n), it
        prev = key
        act = up | dn
        u = np.where(up, 1.0, np.where(dn, -1.0, u))
        mu = np.zeros_like(rp)
        if act.any():
            Aa = (tau * A[act][:, act]).tocsc()
            mu[act] = spla.spsolve(Aa, rp[act] - u[act])
        inact = ~act
        u[inact] = rp[inact] - tau * (A[inact][:, act] @ mu[act])
    raise RuntimeError("active-set iteration did not settle")


def step_b2_any(u_old, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau, z0=None):
    """The step for either sign of xi: (u, z or None)."""
    _, xi, _ = constants(n, delta, kind, amp, sigma, c_F)
    if xi > 0:
        u, z, _ = step_b2(u_old, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau, z0=z0)
        return u, z
    u, _, _ = step_b2_split(u_old, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau)
    return u, None


def step_b2_qp(u_old, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau, iters=200000,
               tol=1e-14, split=False):
    """The same step as a box-constrained QP in u, by accelerated projected
    gradient (FISTA) with dense matrices (tiny lattices only); split=True:
    the xi <= 0 step (xi u at the previous step)."""
    _, xi, _ = constants(n, delta, kind, amp, sigma, c_F)
    Ainv = np.linalg.inv(a_matrix(n, beta1, beta2).toarray())
    M = Ainv / tau + (0.0 if split else xi) * np.eye(n * n)
    u_old = np.asarray(u_old, dtype=np.float64).reshape(-1)
    g = convolve(u_old.reshape(n, n), n, delta, kind, amp, sigma).reshape(-1)
    c = Ainv @ u_old / tau + g - (xi * u_old if split else 0.0)
    ev = np.linalg.eigvalsh(M)
    if ev[0] <= 0:
        raise ValueError("M is not positive definite: the step is not a convex QP")
    L = ev[-1]
    u = np.clip(u_old, -1, 1)
    y, t = u.copy(), 1.0
    for _ in range(iters):
        un = np.clip(y - (M @ y - c) / L, -1.0, 1.0)
        tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        y = un + ((t - 1.0) / tn) * (un - u)
        if np.max(np.abs(un - u)) <= tol:
            u = un
            break
        u, t = un, tn
    return u.reshape(n, n)


def multiplier(u_new, u_old, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau):
    """mu of the step equation: mu = A^{-1}(r - u)/tau - xi u (xi > 0), or
    mu = A^{-1}(r' - u)/tau with r' = u_old + tau A (g - xi u_old) (xi <= 0)."""
    _, xi, _ = constants(n, delta, kind, amp, sigma, c_F)
    A = a_matrix(n, beta1, beta2)
    u_old = np.asarray(u_old, dtype=np.float64).reshape(-1)
    u = np.asarray(u_new, dtype=np.float64).reshape(-1)
    g = convolve(u_old.reshape(n, n), n, delta, kind, amp, sigma).reshape(-1)
    if xi > 0:
        r = u_old + tau * (A @ g)
        return (spla.spsolve(A.tocsc(), r - u) / tau - xi * u).reshape(n, n)
    rp = u_old + tau * (A @ (g - xi * u_old))
    return (spla.spsolve(A.tocsc(), rp - u) / tau).reshape(n, n)


def solve_b2(u0, nsteps, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau):
    """Project u0 onto K and take nsteps steps (for xi > 0 each Newton
    iteration warm-started from the previous z).  Returns (u, mean, f1)."""
    u = np.clip(np.asarray(u0, dtype=np.float64).reshape(n, n), -1.0, 1.0)
    z = None
    for _ in range(nsteps):
        u, z = step_b2_any(u, n, delta, kind, amp, sigma, c_F, beta1, beta2, tau, z0=z)
    mean = float(np.sum(u) / (n * n))
    return u, mean, 0.5 * (1.0 + mean)
