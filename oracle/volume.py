"""FP64 reference of the step on the bounded domain Omega = (0, 1)^2 with a
volume constraint on the interaction region Omega_I (arXiv 2310.10750,
Sec. 2.1: eq. nonl_operator integrates over Omega united with Omega_I, the
set of points outside Omega within delta of it; eq. xi_constant).  Case
beta2 = 0, as for the periodic step.  TEST INFRASTRUCTURE ONLY (see the
package docstring).

Reading (the paper names Omega_I but does not state the values imposed there):
u on Omega_I is data that the evolution does not change (a volume constraint),
the initial datum extended to Omega_I unless the caller supplies other values.
The lattice of Omega is n x n with h = 1/n; it is continued by m = floor(sqrt(R2))
nodes on every side, which holds every node of Omega_I that a disc centred in
Omega reaches.  A state is the (n + 2m) x (n + 2m) array; its inner n x n block
(rows and columns m .. m + n - 1) is Omega, the ring of width m is Omega_I.

Because every disc centred in Omega lies inside Omega united with Omega_I,
c_gamma_h is the same full-disc sum as on the torus at every node of Omega,
which is the constancy of c_gamma over Omega stated after eq. nonl_operator.
The step at a node i of Omega is the periodic scheme's (implicit Euler, the
convolution explicit, Sec. 4):

    u_i^k = clamp((u_i^{k-1} + tau beta1 (gamma * u^{k-1})_i) / (1 + tau beta1 xi_h)),
    (gamma * u)_i = sum_{d in D} w_d u_{i+d}   (neighbours in Omega or Omega_I),

and the ring keeps its values.  The output of interest is the mean over the
n^2 nodes of Omega (eq. ooi with |Omega| = 1).  The initial projection onto
[-1, 1] applies to every node, ring included (the identity on admissible
data).
"""
from __future__ import annotations

import numpy as np

from . import disc, weights


def ring_width(n: int, delta: float) -> int:
    """m: the number of Omega_I lattice rows a disc centred in Omega reaches."""
    return disc(n, delta)[1]


def convolve_interior(U, n, delta, kind, amp, sigma):
    """(gamma * u) at the n x n nodes of Omega of the extended state U
    ((n + 2m) x (n + 2m)), accumulated offset by offset in canonical order."""
    ddy, ddx, wd, _ = weights(n, delta, kind, amp, sigma)
    m = ring_width(n, delta)
    U = np.asarray(U, dtype=np.float64)
    if U.shape != (n + 2 * m, n + 2 * m):
        raise ValueError("state must be (n + 2m) x (n + 2m) = %d^2" % (n + 2 * m))
    g = np.zeros((n, n))
    for dy, dx, w in zip(ddy, ddx, wd):
        g += w * U[m + dy:m + dy + n, m + dx:m + dx + n]
    return g


def step(U, n, delta, kind, amp, sigma, c_F, beta1, tau):
    """One step of the extended state U (no initial projection): Omega's nodes
    advance, the ring is copied."""
    ddy, ddx, wd, c_gamma = weights(n, delta, kind, amp, sigma)
    m = ring_width(n, delta)
    xi = c_gamma - c_F
    den = 1.0 + tau * beta1 * xi
    if not den > 0.0:
        raise ValueError("1 + tau beta1 xi_h must be > 0")
    U = np.asarray(U, dtype=np.float64)
    g = convolve_interior(U, n, delta, kind, amp, sigma)
    out = U.copy()
    inner = U[m:m + n, m:m + n]
    out[m:m + n, m:m + n] = np.clip((inner + tau * beta1 * g) / den, -1.0, 1.0)
    return out


def step_sites(U, sites, n, delta, kind, amp, sigma, c_F, beta1, tau):
    """One step evaluated only at the listed nodes of Omega (flat indices
    y n + x of Omega's n x n lattice), for large lattices."""
    ddy, ddx, wd, c_gamma = weights(n, delta, kind, amp, sigma)
    m = ring_width(n, delta)
    den = 1.0 + tau * beta1 * (c_gamma - c_F)
    if not den > 0.0:
        raise ValueError("1 + tau beta1 xi_h must be > 0")
    U = np.asarray(U, dtype=np.float64)
    sites = np.asarray(sites, dtype=np.int64)
    y = sites // n + m
    x = sites % n + m
    g = np.zeros(sites.size)
    for dy, dx, w in zip(ddy, ddx, wd):
        g += w * U[y + dy, x + dx]
    return np.clip((U[y, x] + tau * beta1 * g) / den, -1.0, 1.0)


def ooi(U, n, m):
    """(mean over Omega, f_1 = (1 + mean) / 2)."""
    inner = np.asarray(U, dtype=np.float64)[m:m + n, m:m + n]
    mean = float(np.sum(inner) / (n * n))
    return mean, 0.5 * (1.0 + mean)


def solve(U0, nsteps, n, delta, kind, amp, sigma, c_F, beta1, tau):
    """Project U0 (every node) onto [-1, 1], take nsteps steps.
    Returns (U, mean, f1)."""
    m = ring_width(n, delta)
    U = np.clip(np.asarray(U0, dtype=np.float64), -1.0, 1.0)
    for _ in range(nsteps):
        U = step(U, n, delta, kind, amp, sigma, c_F, beta1, tau)
    mean, f1 = ooi(U, n, m)
    return U, mean, f1
