"""Seeded synthetic inputs and the workload recipes.

This module only draws random numbers and lays out parameters; it holds none of
the solver's arithmetic (no projection, no kernel sums, no update), so both the
GPU path and the CPU oracle can take their inputs from it.

Random streams: sample ``s`` of a workload with seed ``k`` draws from
``numpy.random.default_rng([k, s])`` in FP64, so a sample's inputs do not
depend on how many other samples are drawn.  Nested multifidelity levels reuse
the same sample streams, i.e. level j evaluates draws 0..m_j-1.

Initial data (arXiv 2310.10750, Sec. 4):

* ``iid``: u0 ~ U(-0.1, 0.1) independently per lattice node;
* ``nuclei``: four nuclei of phase -1 (eq. ic),
  ``u0(x) = 1 - 2 sum_i mu_i exp(-36 |x - xbar_i - eta_i|^2)``, centres
  xbar = (0.25, 0.5), (0.75, 0.5), (0.5, 0.25), (0.5, 0.75) as (x, y), with
  theta_i = (mu_i, eta_i) ~ U([0.9, 1] x [-0.025, 0.025]^2); on the periodic
  unit square the distance is the minimum-image distance.  u0 can leave
  [-1, 1] slightly; projecting it is the solver's first step, not done here.

Arrays are row-major ``[y, x]``, node (x, y) sitting at (x/n, y/n).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List

import numpy as np

KERNEL_CONSTANT = 0
KERNEL_GAUSSIAN = 1

# Integer points (dy, dx) with dy^2 + dx^2 <= r^2 (Gauss circle counts) for
# the integer horizons the recipes use; they set the constant-kernel amplitude
# so that the discrete kernel mass is exactly 1 + xi.
GAUSS_CIRCLE = {1: 5, 2: 13, 3: 29, 4: 49, 8: 197, 16: 797, 32: 3209}

NUCLEI_CENTRES = ((0.25, 0.5), (0.75, 0.5), (0.5, 0.25), (0.5, 0.75))


@dataclass(frozen=True)
class Model:
    """One fidelity level: lattice n x n on the unit torus, horizon delta,
    kernel gamma (constant amp, or amp*exp(-r^2/sigma^2)) on |r| <= delta,
    potential constant c_F, evolution parameters beta1, beta2, time step tau."""
    n: int
    delta: float
    kernel: int
    amp: float
    sigma: float
    c_F: float = 1.0
    beta1: float = 1.0
    beta2: float = 0.0
    tau: float = 0.01
    boundary: int = 0  # 0: periodic torus; 1: Omega = (0,1)^2, fixed data on Omega_I


def state_side(m: Model) -> int:
    """Side of a sample's stored array: n on the torus, n + 2r with the ring
    of r = isqrt(floor((delta n)^2 + 1e-9)) lattice rows of Omega_I data under
    a volume constraint (the layout of the C ABI)."""
    if not m.boundary:
        return m.n
    t = m.delta * m.n
    r = math.isqrt(int(math.floor(t * t + 1e-9)))
    return m.n + 2 * r


@dataclass(frozen=True)
class Sample:
    """One sampled input: which model, its own c_F and kernel amplitude, and
    how its initial datum is drawn."""
    model: int
    c_F: float
    amp: float
    ic: str            # "iid" or "nuclei"
    seed: int
    index: int         # stream index s of default_rng([seed, s])
    theta: tuple = ()  # nuclei parameters (mu1, eta1x, eta1y, ..., mu4, ...)


@dataclass
class Workload:
    name: str
    models: List[Model]
    samples: List[Sample]
    nsteps: int
    precision: str     # "f64", "f32" or "f16"
    description: str = ""
    level_counts: List[int] = field(default_factory=list)

    def site_steps(self) -> int:
        return sum(self.models[s.model].n ** 2 for s in self.samples) * self.nsteps


def rng_for(seed: int, index: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(index)])


def draw_theta(rng: np.random.Generator) -> tuple:
    """Four nuclei parameter triples (mu, eta_x, eta_y), drawn in that order."""
    out = []
    for _ in range(4):
        out.append(rng.uniform(0.9, 1.0))
        out.append(rng.uniform(-0.025, 0.025))
        out.append(rng.uniform(-0.025, 0.025))
    return tuple(float(v) for v in out)


def ic_iid(n: int, seed: int, index: int, lo: float = -0.1, hi: float = 0.1):
    return rng_for(seed, index).uniform(lo, hi, size=(n, n))


def ic_nuclei(n: int, theta) -> np.ndarray:
    """Eq. ic on the n x n periodic lattice (FP64, not projected)."""
    coords = np.arange(n, dtype=np.float64) / n
    X = coords[None, :]
    Y = coords[:, None]
    u = np.ones((n, n), dtype=np.float64)
    for i, (cx, cy) in enumerate(NUCLEI_CENTRES):
        mu, ex, ey = theta[3 * i], theta[3 * i + 1], theta[3 * i + 2]
        dx = X - (cx + ex)
        dy = Y - (cy + ey)
        dx = dx - np.round(dx)   # minimum image on the unit torus
        dy = dy - np.round(dy)
        u = u - 2.0 * mu * np.exp(-36.0 * (dx * dx + dy * dy))
    return u


def theta_block(seed: int, block: int, size: int = 4096) -> np.ndarray:
    """Nuclei parameters of samples block*size .. block*size+size-1 of a
    large study (one generator per block of draws): rows (mu1, eta1x, eta1y,
    ..., mu4, eta4x, eta4y) with mu ~ U[0.9, 1], eta ~ U[-0.025, 0.025]."""
    u = rng_for(seed, block).uniform(size=(size, 12))
    lo = np.tile([0.9, -0.025, -0.025], 4)
    width = np.tile([0.1, 0.05, 0.05], 4)
    return lo + width * u


def ic_nuclei_batch(n: int, thetas, device="cuda:0"):
    """Eq. ic for a batch of parameter rows (as theta_block), computed with
    torch on `device` in FP64: a (B, n*n) tensor, not projected.  Same formula
    and minimum-image distance as ic_nuclei."""
    import torch
    th = torch.as_tensor(np.asarray(thetas, dtype=np.float64), device=device)
    coords = torch.arange(n, dtype=torch.float64, device=device) / n
    X = coords[None, None, :]
    Y = coords[None, :, None]
    u = torch.ones((th.shape[0], n, n), dtype=torch.float64, device=device)
    for i, (cx, cy) in enumerate(NUCLEI_CENTRES):
        mu = th[:, 3 * i, None, None]
        dx = X - (cx + th[:, 3 * i + 1, None, None])
        dy = Y - (cy + th[:, 3 * i + 2, None, None])
        dx = dx - torch.round(dx)
        dy = dy - torch.round(dy)
        u = u - 2.0 * mu * torch.exp(-36.0 * (dx * dx + dy * dy))
    return u.reshape(th.shape[0], n * n)


def initial_state(w: Workload, s: Sample) -> np.ndarray:
    """The sample's stored initial array (state_side x state_side; under a
    volume constraint its ring is the Omega_I data)."""
    m = w.models[s.model]
    n = state_side(m)
    if s.ic == "iid":
        return ic_iid(n, s.seed, s.index)
    if s.ic == "nuclei" and not m.boundary:
        return ic_nuclei(n, s.theta)
    raise ValueError("unknown initial datum kind %r" % s.ic)


def constant_amp(n: int, r: int, mass: float) -> float:
    """Constant-kernel amplitude whose discrete mass h^2 * N * amp equals
    ``mass`` on the disc of integer radius r (N from GAUSS_CIRCLE)."""
    return mass / (GAUSS_CIRCLE[r] / float(n * n))


def gaussian_params(delta_hf: float, eps2_ref: float = 0.00178,
                    delta_ref: float = 0.25):
    """Eq. kernel_gauss with sigma = delta_hf/3 and the 2-D normalisation
    4 eps^2 / (pi sigma^4); eps^2 scaled with delta_hf^2 from the paper's
    (eps^2 = 0.00178, delta_hf = 0.25) so that xi stays about 0.025."""
    sigma = delta_hf / 3.0
    eps2 = eps2_ref * (delta_hf / delta_ref) ** 2
    amp = 4.0 * eps2 / (math.pi * sigma ** 4)
    return amp, sigma, eps2


XI_PAPER = 0.0253   # nonlocal interface parameter of Sec. 4


def workload(name: str, n_samples: int = None, nsteps: int = None,
             precision: str = None, n: int = None) -> Workload:
    """The five recipes (C1..C5); optional overrides shrink them for tests."""
    name = name.upper()
    if name == "C1":
        nn = n or 64
        r = 4
        m = Model(n=nn, delta=r / nn, kernel=KERNEL_CONSTANT,
                  amp=constant_amp(nn, r, 1.0 + XI_PAPER), sigma=0.0,
                  c_F=1.0, tau=0.05)
        S = n_samples or 1
        samples = [Sample(0, m.c_F, m.amp, "iid", 1, s) for s in range(S)]
        w = Workload("C1", [m], samples, nsteps or 200, precision or "f64",
                     "64x64 periodic, delta=4h, constant kernel, iid U(-0.1,0.1)"
                     " initial data, 200 steps of tau=0.05")
    elif name == "C2":
        nn = n or 512
        r = 16
        S = n_samples or 1
        samples = []
        models = []
        for s in range(S):
            rng = rng_for(2, s)
            xi = float(rng.uniform(0.0, 0.05))
            theta = draw_theta(rng)
            amp = constant_amp(nn, r, 1.0 + xi)
            samples.append(Sample(0, 1.0, amp, "nuclei", 2, s, theta))
        models.append(Model(n=nn, delta=r / nn, kernel=KERNEL_CONSTANT,
                            amp=samples[0].amp, sigma=0.0, c_F=1.0, tau=0.01))
        w = Workload("C2", models, samples, nsteps or 1000, precision or "f32",
                     "512x512 periodic, delta=16h (797-point disc), constant "
                     "kernel with xi~U[0,0.05], four-nuclei initial data")
    elif name == "C3":
        nn = n or 128
        r = 8
        amp = constant_amp(nn, r, 1.0 + XI_PAPER)
        m = Model(n=nn, delta=r / nn, kernel=KERNEL_CONSTANT, amp=amp,
                  sigma=0.0, c_F=1.0, tau=0.02)
        S = 4096 if n_samples is None else n_samples
        samples = []
        for s in range(S):
            # c_F ~ U[0.95, 1.05] comes from a stream of its own so that the
            # initial datum of sample s is the same whatever is drawn first.
            cF = float(rng_for(3 + 1000, s).uniform(0.95, 1.05))
            samples.append(Sample(0, cF, amp, "iid", 3, s))
        w = Workload("C3", [m], samples, nsteps or 500, precision or "f32",
                     "4096 samples of 128x128, delta=8h (197-point disc), "
                     "constant kernel, per-sample c_F~U[0.95,1.05], iid initial"
                     " data, 500 steps of tau=0.02")
    elif name == "C4":
        delta = 1.0 / 32.0
        amp, sigma, _ = gaussian_params(delta)
        grids = (1024, 256, 128, 64)
        counts = (8, 64, 512, 4096)
        if n_samples is not None:
            scale = n_samples / 4096.0
            counts = tuple(max(2, int(round(c * scale))) for c in counts)
            counts = tuple(sorted(counts))
        models = [Model(n=g, delta=delta, kernel=KERNEL_GAUSSIAN, amp=amp,
                        sigma=sigma, c_F=1.0, tau=0.01) for g in grids]
        samples = []
        for lvl, cnt in enumerate(counts):
            for s in range(cnt):
                theta = draw_theta(rng_for(4, s))
                samples.append(Sample(lvl, 1.0, amp, "nuclei", 4, s, theta))
        w = Workload("C4", models, samples, nsteps or 100, precision or "f32",
                     "MFMC ensemble: 1024^2 x8, 256^2 x64, 128^2 x512, 64^2 x4096,"
                     " delta=1/32, Gaussian kernel, shared four-nuclei draws, "
                     "100 steps of tau=0.01", list(counts))
    elif name == "V3":
        # C3 on the bounded domain: the ring of Omega_I data is drawn like
        # the interior and then held fixed (volume constraint)
        nn = n or 128
        r = 8
        amp = constant_amp(nn, r, 1.0 + XI_PAPER)
        m = Model(n=nn, delta=r / nn, kernel=KERNEL_CONSTANT, amp=amp,
                  sigma=0.0, c_F=1.0, tau=0.02, boundary=1)
        S = 4096 if n_samples is None else n_samples
        samples = []
        for s in range(S):
            cF = float(rng_for(7 + 1000, s).uniform(0.95, 1.05))
            samples.append(Sample(0, cF, amp, "iid", 7, s))
        w = Workload("V3", [m], samples, nsteps or 500, precision or "f32",
                     "4096 samples of 128x128 on Omega=(0,1)^2 with a volume "
                     "constraint (ring of 8 fixed rows, 144x144 stored), delta=8h "
                     "(197-point disc), constant kernel, per-sample c_F~U[0.95,1.05],"
                     " iid initial data, 500 steps of tau=0.02")
    elif name == "B2":
        # the paper's experimental model: beta1 = 1, beta2 = 0.05, Gaussian
        # kernel of delta = delta_hf = 0.25 (eps^2 = 0.00178), tau = 0.01,
        # four-nuclei data, on the high-fidelity 128^2 lattice
        nn = n or 128
        amp, sigma, _ = gaussian_params(0.25)
        m = Model(n=nn, delta=0.25, kernel=KERNEL_GAUSSIAN, amp=amp, sigma=sigma,
                  c_F=1.0, beta2=0.05, tau=0.01)
        S = 2048 if n_samples is None else n_samples
        samples = [Sample(0, 1.0, amp, "nuclei", 6, s, draw_theta(rng_for(6, s)))
                   for s in range(S)]
        w = Workload("B2", [m], samples, nsteps or 10, precision or "f32",
                     "2048 samples of 128x128, beta1=1, beta2=0.05, delta=0.25 (32h, "
                     "3209-point disc), Gaussian kernel, four-nuclei initial data, "
                     "10 steps of tau=0.01")
    elif name == "C5":
        nn = n or 2048
        r = 32
        amp = constant_amp(nn, r, 1.0 + XI_PAPER)
        m = Model(n=nn, delta=r / nn, kernel=KERNEL_CONSTANT, amp=amp,
                  sigma=0.0, c_F=1.0, tau=0.01)
        S = n_samples or 64
        samples = [Sample(0, 1.0, amp, "nuclei", 5, s,
                          draw_theta(rng_for(5, s))) for s in range(S)]
        w = Workload("C5", [m], samples, nsteps or 100, precision or "f16",
                     "64 samples of 2048x2048, delta=32h (3209-point disc), "
                     "constant kernel, four-nuclei initial data, FP16 state")
    else:
        raise ValueError("unknown workload %r" % name)
    return w


def shrink_model(m: Model, **kw) -> Model:
    return replace(m, **kw)
