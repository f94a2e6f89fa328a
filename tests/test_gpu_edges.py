"""GPU edge cases against the FP64 oracle, through the C ABI: the degenerate
horizon delta = 0 (the disc is the site itself, so the nonlocal operator
vanishes), the widest horizon the direct kernel takes (m = 48), the smallest
lattices a disc allows (n = 2m + 1), a solve of zero steps (projection and
output of interest only), and a lattice whose indices pass 2^31 bytes."""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TDT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}
NPD = {"f64": np.float64, "f32": np.float32, "f16": np.float16}
TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 1e-3}
A = {"direct": nlch.NLCH_ALGO_DIRECT, "rowrun": nlch.NLCH_ALGO_ROWRUN}


def _model(n, R2, kind=0, c_F=1.0, tau=0.05):
    delta = math.sqrt(R2 + 0.25) / n if R2 > 0 else 0.0
    _, m, N, _ = nlch.nlch_disc(n, delta)
    assert m * m <= R2 < (m + 1) ** 2
    sigma = max(delta, 1.0 / n) / 3
    amp = 1.0253 * n * n / N if kind == 0 else 1.0253 / (math.pi * sigma * sigma)
    return nlch.make_model(n, delta, kind, amp, sigma, c_F=c_F, tau=tau)


def _state(n, seed, prec, lo=-1.0, hi=1.0):
    u = np.random.default_rng(seed).uniform(lo, hi, (n, n))
    return u.astype(NPD[prec]).astype(np.float64)


def _step(md, prec, algo, u):
    x = torch.from_numpy(u.reshape(-1)).to(TDT[prec]).to(DEV)
    y = torch.full_like(x, 5.0)
    nlch.nlch_step(md, nlch.PRECISIONS[prec], A[algo], x, y, None)
    torch.cuda.synchronize()
    return y.double().cpu().numpy().reshape(md.n, md.n)


def _oracle(orc, md, u):
    return orc.step(u, md.n, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma, md.c_F,
                    md.beta1, md.tau)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("kind", [0, 1])
def test_zero_horizon_is_the_local_reaction(orc, kind, prec):
    """delta = 0: N = 1, the operator sum is empty, and the step is the local
    map u -> clamp(u (1 + tau beta1 (w0 - ... )) / (1 + tau beta1 xi))."""
    n = 40
    md = _model(n, 0, kind)
    R2, m, N, _ = nlch.nlch_disc(n, md.delta)
    assert (R2, m, N) == (0, 0, 1)
    u = _state(n, 3, prec)
    got = _step(md, prec, "direct", u)
    ref = _oracle(orc, md, u)
    assert np.max(np.abs(got - ref)) <= TOL[prec]
    c, xi, _ = nlch.nlch_model_constants(md)
    tb = md.tau * md.beta1
    local = np.clip((u + tb * c * u) / (1.0 + tb * xi), -1, 1)
    assert np.max(np.abs(ref - local)) <= 1e-15


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_widest_direct_horizon(orc, prec):
    """m = 48 (R2 = 2304, 7241 disc points) on a 100-lattice: the direct
    kernel's largest LDS tile."""
    md = _model(100, 48 * 48, 1)
    u = _state(100, 5, prec, -0.7, 0.7)
    got = _step(md, prec, "direct", u)
    assert np.max(np.abs(got - _oracle(orc, md, u))) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("algo", ["direct", "rowrun"])
@pytest.mark.parametrize("n,R2", [(3, 1), (5, 4), (9, 16), (11, 25)])
def test_smallest_lattice_for_a_disc(orc, n, R2, algo, prec):
    """n = 2m + 1: every disc offset reaches a distinct site of the torus, and
    a single strip and band cover the lattice with most lanes idle."""
    md = _model(n, R2, 0)
    u = _state(n, 11 + n, prec)
    got = _step(md, prec, algo, u)
    assert np.max(np.abs(got - _oracle(orc, md, u))) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("algo", [nlch.NLCH_ALGO_AUTO, nlch.NLCH_ALGO_DIRECT])
def test_zero_steps_projects_and_reduces(algo, prec):
    """nsteps = 0: the state comes back projected onto [-1, 1] and the output
    of interest is its mean (64^2 runs LDS-resident under AUTO)."""
    n = 64
    md = _model(n, 16)
    u0 = _state(n, 21, prec, -1.5, 1.5)
    x = torch.from_numpy(u0.reshape(-1)).to(TDT[prec]).to(DEV)
    scr = torch.empty_like(x)
    ooi = torch.zeros(2, dtype=torch.float64, device=DEV)
    smp = [nlch.nlch_sample(0, 0, 1.0, md.kernel_amp, 0)]
    nlch.nlch_solve_batch([md], smp, 0, nlch.PRECISIONS[prec], algo, x, scr, ooi)
    torch.cuda.synchronize()
    got = x.double().cpu().numpy().reshape(n, n)
    assert np.array_equal(got, np.clip(u0, -1, 1))
    o = ooi.cpu().numpy()
    assert abs(o[0] - got.mean()) <= 1e-13
    assert abs(o[1] - 0.5 * (1 + got.mean())) <= 1e-13


@pytest.mark.parametrize("algo", ["rowrun", "direct"])
def test_large_lattice_indexing(orc, algo):
    """A 20000^2 lattice (4e8 sites, 1.6 GB per FP32 state; offsets past 2^31
    bytes and 2^28 elements): one step at sampled sites, including the last
    rows and columns, against the oracle evaluated at those sites."""
    n = 20000
    md = _model(n, 64, 0)
    rng = np.random.default_rng(8)
    u = rng.uniform(-0.9, 0.9, n * n).astype(np.float32)
    x = torch.from_numpy(u).to(DEV)
    y = torch.empty_like(x)
    ooi = torch.zeros(2, dtype=torch.float64, device=DEV)
    nlch.nlch_step(md, nlch.NLCH_F32, A[algo], x, y, ooi)
    torch.cuda.synchronize()
    sites = np.concatenate([[0, n - 1, n * n - n, n * n - 1, (n // 2) * n + n // 2],
                            rng.integers(0, n * n, 2000)])
    got = y[torch.from_numpy(sites).to(DEV)].double().cpu().numpy()
    ref = orc.step_sites(u.astype(np.float64).reshape(n, n), sites, n, md.delta, md.kernel,
                         md.kernel_amp, md.kernel_sigma, md.c_F, md.beta1, md.tau)
    assert np.max(np.abs(got - ref)) <= TOL["f32"]
    mean = float(y.double().mean().item())
    assert abs(ooi.cpu().numpy()[0] - mean) <= 1e-12
    del x, y
    torch.cuda.empty_cache()
