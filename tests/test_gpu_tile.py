"""The tiled one-step kernel (k_tile, 32 x 32 output tiles staged with their
halo in LDS), used by default for one or a few samples of a lattice and
forced with nlch_set_stream_shape(R=4):

* every site of one step against the FP64 oracle, for every disc it is built
  for, both kernels, FP32 and FP16 storage, lattices that are not a multiple
  of the tile and lattices smaller than a tile (the halo wraps more than once);
* whole trajectories bit for bit equal to the streaming kernel with one wave
  per band (the same window sums, added in the same order);
* the bounded domain with a volume constraint.
"""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch, synth
from tests.gpu_harness import DeviceBatch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TDT = {"f32": torch.float32, "f16": torch.float16}
NPD = {"f32": np.float32, "f16": np.float16}
TOL = {"f32": 1e-6, "f16": 1e-3}
TILE_R2 = [1, 4, 9, 16, 25, 64, 121, 144, 256, 272]


@pytest.fixture(autouse=True)
def _default_shape():
    yield
    nlch.nlch_set_stream_shape(0, 0, 0, 0)


def _model(n, R2, kind, tau=0.05, boundary=0):
    delta = math.sqrt(R2 + 0.25) / n
    _, m, N, _ = nlch.nlch_disc(n, delta)
    sigma = delta / 3
    amp = 1.0253 * n * n / N if kind == 0 else 1.0253 / (math.pi * sigma * sigma)
    return nlch.make_model(n, delta, kind, amp, sigma, c_F=0.98, tau=tau, boundary=boundary)


def _side(md):
    if not md.boundary:
        return md.n
    _, m, _, _ = nlch.nlch_disc(md.n, md.delta)
    return md.n + 2 * m


def _solve(md, prec, u, nsteps, R, samples=1):
    """nsteps of the ROWRUN algorithm (no initial change: u is admissible)
    with streaming shape R (4: tiled) on `samples` copies of u."""
    nlch.nlch_set_stream_shape(R, 0, 0, 0)
    side = _side(md)
    host = np.concatenate([u.reshape(-1)] * samples).astype(NPD[prec])
    x = torch.from_numpy(host).to(DEV)
    scr = torch.empty_like(x)
    ooi = torch.zeros(2 * samples, dtype=torch.float64, device=DEV)
    smp = [nlch.nlch_sample(0, 0, md.c_F, md.kernel_amp, k * side * side) for k in range(samples)]
    nlch.nlch_solve_batch([md], smp, nsteps, nlch.PRECISIONS[prec], nlch.NLCH_ALGO_ROWRUN, x, scr,
                          ooi)
    torch.cuda.synchronize()
    return x.double().cpu().numpy().reshape(samples, side, side), ooi.cpu().numpy()


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("R2", TILE_R2)
def test_tile_one_step_every_site(orc, R2, kind, prec):
    m = math.isqrt(R2)
    for n in (max(2 * m + 1, 20), 70, 96):
        print("tile R2=%d kernel=%d %s n=%d" % (R2, kind, prec, n), flush=True)
        md = _model(n, R2, kind)
        u = np.clip(np.random.default_rng(n + R2).uniform(-1.2, 1.2, (n, n)), -1, 1)
        u = u.astype(NPD[prec]).astype(np.float64)
        got, ooi = _solve(md, prec, u, 1, 4)
        ref = orc.step(u, n, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma, md.c_F,
                       md.beta1, md.tau)
        assert np.max(np.abs(got[0] - ref)) <= TOL[prec], n
        assert abs(ooi[0] - got[0].mean()) <= 1e-12


@pytest.mark.parametrize("R2,kind,prec", [(256, 0, "f32"), (64, 1, "f32"), (121, 0, "f16"),
                                          (9, 1, "f16"), (272, 1, "f32")])
def test_tile_trajectory_equals_streaming(R2, kind, prec):
    n = 100 if R2 < 256 else 130
    print("tile vs stream R2=%d" % R2, flush=True)
    md = _model(n, R2, kind, tau=0.05)
    u = np.random.default_rng(R2).uniform(-0.3, 0.3, (n, n))
    a, oa = _solve(md, prec, u, 30, 4, samples=3)
    b, ob = _solve(md, prec, u, 30, 1, samples=3)
    assert np.array_equal(a, b)
    assert np.array_equal(oa, ob)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_tile_volume_constraint(orc, prec):
    """Omega's 80^2 lattice inside a ring of m = 8 fixed rows: the ring is
    copied, Omega's sites step as in the bounded-domain oracle."""
    from oracle import volume
    n, R2 = 80, 64
    md = _model(n, R2, 0, boundary=1)
    side = _side(md)
    u = np.clip(np.random.default_rng(3).uniform(-1.2, 1.2, (side, side)), -1, 1)
    u = u.astype(NPD[prec]).astype(np.float64)
    got, _ = _solve(md, prec, u, 1, 4)
    ref = volume.step(u, n, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma, md.c_F,
                      md.beta1, md.tau)
    assert np.max(np.abs(got[0] - ref)) <= TOL[prec]


def test_single_high_fidelity_sample_default_is_tiled():
    """C2 (one 512^2 sample, 797-point disc): the default shape runs the tiled
    kernel, and its 100-step states equal the streaming kernel's."""
    print("C2 tile default", flush=True)
    w = synth.workload("C2")
    b = DeviceBatch(w)
    b.solve(algo=nlch.NLCH_ALGO_AUTO, nsteps=100)
    torch.cuda.synchronize()
    nlch.nlch_set_stream_shape(1, 1, 0, 32)
    c = DeviceBatch(w)
    c.solve(algo=nlch.NLCH_ALGO_AUTO, nsteps=100)
    torch.cuda.synchronize()
    assert torch.equal(b.state, c.state)
