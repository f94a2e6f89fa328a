"""GPU parity of the bounded-domain mode (Omega = (0,1)^2 with fixed data on
the interaction region Omega_I, Sec. 2.1) against the FP64 oracle
(oracle.volume), through the C ABI.

Every case checks the updated block against the oracle (one-step bars as for
the torus: 1e-13 FP64, 1e-6 FP32, 1e-3 FP16 storage; trajectories: OoI
relative 1e-12 / 1e-6 / 1e-3 and states 1e-10 / 1e-4), that the ring of both
buffers equals the projected input ring bit-exactly, and that the output of
interest is the mean over Omega alone."""
import math

import numpy as np
import pytest

from oracle import volume as vol
from paper_2310_10750_amd import nlch, synth
from tests.gpu_harness import DeviceBatch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TDT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}
NPD = {"f64": np.float64, "f32": np.float32, "f16": np.float16}
ONE_STEP_TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 1e-3}
TRAJ_TOL = {"f64": (1e-12, 1e-10), "f32": (1e-6, 1e-4), "f16": (1e-3, None)}
A = {"auto": nlch.NLCH_ALGO_AUTO, "direct": nlch.NLCH_ALGO_DIRECT,
     "rowrun": nlch.NLCH_ALGO_ROWRUN, "resident": nlch.NLCH_ALGO_RESIDENT}


def _model(n, R2, kind, tau=0.02, c_F=1.0):
    delta = math.sqrt(R2 + 0.25) / n
    sigma = delta / 3
    r = math.isqrt(R2)
    N = sum(2 * math.isqrt(R2 - dy * dy) + 1 for dy in range(-r, r + 1))
    amp = 1.0253 * n * n / N if kind == 0 else 4 * 0.00178 * (delta / 0.25) ** 2 / (
        math.pi * sigma ** 4)
    return synth.Model(n, delta, kind, amp, sigma, c_F=c_F, tau=tau, boundary=1)


def _input(side, seed, prec):
    U = np.random.default_rng(seed).uniform(-1.2, 1.2, (side, side))
    return U.astype(NPD[prec]).astype(np.float64)


def _ring_mask(side, r):
    mask = np.ones((side, side), dtype=bool)
    mask[r:side - r, r:side - r] = False
    return mask


def _skip_unbuilt(algo, prec, R2):
    if algo == "rowrun" and R2 not in nlch.nlch_rowrun_supported(nlch.PRECISIONS[prec]):
        pytest.skip("no row-run kernel for R2 = %d at %s" % (R2, prec))


CASES = [  # n, R2, kernel, precision, algorithm
    (100, 16, 0, "f64", "rowrun"), (150, 64, 1, "f32", "rowrun"), (72, 9, 0, "f16", "rowrun"),
    (200, 256, 1, "f32", "rowrun"), (64, 1, 0, "f32", "rowrun"), (80, 1024, 0, "f32", "rowrun"),
    (90, 121, 1, "f32", "auto"), (96, 25, 1, "f64", "direct"), (130, 64, 0, "f32", "direct"),
    (70, 36, 1, "f16", "direct"), (129, 64, 0, "f16", "rowrun"),
    # LDS-resident (n = 64, 128; nlch_solve_batch only)
    (128, 64, 0, "f32", "resident"), (64, 16, 1, "f16", "resident"),
    (128, 25, 1, "f32", "auto"), (64, 9, 0, "f64", "resident"), (128, 1, 1, "f16", "resident")]


@pytest.mark.parametrize("n,R2,kind,prec,algo", [c for c in CASES if c[4] != "resident"])
def test_volume_one_step(orc, n, R2, kind, prec, algo):
    _skip_unbuilt(algo, prec, R2)
    print("volume one-step n=%d R2=%d kernel=%d %s %s" % (n, R2, kind, prec, algo), flush=True)
    m = _model(n, R2, kind)
    r = vol.ring_width(n, m.delta)
    side = synth.state_side(m)
    assert side == n + 2 * r
    md = nlch.make_model(m.n, m.delta, m.kernel, m.amp, m.sigma, m.c_F, tau=m.tau,
                         boundary=1)
    U = np.clip(_input(side, 100 + n, prec), -1, 1)
    x = torch.from_numpy(U.reshape(-1)).to(TDT[prec]).to(DEV)
    y = torch.full_like(x, 7.0)
    ooi = torch.zeros(2, dtype=torch.float64, device=DEV)
    nlch.nlch_step(md, nlch.PRECISIONS[prec], A[algo], x, y, ooi)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy().reshape(side, side)
    ref = vol.step(U, n, m.delta, m.kernel, m.amp, m.sigma, m.c_F, m.beta1, m.tau)
    ring = _ring_mask(side, r)
    assert np.array_equal(got[ring], U[ring])
    err = np.max(np.abs(got[~ring] - ref[~ring]))
    assert err <= ONE_STEP_TOL[prec], err
    mean = got[r:r + n, r:r + n].mean()
    o = ooi.cpu().numpy()
    assert abs(o[0] - mean) <= 1e-12 and abs(o[1] - 0.5 * (1 + mean)) <= 1e-12


def _workload(n, R2, kind, prec, S=3, nsteps=8):
    m = _model(n, R2, kind)
    smp = [synth.Sample(0, 1.0 + 0.02 * (k - 1), m.amp * (1 + 0.01 * k), "iid", 11, k)
           for k in range(S)]
    w = synth.Workload("vol", [m], smp, nsteps, prec)
    return w, m


@pytest.mark.parametrize("n,R2,kind,prec,algo", CASES)
def test_volume_trajectory(orc, n, R2, kind, prec, algo):
    """nlch_solve_batch over 8 steps (the initial projection covers the ring)
    against the oracle's solve; both buffers keep the projected ring."""
    _skip_unbuilt(algo, prec, R2)
    print("volume trajectory n=%d R2=%d kernel=%d %s %s" % (n, R2, kind, prec, algo),
          flush=True)
    w, m = _workload(n, R2, kind, prec)
    b = DeviceBatch(w, prec)
    # inputs outside [-1, 1] exercise the projection of the ring
    side = synth.state_side(m)
    r = (side - n) // 2
    b.state.mul_(15.0)
    b.init.copy_(b.state)
    b.solve(A[algo])
    torch.cuda.synchronize()
    o = b.ooi_host()
    ring = _ring_mask(side, r)
    rel, utol = TRAJ_TOL[prec]
    for i, s in enumerate(w.samples):
        off = b.samples[i].offset
        U0 = b.init[off:off + side * side].double().cpu().numpy().reshape(side, side)
        ref, mean, f1 = vol.solve(U0, w.nsteps, n, m.delta, m.kernel, s.amp, m.sigma, s.c_F,
                                  m.beta1, m.tau)
        got = b.sample_state(i)
        assert np.array_equal(got[ring], np.clip(U0, -1, 1)[ring])
        if algo in ("direct", "rowrun"):  # the streaming ping-pong partner
            scr = b.scratch[off:off + side * side].double().cpu().numpy().reshape(side, side)
            assert np.array_equal(scr[ring], np.clip(U0, -1, 1)[ring])
        assert abs(o[i, 1] - f1) <= rel * abs(f1), (i, o[i, 1], f1)
        if utol is not None:
            assert np.max(np.abs(got - ref)) <= utol
        own = got[r:r + n, r:r + n].mean()
        assert abs(o[i, 0] - own) <= 1e-12


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("R2", [1, 4, 9, 16, 25, 64])
def test_volume_resident_layouts(orc, R2, kind):
    """128^2 Omega inside its ring, FP32, LDS-resident: the default layout
    (four columns per lane in split bands; the ring columns stay in the LDS
    halo, the ring rows' fixed sums reach Omega's first and last m rows in
    place of a neighbour's hand-over) against the oracle at every node after
    one step, and against the two-column layout along 8 steps; the ring is
    the projected input in both."""
    print("volume resident layouts R2=%d kernel=%d" % (R2, kind), flush=True)
    n = 128
    out = {}
    for shape in ((0, 0), (2, 16)):
        nlch.nlch_set_resident_shape(*shape)
        try:
            for nsteps in (1, 8):
                w, m = _workload(n, R2, kind, "f32", S=2, nsteps=nsteps)
                b = DeviceBatch(w, "f32")
                b.state.mul_(3.0)
                b.init.copy_(b.state)
                b.solve(nlch.NLCH_ALGO_RESIDENT)
                torch.cuda.synchronize()
                out[shape, nsteps] = (b, w, m)
        finally:
            nlch.nlch_set_resident_shape(0, 0)
    b1, w, m = out[(0, 0), 1]
    side = synth.state_side(m)
    r = (side - n) // 2
    ring = _ring_mask(side, r)
    for i, s in enumerate(w.samples):
        off = b1.samples[i].offset
        U0 = b1.init[off:off + side * side].double().cpu().numpy().reshape(side, side)
        got = b1.sample_state(i)
        ref = vol.step(np.clip(U0, -1, 1), n, m.delta, m.kernel, s.amp, m.sigma, s.c_F,
                       m.beta1, m.tau)
        assert np.array_equal(got[ring], np.clip(U0, -1, 1)[ring])
        assert np.max(np.abs(got[~ring] - ref[~ring])) <= ONE_STEP_TOL["f32"], i
    b8, _, _ = out[(0, 0), 8]
    c8, _, _ = out[(2, 16), 8]
    for i in range(len(w.samples)):
        assert np.max(np.abs(b8.sample_state(i) - c8.sample_state(i))) <= 1e-4, i
        assert np.array_equal(b8.sample_state(i)[ring], c8.sample_state(i)[ring]), i
    np.testing.assert_allclose(b8.ooi_host(), c8.ooi_host(), rtol=1e-6)


@pytest.mark.parametrize("shape", [(2, 1, 0, 0, 0), (1, 2, 1, 0, 0), (2, 4, 2, 0, 0),
                                   (1, 8, 1, 0, 0), (1, 1, 0, 40, 0), (1, 1, 0, 0, 2),
                                   (2, 1, 0, 37, 2)])
def test_volume_stream_shapes(orc, shape):
    """Forced launch shapes of the streaming kernels (columns per lane, waves
    per band, periods, band rows, row phases per wave) on the bounded domain,
    FP32, m = 8 and a ragged 150-node lattice: one step against the oracle at
    every node."""
    R, W, k, B, ph = shape
    print("volume shape R=%d W=%d k=%d B=%d phases=%d" % shape, flush=True)
    w, m = _workload(150, 64, 1, "f32", S=2, nsteps=1)
    nlch.nlch_set_stream_shape(R, W, k, B)
    nlch.nlch_set_stream_phases(ph)
    try:
        b = DeviceBatch(w, "f32")
        b.solve(nlch.NLCH_ALGO_ROWRUN)
        torch.cuda.synchronize()
    finally:
        nlch.nlch_set_stream_shape(0, 0, 0, 0)
        nlch.nlch_set_stream_phases(0)
    side = synth.state_side(m)
    for i, s in enumerate(w.samples):
        off = b.samples[i].offset
        U0 = np.clip(b.init[off:off + side * side].double().cpu().numpy(), -1, 1)
        ref = vol.step(U0.reshape(side, side), 150, m.delta, m.kernel, s.amp, m.sigma, s.c_F,
                       m.beta1, m.tau)
        assert np.max(np.abs(b.sample_state(i) - ref)) <= ONE_STEP_TOL["f32"]


def test_volume_next_to_periodic_in_one_batch(orc):
    """A bounded-domain group and a periodic group in one call: each sample
    equals its own single-group solve bit for bit."""
    mv = _model(96, 16, 1)
    mp = synth.Model(96, mv.delta, 1, mv.amp, mv.sigma, tau=mv.tau)
    smp = [synth.Sample(k % 2, 1.0, mv.amp, "iid", 12, k) for k in range(4)]
    w = synth.Workload("mixed", [mv, mp], smp, 6, "f32")
    both = DeviceBatch(w)
    both.solve(nlch.NLCH_ALGO_AUTO)
    torch.cuda.synchronize()
    for k in range(4):
        single = synth.Workload("one", [w.models[k % 2]],
                                [synth.Sample(0, 1.0, mv.amp, "iid", 12, k)], 6, "f32")
        one = DeviceBatch(single)
        one.solve(nlch.NLCH_ALGO_AUTO)
        torch.cuda.synchronize()
        assert np.array_equal(both.sample_state(k), one.sample_state(0)), k
        assert np.array_equal(both.ooi_host()[k], one.ooi_host()[0]), k


def test_volume_full_size_sampled(orc):
    """The benchmark's bounded-domain workload at full size (4096 samples of
    128^2 with the 8-row ring, FP32) in the benchmark's launch configuration
    (AUTO with the autotuner): one step, sampled nodes of sampled samples
    against the oracle, the rings untouched, OoI against each state's mean."""
    w = synth.workload("V3", nsteps=1)
    m = w.models[0]
    b = DeviceBatch(w)
    b.solve(nlch.NLCH_ALGO_AUTO | nlch.NLCH_ALGO_AUTOTUNE)
    torch.cuda.synchronize()
    side = synth.state_side(m)
    r = (side - m.n) // 2
    ring = _ring_mask(side, r)
    o = b.ooi_host()
    rng = np.random.default_rng(5)
    for i in [0, 1, 2047, 4095] + list(rng.choice(4096, 4, replace=False)):
        s = w.samples[i]
        U0 = np.clip(synth.initial_state(w, s).astype(np.float32).astype(np.float64), -1, 1)
        got = b.sample_state(i)
        assert np.array_equal(got[ring], U0[ring]), i
        sites = rng.choice(m.n * m.n, 600, replace=False)
        ref = vol.step_sites(U0, sites, m.n, m.delta, m.kernel, s.amp, m.sigma, s.c_F,
                             m.beta1, m.tau)
        inner = got[r:r + m.n, r:r + m.n].reshape(-1)
        assert np.max(np.abs(inner[sites] - ref)) <= ONE_STEP_TOL["f32"], i
        assert abs(o[i, 0] - inner.mean()) <= 1e-12, i
