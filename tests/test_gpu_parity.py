"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (from the arithmetic): FP64 paths agree with the oracle to 1e-13
per step (only summation order differs); FP32 one-step results differ by FP32
rounding of the state plus accumulation rounding scaled by the small update
coefficient (bound 1e-6 absolute); FP16 storage adds half an FP16 ulp per
stored value (bound 1e-3).  Whole trajectories: OoI relative error <= 1e-6
(FP32), <= 1e-12 (FP64).
"""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch, synth
from tests.gpu_harness import DeviceBatch, oracle_samples

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ONE_STEP_TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 1e-3}
TDT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}
NPD = {"f64": np.float64, "f32": np.float32, "f16": np.float16}


def _model(n, R2, kind, tau=0.05, c_F=1.0):
    delta = math.sqrt(R2) / n
    _, m, N, _ = nlch.nlch_disc(n, delta)
    if kind == 0:
        amp, sigma = 1.0253 * n * n / N, 0.0
    else:
        sigma = delta / 3
        amp = 1.0253 / (math.pi * sigma * sigma)
    return nlch.make_model(n, delta, kind, amp, sigma, c_F=c_F, tau=tau)


def _rand_state(n, seed, prec):
    rng = np.random.default_rng(seed)
    u = np.clip(rng.uniform(-1.5, 1.5, (n, n)), -1, 1)
    return u.astype(NPD[prec]).astype(np.float64)


def _step_gpu(md, prec, algo, u):
    x = torch.from_numpy(u.reshape(-1)).to(TDT[prec]).to(DEV)
    y = torch.empty_like(x)
    ooi = torch.zeros(2, dtype=torch.float64, device=DEV)
    nlch.nlch_step(md, nlch.PRECISIONS[prec], algo, x, y, ooi)
    torch.cuda.synchronize()
    return y.double().cpu().numpy().reshape(md.n, md.n), ooi.cpu().numpy()


def _step_oracle(orc, md, u):
    return orc.step(u, md.n, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma,
                    md.c_F, md.beta1, md.tau)


CASES = [(40, 9, 0), (40, 9, 1), (96, 64, 0), (96, 64, 1), (88, 272, 0),
         (130, 1024, 1), (70, 16, 0), (50, 25, 1), (33, 1, 0), (64, 4, 1),
         # horizons of the MFMC study's models (row-run built for FP32 arithmetic)
         (88, 121, 1), (64, 144, 1), (90, 484, 0), (128, 576, 1)]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("algo", [nlch.NLCH_ALGO_DIRECT, nlch.NLCH_ALGO_ROWRUN])
@pytest.mark.parametrize("n,R2,kind", CASES)
def test_one_step_parity(orc, n, R2, kind, algo, prec):
    print("one-step n=%d R2=%d kernel=%d algo=%d %s" % (n, R2, kind, algo, prec), flush=True)
    if algo == nlch.NLCH_ALGO_ROWRUN and R2 not in nlch.nlch_rowrun_supported(
            nlch.PRECISIONS[prec]):
        pytest.skip("no row-run kernel for R2 = %d at %s (direct kernel covers it)" % (R2, prec))
    md = _model(n, R2, kind)
    u = _rand_state(n, 100 + n + R2, prec)
    got, ooi = _step_gpu(md, prec, algo, u)
    ref = _step_oracle(orc, md, u)
    err = np.max(np.abs(got - ref))
    assert err <= ONE_STEP_TOL[prec], err
    assert np.all(np.abs(got) <= 1)
    mean = got.mean()
    assert abs(ooi[0] - mean) <= 1e-12 and abs(ooi[1] - 0.5 * (1 + mean)) <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_direct_any_horizon(orc, prec):
    """Horizons without a compiled row-run kernel run on the direct kernel."""
    for n, R2, kind in [(48, 7, 0), (48, 13, 1), (100, 150, 0)]:
        md = _model(n, R2, kind)
        u = _rand_state(n, 7 + R2, prec)
        got, _ = _step_gpu(md, prec, nlch.NLCH_ALGO_AUTO, u)
        assert np.max(np.abs(got - _step_oracle(orc, md, u))) <= ONE_STEP_TOL[prec]


@pytest.mark.parametrize("algo", [nlch.NLCH_ALGO_DIRECT, nlch.NLCH_ALGO_ROWRUN])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_step_invariants_bit_exact(algo, prec):
    """Constant states +-1 and 0 are stationary; step(-u) = -step(u); lattice
    translations commute with the step -- all bit-exactly."""
    md = _model(96, 64, 1)
    n = md.n
    for c in (1.0, -1.0, 0.0):
        got, _ = _step_gpu(md, prec, algo, np.full((n, n), c))
        assert np.all(got == c)
    u = _rand_state(n, 3, prec)
    s, _ = _step_gpu(md, prec, algo, u)
    sm, _ = _step_gpu(md, prec, algo, -u)
    assert np.array_equal(sm, -s)
    for sh in [(1, 0), (0, 37), (50, 71)]:
        st, _ = _step_gpu(md, prec, algo, np.roll(u, sh, (0, 1)))
        assert np.array_equal(st, np.roll(s, sh, (0, 1))), sh


TRAJ_TOL = {"f64": (1e-12, 1e-10), "f32": (1e-6, 1e-4)}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("algo", [nlch.NLCH_ALGO_AUTO, nlch.NLCH_ALGO_DIRECT,
                                  nlch.NLCH_ALGO_ROWRUN])
def test_c1_trajectory(orc, algo, prec):
    """64x64, delta = 4h, 200 steps of tau = 0.05 (obstacle active on ~90% of
    the sites at the end)."""
    print("C1 trajectory algo=%d %s" % (algo, prec), flush=True)
    w = synth.workload("C1")
    b = DeviceBatch(w, prec)
    b.solve(algo)
    torch.cuda.synchronize()
    ref = oracle_samples(orc, w, [0], prec)[0]
    got = b.sample_state(0)
    f1 = b.ooi_host()[0, 1]
    rel_tol, u_tol = TRAJ_TOL[prec]
    assert abs(f1 - ref[2]) <= rel_tol * abs(ref[2]), (f1, ref[2])
    assert np.max(np.abs(got - ref[0])) <= u_tol
    assert np.mean(np.abs(got) == 1) > 0.8


def test_c1_fp16_storage(orc):
    w = synth.workload("C1")
    b = DeviceBatch(w, "f16")
    b.solve()
    torch.cuda.synchronize()
    ref = oracle_samples(orc, w, [0], "f16")[0]
    f1 = b.ooi_host()[0, 1]
    assert abs(f1 - ref[2]) <= 1e-3 * abs(ref[2])


def test_resume_is_bit_exact():
    w = synth.workload("C1", nsteps=60)
    for algo in (nlch.NLCH_ALGO_AUTO, nlch.NLCH_ALGO_ROWRUN, nlch.NLCH_ALGO_DIRECT):
        a = DeviceBatch(w, "f32")
        a.solve(algo, nsteps=60)
        b = DeviceBatch(w, "f32")
        b.solve(algo, nsteps=25)
        b.solve(algo, nsteps=35)
        torch.cuda.synchronize()
        assert torch.equal(a.state, b.state)
        assert torch.equal(a.ooi, b.ooi)


def test_graph_replay_matches_direct_enqueue():
    w = synth.workload("C1", nsteps=31, n=64)
    ref = DeviceBatch(w, "f32")
    ref.solve(nlch.NLCH_ALGO_ROWRUN | nlch.NLCH_ALGO_NOGRAPH)
    b = DeviceBatch(w, "f32")
    s = torch.cuda.Stream()
    for _ in range(3):
        b.reset()
        b.solve(nlch.NLCH_ALGO_ROWRUN, stream=s)
        s.synchronize()
        # eager work between replays
        _ = (b.scratch * 2).sum().item()
        assert torch.equal(b.state, ref.state)
        assert torch.equal(b.ooi, ref.ooi)


RESIDENT_R2 = [1, 4, 9, 16, 25, 64]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("R2", RESIDENT_R2)
def test_resident_one_step_every_disc(orc, R2, n, kind, prec):
    """Every compiled LDS-resident kernel (disc, lattice, kernel, storage)
    against the oracle at every site after one and after three steps, from a
    random admissible state (three samples with their own c_F)."""
    md = _model(n, R2, kind)
    algo = nlch.NLCH_ALGO_RESIDENT
    u = [_rand_state(n, 40 + k, prec) for k in range(3)]
    host = np.concatenate([v.reshape(-1) for v in u])
    smp = [nlch.nlch_sample(0, 0, 1.0 + 0.02 * k, md.kernel_amp, k * n * n) for k in range(3)]
    for nsteps in (1, 3):
        x = torch.from_numpy(host).to(TDT[prec]).to(DEV)
        ooi = torch.zeros(6, dtype=torch.float64, device=DEV)
        try:
            nlch.nlch_solve_batch([md], smp, nsteps, nlch.PRECISIONS[prec], algo, x, None, ooi)
        except nlch.NlchError as e:
            assert e.code == nlch.NLCH_EUNSUPPORTED
            pytest.skip("no resident kernel for n=%d R2=%d at %s" % (n, R2, prec))
        torch.cuda.synchronize()
        got = x.double().cpu().numpy().reshape(3, n, n)
        for k in range(3):
            ref = u[k]
            for _ in range(nsteps):
                ref = orc.step(ref, n, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma,
                               smp[k].c_F, md.beta1, md.tau)
            tol = ONE_STEP_TOL[prec] * (1 if nsteps == 1 else 10)
            assert np.max(np.abs(got[k] - ref)) <= tol, (k, nsteps)
            assert abs(ooi.cpu().numpy()[2 * k] - got[k].mean()) <= 1e-12


def test_graph_cache_eviction_keeps_results():
    """More distinct call signatures (step counts) than a batch caches graphs
    for: every call still equals the direct enqueue, also after the cache was
    dropped, and a repeated signature replays correctly."""
    w = synth.workload("C1", n_samples=2, nsteps=1, n=64)
    b = DeviceBatch(w, "f32")
    ref = DeviceBatch(w, "f32")
    for k in list(range(1, 21)) + [3, 20]:
        b.reset()
        b.solve(nlch.NLCH_ALGO_ROWRUN, nsteps=k)
        ref.reset()
        ref.solve(nlch.NLCH_ALGO_ROWRUN | nlch.NLCH_ALGO_NOGRAPH, nsteps=k)
        torch.cuda.synchronize()
        assert torch.equal(b.state, ref.state), k
        assert torch.equal(b.ooi, ref.ooi), k


def test_mixed_batch_uneven_sizes(orc):
    """Gaussian kernel, fixed physical horizon, three lattices in one call
    (row-run for 256^2, LDS-resident for 128^2 and 64^2)."""
    delta = 1.0 / 32
    amp, sigma, _ = synth.gaussian_params(delta)
    models = [synth.Model(256, delta, 1, amp, sigma, tau=0.01),
              synth.Model(128, delta, 1, amp, sigma, tau=0.01),
              synth.Model(64, delta, 1, amp, sigma, tau=0.01)]
    samples = []
    for lvl, cnt in enumerate((2, 3, 5)):
        for s in range(cnt):
            samples.append(synth.Sample(lvl, 1.0, amp, "nuclei", 4, s,
                                        synth.draw_theta(synth.rng_for(4, s))))
    w = synth.Workload("mixed", models, samples, 41, "f32")
    b = DeviceBatch(w)
    b.solve()
    torch.cuda.synchronize()
    ref = oracle_samples(orc, w, range(len(samples)), "f32")
    o = b.ooi_host()
    for i in range(len(samples)):
        assert abs(o[i, 1] - ref[i][2]) <= 1e-6 * abs(ref[i][2]), i
        assert np.max(np.abs(b.sample_state(i) - ref[i][0])) <= 1e-4
    # every sample equals its own single-sample solve
    for i in (0, 2, 9):
        wi = synth.Workload("one", models, [samples[i]], 41, "f32")
        bi = DeviceBatch(wi)
        bi.solve()
        torch.cuda.synchronize()
        assert np.array_equal(bi.sample_state(0), b.sample_state(i))


def test_check_finite_rejects_nan_without_writes():
    w = synth.workload("C1", nsteps=5)
    b = DeviceBatch(w, "f32")
    b.state[123] = float("nan")
    before = b.state.clone()
    with pytest.raises(nlch.NlchError) as e:
        b.solve(nlch.NLCH_ALGO_CHECK_FINITE)
    assert e.value.code == nlch.NLCH_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(torch.isnan(b.state), torch.isnan(before))
    assert torch.equal(torch.nan_to_num(b.state), torch.nan_to_num(before))
    # without the check NaN propagates to the output of interest
    b.solve()
    torch.cuda.synchronize()
    assert math.isnan(b.ooi_host()[0, 1])


def test_mfmc_estimate_matches_oracle():
    from oracle import mfmc
    rng = np.random.default_rng(8)
    m = [8, 64, 512, 4096]
    z = rng.normal(0.5, 0.01, 4096)
    ys = [z + 1e-4 * rng.normal(size=4096) * k for k in (1, 2, 3, 5)]
    dev = [torch.from_numpy(y).to(DEV) for y in ys]
    for alpha in (None, [0.9, 1.1, 0.7]):
        got = nlch.mfmc_estimate(dev, m, alpha)
        ref = mfmc.mfmc_estimate(ys, m, alpha)
        assert abs(got["q_mfmc"] - ref["q_mfmc"]) <= 1e-14
        assert abs(got["q_mc"] - ref["q_mc"]) <= 1e-14
        for k in ("mean_mj", "var", "rho", "alpha"):
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-11, atol=1e-15)
        np.testing.assert_allclose(got["mean_mjm1"][1:], ref["mean_mjm1"][1:], rtol=1e-13)


def _shape_workload(prec="f32", nsteps=9, big=True):
    delta = 1.0 / 32
    amp, sigma, _ = synth.gaussian_params(delta)
    models = [synth.Model(256, delta, 1, amp, sigma, tau=0.01),
              synth.Model(300, 16 / 300, 0, 1.0253 * 300 * 300 / 797, 0.0, tau=0.01),
              synth.Model(130, 32 / 130, 1, 4e-3 / (math.pi * (32 / 390) ** 4),
                          32 / 390, tau=0.01),
              # m = 32 on a lattice of several ragged shared bands
              synth.Model(400, 32 / 400, 0, 1.0253 * 400 * 400 / 3209, 0.0, tau=0.01),
              synth.Model(1024, 1 / 32, 1, amp, sigma, tau=0.01)]
    samples = [synth.Sample(0, 1.0, amp, "nuclei", 4, s, synth.draw_theta(synth.rng_for(4, s)))
               for s in range(3)]
    samples += [synth.Sample(1, 1.0, models[1].amp, "iid", 7, s) for s in range(2)]
    samples += [synth.Sample(2, 1.0, models[2].amp, "iid", 8, s) for s in range(2)]
    samples += [synth.Sample(3, 1.0, models[3].amp, "iid", 9, 0)]
    if big:
        samples += [synth.Sample(4, 1.0, amp, "nuclei", 4, 9,
                                 synth.draw_theta(synth.rng_for(4, 9)))]
    else:
        models = models[:4]
    return synth.Workload("shapes", models, samples, nsteps, prec)


@pytest.fixture
def reset_shape():
    yield
    nlch.nlch_set_stream_shape(0, 0, 0, 0)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_single_wave_shapes_give_identical_results(reset_shape, prec):
    """With one wave per band the launch shape (columns per lane, band
    height) does not change any result: every site sums the same window sums
    in the same row order, with FP32 or FP16 storage."""
    w = _shape_workload(prec)
    ref = DeviceBatch(w)
    ref.solve(nlch.NLCH_ALGO_ROWRUN)
    torch.cuda.synchronize()
    for R, B in ((1, 16), (2, 40), (1, 97), (2, 0), (1, 1024)):
        print("shape %s R=%d W=1 B=%d" % (prec, R, B), flush=True)
        nlch.nlch_set_stream_shape(R, 1, 0, B)
        b = DeviceBatch(w)
        b.solve(nlch.NLCH_ALGO_ROWRUN)
        torch.cuda.synchronize()
        assert torch.equal(ref.state, b.state), (R, B)
        assert torch.equal(ref.ooi, b.ooi), (R, B)


SHAPES_MW = [(1, 2, 1), (2, 2, 2), (1, 4, 1), (2, 4, 1), (1, 8, 1), (1, 4, 4), (2, 8, 2)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("R,W,k", SHAPES_MW)
def test_multiwave_bands_one_step(orc, reset_shape, R, W, k, prec):
    """Bands shared by W waves (partial sums handed over in LDS): one step
    from random states against the oracle on every site, lattices with ragged
    strips and bands (300^2), a band taller than the lattice, and groups the
    shared-band kernel is not built for (FP64), which use one wave per band;
    m = 32 on 130^2 (one band) and 400^2 (ragged bands); with the energy
    trace on."""
    w = _shape_workload(prec, nsteps=1, big=False)
    print("multiwave R=%d W=%d periods=%d %s" % (R, W, k, prec), flush=True)
    nlch.nlch_set_stream_shape(R, W, k, 0)
    b = DeviceBatch(w, prec)
    rng = np.random.default_rng(5)
    host = np.clip(rng.uniform(-1.5, 1.5, b.total), -1, 1).astype(NPD[prec])
    b.state.copy_(torch.from_numpy(host).to(DEV))
    b.init.copy_(b.state)
    e = b.solve_energy(nlch.NLCH_ALGO_ROWRUN, nsteps=1)
    torch.cuda.synchronize()
    E = e.cpu().numpy()
    for i, smp in enumerate(w.samples):
        m = w.models[smp.model]
        off = b.samples[i].offset
        u0 = host[off:off + m.n * m.n].astype(np.float64).reshape(m.n, m.n)
        ref = orc.step(u0, m.n, m.delta, m.kernel, smp.amp, m.sigma, smp.c_F, m.beta1, m.tau)
        got = b.sample_state(i)
        assert np.max(np.abs(got - ref)) <= ONE_STEP_TOL[prec], (i, m.n)
        e0 = orc.energy(u0, m.n, m.delta, m.kernel, smp.amp, m.sigma, smp.c_F)
        e1 = orc.energy(got, m.n, m.delta, m.kernel, smp.amp, m.sigma, smp.c_F)
        etol = 1e-11 if prec == "f64" else 1e-5
        assert abs(E[0, i] - e0) <= etol * abs(e0), (i, E[0, i], e0)
        assert abs(E[1, i] - e1) <= etol * abs(e1), (i, E[1, i], e1)


def test_multiwave_trajectory_and_repeatability(orc, reset_shape):
    """Nine steps with W = 4 waves per band: the OoI stays within the FP32
    trajectory bar of the oracle, and the same shape repeats bit-exactly."""
    w = _shape_workload("f32", nsteps=9)
    nlch.nlch_set_stream_shape(1, 4, 1, 0)
    a = DeviceBatch(w)
    a.solve(nlch.NLCH_ALGO_ROWRUN)
    b = DeviceBatch(w)
    b.solve(nlch.NLCH_ALGO_ROWRUN)
    torch.cuda.synchronize()
    assert torch.equal(a.state, b.state)
    ref = oracle_samples(orc, w, [0, 3, 5], "f32")
    o = a.ooi_host()
    for i in (0, 3, 5):
        assert abs(o[i, 1] - ref[i][2]) <= 1e-6 * abs(ref[i][2]), i
        assert np.max(np.abs(a.sample_state(i) - ref[i][0])) <= 1e-4


SHAPES_PH = [(1, 0), (2, 0), (1, 16), (2, 33), (1, 97), (2, 1024)]


@pytest.fixture
def reset_phases():
    yield
    nlch.nlch_set_stream_phases(0)
    nlch.nlch_set_stream_shape(0, 0, 0, 0)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("R,B", SHAPES_PH)
def test_two_phase_bands_one_step(orc, reset_phases, R, B, prec):
    """Two row phases per wave (the half-waves walk alternate input rows and
    add each other's partial sums with a lane swap): one step from random
    states against the oracle on every site, with odd and even band heights
    (an odd count of input rows leaves the last one to one half), the
    default height, bands taller than the lattice, ragged strips of 32R
    columns and ragged bands (300^2, 130^2, 400^2), m = 8 to 32, both
    kernels, and the energy trace on; FP64 groups keep one phase."""
    w = _shape_workload(prec, nsteps=1, big=False)
    print("two-phase R=%d B=%d %s" % (R, B, prec), flush=True)
    nlch.nlch_set_stream_shape(R, 1, 0, B)
    nlch.nlch_set_stream_phases(2)
    b = DeviceBatch(w, prec)
    rng = np.random.default_rng(6)
    host = np.clip(rng.uniform(-1.5, 1.5, b.total), -1, 1).astype(NPD[prec])
    b.state.copy_(torch.from_numpy(host).to(DEV))
    b.init.copy_(b.state)
    e = b.solve_energy(nlch.NLCH_ALGO_ROWRUN, nsteps=1)
    torch.cuda.synchronize()
    E = e.cpu().numpy()
    for i, smp in enumerate(w.samples):
        m = w.models[smp.model]
        off = b.samples[i].offset
        u0 = host[off:off + m.n * m.n].astype(np.float64).reshape(m.n, m.n)
        ref = orc.step(u0, m.n, m.delta, m.kernel, smp.amp, m.sigma, smp.c_F, m.beta1, m.tau)
        got = b.sample_state(i)
        assert np.max(np.abs(got - ref)) <= ONE_STEP_TOL[prec], (i, m.n)
        e0 = orc.energy(u0, m.n, m.delta, m.kernel, smp.amp, m.sigma, smp.c_F)
        e1 = orc.energy(got, m.n, m.delta, m.kernel, smp.amp, m.sigma, smp.c_F)
        etol = 1e-11 if prec == "f64" else 1e-5
        assert abs(E[0, i] - e0) <= etol * abs(e0), (i, E[0, i], e0)
        assert abs(E[1, i] - e1) <= etol * abs(e1), (i, E[1, i], e1)


def test_two_phase_trajectory_and_repeatability(orc, reset_phases):
    """Nine steps with two row phases per wave: the OoI stays within the FP32
    trajectory bar of the oracle, the same shape repeats bit-exactly, and
    the states stay within rounding of the one-phase shape."""
    w = _shape_workload("f32", nsteps=9)
    one = DeviceBatch(w)
    one.solve(nlch.NLCH_ALGO_ROWRUN)
    nlch.nlch_set_stream_shape(1, 1, 0, 64)
    nlch.nlch_set_stream_phases(2)
    a = DeviceBatch(w)
    a.solve(nlch.NLCH_ALGO_ROWRUN)
    b = DeviceBatch(w)
    b.solve(nlch.NLCH_ALGO_ROWRUN)
    torch.cuda.synchronize()
    assert torch.equal(a.state, b.state)
    assert not torch.equal(a.state, one.state)  # the two-phase kernel ran
    assert torch.max(torch.abs(a.state - one.state)).item() <= 1e-5
    ref = oracle_samples(orc, w, [0, 3, 5], "f32")
    o = a.ooi_host()
    for i in (0, 3, 5):
        assert abs(o[i, 1] - ref[i][2]) <= 1e-6 * abs(ref[i][2]), i
        assert np.max(np.abs(a.sample_state(i) - ref[i][0])) <= 1e-4


def test_autotune_is_repeatable(reset_shape):
    """The autotuner keeps one shape per batch signature: later calls repeat
    exactly; results stay within rounding of the default shape."""
    w = _shape_workload()
    ref = DeviceBatch(w)
    ref.solve(nlch.NLCH_ALGO_ROWRUN)
    b = DeviceBatch(w)
    b.solve(nlch.NLCH_ALGO_ROWRUN | nlch.NLCH_ALGO_AUTOTUNE)
    first = b.state.clone()
    b.reset()
    b.solve(nlch.NLCH_ALGO_ROWRUN | nlch.NLCH_ALGO_AUTOTUNE)
    torch.cuda.synchronize()
    assert torch.equal(first, b.state)
    assert torch.max(torch.abs(b.state - ref.state)).item() <= 1e-5
    np.testing.assert_allclose(b.ooi_host(), ref.ooi_host(), rtol=1e-6)
