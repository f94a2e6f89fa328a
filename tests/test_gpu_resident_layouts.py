"""Layouts of the LDS-resident kernel (FP32, 128^2), set with
nlch_set_resident_shape(columns, rows per lane):

* (2, 16): two columns per lane, one 16-row band per wave;
* (4, 16): four columns per lane, two bands per wave, 16-byte window loads.
  Every site sums the same window sums in the same order as in (2, 16), so
  the states are bit-identical;
* (4, 8): one band per wave, each half-wave walking 8 rows.  Each band sum
  is formed in two parts, so it differs from (2, 16) by FP32 rounding.  It
  is checked against the FP64 oracle at every site, and against (2, 16)
  along a trajectory.

64^2 lattices (FP32) run one column per lane with bands of 8 (m <= 8), 16 or
32 rows, set with (1, 8), (1, 16), (1, 32): the partial sums handed between
bands group the disc rows differently, so they differ by FP32 rounding; each
is checked against the FP64 oracle at every site and against (1, 16) along
a trajectory.  NLCH_ALGO_AUTOTUNE picks one of the layouts per batch
signature; its results stay within rounding of the default and repeat
exactly once the pick is cached.

The outputs of interest are FP64 sums of the states in a layout-dependent
order, so for bit-identical states they agree to FP64 rounding."""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch, synth
from tests.gpu_harness import DeviceBatch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SHAPES = [(2, 16), (4, 16), (4, 8)]


@pytest.fixture(autouse=True)
def _default_layout():
    yield
    nlch.nlch_set_resident_shape(0, 0)


def _model(n, R2, kind, tau=0.05):
    delta = math.sqrt(R2) / n
    _, m, N, _ = nlch.nlch_disc(n, delta)
    if kind == 0:
        amp, sigma = 1.0253 * n * n / N, 0.0
    else:
        sigma = delta / 3
        amp = 1.0253 / (math.pi * sigma * sigma)
    return nlch.make_model(n, delta, kind, amp, sigma, tau=tau)


def _solve(md, smp, host, nsteps, shape):
    nlch.nlch_set_resident_shape(*shape)
    x = torch.from_numpy(host).to(DEV)
    ooi = torch.zeros(2 * len(smp), dtype=torch.float64, device=DEV)
    nlch.nlch_solve_batch([md], smp, nsteps, nlch.NLCH_F32, nlch.NLCH_ALGO_RESIDENT, x, None,
                          ooi)
    torch.cuda.synchronize()
    return x.cpu().numpy(), ooi.cpu().numpy()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("R2", [1, 4, 9, 16, 25, 64])
def test_layouts_of_the_resident_kernel(orc, R2, kind):
    print("layouts R2=%d kernel=%d" % (R2, kind), flush=True)
    n, S = 128, 5
    md = _model(n, R2, kind)
    rng = np.random.default_rng(R2 * 10 + kind)
    host = rng.uniform(-1.2, 1.2, S * n * n).astype(np.float32)
    smp = [nlch.nlch_sample(0, 0, 0.96 + 0.02 * k, md.kernel_amp, k * n * n) for k in range(S)]
    for nsteps in (0, 1, 7, 40):
        out = {sh: _solve(md, smp, host, nsteps, sh) for sh in SHAPES}
        s2, o2 = out[(2, 16)]
        s4, o4 = out[(4, 16)]
        sh8, oh8 = out[(4, 8)]
        assert np.array_equal(s2, s4), nsteps
        np.testing.assert_allclose(o4, o2, rtol=0, atol=1e-15)
        # the split-band layout: FP32 rounding of the band sums, growing along
        # the trajectory; each state's mean is its output of interest
        assert np.max(np.abs(sh8.astype(np.float64) - s2)) <= (1e-6 if nsteps <= 1 else 1e-4)
        for k in range(S):
            assert abs(oh8[2 * k] - np.mean(sh8[k * n * n:(k + 1) * n * n].astype(np.float64))) \
                <= 1e-12
        if nsteps == 1:
            # every site against the FP64 oracle
            for k in range(S):
                u0 = np.clip(host[k * n * n:(k + 1) * n * n].astype(np.float64), -1, 1)
                ref = orc.step(u0.reshape(n, n), n, md.delta, md.kernel, md.kernel_amp,
                               md.kernel_sigma, smp[k].c_F, md.beta1, md.tau)
                got = sh8[k * n * n:(k + 1) * n * n].astype(np.float64).reshape(n, n)
                assert np.max(np.abs(got - ref)) <= 1e-6


def test_benchmark_workload_layouts_agree(orc):
    """256 samples of the benchmark workload (128^2, 197-point disc, per-sample
    c_F, 500 steps): (2, 16) and (4, 16) give the same states; (4, 8) meets
    the OoI bar against the FP64 oracle."""
    print("C3 layouts", flush=True)
    w = synth.workload("C3", n_samples=256)
    out = {}
    for sh in SHAPES:
        nlch.nlch_set_resident_shape(*sh)
        b = DeviceBatch(w)
        b.solve(algo=nlch.NLCH_ALGO_AUTO)
        torch.cuda.synchronize()
        out[sh] = (b.state.cpu().numpy(), b.ooi_host())
    assert np.array_equal(out[(2, 16)][0], out[(4, 16)][0])
    np.testing.assert_allclose(out[(4, 16)][1], out[(2, 16)][1], rtol=0, atol=1e-15)
    from tests.gpu_harness import oracle_samples
    ref = oracle_samples(orc, w, [0, 1, 255], "f32")
    for i in (0, 1, 255):
        assert abs(out[(4, 8)][1][i, 1] - ref[i][2]) <= 1e-6 * abs(ref[i][2])


SHAPES64 = [(1, 8), (1, 16), (1, 32)]


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("R2", [1, 4, 9, 16, 25, 64])
def test_band_heights_of_the_64sq_resident_kernel(orc, R2, kind):
    print("64^2 band heights R2=%d kernel=%d" % (R2, kind), flush=True)
    n, S = 64, 6
    md = _model(n, R2, kind)
    rng = np.random.default_rng(R2 * 7 + kind)
    host = rng.uniform(-1.2, 1.2, S * n * n).astype(np.float32)
    smp = [nlch.nlch_sample(0, 0, 0.97 + 0.01 * k, md.kernel_amp, k * n * n) for k in range(S)]
    for nsteps in (1, 30):
        out = {sh: _solve(md, smp, host, nsteps, sh) for sh in SHAPES64}
        base, obase = out[(1, 16)]
        for sh in SHAPES64:
            st, oo = out[sh]
            assert np.max(np.abs(st.astype(np.float64) - base)) <= \
                (1e-6 if nsteps == 1 else 1e-4), sh
            for k in range(S):
                assert abs(oo[2 * k] - np.mean(st[k * n * n:(k + 1) * n * n].astype(np.float64))) \
                    <= 1e-12
            if nsteps == 1:
                for k in (0, S - 1):
                    u0 = np.clip(host[k * n * n:(k + 1) * n * n].astype(np.float64), -1, 1)
                    ref = orc.step(u0.reshape(n, n), n, md.delta, md.kernel, md.kernel_amp,
                                   md.kernel_sigma, smp[k].c_F, md.beta1, md.tau)
                    got = st[k * n * n:(k + 1) * n * n].astype(np.float64).reshape(n, n)
                    assert np.max(np.abs(got - ref)) <= 1e-6, sh


@pytest.mark.parametrize("kind", [0, 1])
def test_default_layout_invariants_bit_exact(kind):
    """The default 128^2 FP32 layout (four columns per lane, split bands;
    for the constant kernel the windows come from running sums shared by a
    lane's four columns): the step commutes with negation, keeps u = 1, -1
    and 0 fixed, and commutes with translations by whole bands (16 rows) and
    whole four-column groups, all bit for bit, over three steps."""
    n, S, nsteps = 128, 1, 3
    md = _model(n, 64, kind)
    smp = [nlch.nlch_sample(0, 0, 0.98, md.kernel_amp, 0)]
    rng = np.random.default_rng(40 + kind)
    u = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    base, _ = _solve(md, smp, u.reshape(-1), nsteps, (0, 0))
    base = base.reshape(n, n)
    neg, _ = _solve(md, smp, (-u).reshape(-1), nsteps, (0, 0))
    assert np.array_equal(neg.reshape(n, n), -base)
    for c in (1.0, -1.0, 0.0):
        st, _ = _solve(md, smp, np.full(n * n, c, dtype=np.float32), nsteps, (0, 0))
        assert np.array_equal(st, np.full(n * n, c, dtype=np.float32)), c
    for sh in ((16, 0), (0, 4), (32, 8), (48, 124)):
        st, _ = _solve(md, smp, np.roll(u, sh, (0, 1)).reshape(-1), nsteps, (0, 0))
        assert np.array_equal(st.reshape(n, n), np.roll(base, sh, (0, 1))), sh


def _solve64(md, smp, host, nsteps, shape):
    nlch.nlch_set_resident_shape(*shape)
    x = torch.from_numpy(host).to(DEV)
    ooi = torch.zeros(2 * len(smp), dtype=torch.float64, device=DEV)
    nlch.nlch_solve_batch([md], smp, nsteps, nlch.NLCH_F64, nlch.NLCH_ALGO_RESIDENT, x, None,
                          ooi)
    torch.cuda.synchronize()
    return x.cpu().numpy(), ooi.cpu().numpy()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("R2", [1, 4, 9, 16, 25, 64])
def test_fp64_band_heights_of_the_64sq_resident_kernel(orc, R2, kind):
    """FP64 64^2 in 8-row bands (8 waves for a sample, the single-sample
    latency case) against 16-row bands and the FP64 oracle at every site."""
    print("64^2 FP64 band heights R2=%d kernel=%d" % (R2, kind), flush=True)
    n, S = 64, 3
    md = _model(n, R2, kind)
    rng = np.random.default_rng(R2 * 11 + kind)
    host = rng.uniform(-1.2, 1.2, S * n * n)
    smp = [nlch.nlch_sample(0, 0, 0.97 + 0.02 * k, md.kernel_amp, k * n * n) for k in range(S)]
    for nsteps in (1, 30):
        s16, o16 = _solve64(md, smp, host, nsteps, (1, 16))
        s8, o8 = _solve64(md, smp, host, nsteps, (1, 8))
        assert np.max(np.abs(s8 - s16)) <= (1e-14 if nsteps == 1 else 1e-11)
        np.testing.assert_allclose(o8, o16, rtol=1e-12, atol=1e-15)
        if nsteps == 1:
            for k in range(S):
                u0 = np.clip(host[k * n * n:(k + 1) * n * n], -1, 1)
                ref = orc.step(u0.reshape(n, n), n, md.delta, md.kernel, md.kernel_amp,
                               md.kernel_sigma, smp[k].c_F, md.beta1, md.tau)
                assert np.max(np.abs(s8[k * n * n:(k + 1) * n * n].reshape(n, n) - ref)) \
                    <= 1e-13


def test_fp64_single_sample_trajectory_in_8_row_bands(orc):
    """The C1 recipe (one 64^2 sample, m = 4, 200 steps, FP64) in 8-row
    bands: the OoI and every site against the FP64 oracle's trajectory."""
    from tests.gpu_harness import oracle_samples
    w = synth.workload("C1")
    nlch.nlch_set_resident_shape(1, 8)
    b = DeviceBatch(w)
    b.solve(nlch.NLCH_ALGO_RESIDENT)
    torch.cuda.synchronize()
    ref = oracle_samples(orc, w, [0], "f64")[0]
    assert abs(b.ooi_host()[0, 1] - ref[2]) <= 1e-12 * abs(ref[2])
    assert np.max(np.abs(b.sample_state(0) - ref[0])) <= 1e-10


@pytest.mark.parametrize("n,R2", [(64, 4), (128, 64)])
def test_autotuned_resident_layout(n, R2):
    """AUTOTUNE times the resident layouts for the batch signature: results
    within rounding of the default layout, and exactly repeatable once the
    pick is cached."""
    print("resident autotune n=%d R2=%d" % (n, R2), flush=True)
    S = 512
    md = _model(n, R2, 1)
    host = np.random.default_rng(n + R2).uniform(-1, 1, S * n * n).astype(np.float32)
    smp = [nlch.nlch_sample(0, 0, 1.0, md.kernel_amp, k * n * n) for k in range(S)]

    def run(algo):
        x = torch.from_numpy(host).to(DEV)
        ooi = torch.zeros(2 * S, dtype=torch.float64, device=DEV)
        nlch.nlch_solve_batch([md], smp, 40, nlch.NLCH_F32, algo, x, None, ooi)
        torch.cuda.synchronize()
        return x.cpu().numpy(), ooi.cpu().numpy()

    d, od = run(nlch.NLCH_ALGO_RESIDENT)
    t1, o1 = run(nlch.NLCH_ALGO_RESIDENT | nlch.NLCH_ALGO_AUTOTUNE)
    t2, o2 = run(nlch.NLCH_ALGO_RESIDENT | nlch.NLCH_ALGO_AUTOTUNE)
    assert np.array_equal(t1, t2) and np.array_equal(o1, o2)
    assert np.max(np.abs(t1.astype(np.float64) - d)) <= 1e-4
    assert np.max(np.abs(o1[1::2] - od[1::2])) <= 1e-6
