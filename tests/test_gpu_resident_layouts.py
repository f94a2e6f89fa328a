"""The LDS-resident kernel's layouts give bit-identical states: two columns
per lane with one 16-row band per wave, and four columns per lane with two
bands per wave and 16-byte window loads (FP32, 128^2).  Every site sums the
same window sums in the same order in both.  The outputs of interest are
FP64 sums of the same values in a different order, so they agree to FP64
rounding.  The oracle comparison of every built resident kernel at every site
is in test_gpu_parity.py."""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch, synth
from tests.gpu_harness import DeviceBatch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _default_layout():
    yield
    nlch.nlch_set_resident_shape(0)


def _model(n, R2, kind, tau=0.05):
    delta = math.sqrt(R2) / n
    _, m, N, _ = nlch.nlch_disc(n, delta)
    if kind == 0:
        amp, sigma = 1.0253 * n * n / N, 0.0
    else:
        sigma = delta / 3
        amp = 1.0253 / (math.pi * sigma * sigma)
    return nlch.make_model(n, delta, kind, amp, sigma, tau=tau)


def _solve(md, smp, host, nsteps, cols):
    nlch.nlch_set_resident_shape(cols)
    x = torch.from_numpy(host).to(DEV)
    ooi = torch.zeros(2 * len(smp), dtype=torch.float64, device=DEV)
    nlch.nlch_solve_batch([md], smp, nsteps, nlch.NLCH_F32, nlch.NLCH_ALGO_RESIDENT, x, None,
                          ooi)
    torch.cuda.synchronize()
    return x.cpu().numpy(), ooi.cpu().numpy()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("R2", [1, 4, 9, 16, 25, 64])
def test_four_columns_equal_two_columns(R2, kind):
    print("layouts R2=%d kernel=%d" % (R2, kind), flush=True)
    n, S = 128, 5
    md = _model(n, R2, kind)
    rng = np.random.default_rng(R2 * 10 + kind)
    host = rng.uniform(-1.2, 1.2, S * n * n).astype(np.float32)
    smp = [nlch.nlch_sample(0, 0, 0.96 + 0.02 * k, md.kernel_amp, k * n * n) for k in range(S)]
    for nsteps in (0, 1, 7, 40):
        s2, o2 = _solve(md, smp, host, nsteps, 2)
        s4, o4 = _solve(md, smp, host, nsteps, 4)
        assert np.array_equal(s2, s4), nsteps
        np.testing.assert_allclose(o4, o2, rtol=0, atol=1e-15)


def test_benchmark_workload_layouts_agree():
    """256 samples of the benchmark workload (128^2, 197-point disc, per-sample
    c_F, 500 steps): the two layouts give the same final states."""
    print("C3 layouts", flush=True)
    w = synth.workload("C3", n_samples=256)
    out = []
    for cols in (2, 4):
        nlch.nlch_set_resident_shape(cols)
        b = DeviceBatch(w)
        b.solve(algo=nlch.NLCH_ALGO_AUTO)
        torch.cuda.synchronize()
        out.append((b.state.cpu().numpy(), b.ooi_host()))
    assert np.array_equal(out[0][0], out[1][0])
    np.testing.assert_allclose(out[1][1], out[0][1], rtol=0, atol=1e-15)
