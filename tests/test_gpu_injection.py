"""Error paths on the GPU, forced from the host: nlch_debug_inject_device_error
makes the nth checked HIP call of the library report failure without making
it.  For every n up to the number of checked calls a solve makes, the call
returns NLCH_EDEVICE naming the injection, and the same solve repeated
without injection gives the reference result bit for bit -- through device
set-up, batch tables, autotuning, graph capture and replay, and two launch
groups on forked streams.  Nothing invalid is issued to the device: the
injected call is skipped, and the kernels that did run were valid launches."""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _disarm():
    yield
    nlch.nlch_debug_inject_device_error(0)


def _models():
    # a streaming group (96^2) and an LDS-resident group (64^2)
    out = []
    for n, r2 in ((96, 16), (64, 9)):
        delta = math.sqrt(r2) / n
        _, m, N, _ = nlch.nlch_disc(n, delta)
        out.append(nlch.make_model(n, delta, 0, 1.0253 * n * n / N, 0.0, tau=0.05))
    return out


SIDES = (96, 96, 64)


def _solve(models, base, nsteps, algo, u0, state, scratch, ooi):
    """The three samples at offsets base.. of the state buffer (base a
    multiple of 4 floats: the batch signature changes, the kernels do not)."""
    total = int(u0.numel())
    offs = [base, base + 96 * 96, base + 2 * 96 * 96]
    smp = [nlch.nlch_sample(k, 0, 1.0, models[k].kernel_amp, offs[i])
           for i, k in enumerate((0, 0, 1))]
    state.zero_()
    state[base:base + total].copy_(u0)
    ooi.zero_()
    nlch.nlch_solve_batch(models, smp, nsteps, nlch.NLCH_F32, algo, state, scratch, ooi)
    torch.cuda.synchronize()
    return state[base:base + total].clone(), ooi.clone()


@pytest.mark.parametrize("algo", [nlch.NLCH_ALGO_AUTO,
                                  nlch.NLCH_ALGO_AUTO | nlch.NLCH_ALGO_AUTOTUNE,
                                  nlch.NLCH_ALGO_AUTO | nlch.NLCH_ALGO_NOGRAPH])
def test_every_injected_failure_leaves_the_library_usable(algo):
    models = _models()
    total = 2 * 96 * 96 + 64 * 64
    u0 = torch.from_numpy(
        np.random.default_rng(5).uniform(-1, 1, total).astype(np.float32)).to(DEV)
    state = torch.empty(total + 4 * 400, dtype=torch.float32, device=DEV)
    scratch = torch.empty_like(state)
    ooi = torch.zeros(6, dtype=torch.float64, device=DEV)
    ref = _solve(models, 0, 7, algo, u0, state, scratch, ooi)
    failed = 0
    for n in range(1, 400):
        print("algo 0x%x: failure injected at checked call %d" % (algo, n), flush=True)
        nlch.nlch_debug_inject_device_error(n)
        try:
            _solve(models, 4 * n, 7, algo, u0, state, scratch, ooi)
        except nlch.NlchError as e:
            assert e.code == nlch.NLCH_EDEVICE and "injected" in str(e), str(e)
            failed += 1
        else:
            # the solve makes fewer than n checked calls: every call was covered
            break
        finally:
            nlch.nlch_debug_inject_device_error(0)
        again = _solve(models, 4 * n, 7, algo, u0, state, scratch, ooi)
        assert torch.equal(again[0], ref[0]) and torch.equal(again[1], ref[1]), n
    else:
        pytest.fail("a solve made 400 or more checked calls")
    assert failed >= 5


def test_injected_failure_of_a_single_step_and_the_moments():
    models = _models()
    u = torch.from_numpy(np.random.default_rng(6).uniform(-1, 1, 96 * 96).astype(np.float32)).to(DEV)
    y0 = torch.empty_like(u)
    nlch.nlch_step(models[0], nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, u, y0, None)
    torch.cuda.synchronize()
    for n in range(1, 40):
        nlch.nlch_debug_inject_device_error(n)
        y = torch.full_like(u, 7.0)
        try:
            nlch.nlch_step(models[0], nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, u, y, None)
        except nlch.NlchError as e:
            assert e.code == nlch.NLCH_EDEVICE and "injected" in str(e)
        else:
            break
        finally:
            nlch.nlch_debug_inject_device_error(0)
        y = torch.empty_like(u)
        nlch.nlch_step(models[0], nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, u, y, None)
        torch.cuda.synchronize()
        assert torch.equal(y, y0), n
