"""The library caches device tables per call signature.  These tests run
sequences of calls that share a model and a sample and check every result
against the FP64 oracle:

* nlch_step and a batch solve of the same model and sample keep separate
  tables.  The solve may pick the LDS-resident kernel, which needs no scratch
  buffer, while the step uses a per-step kernel and an OoI reduction.  Both
  orders are covered.
* Two solves with one signature, enqueued on two streams into different
  buffers, share the signature's OoI chunk sums.  The library orders them,
  so both outputs are right.
"""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _model(n, r, tau=0.05):
    _, m, N, _ = nlch.nlch_disc(n, r / n)
    amp = 1.0253 * n * n / N
    return nlch.make_model(n, r / n, nlch.NLCH_KERNEL_CONSTANT, amp, tau=tau)


def _u0(n, seed):
    u = np.random.default_rng(seed).uniform(-0.3, 0.3, (n, n))
    return u.astype(np.float32).astype(np.float64)


def _oracle_solve(orc, md, u0, nsteps):
    return orc.solve(u0, nsteps, md.n, md.delta, md.kernel, md.kernel_amp,
                     md.kernel_sigma, md.c_F, md.beta1, md.tau)


def test_step_then_resident_solve_without_scratch(orc):
    print("step then resident solve", flush=True)
    md = _model(64, 4)
    u0 = _u0(64, 1)
    x = torch.from_numpy(u0.reshape(-1)).float().to(DEV)
    y = torch.empty_like(x)
    o1 = torch.zeros(2, dtype=torch.float64, device=DEV)
    nlch.nlch_step(md, nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, x, y, o1)
    torch.cuda.synchronize()
    ref1 = orc.step(u0, 64, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma, md.c_F,
                    md.beta1, md.tau)
    assert np.max(np.abs(y.double().cpu().numpy().reshape(64, 64) - ref1)) <= 1e-6
    # the same model and sample as a batch: the resident kernel, no scratch
    smp = [nlch.nlch_sample(0, 0, md.c_F, md.kernel_amp, 0)]
    st = x.clone()
    o2 = torch.zeros(2, dtype=torch.float64, device=DEV)
    nlch.nlch_solve_batch([md], smp, 30, nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, st, None, o2)
    torch.cuda.synchronize()
    ref, mean, f1 = _oracle_solve(orc, md, u0, 30)
    assert np.max(np.abs(st.double().cpu().numpy().reshape(64, 64) - ref)) <= 1e-5
    assert abs(o2[1].item() - f1) <= 1e-6 * abs(f1)


def test_resident_solve_then_step_with_ooi(orc):
    print("resident solve then step", flush=True)
    md = _model(64, 3, tau=0.04)
    u0 = _u0(64, 2)
    smp = [nlch.nlch_sample(0, 0, md.c_F, md.kernel_amp, 0)]
    st = torch.from_numpy(u0.reshape(-1)).float().to(DEV)
    o = torch.zeros(2, dtype=torch.float64, device=DEV)
    nlch.nlch_solve_batch([md], smp, 10, nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, st, None, o)
    torch.cuda.synchronize()
    ref, _, f1 = _oracle_solve(orc, md, u0, 10)
    assert abs(o[1].item() - f1) <= 1e-6 * abs(f1)
    # a step of the same model and sample, with its output of interest
    x = torch.from_numpy(u0.reshape(-1)).float().to(DEV)
    y = torch.empty_like(x)
    o1 = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
    nlch.nlch_step(md, nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, x, y, o1)
    torch.cuda.synchronize()
    ref1 = orc.step(u0, 64, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma, md.c_F,
                    md.beta1, md.tau)
    got = y.double().cpu().numpy().reshape(64, 64)
    assert np.max(np.abs(got - ref1)) <= 1e-6
    assert abs(o1[0].item() - float(np.mean(got))) <= 1e-12


def test_same_signature_on_two_streams(orc):
    """A lattice that runs on the per-step kernels (n = 96, not resident), one
    signature, two streams, two state buffers: both OoIs are the oracle's."""
    print("same signature on two streams", flush=True)
    n, steps = 96, 40
    md = _model(n, 4)
    u0 = _u0(n, 3)
    smp = [nlch.nlch_sample(0, 0, md.c_F, md.kernel_amp, 0)]
    bufs = []
    for _ in range(2):
        st = torch.from_numpy(u0.reshape(-1)).float().to(DEV)
        bufs.append((st, torch.empty_like(st), torch.zeros(2, dtype=torch.float64, device=DEV)))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        for (st, sc, o), s in zip(bufs, (s1, s2)):
            st.copy_(torch.from_numpy(u0.reshape(-1)).float().to(DEV))
            torch.cuda.synchronize()
        for (st, sc, o), s in zip(bufs, (s1, s2)):
            nlch.nlch_solve_batch([md], smp, steps, nlch.NLCH_F32,
                                  nlch.NLCH_ALGO_ROWRUN, st, sc, o, s.cuda_stream)
        torch.cuda.synchronize()
        _, _, f1 = _oracle_solve(orc, md, u0, steps)
        for st, sc, o in bufs:
            assert abs(o[1].item() - f1) <= 1e-6 * abs(f1)
            assert math.isfinite(o[0].item())
