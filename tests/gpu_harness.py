"""Helpers shared by the GPU parity tests and the benchmark: device buffers for
a synthetic workload, and the matching FP64 oracle runs.

The oracle is always fed exactly the values the GPU starts from (the synthetic
FP64 initial data rounded to the state type), so a comparison isolates the
kernels' arithmetic.
"""
from __future__ import annotations

import numpy as np

from paper_2310_10750_amd import nlch, synth

TORCH_DTYPE = {"f64": "float64", "f32": "float32", "f16": "float16"}
NP_DTYPE = {"f64": np.float64, "f32": np.float32, "f16": np.float16}


def rounded_initial(w, s, prec):
    """Initial datum of sample s rounded (RNE) to the state type, as FP64."""
    return synth.initial_state(w, s).astype(NP_DTYPE[prec]).astype(np.float64)


class DeviceBatch:
    """State / scratch / OoI buffers of a workload on cuda:0."""

    def __init__(self, w, prec=None, device="cuda:0", samples=None):
        import torch
        self.w = w
        self.prec = prec or w.precision
        self.models, self.samples, self.total = nlch.structs_for(w)
        self.dtype = getattr(torch, TORCH_DTYPE[self.prec])
        host = np.empty(self.total, dtype=NP_DTYPE[self.prec])
        for i, s in enumerate(w.samples):
            n = synth.state_side(w.models[s.model])
            off = self.samples[i].offset
            host[off:off + n * n] = synth.initial_state(w, s).astype(
                NP_DTYPE[self.prec]).reshape(-1)
        self.host0 = host
        self.state = torch.from_numpy(host).to(device)
        self.init = self.state.clone()
        self.scratch = torch.empty_like(self.state)
        self.ooi = torch.zeros(2 * len(w.samples), dtype=torch.float64, device=device)

    def reset(self):
        self.state.copy_(self.init)

    def solve(self, algo=nlch.NLCH_ALGO_AUTO, nsteps=None, stream=None):
        nlch.nlch_solve_batch(self.models, self.samples,
                              self.w.nsteps if nsteps is None else nsteps,
                              nlch.PRECISIONS[self.prec], algo, self.state,
                              self.scratch, self.ooi, stream)

    def solve_energy(self, algo=nlch.NLCH_ALGO_AUTO, nsteps=None, stream=None):
        """Solve with the energy trace; returns the (nsteps + 1, n_samples)
        device array of E_h(u^k)."""
        import torch
        k = self.w.nsteps if nsteps is None else nsteps
        e = torch.full(((k + 1) * len(self.w.samples),), float("nan"), dtype=torch.float64,
                       device=self.state.device)
        nlch.nlch_solve_batch_energy(self.models, self.samples, k, nlch.PRECISIONS[self.prec],
                                     algo, self.state, self.scratch, self.ooi, e, stream)
        return e.view(k + 1, len(self.w.samples))

    def sample_state(self, i):
        """Sample i's stored array (with the ring under a volume constraint)."""
        n = synth.state_side(self.w.models[self.w.samples[i].model])
        off = self.samples[i].offset
        return self.state[off:off + n * n].double().cpu().numpy().reshape(n, n)

    def ooi_host(self):
        return self.ooi.cpu().numpy().reshape(-1, 2)


def oracle_samples(orc, w, idx, prec, nsteps=None):
    """FP64 oracle trajectories of the listed samples (grouped by model)."""
    nsteps = w.nsteps if nsteps is None else nsteps
    out = {}
    by_model = {}
    for i in idx:
        by_model.setdefault(w.samples[i].model, []).append(i)
    for mi, ids in by_model.items():
        m = w.models[mi]
        u0 = np.stack([rounded_initial(w, w.samples[i], prec) for i in ids])
        U, mean, f1 = orc.solve_many(u0, nsteps, m.n, m.delta, m.kernel, m.sigma,
                                     m.beta1, m.tau, [w.samples[i].c_F for i in ids],
                                     [w.samples[i].amp for i in ids])
        for k, i in enumerate(ids):
            out[i] = (U[k], mean[k], f1[k])
    return out


def one_step_sites(orc, w, batch, i, nsites=1500, seed=0):
    """Max |GPU step - oracle step| over random sites of sample i, both
    stepping from the GPU's current state of that sample (taken as stored).
    Advances the sample by one step on the GPU."""
    from paper_2310_10750_amd import nlch
    s = w.samples[i]
    m = w.models[s.model]
    u = batch.sample_state(i)
    rng = np.random.default_rng(seed)
    sites = rng.choice(m.n * m.n, size=min(nsites, m.n * m.n), replace=False)
    ref = orc.step_sites(u, sites, m.n, m.delta, m.kernel, s.amp, m.sigma, s.c_F,
                         m.beta1, m.tau)
    one = nlch.nlch_sample(s.model, 0, s.c_F, s.amp, 0)
    off = batch.samples[i].offset
    x = batch.state[off:off + m.n * m.n]
    scr = batch.scratch[off:off + m.n * m.n]
    import torch
    o = torch.zeros(2, dtype=torch.float64, device=batch.state.device)
    nlch.nlch_solve_batch(batch.models, [one], 1, nlch.PRECISIONS[batch.prec],
                          nlch.NLCH_ALGO_AUTO, x, scr, o)
    torch.cuda.synchronize()
    got = batch.sample_state(i).reshape(-1)[sites]
    return float(np.max(np.abs(got - ref)))
