"""Multifidelity Monte Carlo study on synthetic draws (arXiv 2310.10750, Sec. 4).

The paper's pipeline, driven through the library on one GPU:

1. nine models f_1..f_9 pairing the lattices h = 1/128, 1/88, 1/64 with the
   horizons delta = 0.25, 0.1875, 0.125 (Table 1's (h, delta) pairs, f_1 the
   high-fidelity one), Gaussian kernel of eq. kernel_gauss with
   delta_hf = 0.25, eps^2 = 0.00178 (2-D normalisation), c_F = 1, beta1 = 1,
   tau = 0.01, T = 1, four-nuclei initial data (eq. ic) drawn per sample and
   shared by all models (nesting);
2. pilot: sample standard deviations sigma_k and correlations rho_{1,k} from
   P shared draws, and per-sample costs C_k measured as GPU solve time per
   sample at a fixed batch size (Sec. 4 uses 50 pilot samples and CPU times);
3. model selection (mfmc_select: conditions (a), (b), V, B_min) and the five
   cases of Sec. 4 -- lowest V, second lowest V, lowest B_min, the three-h
   subset {f_1, f_4, f_8} and the three-delta subset {f_1, f_2, f_5} -- plus
   plain Monte Carlo on f_1;
4. for 8 budgets log-spaced over the same range as the paper's
   10^3..10^{16/3} seconds expressed in units of C_1 (63.089 s there), the
   sample allocation (mfmc_allocate, with the below-B_min rule), R
   independent replicates of every estimator (mfmc_estimate with the pilot's
   alpha_j = rho_{1,j} sigma_1 / sigma_j) and their mean-squared error
   against Q_validation, the mean of f_1 over V further draws;
5. the theoretical MSE: sigma_1^2 C_1 V / B for B >= B_min (eq.
   error_theory with m_1* of eq. samples), sigma_1^2 / m for Monte Carlo.

Model outputs f_k(theta_i) for draw i come from the batched solver with the
same draw stream for every model, so replicate r of every estimator uses the
draws r*D .. r*D + m_j - 1 (D the largest per-replicate count of any model).
Everything here is orchestration of the library's entry points; the only
arithmetic done on the host is the pilot statistics, the theory curves and
the squared errors.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import nlch, synth

# (label, lattice n, horizon delta) in Table 1's model numbering.
MODELS9 = [("f1", 128, 0.25), ("f2", 128, 0.1875), ("f3", 88, 0.1875),
           ("f4", 88, 0.25), ("f5", 128, 0.125), ("f6", 88, 0.125),
           ("f7", 64, 0.1875), ("f8", 64, 0.25), ("f9", 64, 0.125)]
PAPER_C1_SECONDS = 63.089
PAPER_BUDGETS_SECONDS = [10 ** (3 + i / 3) for i in range(8)]

PILOT_SEED, STUDY_SEED, VALIDATION_SEED = 41, 42, 43


def study_models(lattices=MODELS9, delta_hf=0.25, tau=0.01, beta2=0.0):
    """The study's models; beta2 = 0.05 is the paper's (a coupled step per
    time step: Newton for xi_h > 0, the split step for the truncated kernels'
    xi_h <= 0)."""
    amp, sigma, _ = synth.gaussian_params(delta_hf)
    return [synth.Model(n, delta, synth.KERNEL_GAUSSIAN, amp, sigma, beta2=beta2, tau=tau)
            for _, n, delta in lattices]


class Runner:
    """Evaluates the output of interest f_1 = (1 + mean u(T))/2 of one model
    for given draw indices of a seed, in fixed-size batches on the GPU."""

    def __init__(self, models, nsteps=100, precision="f32", chunk=4096, device="cuda:0",
                 algo=nlch.NLCH_ALGO_AUTO | nlch.NLCH_ALGO_AUTOTUNE, block=4096, log=None):
        import torch
        self.torch = torch
        self.log = log  # progress lines of long output runs (every ~30 s)
        self.models = models
        self.nsteps = nsteps
        self.prec = precision
        self.dtype = {"f64": torch.float64, "f32": torch.float32,
                      "f16": torch.float16}[precision]
        self.chunk = chunk
        self.device = device
        self.algo = algo
        self.block = block
        self.stream = torch.cuda.Stream(device=device)
        self._buf = {}
        self._theta = {}

    def _buffers(self, k):
        if k not in self._buf:
            m = self.models[k]
            nn = m.n * m.n
            st = self.torch.empty(self.chunk * nn, dtype=self.dtype, device=self.device)
            md = (nlch.nlch_model * 1)(nlch.make_model(m.n, m.delta, m.kernel, m.amp, m.sigma,
                                                       c_F=m.c_F, beta1=m.beta1,
                                                       beta2=m.beta2, tau=m.tau))
            smp = (nlch.nlch_sample * self.chunk)(*[
                nlch.nlch_sample(0, 0, m.c_F, m.amp, i * nn) for i in range(self.chunk)])
            ooi = self.torch.zeros(2 * self.chunk, dtype=self.torch.float64, device=self.device)
            self._buf[k] = (st, self.torch.empty_like(st), ooi, md, smp)
        return self._buf[k]

    def thetas(self, seed, idx):
        """Parameter rows of the given draw indices (theta_block layout)."""
        idx = np.asarray(idx, dtype=np.int64)
        out = np.empty((idx.size, 12))
        blocks = idx // self.block
        for b in np.unique(blocks):
            key = (seed, int(b))
            if key not in self._theta:
                if len(self._theta) > 256:
                    self._theta.clear()
                self._theta[key] = synth.theta_block(seed, int(b), self.block)
            sel = blocks == b
            out[sel] = self._theta[key][idx[sel] % self.block]
        return out

    def outputs(self, k, seed, idx):
        """f_1 of model k for the draws idx of `seed` (numpy FP64 array)."""
        idx = np.asarray(idx, dtype=np.int64)
        m = self.models[k]
        st, scr, ooi, md, smp = self._buffers(k)
        res = np.empty(idx.size)
        torch = self.torch
        t_last = time.time()
        for lo in range(0, idx.size, self.chunk):
            if self.log and time.time() - t_last > 30.0:
                self.log("  model %d: %d of %d draws" % (k, lo, idx.size))
                t_last = time.time()
            part = idx[lo:lo + self.chunk]
            # a full batch every time (one batch signature, one graph): the
            # tail repeats the last draw
            full = np.concatenate([part, np.full(self.chunk - part.size, part[-1])])
            with torch.cuda.stream(self.stream):
                u0 = synth.ic_nuclei_batch(m.n, self.thetas(seed, full), self.device)
                st.copy_(u0.reshape(-1).to(self.dtype))
                nlch.nlch_solve_batch(md, smp, self.nsteps, nlch.PRECISIONS[self.prec],
                                      self.algo, st, scr, ooi, self.stream)
            self.stream.synchronize()
            res[lo:lo + part.size] = ooi.view(-1, 2)[:part.size, 1].cpu().numpy()
        return res

    def cost(self, k, reps=3):
        """GPU seconds per sample of model k: a full batch's solve time
        (HIP events on the solver's stream, after a warm-up) / batch size."""
        torch = self.torch
        self.outputs(k, PILOT_SEED, np.arange(self.chunk))  # warm-up, autotune
        st, scr, ooi, md, smp = self._buffers(k)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(reps):
            with torch.cuda.stream(self.stream):
                e0.record(self.stream)
                nlch.nlch_solve_batch(md, smp, self.nsteps, nlch.PRECISIONS[self.prec],
                                      self.algo, st, scr, ooi, self.stream)
                e1.record(self.stream)
            self.stream.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3 / self.chunk)
        return best


def pilot_statistics(y):
    """sigma_k (sample standard deviation) and rho_{1,k} from a (K, P) array
    of pilot outputs on shared draws."""
    y = np.asarray(y, dtype=np.float64)
    sigma = y.std(axis=1, ddof=1)
    rho = np.array([1.0] + [float(np.corrcoef(y[0], y[k])[0, 1]) for k in range(1, len(y))])
    return sigma, rho


def choose_cases(feasible, labels):
    """The five cases of Sec. 4 from the feasible subsets (sorted by V)."""
    idx = {lab: i for i, lab in enumerate(labels)}
    by_set = {frozenset(s): (s, V, b) for s, V, b in feasible}
    cases = {"case1 lowest V": feasible[0]}
    if len(feasible) > 1:
        cases["case2 second lowest V"] = feasible[1]
    cases["case3 lowest B_min"] = min(feasible, key=lambda t: t[2])
    for name, labs in (("case4 three-h", ("f1", "f4", "f8")),
                       ("case5 three-delta", ("f1", "f2", "f5"))):
        if all(l in idx for l in labs):
            key = frozenset(idx[l] for l in labs)
            if key in by_set:
                cases[name] = by_set[key]
    return cases


def run_study(models=None, labels=None, pilot=50, replicates=100, validation=360000,
              budgets_c1=None, nsteps=100, precision="f32", chunk=4096, log=print,
              costs_only=False):
    import torch
    models = models or study_models()
    labels = labels or [lab for lab, _, _ in MODELS9]
    K = len(models)
    budgets_c1 = budgets_c1 or [b / PAPER_C1_SECONDS for b in PAPER_BUDGETS_SECONDS]
    run = Runner(models, nsteps=nsteps, precision=precision, chunk=chunk, log=log)
    t0 = time.time()

    # 2. pilot statistics and costs
    yp = np.stack([run.outputs(k, PILOT_SEED, np.arange(pilot)) for k in range(K)])
    sigma, rho = pilot_statistics(yp)
    cost = np.zeros(K)
    for k in range(K):
        cost[k] = run.cost(k)
        log("cost of %s: %.1f us per sample (%.1fs)" % (labels[k], 1e6 * cost[k],
                                                         time.time() - t0))
    log("pilot (%d draws) and costs: %.1fs" % (pilot, time.time() - t0))
    if costs_only:
        return {"models": [{"label": labels[k], "n": models[k].n, "delta": models[k].delta,
                            "beta2": models[k].beta2, "rho": float(rho[k]),
                            "sigma": float(sigma[k]), "cost_s": float(cost[k])}
                           for k in range(K)], "seconds": time.time() - t0}

    # 3. selection
    feasible, ncand = nlch.mfmc_select(list(cost / cost[0]), list(rho))
    cases = choose_cases(feasible, labels)

    # 4. allocations for every case and budget
    alloc = {}
    D = np.zeros(K, dtype=np.int64)
    for b in budgets_c1:
        B = b * cost[0]
        m_mc = int(math.floor(b))
        alloc[("mc", b)] = ((0,), [m_mc], True)
        D[0] = max(D[0], m_mc)
        for name, (sub, V, bmin) in cases.items():
            try:
                _, mi, m1 = nlch.mfmc_allocate(sub, list(cost), list(rho), B)
            except nlch.NlchError:
                alloc[(name, b)] = None  # below sum_l l C_{i_l}: no estimator
                continue
            alloc[(name, b)] = (sub, list(mi), m1 >= 1.0)
            for j, k in enumerate(sub):
                D[k] = max(D[k], mi[j])
    stride = int(D.max())
    # model outputs of every replicate's draws, on the device, (R, D_k) each
    Y = []
    for k in range(K):
        if D[k] == 0:
            Y.append(None)
            continue
        idx = (np.arange(replicates)[:, None] * stride + np.arange(D[k])[None, :]).reshape(-1)
        Y.append(torch.from_numpy(run.outputs(k, STUDY_SEED, idx).reshape(replicates, D[k]))
                 .to(run.device))
        log("model %s: %d draws per replicate (%.1fs)" % (labels[k], D[k], time.time() - t0))
    yv = run.outputs(0, VALIDATION_SEED, np.arange(validation))
    q_val = float(np.mean(yv))
    log("validation: %d draws of %s, Q = %.9f (%.1fs)" % (validation, labels[0], q_val,
                                                          time.time() - t0))

    # estimators and their mean-squared error
    alpha = {k: float(rho[k] * sigma[0] / sigma[k]) for k in range(K)}
    rows = []
    for (name, b), a in sorted(alloc.items(), key=lambda t: (t[0][0], t[0][1])):
        if a is None:
            rows.append({"case": name, "budget_c1": b, "mse": None})
            continue
        sub, m, above = a
        q = []
        for r in range(replicates):
            ptrs = [Y[k].data_ptr() + 8 * r * int(D[k]) for k in sub]
            est = nlch.mfmc_estimate(ptrs, m, [alpha[k] for k in sub[1:]] or None,
                                     stream=run.stream)
            q.append(est["q_mfmc"])
        q = np.array(q)
        mse = float(np.mean((q - q_val) ** 2))
        if name == "mc":
            theory = float(sigma[0] ** 2 / m[0])
        else:
            V = cases[name][1]
            theory = float(sigma[0] ** 2 * V / b) if above else None
        rows.append({"case": name, "budget_c1": b, "budget_paper_seconds": b * PAPER_C1_SECONDS,
                     "subset": [labels[k] for k in sub], "m": [int(v) for v in m],
                     "above_bmin": bool(above), "mse": mse, "mse_theory": theory,
                     "mean_estimate": float(np.mean(q))})
    return {
        "models": [{"label": labels[k], "n": models[k].n, "delta": models[k].delta,
                    "rho": float(rho[k]), "sigma": float(sigma[k]),
                    "cost_s": float(cost[k]), "cost_ratio": float(cost[k] / cost[0])}
                   for k in range(K)],
        "beta2": models[0].beta2, "nsteps": nsteps, "chunk": chunk,
        "pilot": pilot, "replicates": replicates, "validation": validation,
        "q_validation": q_val, "n_candidates": ncand, "n_feasible": len(feasible),
        "feasible_top": [{"subset": [labels[k] for k in s], "V": V, "bmin_over_c1": bm}
                         for s, V, bm in feasible[:10]],
        "cases": {name: {"subset": [labels[k] for k in s], "V": V, "bmin_over_c1": bm}
                  for name, (s, V, bm) in cases.items()},
        "rows": rows, "seconds": time.time() - t0,
    }


def report_markdown(res):
    out = ["| model | n | delta | rho_1k | sigma_k | C_k (GPU us) | C_k/C_1 |",
           "|---|---|---|---|---|---|---|"]
    for m in res["models"]:
        out.append("| %s | %d | %.4f | %.7f | %.3e | %.2f | %.4f |" % (
            m["label"], m["n"], m["delta"], m["rho"], m["sigma"], 1e6 * m["cost_s"],
            m["cost_ratio"]))
    out += ["", "%d of %d subsets feasible; cases:" % (res["n_feasible"], res["n_candidates"]), ""]
    for name, c in res["cases"].items():
        out.append("* %s: {%s}, V = %.5f, B_min/C_1 = %.2f" % (
            name, ", ".join(c["subset"]), c["V"], c["bmin_over_c1"]))
    out += ["", "| case | B/C_1 | MSE | MSE theory | m |", "|---|---|---|---|---|"]
    for r in res["rows"]:
        if r["mse"] is None:
            out.append("| %s | %.1f | below sum l C | | |" % (r["case"], r["budget_c1"]))
            continue
        th = "%.3e" % r["mse_theory"] if r["mse_theory"] is not None else "(below B_min)"
        out.append("| %s | %.1f | %.3e | %s | %s |" % (r["case"], r["budget_c1"], r["mse"], th,
                                                      r["m"]))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--pilot", type=int, default=50)
    ap.add_argument("--replicates", type=int, default=100)
    ap.add_argument("--validation", type=int, default=360000)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--beta2", type=float, default=0.0,
                    help="beta2 of every model (the paper's experiments: 0.05)")
    ap.add_argument("--budgets", type=int, default=8,
                    help="use the first N of the paper's 8 budgets")
    ap.add_argument("--chunk", type=int, default=4096, help="samples per solver call")
    ap.add_argument("--costs-only", action="store_true",
                    help="stop after the pilot statistics and the costs")
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    a = ap.parse_args(argv)
    budgets = [b / PAPER_C1_SECONDS for b in PAPER_BUDGETS_SECONDS[:a.budgets]]
    res = run_study(models=study_models(beta2=a.beta2), pilot=a.pilot,
                    replicates=a.replicates, validation=a.validation, budgets_c1=budgets,
                    precision=a.precision, chunk=a.chunk, costs_only=a.costs_only,
                    log=lambda *x: print(*x, file=sys.stderr, flush=True))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    if not a.costs_only:
        print(report_markdown(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
