#!/usr/bin/env python3
"""Benchmark of the batched solve on one MI355X.

One benchmark step is one pass of the whole path over one batch: reset the
state buffer to the initial data (a device-to-device copy, inputs already in
HBM), the batched solve (initial projection, every time step with the
obstacle-constrained update, per-sample FP64 output of interest), and the FP64
Monte Carlo moments of the outputs.  Default workload: 4096 samples of a
128 x 128 periodic lattice, horizon 8h (197-point disc), constant kernel,
per-sample c_F, 500 steps, FP32 state and arithmetic.

Prints one JSON line on stdout (diagnostics go to stderr), with
  roofline     -- the dominant kernel's algorithmic work rate against its bound,
                  timed live with HIP events on the stream it runs on;
  cpu_baseline -- the FP64 CPU oracle timed on a bounded sample of the same
                  workload on the host cores (and the OoI error against it);
  fp64_one_sample -- the same workload's throughput in FP64 with one sample per
                  call and one launch per step (no graph) on the same GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("site-steps/s & HBM/LDS GB/s: batched FP32 vs 1-sample FP64, "
          "OoI err stated")
# FP32 vector peak of MI355X in lane-operations (one add, multiply or fused
# multiply-add each): 256 CUs x 128 FP32 lanes per clock x 2.4 GHz = 78.6 T/s,
# the published 157.3 TFLOP/s with a fused multiply-add counted as one.
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
FP32_PEAK_TFLOPS = 157.3
# FP64 vector: half the FP32 lane rate (the published 78.6 TFLOP/s).
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# Rates the peak-measurement program (paper_2310_10750_amd/peaks) reaches on
# MI355X with the library's compile flags: FP32 adds, and LDS reads of 8 and 16 bytes
# per lane (lane-contiguous).  No LDS bandwidth of CDNA4 is published beside
# the 160 KB capacity; the measured rates are the LDS ceiling used here.
MEASURED_ADD_TOPS = 71.9
MEASURED_LDS_GBS = {"8B": 72800.0, "16B": 95300.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources each measured kernel is compiled from (its template, the device
# helpers and structures it includes, and the unit that instantiates it).
KERNEL_SOURCES = {
    "k_resident": ["kern_rowrun_impl.h", "kern_rowrun_dispatch.h", "kern_rowrun_f32.hip",
                   "nlch_device.h", "nlch_internal.h"],
    "k_resident4": ["kern_rowrun_impl.h", "kern_resident4.hip", "nlch_device.h",
                    "nlch_internal.h"],
    "k_resident4h": ["kern_rowrun_impl.h", "kern_resident4.hip", "nlch_device.h",
                     "nlch_internal.h"],
}


def _code_only(text: str) -> str:
    """A C++ source without its comments, trailing blanks and blank lines
    (the kernel sources hold no comment markers inside string literals)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def kernel_source_hash(kernel="k_resident"):
    """Hash of a kernel's sources, to tell whether stored counter data still
    describe the current kernel.  Comments do not count: a change to them
    alone leaves the compiled kernel as it was."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2310_10750_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, sorted(os.listdir(csrc))):
        h.update(f.encode())
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def algorithmic_ops(m: int, kernel: int) -> int:
    """VALU lane-operations per site-step of the row-run evaluation: 2m for the
    window sums (m pair adds, m accumulations -- fused multiply-adds for the
    Gaussian kernel), 2m+1 for adding the window sums of the 2m+1 disc rows
    (adds, or fused multiply-adds), and 5 for the update from the disc sum
    (a multiply, a fused multiply-add, an add) and the projection (a maximum
    and a minimum).  A fused multiply-add counts as one lane-operation."""
    return 2 * m + (2 * m + 1) + 5


def split_window_ops(R2: int, C: int = 4) -> float:
    """VALU lane-operations per site-step of k_resident4h on the constant
    kernel, whose C columns per lane share running sums of their window: the
    window win[0 .. 2m + C) is summed leftwards from its middle and
    rightwards from it (2m + C - 2 additions per lane and row), and each
    column's window sum of a half-width the disc uses is one addition of a
    left and a right running sum when the window straddles the middle (else
    a direct sum, 2w additions); then the 2m+1 disc-row additions and the 5
    of the update, as in algorithmic_ops."""
    m = math.isqrt(R2)
    isqrt = math.isqrt
    widths = sorted({isqrt(R2 - a * a) for a in range(m + 1)})
    S = m + C // 2
    per_lane = 2 * m + C - 2
    for w in widths:
        for c in range(C):
            lo, hi = m + c - w, m + c + w
            per_lane += 1 if (lo <= S - 1 and hi >= S) else 2 * w
    return per_lane / C + (2 * m + 1) + 5


def algorithmic_flops(m: int, kernel: int) -> int:
    """The same work in floating-point operations, a fused multiply-add
    counted as two and the projection's maximum and minimum as none: constant
    kernel 2m + (2m+1) + 4; Gaussian kernel (m of the window terms and all
    2m+1 row sums are fused multiply-adds) 3m + 2(2m+1) + 4."""
    if kernel == 1:
        return 3 * m + 2 * (2 * m + 1) + 4
    return 2 * m + (2 * m + 1) + 4


def stored_counters(kernel_name: str, workload: str):
    """The committed counter summary of the kernel (profiles/traffic.json),
    if it was measured on this workload and on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    e = d.get(kernel_name)
    if not e or e.get("source_hash") != kernel_source_hash(kernel_name):
        return None
    if not e.get("workload", "").startswith(workload + ":"):
        return None
    return e


def stored_traffic(kernel_name: str, workload: str):
    """HBM bytes per launch of the kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None."""
    e = stored_counters(kernel_name, workload)
    return e.get("bytes_per_launch") if e else None


def host_info():
    """The CPU the oracle baseline ran on: model name, logical CPUs, and the
    CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--algo", type=lambda v: int(v, 0), default=0x800,
                    help="nlch algorithm word (default AUTO | AUTOTUNE)")
    ap.add_argument("--cpu-samples", type=int, default=512,
                    help="most samples the CPU oracle baseline may time")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="the CPU oracle baseline adds chunks of up to 16 samples until "
                         "this much oracle time is spent")
    ap.add_argument("--fp64-samples", type=int, default=4)
    ap.add_argument("--resident-shape", default="0,0",
                    help="layout of the LDS-resident kernel: columns,rows per lane "
                         "(0,0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(samples would shard by sample index, with one FP64 all-reduce of "
              "the moment sums).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2310_10750_amd import nlch, synth
    if not os.path.exists(nlch.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    dev = torch.device("cuda:0")
    w = synth.workload(args.workload)
    prec = args.precision or w.precision
    tdt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}[prec]
    ndt = {"f64": np.float64, "f32": np.float32, "f16": np.float16}[prec]
    models, samples, total = nlch.structs_for(w)
    S = len(w.samples)
    site_steps = w.site_steps()
    log("workload %s: %d samples, %d site-steps per solve" % (w.name, S, site_steps))

    t0 = time.time()
    host = np.empty(total, dtype=ndt)
    for i, s in enumerate(w.samples):
        n = synth.state_side(w.models[s.model])
        off = samples[i].offset
        host[off:off + n * n] = synth.initial_state(w, s).astype(ndt).reshape(-1)
    init = torch.from_numpy(host).to(dev)
    state = torch.empty_like(init)
    scratch = torch.empty_like(init)
    ooi = torch.zeros(2 * S, dtype=torch.float64, device=dev)
    log("inputs generated in %.1fs" % (time.time() - t0))

    stream = torch.cuda.Stream(device=dev)
    precision = nlch.PRECISIONS[prec]
    nlch.nlch_set_resident_shape(*[int(v) for v in args.resident_shape.split(",")])
    level_counts = w.level_counts or [S]
    # MFMC moments: levels are contiguous in sample order, HF first.
    level_ptrs, off = [], 0
    for c in level_counts:
        level_ptrs.append(ooi.data_ptr() + 8 * (2 * off + 1))
        off += c

    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]

    def one_step(i=None):
        with torch.cuda.stream(stream):
            state.copy_(init)
            if i is not None:
                ev_s[i].record(stream)
            nlch.nlch_solve_batch(models, samples, w.nsteps, precision, args.algo, state,
                                  scratch, ooi, stream)
            if i is not None:
                ev_e[i].record(stream)
        if level_counts[0] < 2:  # a single high-fidelity draw: no moments
            stream.synchronize()
            return None
        return nlch.mfmc_estimate(level_ptrs, level_counts, stream=stream, y_stride=2)

    # A plain elementwise copy of known size (the state buffer), run once
    # outside the timed region: its HBM counters calibrate the solver's.
    with torch.cuda.stream(stream):
        torch.add(init, 0, out=scratch)
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        est = one_step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_start
    ms_per_step = 1e3 * dt / max(1, args.steps)
    value = site_steps / (dt / max(1, args.steps))
    solve_ms = float(np.mean([ev_s[i].elapsed_time(ev_e[i]) for i in range(args.steps)]))
    log("%.3f ms/step, solve %.3f ms, %.3e site-steps/s" % (ms_per_step, solve_ms, value))

    # Dominant kernel: with every sample LDS-resident the solve is one launch.
    m0 = w.models[0]
    R2, mdisc, N, _ = nlch.nlch_disc(m0.n, m0.delta)
    resident = all(mm.n in (64, 128) and mm.beta2 == 0 for mm in w.models) and \
        (args.algo & 0xff) in (0, 3)
    kname = "k_resident" if resident else "k_rowrun"
    shape = tuple(int(v) for v in args.resident_shape.split(","))
    # FP32 128^2 (periodic, or Omega inside its ring): four columns per lane
    # in split bands by default; (4, 16) is built for the periodic lattice
    # only (a bounded domain then runs the two-column kernel)
    boundary = any(mm.boundary for mm in w.models)
    if resident and prec == "f32" and all(mm.n == 128 for mm in w.models) and mdisc <= 8:
        if shape == (4, 16):
            kname = "k_resident" if boundary else "k_resident4"
        elif shape != (2, 16):
            kname = "k_resident4h"
    # k_resident4h evaluates the constant kernel's windows (m >= 3) from
    # running sums shared by a lane's four columns (fewer operations than
    # 4m + 6)
    def split(m, kernel):
        return kname == "k_resident4h" and kernel == 0 and m >= 3

    def ops_of(m, kernel, R2):
        return split_window_ops(R2) if split(m, kernel) else algorithmic_ops(m, kernel)

    def flops_of(m, kernel, R2):
        # all window and row operations are additions; the update is 4 flops
        return split_window_ops(R2) - 1 if split(m, kernel) else algorithmic_flops(m, kernel)

    def per_site(fn):
        tot = 0
        for s in w.samples:
            mm = w.models[s.model]
            r2, md, _, _ = nlch.nlch_disc(mm.n, mm.delta)
            tot += fn(md, mm.kernel, r2) * mm.n ** 2
        return tot * w.nsteps
    ops, flops = per_site(ops_of), per_site(flops_of)
    achieved = ops / (solve_ms * 1e-3) / 1e12
    tflops = flops / (solve_ms * 1e-3) / 1e12
    traffic = stored_traffic(kname, w.name)
    # FP64 arithmetic (FP64 state, or the ACC64 flag) runs at half the lane rate
    f64 = prec == "f64" or bool(args.algo & nlch.NLCH_ALGO_ACC64)
    peak_ops = VALU_PEAK_TOPS / 2 if f64 else VALU_PEAK_TOPS
    peak_tf = FP64_PEAK_TFLOPS if f64 else FP32_PEAK_TFLOPS
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak_ops, 3),
                "unit": "T lane-ops/s", "frac": round(achieved / peak_ops, 4),
                "traffic": traffic, "kernel": kname,
                "arithmetic": "f64" if f64 else "f32",
                "ops_per_site_step": ops_of(mdisc, m0.kernel, R2),
                "flops_per_site_step": flops_of(mdisc, m0.kernel, R2),
                "achieved_tflops": round(tflops, 3), "peak_tflops": peak_tf,
                "frac_flops": round(tflops / peak_tf, 4)}
    if not f64:
        roofline["frac_measured_add_rate"] = round(achieved / MEASURED_ADD_TOPS, 4)
    if any(mm.beta2 > 0 for mm in w.models):
        # an iterative solve per step (Newton with conjugate-gradient inner
        # solves): no fixed algorithmic count per site-step to price
        roofline = None
    state_bytes = total * np.dtype(ndt).itemsize
    hbm_gbs = 2 * state_bytes / (solve_ms * 1e-3) / 1e9
    # LDS bytes per launch from the committed counters (SQ_INSTS_LDS_LOAD- and
    # _STORE_BANDWIDTH, 64-byte units), over this run's launch duration
    ctr = stored_counters(kname, w.name)
    lds = None
    if ctr and ctr.get("lds_bytes_per_launch") and roofline is not None:
        lb = ctr["lds_bytes_per_launch"]
        gbs = lb / (solve_ms * 1e-3) / 1e9
        width = ctr.get("lds_read_width", "8B")
        lds = {"bytes_per_launch": lb, "bytes_per_site_step": round(lb / site_steps, 2),
               "achieved_gbs": round(gbs, 1), "read_width": width,
               "frac_measured_8B": round(gbs / MEASURED_LDS_GBS["8B"], 4),
               "frac_measured_16B": round(gbs / MEASURED_LDS_GBS["16B"], 4)}
        # the pipe nearer its ceiling: VALU against the measured add rate, LDS
        # against the measured rate of the kernel's read width
        f_lds = gbs / MEASURED_LDS_GBS[width]
        f_valu = roofline.get("frac_measured_add_rate", roofline["frac"])
        roofline["binding_pipe"] = "lds" if f_lds > f_valu else "valu"
        roofline["frac_lds"] = round(f_lds, 4)

    out = {
        "metric": METRIC, "value": value, "unit": "site-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "%s: %s" % (w.name, w.description), "samples": S,
                   "n": [mm.n for mm in w.models], "R2": R2, "disc_points": N,
                   "time_steps": w.nsteps, "precision": prec, "algo": args.algo},
        "roofline": roofline,
        # one solve's wall time on the device per time step (for a single
        # sample: the latency of one step of the high-fidelity model)
        "latency": {"us_per_time_step": round(1e3 * solve_ms / max(1, w.nsteps), 3),
                    "samples": S, "time_steps": w.nsteps},
        "hbm_state_gbs": round(hbm_gbs, 1),
        "lds": lds,
    }
    if est is not None:
        out["mfmc_estimate"] = {"q_mfmc": est["q_mfmc"], "q_mc": est["q_mc"],
                                "levels": level_counts, "alpha": est["alpha"]}

    # FP64, one sample per call, one launch per step, no graph.
    if not args.no_fp64_baseline:
        k = min(args.fp64_samples, S)
        mods = (nlch.nlch_model * len(w.models))(*models)
        u64 = [torch.from_numpy(synth.initial_state(w, w.samples[i]).reshape(-1)).to(dev)
               for i in range(k)]
        scr = torch.empty_like(u64[0])
        o64 = torch.zeros(2, dtype=torch.float64, device=dev)
        algo64 = nlch.NLCH_ALGO_DIRECT | nlch.NLCH_ALGO_NOGRAPH
        one = lambda i: nlch.nlch_solve_batch(
            mods, [nlch.nlch_sample(samples[i].model, 0, samples[i].c_F,
                                    samples[i].kernel_amp, 0)],
            w.nsteps, nlch.NLCH_F64, algo64, u64[i], scr, o64, stream)
        one(0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(k):
            one(i)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t
        ss64 = sum(w.models[w.samples[i].model].n ** 2 for i in range(k)) * w.nsteps
        v64 = ss64 / t64
        out["fp64_one_sample"] = {"value": v64, "unit": "site-steps/s", "samples": k,
                                  "algo": "direct, 1 launch per step, no graph",
                                  "speedup": value / v64}
        log("fp64 one-sample: %.3e site-steps/s, speedup %.1fx" % (v64, value / v64))

    # CPU oracle on a bounded sample (also the OoI error statement).
    if not args.no_cpu_baseline:
        import oracle
        o = ooi.view(-1, 2).cpu().numpy()
        cores = oracle.threads()

        def run_oracle(ids, nsteps):
            """FP64 oracle outputs f1 of samples ids (all of one model) after
            nsteps steps, and the threads it used."""
            mm = w.models[w.samples[ids[0]].model]
            u0 = np.stack([synth.initial_state(w, w.samples[i]).astype(ndt).astype(np.float64)
                           for i in ids])
            if mm.beta2 > 0:
                # the beta2 > 0 oracle (sparse direct Newton solves, one thread)
                from oracle import b2
                return [b2.solve_b2(u0[j], nsteps, mm.n, mm.delta, mm.kernel, w.samples[i].amp,
                                    mm.sigma, w.samples[i].c_F, mm.beta1, mm.beta2, mm.tau)[2]
                        for j, i in enumerate(ids)], 1
            if mm.boundary:
                # the bounded-domain oracle (numpy, one thread)
                from oracle import volume
                return [volume.solve(u0[j], nsteps, mm.n, mm.delta, mm.kernel,
                                     w.samples[i].amp, mm.sigma, w.samples[i].c_F, mm.beta1,
                                     mm.tau)[2] for j, i in enumerate(ids)], 1
            _, _, f1 = oracle.solve_many(u0, nsteps, mm.n, mm.delta, mm.kernel, mm.sigma,
                                         mm.beta1, mm.tau, [w.samples[i].c_F for i in ids],
                                         [w.samples[i].amp for i in ids], want_states=False)
            return f1, cores

        # one step of sample 0 first: its time decides how large a sample the
        # budget allows
        t = time.perf_counter()
        _, cores = run_oracle([0], 1)
        t1 = time.perf_counter() - t
        n0 = w.models[w.samples[0].model].n
        if t1 * w.nsteps > args.cpu_seconds:
            # not even one whole sample fits: the first steps of sample 0
            ksteps = max(1, min(w.nsteps, int(args.cpu_seconds / max(t1, 1e-9))))
            t = time.perf_counter()
            run_oracle([0], ksteps)
            tcpu = time.perf_counter() - t
            sscpu = n0 ** 2 * ksteps
            sample = ("sample 0 of %d, its first %d of %d steps (%.1f s of oracle time)"
                      % (S, ksteps, w.nsteps, tcpu))
            rel, k = [], 0
        else:
            rel, tcpu, sscpu, k = [], 0.0, 0, 0
            cap = min(args.cpu_samples, S)
            # (the oracle spreads a chunk's samples over its threads, so a
            # chunk of c samples takes about c / threads of c single runs)
            chunk = int(max(1, min(16, args.cpu_seconds * cores / (2 * t1 * w.nsteps))))
            # chunks of consecutive samples (all steps each) until the time
            # budget is spent; the sample count is reported
            while k < cap and tcpu < args.cpu_seconds:
                idx = list(range(k, min(k + chunk, cap)))
                by_model = {}
                for i in idx:
                    by_model.setdefault(w.samples[i].model, []).append(i)
                for mi, ids in by_model.items():
                    t = time.perf_counter()
                    f1, cores = run_oracle(ids, w.nsteps)
                    tcpu += time.perf_counter() - t
                    sscpu += len(ids) * w.models[mi].n ** 2 * w.nsteps
                    for j, i in enumerate(ids):
                        rel.append(abs(o[i, 1] - f1[j]) / abs(f1[j]))
                k = idx[-1] + 1
            sample = ("samples 0..%d of %d, all %d steps each (%.1f s of oracle time)"
                      % (k - 1, S, w.nsteps, tcpu))
        out["cpu_baseline"] = {"value": sscpu / tcpu, "unit": "site-steps/s",
                               "cores": cores, "kind": "oracle", "sample": sample,
                               "host": host_info()}
        if rel:
            out["ooi_rel_err"] = {"max": max(rel), "samples": k, "vs": "FP64 CPU oracle"}
            log("cpu oracle %.3e site-steps/s on %d threads; max OoI rel err %.2e"
                % (sscpu / tcpu, cores, max(rel)))
        else:
            out["ooi_rel_err"] = None  # no whole trajectory fits the CPU budget
            log("cpu oracle %.3e site-steps/s on %d threads (%s)" % (sscpu / tcpu, cores, sample))

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
