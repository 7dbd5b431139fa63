"""Benchmark: semblance evaluations per second of the CMP scan on one MI355X.

Workload (one "step" = one cmp_scan call over the whole batch, i.e. the
energy-coefficient pass plus the scan kernel): 20000 midpoints x fold 60 x
2000 samples at dt = 2 ms (half-offsets U[0, 3000] m, 8 Ricker(30 Hz) events
of random polarity per gather, SNR 2), 201 velocities 1400..5000 m/s, window
15 samples.  Inputs are synthetic (the paper's datasets are not public) and
resident in HBM before the timed region.

Prints one JSON line.  Fields beyond the driver's contract:
  roofline      the scan kernel against the FP32 vector-ALU peak, with the
                paper's per-intersection flop count 12 + 7w (Eq. 2) applied
                to every intersection (12) and to every contributing window
                (7w); time from HIP events around each scan call on the
                stream it runs on;
  cpu_baseline  the FP64 oracle on this host's cores over the first 128
                gathers (same per-evaluation metric);
  crs           the same metric for the 2D-CRS line (512 centrals, 270-trace
                apertures, 21x21x41 parameters, w = 9), one timed call.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 vector peak (published)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cmp_valid_evals(h: np.ndarray, q: np.ndarray, ns: int, dt: float, w: int, ngathers: int) -> int:
    """Exact number of (gather, t0, q, trace) intersections whose window lies on
    the trace, for uniform gathers.  tau(s) = sqrt(s^2 + q h^2/dt^2) grows with s,
    so for each (trace, q) the contributing s form one interval:
    hw <= floor(tau) <= ns - 2 - hw."""
    hw = (w - 1) // 2
    gam = (h.astype(np.float64) ** 2 / (dt * dt))[:, None] * q.astype(np.float64)[None, :]
    top = float(ns - 1 - hw)  # need tau < top
    # largest s with s^2 + gam < top^2
    lim = top * top - gam
    smax = np.where(lim > 0, np.ceil(np.sqrt(np.maximum(lim, 0))) - 1, -1.0)
    smax = np.minimum(smax, ns - 1)
    # smallest s with tau >= hw: s^2 + gam >= hw^2
    low = hw * hw - gam
    smin = np.where(low > 0, np.ceil(np.sqrt(np.maximum(low, 0))), 0.0)
    cnt = np.maximum(smax - smin + 1, 0)
    return int(cnt.sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-crs", action="store_true", help="skip the CRS line measurement")
    ap.add_argument("--gathers", type=int, default=20000, help="(testing only) fewer gathers")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1907_11678_amd as semb

    torch.cuda.set_device(0)
    dev = "cuda"

    # ---- inputs -----------------------------------------------------------
    spec = synth.cmp_large_spec()
    spec.ngathers = args.gathers
    G, F, NS, W = spec.ngathers, spec.fold, spec.ns, 15
    t = time.time()
    host = torch.empty(G * F * NS, dtype=torch.float32).pin_memory()
    h = np.empty(G * F, np.float32)
    synth.cmp_fill(spec, host.numpy(), h)
    log(f"generated {G} gathers in {time.time() - t:.1f} s")
    gs = synth.uniform_cmp_layout(spec, host.numpy(), h)
    jobs = synth.cmp_jobs(gs)
    q_host = synth.cmp_large_grid()
    dg = semb.upload_gathers(host, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset, gs.midpoint,
                             gs.central_x, gs.dt, device=dev)
    dj = semb.upload_jobs(jobs.central, None, None, jobs.out_off, jobs.n_out, device=dev)
    q = torch.from_numpy(q_host).to(dev)
    n = jobs.n_out
    best = torch.empty(n, dtype=torch.int32, device=dev)
    sb = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.float32, device=dev)
    ws = semb.alloc_workspace(dg.nsamples)
    torch.cuda.synchronize()

    evals = G * NS * q_host.size * F
    valid = cmp_valid_evals(h, q_host, NS, gs.dt, W, G) if G == spec.ngathers else None
    flops = 12 * evals + 7 * W * valid

    stream = torch.cuda.current_stream()

    def step():
        semb.cmp_scan(dg, dj, q, W, best, sb, st, ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms_per_step = wall * 1e3 / args.steps
    value = evals / (wall / args.steps)
    k_avg = sum(kms) / len(kms) * 1e-3
    achieved = flops / k_avg / 1e12
    log(f"cmp_large: {ms_per_step:.1f} ms/step (events {[round(x, 1) for x in kms]}), "
        f"{value:.3e} evals/s, valid fraction {valid / evals:.4f}")

    out = {
        "metric": "semblance evals/s (trace-samples x params / s), CMP scan",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "cmp_large: 20000 midpoints x fold 60 x 2000 samples (dt 2 ms), "
                        "201 velocities 1400-5000 m/s, window 15",
            "midpoints": G, "fold": F, "samples": NS, "params": int(q_host.size), "window": W,
            "evals_per_step": evals, "valid_windows_per_step": valid,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": None,
            "kernel": "scan_kernel (CMP, w=15), timed with the energy-coefficient pass it follows",
            "flops_per_launch": flops,
            "avg_launch_ms": k_avg * 1e3,
        },
    }

    # ---- CRS line (context) -------------------------------------------------
    if not args.no_crs:
        del dg, ws
        torch.cuda.empty_cache()
        wl = synth.crs_line()
        cg, cj = wl.gathers, wl.jobs
        dgc = semb.upload_gathers(cg.samples, cg.sample_off, cg.trace_ptr, cg.ns, cg.half_offset,
                                  cg.midpoint, cg.central_x, cg.dt, device=dev)
        djc = semb.upload_jobs(cj.central, cj.apert_ptr, cj.apert_gather, cj.out_off, cj.n_out, device=dev)
        nc = cj.n_out
        cb = torch.empty(nc, dtype=torch.int32, device=dev)
        cs = torch.empty(nc, dtype=torch.float32, device=dev)
        ct = torch.empty(nc, dtype=torch.float32, device=dev)
        wsc = semb.alloc_workspace(dgc.nsamples)
        A, B, qc = (torch.from_numpy(x).to(dev) for x in (wl.grid.A, wl.grid.B, wl.grid.q))
        semb.crs_scan(dgc, djc, A, B, qc, wl.w, cb, cs, ct, wsc, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        semb.crs_scan(dgc, djc, A, B, qc, wl.w, cb, cs, ct, wsc, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        cev = synth.count_evals(cg, cj, wl.grid)
        out["crs"] = {"workload": "crs_line: 512 centrals, +-4 gathers x fold 30 (270 traces), "
                                  "1000 samples (dt 4 ms), 21x21x41 parameters, window 9",
                      "value": cev / (ms * 1e-3), "unit": "evals/s", "ms": ms,
                      "tflops_nominal": cev * (12 + 7 * wl.w) / (ms * 1e-3) / 1e12}
        log(f"crs_line: {ms:.1f} ms, {cev / (ms * 1e-3):.3e} evals/s")

    # ---- CPU oracle baseline ---------------------------------------------
    if not args.no_cpu:
        import oracle
        ng = min(128, G)
        sub = synth.Gathers(gs.samples[:ng * F * NS], gs.sample_off[:ng], gs.trace_ptr[:ng + 1],
                            gs.ns[:ng], gs.half_offset[:ng * F], gs.midpoint[:ng * F],
                            gs.central_x[:ng], gs.dt)
        sj = synth.cmp_jobs(sub)
        nt = oracle.max_threads()
        t = time.perf_counter()
        oracle.scan("cmp", sub, sj, synth.Grid(q=q_host), W, nthreads=nt)
        dtc = time.perf_counter() - t
        cev = ng * NS * q_host.size * F
        out["cpu_baseline"] = {"value": cev / dtc, "unit": "evals/s", "cores": nt, "kind": "oracle",
                               "sample": f"first {ng} of the {G} gathers ({cev:.3e} evals, FP64, "
                                         f"{dtc:.1f} s)"}
        log(f"cpu oracle: {cev / dtc:.3e} evals/s on {nt} threads")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
