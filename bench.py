"""Benchmark: semblance evaluations per second of the parameter scan on one MI355X.

The step (the timed unit, K of them): one cmp_scan call over the CMP-large
workload -- 20000 midpoints x fold 60 x 2000 samples at dt = 2 ms
(half-offsets U[0, 3000] m, 8 Ricker(30 Hz) events of random polarity per
gather, SNR 2), 201 velocities 1400..5000 m/s, window 15.  A call is the
window-energy pre-pass plus the scan kernel.  Inputs are synthetic (the
paper's datasets are not public) and resident in HBM before the timed region.
value = intersections (midpoints x samples x velocities x traces, every one
counted) / wall-clock seconds per step.

Prints one JSON line.  Fields beyond the step itself:
  roofline      the scan kernel against the FP32 vector-ALU peak.  Work per
                launch = the paper's per-intersection flop count 12 + 7w
                (Eq. 2), 12 on every intersection and 7w on every window that
                lies on its trace (counted exactly in closed form); time =
                HIP events recorded by the library around each scan-kernel
                launch, on the stream it runs on, averaged over the K steps.
                traffic = HBM bytes per launch from the rocprofv3 FETCH_SIZE /
                WRITE_SIZE record in profiles/, or null when that record was
                taken on other kernel sources than the ones built now;
  crs           the 2D-CRS line: 512 centrals, +-4 gathers x fold 30 (270
                traces), 1000 samples at 4 ms, A 21 x B 21 x v 41, window 9;
  batched       4096 gathers of fold 8..120 and 500..2000 samples, 2867 CMP
                jobs (101 velocities, w 11) and 1229 CRS jobs (11 x 11 x 21,
                +-2 gathers, w 9), one persistent launch replayed from a
                captured HIP graph;
  refine        the CRS line again: a coarse 7 x 7 x 11 scan + 8 gradient-
                ascent steps per output sample, captured in one HIP graph,
                against the exhaustive 21 x 21 x 41 scan (time and semblance);
                also from the 4 best local maxima of the coarse panel, the
                best two also shifted in q, 16 steps per start (multistart);
  cpu_baseline  the FP64 oracle on this host's cores over the first gathers
                of the CMP-large workload (same per-intersection metric).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 vector peak (published)
# LDS: 256 bytes per clock per CU, 256 CUs, 2.4 GHz.  The 16-byte read probe
# (semb_probe) measures about 145 TB/s, 236 B per clock at the spec clock, so
# the 128 B per clock of earlier CDNA parts is not this part's figure.
PEAK_LDS_TBPS = 256 * 256 * 2.4e9 / 1e12
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "scan_kernel_cmp_large_traffic.txt")
COUNTER_RECORD = os.path.join(ROOT, "profiles", "scan_kernel_counters.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eq2_flops(evals: int, valid: int, w: int) -> int:
    """Eq. 2 work: 12 per intersection, 7w per window on its trace."""
    return 12 * evals + 7 * w * valid


CEILINGS: dict = {}


def measure_ceilings(semb) -> dict:
    """The probes of the library: plain FP32 and FP64 FMA rates (TFLOP/s),
    v_rsq_f64 results (T/s), LDS read bandwidth (TB/s) with 16-byte reads and
    with the paired 4-byte reads the scan windows use, each the best of 3
    runs of 5 launches."""
    out = {}
    for name, key in (("fma_f32", "fp32_fma_tflops"), ("fma_f64", "fp64_fma_tflops"),
                      ("rsq_f64", "rsq_f64_tps"), ("lds_read", "lds_read_tbps"),
                      ("lds_read2", "lds_read2_tbps")):
        out[key] = max(semb.probe(name, reps=5)[0] for _ in range(3)) / 1e12
    return out


def roofline(kernel: str, evals: int, valid: int, w: int, kernel_ms: float, call_ms: float | None,
             traffic=None, flops: int | None = None, work: str | None = None) -> dict:
    """The roofline object of one leg's dominant kernel.

    achieved = Eq. (2)'s work (12 flops per intersection, 7w per contributing
    window) / the kernel's mean launch time (HIP events around its launches),
    against the FP32 vector peak.  This counts the paper's per-intersection
    work, not the instructions issued: the kernels form a window's energy from
    a precomputed Gram form, so a window costs them 2w + 3 FP32 FMAs, not 7w.
    frac_whole_call divides by the whole call instead (window-energy pre-pass
    included).  With a counter record of the same kernel sources (profiles/),
    also the executed rates from the counters, at the live kernel time:
    FP32 FMA work against the FP32 peak, VALU instructions per CU clock (at
    2.4 GHz), and LDS bytes read against the LDS peak; and, with the ceilings
    the probes measured in this run, VALU issue against the plain-FMA issue
    ceiling and LDS bytes against the measured LDS bandwidth, the larger of
    which names the binding unit."""
    from paper_1907_11678_amd import profiling
    if flops is None:
        flops = eq2_flops(evals, valid, w)
    t = kernel_ms * 1e-3
    ach = flops / t / 1e12
    out = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
           "frac": ach / PEAK_FP32_TFLOPS, "traffic": traffic, "kernel": kernel,
           "work": work or "Eq. (2) flops: 12 per intersection + 7w per contributing window",
           "evals_per_launch": evals, "valid_windows_per_launch": valid, "flops_per_launch": flops,
           "avg_launch_ms": kernel_ms,
           "timed": "avg_launch_ms is the kernel alone; frac_whole_call also counts the window-energy pass"}
    if call_ms:
        out["call_ms"] = call_ms
        out["frac_whole_call"] = flops / (call_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS
    rec = profiling.current_counters(COUNTER_RECORD, kernel)
    if rec is not None:
        we = evals / 64.0
        fma = rec["fma_f32_per_wave_eval"] * we * 64 * 2 / t / 1e12
        lds = rec["lds_load_bytes_per_lane_eval"] * evals / t / 1e12
        issue = rec["valu_insts_per_wave_eval"] * we / (t * 2.4e9 * 256)
        ex = {
            "fp32_fma_tflops": fma, "fp32_fma_frac": fma / PEAK_FP32_TFLOPS,
            "valu_insts_per_wave_eval": rec["valu_insts_per_wave_eval"],
            "valu_insts_per_clk_per_cu": issue,
            "lds_tbps": lds, "lds_peak_tbps": PEAK_LDS_TBPS, "lds_frac": lds / PEAK_LDS_TBPS,
            "lds_busy_fraction": rec.get("lds_busy_fraction"),
            "binding": "lds" if lds / PEAK_LDS_TBPS > issue else "valu issue",
            "source": os.path.relpath(COUNTER_RECORD, ROOT)}
        if CEILINGS:
            # wave-instructions per second: the probe's plain FMAs (2 flops x 64 lanes each)
            # against every VALU instruction the kernel issued
            v_ceil = CEILINGS["fp32_fma_tflops"] * 1e12 / 128.0
            v_rate = rec["valu_insts_per_wave_eval"] * we / t
            ex["valu_issue_frac_of_measured"] = v_rate / v_ceil
            ex["fp32_fma_frac_of_measured"] = fma / CEILINGS["fp32_fma_tflops"]
            # the kernels read their windows with paired 4-byte reads
            ex["lds_frac_of_measured"] = lds / CEILINGS["lds_read2_tbps"]
            ex["binding"] = "lds" if ex["lds_frac_of_measured"] > ex["valu_issue_frac_of_measured"] else \
                "valu issue"
        out["executed"] = ex
    else:
        out["executed"] = None
    return out


def cmp_valid_evals(h: np.ndarray, q: np.ndarray, ns: int, dt: float, w: int) -> int:
    """Exact number of (gather, t0, q, trace) intersections whose window lies on
    the trace, for gathers of ns samples.  tau(s) = sqrt(s^2 + q h^2 / dt^2)
    grows with s, so for each (trace, q) the contributing s form one interval:
    hw <= tau < ns - 1 - hw."""
    hw = (w - 1) // 2
    gam = (h.astype(np.float64) ** 2 / (dt * dt))[:, None] * q.astype(np.float64)[None, :]
    top = float(ns - 1 - hw)
    lim = top * top - gam
    smax = np.where(lim > 0, np.ceil(np.sqrt(np.maximum(lim, 0))) - 1, -1.0)
    smax = np.minimum(smax, ns - 1)
    low = hw * hw - gam
    smin = np.where(low > 0, np.ceil(np.sqrt(np.maximum(low, 0))), 0.0)
    return int(np.maximum(smax - smin + 1, 0).sum())


def _aperture_traces(gs, jobs, kind):
    """Per (job, aperture trace): job index, trace index, the trace's gather."""
    tp = gs.trace_ptr.astype(np.int64)
    if kind == "crs":
        ap = np.asarray(jobs.apert_ptr, np.int64)
        pj = np.repeat(np.arange(jobs.njobs), np.diff(ap))
        pg = np.asarray(jobs.apert_gather, np.int64)[: int(ap[-1])]
    else:
        pj = np.arange(jobs.njobs)
        pg = np.asarray(jobs.central, np.int64)
    cnt = tp[pg + 1] - tp[pg]
    first = np.cumsum(cnt) - cnt
    tj = np.repeat(pj, cnt)
    tg = np.repeat(pg, cnt)
    ti = np.repeat(tp[pg], cnt) + (np.arange(int(cnt.sum())) - np.repeat(first, cnt))
    return tj, ti, tg


def valid_windows(gs, jobs, grid, w: int, kind: str, device: str = "cpu", chunk: int = 1 << 25) -> int:
    """Exact number of (job, t0, parameter, trace) intersections whose window
    lies on its trace.  With u(s) = T/dt^2 = s^2 + beta s + gamma (convex in s;
    CMP: beta = 0, gamma = q h^2/dt^2; CRS: beta = (4 A dm + 2 B dm^2)/dt,
    gamma = (4 A^2 dm^2 + q h^2)/dt^2) a trace contributes at output sample s
    iff hw^2 <= u(s) < (ns_i - 1 - hw)^2, so for each (trace, parameter) the
    count is the number of integers of [0, ns_c - 1] in the root interval of
    the upper level minus those in the root interval of the lower one.  FP64,
    in chunks of (trace, parameter) pairs, on `device` (torch)."""
    import torch
    hw = (w - 1) // 2
    dt = float(gs.dt)
    tj, ti, tg = _aperture_traces(gs, jobs, kind)
    cen = np.asarray(jobs.central, np.int64)[tj]
    if kind == "crs":
        dm = gs.midpoint[ti].astype(np.float64) - gs.central_x[cen].astype(np.float64)
        A = grid.A.astype(np.float64)
        B = grid.B.astype(np.float64)
    else:
        dm = np.zeros(ti.size)
        A = np.zeros(1)
        B = np.zeros(1)
    h = gs.half_offset[ti].astype(np.float64)
    top = (gs.ns[tg].astype(np.float64) - 1 - hw) ** 2
    n = gs.ns[cen].astype(np.float64)
    dev = torch.device(device)
    f64 = dict(dtype=torch.float64, device=dev)
    tA = torch.tensor(A, **f64).view(1, -1, 1, 1)
    tB = torch.tensor(B, **f64).view(1, 1, -1, 1)
    tq = torch.tensor(grid.q.astype(np.float64), **f64).view(1, 1, 1, -1)
    npar = A.size * B.size * grid.q.size
    rows = max(1, chunk // npar)
    total = 0
    for r0 in range(0, ti.size, rows):
        sl = slice(r0, min(r0 + rows, ti.size))
        d = torch.tensor(dm[sl], **f64).view(-1, 1, 1, 1)
        hh = torch.tensor(h[sl], **f64).view(-1, 1, 1, 1)
        nn = torch.tensor(n[sl], **f64).view(-1, 1, 1, 1)
        beta = (4.0 * tA * d + 2.0 * tB * d * d) / dt
        gamma = (4.0 * tA * tA * d * d + tq * hh * hh) / (dt * dt)

        def below(level):  # integers s in [0, n-1] with u(s) < level
            disc = beta * beta - 4.0 * (gamma - level)
            sq = torch.sqrt(torch.clamp(disc, min=0.0))
            lo = torch.clamp(torch.floor((-beta - sq) / 2) + 1, min=0.0)
            hi = torch.minimum(torch.ceil((-beta + sq) / 2) - 1, nn - 1)
            return torch.where(disc > 0, torch.clamp(hi - lo + 1, min=0.0), torch.zeros_like(disc))

        cnt = below(torch.tensor(top[sl], **f64).view(-1, 1, 1, 1)) - below(float(hw * hw))
        total += int(cnt.sum().item())
    return total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cmp-only", action="store_true", help="skip the CRS, batched and refinement legs")
    ap.add_argument("--legs", default="cmp_plain,crs,refine,batched",
                    help="legs to run after the CMP step (comma list of cmp_plain, crs, refine, batched)")
    ap.add_argument("--gathers", type=int, default=20000, help="(testing only) fewer CMP gathers")
    ap.add_argument("--cpu-gathers", type=int, default=384, help="CMP gathers in the CPU oracle sample")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="also measure the paper's Table 1 dataset shapes (CMP and CRS)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (counter calibration)")
    ap.add_argument("--plain-shape", type=int, default=-1, metavar="S",
                    help="(profiling) run the CMP-plain leg in tile shape S without the tuner")
    ap.add_argument("--batch-shape", type=int, default=-1, metavar="BS",
                    help="(profiling) run the batched leg in batch shape BS, split 256, without the tuner")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "there is no multi-GPU path to run.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1907_11678_amd as semb
    from paper_1907_11678_amd import profiling

    torch.cuda.set_device(0)
    dev = "cuda"
    stream = torch.cuda.current_stream()

    # measured ceilings of this part (microbenchmarks), the executed-rate denominators
    CEILINGS.update(measure_ceilings(semb))
    log("ceilings: " + ", ".join(f"{k} {v:.4g}" for k, v in CEILINGS.items()))

    if args.calibrate_copy > 0:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 3 x {nb} bytes")
        del src, dst

    # ---- CMP large: the step ---------------------------------------------
    spec = synth.cmp_large_spec()
    full_size = args.gathers == spec.ngathers
    spec.ngathers = args.gathers
    G, F, NS, W = spec.ngathers, spec.fold, spec.ns, 15
    t = time.time()
    host = torch.empty(G * F * NS, dtype=torch.float32).pin_memory()
    h = np.empty(G * F, np.float32)
    synth.cmp_fill(spec, host.numpy(), h)
    log(f"generated {G} CMP gathers in {time.time() - t:.1f} s")
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
    valid = cmp_valid_evals(h, q_host, NS, gs.dt, W)

    # tile shape: tuned on the first 1024 midpoints (outside the timed region)
    shape, shape_ms = semb.tune_scan(0, dg, dj, q, W, best, sb, st, ws, sample_jobs=1024, reps=2,
                                     stream=stream)
    log(f"tile shape {shape} ({semb.shape_name(shape)}); per-shape ms on the sample {shape_ms}")

    def step():
        semb.cmp_scan(dg, dj, q, W, best, sb, st, ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    with semb.KernelTimer(args.steps) as kt:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = evals / (wall / args.steps)
    k_avg = sum(kt.ms) / len(kt.ms) * 1e-3
    # the record holds the full workload's per-launch bytes: a reduced run has none
    traffic = profiling.current_traffic(TRAFFIC_RECORD) if full_size else None
    rl = roofline(f"scan_kernel<0, 15, {shape}>", evals, valid, W, k_avg * 1e3, ms_per_step, traffic)
    rl["algorithmic_bytes_per_launch"] = 4 * (gs.samples.size + h.size + 3 * n)
    log(f"cmp_large: {ms_per_step:.1f} ms/step, scan kernel {[round(x, 1) for x in kt.ms]} ms, "
        f"{value:.3e} evals/s, valid fraction {valid / evals:.4f}, {rl['achieved']:.1f} TFLOP/s")

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
            "tile_shape": shape, "tile_shape_ms_on_sample": shape_ms,
        },
        "roofline": rl,
        "ceilings": dict(CEILINGS, source="semb_probe microbenchmarks, this run"),
    }
    # PCIe context (never `value`): the samples' host-to-device copy from pinned
    # memory, timed on its own after the step, and the rate a caller who
    # uploads the data for every step would see
    dst = torch.empty_like(dg.samples)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dst.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    h2d = time.perf_counter() - t0
    out["pcie"] = {"h2d_bytes": host.numel() * 4, "h2d_ms": h2d * 1e3,
                   "h2d_gb_per_s": host.numel() * 4 / h2d / 1e9,
                   "evals_per_s_with_upload": evals / (ms_per_step * 1e-3 + h2d)}
    log(f"pcie: {host.numel() * 4 / 1e9:.2f} GB host-to-device in {h2d * 1e3:.1f} ms "
        f"({host.numel() * 4 / h2d / 1e9:.1f} GB/s); with the upload in every step "
        f"{out['pcie']['evals_per_s_with_upload']:.3e} evals/s")
    del dst, dg, ws, host
    torch.cuda.empty_cache()

    legs = set() if args.cmp_only else {x.strip() for x in args.legs.split(",") if x.strip()}
    if "cmp_plain" in legs:
        out["cmp_plain"] = cmp_plain_leg(torch, synth, semb, dev, stream, fixed_shape=args.plain_shape)
    if legs & {"crs", "refine"}:
        out["crs"], fine = crs_leg(torch, synth, semb, dev, stream)
        if "refine" in legs:
            out["refine"] = refine_leg(torch, synth, semb, dev, stream, fine)
        del fine
        torch.cuda.empty_cache()
    if "batched" in legs:
        out["batched"] = batched_leg(torch, synth, semb, dev, stream, args.batch_shape)

    if args.paper_shapes:
        out["paper_shapes"] = paper_shapes_leg(torch, synth, semb, dev, stream)
        torch.cuda.empty_cache()

    # ---- CPU oracle baseline ---------------------------------------------
    if not args.no_cpu:
        import oracle
        ng = min(args.cpu_gathers, G)
        cs = synth.cmp_large_spec()
        cs.ngathers = ng
        samples = np.empty(ng * F * NS, np.float32)
        hh = np.empty(ng * F, np.float32)
        synth.cmp_fill(cs, samples, hh)
        sub = synth.uniform_cmp_layout(cs, samples, hh)
        sj = synth.cmp_jobs(sub)
        nt = oracle.max_threads()
        t = time.perf_counter()
        oracle.scan("cmp", sub, sj, synth.Grid(q=q_host), W, nthreads=nt)
        dtc = time.perf_counter() - t
        cev = ng * NS * q_host.size * F
        out["cpu_baseline"] = {"value": cev / dtc, "unit": "evals/s", "cores": nt, "kind": "oracle",
                               "sample": f"first {ng} of the {G} CMP-large gathers ({cev:.3e} evals, "
                                         f"FP64, {dtc:.1f} s)",
                               "cpu": _cpu_model()}
        log(f"cpu oracle: {cev / dtc:.3e} evals/s on {nt} threads")

    print(json.dumps(out), flush=True)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _timed_replays(torch, g, stream, n):
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for e0, e1 in ev:
        e0.record(stream)
        g.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in ev]


def cmp_plain_leg(torch, synth, semb, dev, stream, launches: int = 20, fixed_shape: int = -1):
    """64 midpoints x fold 24 x 1000 samples (dt 4 ms), 101 velocities, w 11:
    a call of about a tenth of a millisecond, so `launches` back-to-back
    cmp_scan calls are captured in one HIP graph and replayed; time per call =
    replay time / launches."""
    wl = synth.cmp_plain()
    gs, jobs = wl.gathers, wl.jobs
    dg = semb.upload_gathers(gs.samples, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset, gs.midpoint,
                             gs.central_x, gs.dt, device=dev)
    dj = semb.upload_jobs(jobs.central, None, None, jobs.out_off, jobs.n_out, device=dev)
    n = jobs.n_out
    best = torch.empty(n, dtype=torch.int32, device=dev)
    sb = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.float32, device=dev)
    ws = semb.alloc_workspace(dg.nsamples)
    q = torch.from_numpy(wl.grid.q).to(dev)
    s = torch.cuda.Stream()
    if fixed_shape >= 0:
        shape = fixed_shape
        semb.set_scan_shape(0, wl.w, dg, dj, shape)
    else:
        shape, _ = semb.tune_scan(0, dg, dj, q, wl.w, best, sb, st, ws, sample_jobs=64, reps=5, stream=s)
    with semb.KernelTimer(launches) as kt:
        for _ in range(launches):
            semb.cmp_scan(dg, dj, q, wl.w, best, sb, st, ws, stream=s)
        torch.cuda.synchronize()
    k_ms = sorted(kt.ms)[len(kt.ms) // 2]
    s.wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(launches):
            semb.cmp_scan(dg, dj, q, wl.w, best, sb, st, ws, stream=s)
    g.replay()
    torch.cuda.synchronize()
    reps = sorted(_timed_replays(torch, g, torch.cuda.current_stream(), 5))
    call_ms = reps[len(reps) // 2] / launches
    evals = synth.count_evals(gs, jobs, wl.grid)
    valid = cmp_valid_evals(gs.half_offset, wl.grid.q, int(gs.ns[0]), gs.dt, wl.w)
    rl = roofline(f"scan_kernel<0, 11, {shape}>", evals, valid, wl.w, k_ms, call_ms)
    log(f"cmp_plain: {call_ms * 1e3:.1f} us per call in a {launches}-call graph (scan kernel {k_ms * 1e3:.1f} us "
        f"eager), {evals / (call_ms * 1e-3):.3e} evals/s, {rl['achieved']:.1f} TFLOP/s")
    return {"workload": "cmp_plain: 64 midpoints x fold 24 x 1000 samples (dt 4 ms), 101 velocities 1500-4500 m/s, "
                        "window 11",
            "value": evals / (call_ms * 1e-3), "unit": "evals/s", "ms_per_call": call_ms,
            "graph": f"{launches} back-to-back cmp_scan calls per replay, median of 5 replays",
            "evals": evals, "valid_windows": valid, "kernel_ms_eager_median": k_ms, "tile_shape": shape,
            "roofline": rl}


def crs_leg(torch, synth, semb, dev, stream):
    wl = synth.crs_line()
    cg, cj = wl.gathers, wl.jobs
    dg = semb.upload_gathers(cg.samples, cg.sample_off, cg.trace_ptr, cg.ns, cg.half_offset, cg.midpoint,
                             cg.central_x, cg.dt, device=dev)
    dj = semb.upload_jobs(cj.central, cj.apert_ptr, cj.apert_gather, cj.out_off, cj.n_out, device=dev)
    n = cj.n_out
    best = torch.empty(n, dtype=torch.int32, device=dev)
    sb = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.float32, device=dev)
    ws = semb.alloc_workspace(dg.nsamples)
    A, B, q = (torch.from_numpy(x).to(dev) for x in (wl.grid.A, wl.grid.B, wl.grid.q))
    # 128 centrals x 16 sample blocks: four rounds of workgroups on 256 CUs
    shape, _ = semb.tune_scan(1, dg, dj, q, wl.w, best, sb, st, ws, A=A, B=B, sample_jobs=128, reps=1,
                              stream=stream)
    semb.crs_scan(dg, dj, A, B, q, wl.w, best, sb, st, ws, stream=stream)
    torch.cuda.synchronize()
    with semb.KernelTimer(2) as kt:
        t0 = time.perf_counter()
        for _ in range(2):
            semb.crs_scan(dg, dj, A, B, q, wl.w, best, sb, st, ws, stream=stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / 2
    evals = synth.count_evals(cg, cj, wl.grid)
    valid = valid_windows(cg, cj, wl.grid, wl.w, "crs", device=dev)
    k_ms = sum(kt.ms) / len(kt.ms)
    rl = roofline(f"scan_kernel<1, 9, {shape}>", evals, valid, wl.w, k_ms, wall * 1e3)
    log(f"crs_line: {wall * 1e3:.1f} ms/call, scan kernel {k_ms:.1f} ms, {evals / wall:.3e} evals/s, "
        f"valid fraction {valid / evals:.4f}, {rl['achieved']:.1f} TFLOP/s")
    res = {"workload": "crs_line: 512 centrals, +-4 gathers x fold 30 (270 traces), 1000 samples (dt 4 ms), "
                       "21x21x41 parameters, window 9",
           "value": evals / wall, "unit": "evals/s", "ms_per_call": wall * 1e3, "evals": evals,
           "valid_windows": valid, "kernel_ms": k_ms, "tile_shape": shape, "roofline": rl}
    fine = {"wl": wl, "dg": dg, "dj": dj, "s_best": sb.cpu().numpy().astype(np.float64), "ms": wall * 1e3,
            "best": best.cpu().numpy()}
    return res, fine


def refine_leg(torch, synth, semb, dev, stream, fine):
    wl, dg, dj = fine["wl"], fine["dg"], fine["dj"]
    n = wl.jobs.n_out
    coarse = synth.crs_coarse_grid()
    A, B, q = (torch.from_numpy(x).to(dev) for x in (coarse.A, coarse.B, coarse.q))
    best = torch.empty(n, dtype=torch.int32, device=dev)
    s0 = torch.empty(n, device=dev)
    st0 = torch.empty(n, device=dev)
    theta = torch.empty((n, 3), device=dev)
    S = torch.empty(n, device=dev)
    st = torch.empty(n, device=dev)
    ws = semb.alloc_workspace(dg.nsamples)

    def cell(v):
        v = np.asarray(v, np.float64)
        return float((v.max() - v.min()) / max(v.size - 1, 1))

    scale = (cell(coarse.A), cell(coarse.B), cell(coarse.q))
    lo = (float(coarse.A.min()), float(coarse.B.min()), float(coarse.q.min()))
    hi = (float(coarse.A.max()), float(coarse.B.max()), float(coarse.q.max()))

    s = torch.cuda.Stream()
    shape, _ = semb.tune_scan(1, dg, dj, q, wl.w, best, s0, st0, ws, A=A, B=B, sample_jobs=128, reps=2, stream=s)
    # the coarse scan's kernel time, eager (it is most of the graph below)
    with semb.KernelTimer(3) as kt:
        for _ in range(3):
            semb.crs_scan(dg, dj, A, B, q, wl.w, best, s0, st0, ws, stream=s)
        torch.cuda.synchronize()
    coarse_ms = sum(kt.ms) / len(kt.ms)
    ev_coarse = synth.count_evals(wl.gathers, wl.jobs, coarse)
    val_coarse = valid_windows(wl.gathers, wl.jobs, coarse, wl.w, "crs", device=dev)

    def run():
        semb.crs_scan(dg, dj, A, B, q, wl.w, best, s0, st0, ws, stream=s)
        semb.theta_from_best(best, q, theta, A=A, B=B, stream=s)
        semb.refine(dg, dj, 1, theta, wl.w, S, st, steps=8, eta0=0.5, scale=scale, lo=lo, hi=hi, stream=s)

    s.wait_stream(stream)
    with torch.cuda.stream(s):
        run()
    stream.wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run()
    g.replay()
    torch.cuda.synchronize()
    ms = _timed_replays(torch, g, torch.cuda.current_stream(), 3)
    t_ms = sorted(ms)[1]
    Sr = S.cpu().numpy().astype(np.float64)
    Sf = fine["s_best"]
    sel = Sf > 0.1
    d = (Sr - Sf)[sel]
    res = {"workload": "crs_line data, coarse 7x7x11 scan + 8 ascent steps per output sample, one HIP graph",
           "ms": t_ms, "coarse_tile_shape": shape, "exhaustive_ms": fine["ms"], "speedup_vs_exhaustive": fine["ms"] / t_ms,
           "roofline": roofline(f"scan_kernel<1, 9, {shape}>", ev_coarse, val_coarse, wl.w, coarse_ms, None),
           "coarse_scan_share_of_graph": coarse_ms / t_ms,
           "rows_compared": int(sel.sum()),
           "s_gap_median": float(np.median(d)), "s_gap_p5": float(np.percentile(d, 5)),
           "frac_at_least_fine": float((d >= -1e-4).mean()),
           "mean_s_coarse": float(s0.cpu().numpy().mean()), "mean_s_refined": float(Sr.mean()),
           "mean_s_fine": float(Sf.mean())}
    log(f"refine: {t_ms:.1f} ms vs exhaustive {fine['ms']:.1f} ms; S gap median {res['s_gap_median']:+.4f}, "
        f"p5 {res['s_gap_p5']:+.4f}, >= fine-1e-4 on {res['frac_at_least_fine']:.3f} of {int(sel.sum())} rows")

    # multi-start: the coarse scan's panel, its best local maxima per row, each
    # also shifted along q, as starts (the library's rule); the best of all
    # ascents; one graph
    K, STARTS, STEPS_MS = semb.MULTISTART_PEAKS, semb.MULTISTART_STARTS, semb.MULTISTART_STEPS
    NS = len(STARTS)
    panel = torch.empty((n, coarse.n), device=dev)
    theta_k = torch.empty((NS, n, 3), device=dev)
    s_k = torch.empty((NS, n), device=dev)
    st_k = torch.empty((NS, n), device=dev)
    best_k = torch.empty((K, n), dtype=torch.int32, device=dev)
    peak_s = torch.empty((K, n), device=dev)
    Sm = torch.empty(n, device=dev)
    stm = torch.empty(n, device=dev)
    thm = torch.empty((n, 3), device=dev)

    def run_ms():
        semb.crs_scan(dg, dj, A, B, q, wl.w, best, s0, st0, ws, panel=panel, stream=s)
        semb.refine_multistart(dg, dj, 1, panel, A, B, q, wl.w, K, theta_k, s_k, st_k, best_k, peak_s, Sm, stm,
                               thm, steps=STEPS_MS, eta0=0.5, scale=scale, lo=lo, hi=hi, stream=s, starts=STARTS)

    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run_ms()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gm = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gm, stream=s):
        run_ms()
    gm.replay()
    torch.cuda.synchronize()
    m_ms = sorted(_timed_replays(torch, gm, torch.cuda.current_stream(), 3))[1]
    dm_ = (Sm.cpu().numpy().astype(np.float64) - Sf)[sel]
    # the rows short of the fine grid by more than 0.01: how far is the fine
    # grid's optimum from the nearest start, in coarse cells (max over A, B, q)?
    thf = torch.empty((n, 3), device=dev)
    semb.theta_from_best(torch.from_numpy(fine["best"]).to(dev), torch.from_numpy(wl.grid.q).to(dev), thf,
                         A=torch.from_numpy(wl.grid.A).to(dev), B=torch.from_numpy(wl.grid.B).to(dev))
    th_starts = theta_k.clone()
    for i, (k, off) in enumerate(STARTS):  # the starts themselves (theta_k now holds the refined ones)
        semb.theta_from_best(best_k[k], q, th_starts[i], A=A, B=B)
        if any(off):
            semb.theta_shift(th_starts[i], [off[c] * scale[c] for c in range(3)], lo, hi)
    torch.cuda.synchronize()
    sc = np.asarray(scale, np.float64)
    dist = np.min(np.abs(th_starts.cpu().numpy().astype(np.float64) - thf.cpu().numpy()[None]) / sc, axis=0).max(1)
    short = (Sm.cpu().numpy().astype(np.float64) - Sf < -0.01) & sel
    res["multistart"] = {"peaks": K, "starts_peak_and_offset_in_coarse_cells": [[k, list(o)] for k, o in STARTS],
                         "starts": NS,
                           "steps": STEPS_MS, "ms": m_ms, "speedup_vs_exhaustive": fine["ms"] / m_ms,
                           "s_gap_median": float(np.median(dm_)), "s_gap_p5": float(np.percentile(dm_, 5)),
                           "s_gap_mean": float(dm_.mean()), "frac_at_least_fine": float((dm_ >= -1e-4).mean()),
                           "rows_short_by_0.01": int(short.sum()),
                           "short_rows_with_no_start_within_1_coarse_cell": int((short & (dist > 1.0)).sum())}
    res["s_gap_mean"] = float(d.mean())
    log(f"refine, {NS} starts from {K} peaks x {STEPS_MS} steps: {m_ms:.1f} ms; S gap median {np.median(dm_):+.4f}, "
        f"mean {dm_.mean():+.4f}, p5 {np.percentile(dm_, 5):+.4f}, >= fine-1e-4 on {(dm_ >= -1e-4).mean():.3f}; "
        f"{int(short.sum())} rows short by > 0.01, {int((short & (dist > 1.0)).sum())} of them with no start "
        f"within one coarse cell of the fine grid's optimum")
    return res


def batched_leg(torch, synth, semb, dev, stream, fixed_shape: int = -1):
    t = time.time()
    bw = synth.batched_line()
    log(f"generated the batched line in {time.time() - t:.1f} s")
    gs, jobs = bw.gathers, bw.jobs
    dg = semb.upload_gathers(gs.samples, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset, gs.midpoint,
                             gs.central_x, gs.dt, device=dev)
    dj = semb.upload_jobs(jobs.central, jobs.apert_ptr, jobs.apert_gather, jobs.out_off, jobs.n_out, device=dev)
    kind = torch.from_numpy(bw.kind).to(dev)
    qc = torch.from_numpy(bw.grid_cmp.q).to(dev)
    A, B, qr = (torch.from_numpy(x).to(dev) for x in (bw.grid_crs.A, bw.grid_crs.B, bw.grid_crs.q))
    n = jobs.n_out
    best = torch.empty(n, dtype=torch.int32, device=dev)
    sb = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.float32, device=dev)
    # batch tile shape and parameter split, tuned on the first 512 jobs (outside the timed region)
    t = time.time()
    if fixed_shape >= 0:
        shape, split, tune_ms = fixed_shape, 256, {}
        semb.set_batch_choice(bw.w_cmp, bw.w_crs, dg, dj, shape, split)
    else:
        shape, split, tune_ms = semb.tune_batch(dg, dj, bw.kind, kind, qc, bw.w_cmp, A, B, qr, bw.w_crs,
                                                jobs.central, jobs.apert_ptr, jobs.apert_gather, gs.ns,
                                                gs.trace_ptr, best, sb, st, splits=(256, 1024), reps=1,
                                                sample_jobs=512, stream=stream)
    log(f"batch tile shape {shape} ({semb.batch_shape_name(shape)}), split {split}; ms per shape on the "
        f"512-job sample {tune_ms} ({time.time() - t:.1f} s)")
    tiles, ng, npart = semb.batch_plan(bw.kind, jobs.central, jobs.apert_ptr, jobs.apert_gather, gs.ns,
                                       gs.trace_ptr, bw.grid_cmp.n, bw.grid_crs.n, split)
    dtiles = torch.from_numpy(tiles).to(dev)
    ws = semb.alloc_batch_workspace(dg.nsamples, bw.w_cmp, bw.w_crs, ng, npart)
    s = torch.cuda.Stream()

    def run():
        semb.scan_batch(dg, dj, kind, qc, bw.w_cmp, A, B, qr, bw.w_crs, dtiles, ng, npart, best, sb, st, ws,
                        stream=s)

    s.wait_stream(stream)
    with semb.KernelTimer(2) as kt:
        with torch.cuda.stream(s):
            run()
            run()
        torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run()
    g.replay()
    torch.cuda.synchronize()
    ms = _timed_replays(torch, g, torch.cuda.current_stream(), 3)
    t_ms = sorted(ms)[1]
    ev_c = synth.count_evals(gs, bw.subset(0), bw.grid_cmp)
    ev_r = synth.count_evals(gs, bw.subset(1), bw.grid_crs)
    ev = ev_c + ev_r
    va_c = valid_windows(gs, bw.subset(0), bw.grid_cmp, bw.w_cmp, "cmp", device=dev)
    va_r = valid_windows(gs, bw.subset(1), bw.grid_crs, bw.w_crs, "crs", device=dev)
    k_ms = sum(kt.ms) / len(kt.ms)
    # one launch does both kinds: Eq. (2) work of each at its own window
    fl = eq2_flops(ev_c, va_c, bw.w_cmp) + eq2_flops(ev_r, va_r, bw.w_crs)
    rl = roofline(f"batch_kernel<{bw.w_cmp}, {bw.w_crs}, {shape}>", ev, va_c + va_r, 0, k_ms, t_ms, flops=fl,
                  work="Eq. (2) flops: 12 per intersection + 7w per contributing window, w 11 for the CMP "
                       "jobs and 9 for the CRS jobs")
    log(f"batched: graph {t_ms:.1f} ms (kernel {k_ms:.1f} ms eager), {ev / (t_ms * 1e-3):.3e} evals/s, "
        f"{tiles.shape[0]} tiles, {rl['achieved']:.1f} TFLOP/s")
    return {"workload": "batched_line: 4096 gathers, fold 8-120, 500-2000 samples (dt 4 ms); 2867 CMP jobs "
                        "(101 velocities, w 11) + 1229 CRS jobs (11x11x21, +-2 gathers, w 9); one persistent "
                        "launch in a HIP graph",
            "value": ev / (t_ms * 1e-3), "unit": "evals/s", "graph_ms": t_ms, "kernel_ms_eager": k_ms,
            "evals": ev, "evals_cmp": ev_c, "evals_crs": ev_r, "valid_windows_cmp": va_c, "valid_windows_crs": va_r,
            "tiles": int(tiles.shape[0]), "batch_shape": shape, "split_params": split,
            "tuning_ms_per_shape_on_512_jobs": {str(k): v for k, v in tune_ms.items()}, "roofline": rl}


def _scan_rate(torch, semb, wl, dev, stream, tune_jobs):
    """Tuned shape, then 3 timed calls of the scan over workload wl: evals/s and
    the scan kernel's mean time."""
    import synth
    gs, jobs = wl.gathers, wl.jobs
    crs = wl.kind == "crs"
    dg = semb.upload_gathers(gs.samples, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset, gs.midpoint,
                             gs.central_x, gs.dt, device=dev)
    dj = semb.upload_jobs(jobs.central, jobs.apert_ptr if crs else None, jobs.apert_gather if crs else None,
                          jobs.out_off, jobs.n_out, device=dev)
    n = jobs.n_out
    best = torch.empty(n, dtype=torch.int32, device=dev)
    sb = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.float32, device=dev)
    ws = semb.alloc_workspace(dg.nsamples)
    q = torch.from_numpy(wl.grid.q).to(dev)
    A = torch.from_numpy(wl.grid.A).to(dev) if crs else None
    B = torch.from_numpy(wl.grid.B).to(dev) if crs else None
    shape, _ = semb.tune_scan(1 if crs else 0, dg, dj, q, wl.w, best, sb, st, ws, A=A, B=B,
                              sample_jobs=tune_jobs, reps=1, stream=stream)

    def call():
        if crs:
            semb.crs_scan(dg, dj, A, B, q, wl.w, best, sb, st, ws, stream=stream)
        else:
            semb.cmp_scan(dg, dj, q, wl.w, best, sb, st, ws, stream=stream)

    call()
    torch.cuda.synchronize()
    with semb.KernelTimer(3) as kt:
        t0 = time.perf_counter()
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / 3
    evals = synth.count_evals(gs, jobs, wl.grid)
    return {"evals": evals, "value": evals / wall, "ms_per_call": wall * 1e3,
            "kernel_ms": sum(kt.ms) / len(kt.ms), "tile_shape": shape}


def paper_shapes_leg(torch, synth, semb, dev, stream):
    """The eight dataset shapes of the paper's Table 1 (fold 60 / 1000, 550 /
    1650 samples; the "dt" column read as the window, 19 or 17 samples):
    CMP over a line of gathers (101 velocities) and CRS over +-2 gathers with
    the coarse 7 x 7 x 11 grid.  The numbers of gathers are chosen to keep each
    call in the tens to hundreds of milliseconds (the paper's datasets hold
    61,628 to 2,648,430 CDPs)."""
    cmp_gathers = {(60, 550): 3000, (60, 1650): 1200, (1000, 550): 360, (1000, 1650): 240}
    crs_centrals = {(60, 550): 256, (60, 1650): 128, (1000, 550): 128, (1000, 1650): 64}
    import dataclasses
    res = {}
    k = 2
    for d0 in (1, 3, 5, 7):  # datasets d0 and d0 + 1 share fold, ns and data
        fold, ns, _ = synth.PAPER_DATASETS[d0]
        t = time.time()
        wl0 = synth.paper_shape(d0, cmp_gathers[(fold, ns)])
        nc = crs_centrals[(fold, ns)]
        wc0 = synth.paper_shape(d0, nc + 2 * k, kind="crs", half_aperture=k)
        log(f"generated the fold {fold} x {ns} lines in {time.time() - t:.1f} s")
        for d in (d0, d0 + 1):
            w = synth.paper_window(synth.PAPER_DATASETS[d][2])
            wl = dataclasses.replace(wl0, w=w)
            wc = dataclasses.replace(wc0, w=w)
            r = _scan_rate(torch, semb, wl, dev, stream, tune_jobs=256)
            rc = _scan_rate(torch, semb, wc, dev, stream, tune_jobs=max(16, nc // 2))
            res[f"data{d}"] = {"fold": fold, "samples": ns, "window": w, "cmp_gathers": wl.jobs.njobs,
                               "cmp": r, "crs_centrals": wc.jobs.njobs, "crs": rc}
            log(f"paper data{d} (fold {fold}, ns {ns}, w {w}): CMP {r['value']:.3e} evals/s, "
                f"CRS {rc['value']:.3e} evals/s")
        del wl0, wc0, wl, wc
        torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
