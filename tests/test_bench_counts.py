"""Host-side counts that bench.py's roofline figures rest on: the number of
intersections whose window lies on the trace, from closed forms, against a
direct evaluation of the validity rule on every (t0, parameter, trace)."""
from __future__ import annotations

import numpy as np

import bench
import synth


def _brute_valid(gs, jobs, grid, w):
    hw = (w - 1) // 2
    tp = gs.trace_ptr.astype(np.int64)
    A = grid.A.astype(np.float64)[:, None, None, None]
    B = grid.B.astype(np.float64)[None, :, None, None]
    q = grid.q.astype(np.float64)[None, None, :, None]
    valid = total = 0
    for j in range(jobs.njobs):
        c = int(jobs.central[j])
        s = np.arange(int(gs.ns[c]))[None, None, None, :] * gs.dt
        for g in jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]:
            for i in range(tp[g], tp[g + 1]):
                dm = float(gs.midpoint[i]) - float(gs.central_x[c])
                h = float(gs.half_offset[i])
                T = (s + 2 * A * dm) ** 2 + 2 * s * B * dm * dm + q * h * h
                k = np.floor(np.sqrt(np.maximum(T, 0)) / gs.dt)
                ok = (T >= 0) & (k >= hw) & (k + hw + 1 <= int(gs.ns[g]) - 1)
                valid += int(ok.sum())
                total += ok.size
    return valid, total


def test_cmp_valid_count_is_exact():
    wl = synth.cmp_plain(ids=[0, 1, 2])
    gs = wl.gathers
    v, _ = _brute_valid(gs, wl.jobs, wl.grid, wl.w)
    assert bench.cmp_valid_evals(gs.half_offset, wl.grid.q, int(gs.ns[0]), gs.dt, wl.w) == v


def test_crs_valid_count_is_exact():
    wl = synth.crs_line(centrals=[20, 300], grid=synth.crs_coarse_grid())
    v, t = _brute_valid(wl.gathers, wl.jobs, wl.grid, wl.w)
    assert bench.valid_windows(wl.gathers, wl.jobs, wl.grid, wl.w, "crs") == v
    # small chunks: the same count
    assert bench.valid_windows(wl.gathers, wl.jobs, wl.grid, wl.w, "crs", chunk=1000) == v


def test_valid_count_of_uneven_jobs_and_negative_radicands():
    """Uneven fold and ns (neighbours of another length), CRS with B < 0
    making T < 0, w = 1 (where T < 0 alone decides) and w = 9, CMP jobs."""
    from tests import helpers
    rng = np.random.default_rng(5)
    gs = helpers.random_line(rng, 6, fold_range=(1, 4), ns_range=(30, 90), hmax=400.0)
    grid = synth.Grid(A=np.array([-3e-3, 0.0, 2e-3], np.float32), B=np.array([-2e-5, 0.0, 1e-5], np.float32),
                      q=synth.velocity_grid(700, 3000, 4))
    for w in (1, 9):
        jobs = synth.line_crs_jobs(gs, list(range(6)), 2)
        v, _ = _brute_valid(gs, jobs, grid, w)
        assert bench.valid_windows(gs, jobs, grid, w, "crs") == v
        cj = synth.cmp_jobs(gs)
        cg = synth.Grid(A=np.zeros(1, np.float32), B=np.zeros(1, np.float32), q=grid.q)
        v, _ = _brute_valid(gs, synth.line_crs_jobs(gs, list(range(6)), 0), cg, w)
        assert bench.valid_windows(gs, cj, synth.Grid(q=grid.q), w, "cmp") == v


def test_eq2_flops():
    assert bench.eq2_flops(10, 7, 9) == 120 + 7 * 9 * 7


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU; asking for more exits with a message before
    touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_roofline_executed_fractions(tmp_path, monkeypatch):
    """The executed object: rates from a counter record (matching digest) at
    the live kernel time, against the published peaks and the probes'
    ceilings, and the unit nearer its measured ceiling named as binding."""
    from paper_1907_11678_amd import profiling
    rec = {"scan_kernel<0, 15, 0>": {"evals_per_launch": 64e6, "valu_insts_per_wave_eval": 50.0,
                                     "fma_f32_per_wave_eval": 32.0, "lds_load_bytes_per_lane_eval": 80.0,
                                     "lds_busy_fraction": 0.8}}
    path = str(tmp_path / "counters.txt")
    profiling.write_counter_record(rec, path)
    monkeypatch.setattr(bench, "COUNTER_RECORD", path)
    monkeypatch.setattr(bench, "CEILINGS", {"fp32_fma_tflops": 128.0, "lds_read2_tbps": 80.0})
    evals, t_ms = 64_000_000, 1.0  # 1e6 wave-evaluations in 1 ms
    r = bench.roofline("scan_kernel<0, 15, 0>", evals, evals, 15, t_ms, 2.0)
    ex = r["executed"]
    assert r["frac"] == bench.eq2_flops(evals, evals, 15) / 1e-3 / 1e12 / bench.PEAK_FP32_TFLOPS
    assert r["frac_whole_call"] == r["frac"] / 2
    assert abs(ex["fp32_fma_tflops"] - 32.0 * 1e6 * 64 * 2 / 1e-3 / 1e12) < 1e-9        # 4.096
    assert abs(ex["lds_tbps"] - 80.0 * evals / 1e-3 / 1e12) < 1e-9                       # 5.12
    assert abs(ex["valu_issue_frac_of_measured"] - (50.0 * 1e6 / 1e-3) / (128e12 / 128)) < 1e-12  # 0.05
    assert abs(ex["lds_frac_of_measured"] - 5.12 / 80.0) < 1e-12                         # 0.064
    assert ex["binding"] == "lds"
    monkeypatch.setattr(bench, "CEILINGS", {"fp32_fma_tflops": 64.0, "lds_read2_tbps": 80.0})
    assert bench.roofline("scan_kernel<0, 15, 0>", evals, evals, 15, t_ms, None)["executed"]["binding"] == "valu issue"
    # another kernel, or a record of other sources, gives no executed object
    assert bench.roofline("scan_kernel<1, 9, 2>", evals, evals, 9, t_ms, None)["executed"] is None
    monkeypatch.setattr(profiling, "source_digest", lambda: "0000000000000000")
    assert bench.roofline("scan_kernel<0, 15, 0>", evals, evals, 15, t_ms, None)["executed"] is None
