"""Small-case builders and an independent brute-force scan for the oracle pins.

The brute force below is a second, deliberately different implementation of
the definition the oracle follows (Eq. (1) with the 1/M normalisation, the
window of Algorithm 1, the grid search of section 3.2): window samples come
from ``numpy.interp`` at positions tau - hw + j instead of an explicit
floor/fraction split, the semblance is formed from the [M, w] matrix of
corrected window samples, and the pick is ``numpy.argmax`` over the panel.
It is meant for tiny gathers only (pure Python loops).
"""
from __future__ import annotations

import math

import numpy as np

import synth


def ramp(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float32)


def gathers_from_case(case: dict) -> tuple:
    """Build (Gathers, Jobs, Grid, kind, w) from a golden hand case."""
    ns = case["ns"]

    def tr(t):
        return ramp(ns) if t == "ramp8" else np.asarray(t, np.float32)

    if case["kind"] == "cmp":
        traces = np.stack([tr(t) for t in case["traces"]])
        gs = synth.pack_gathers([traces], [case["half_offset"]], [np.zeros(len(traces))], [0.0],
                                case["dt"])
        jobs = synth.cmp_jobs(gs)
        grid = synth.Grid(q=np.asarray(case["q"], np.float32))
    else:
        tl, hl, ml, xc = [], [], [], []
        for g in case["gathers"]:
            tl.append(np.stack([tr(t) for t in g["traces"]]))
            hl.append(g["half_offset"])
            ml.append(np.full(len(g["traces"]), g["x"], np.float32))
            xc.append(g["x"])
        gs = synth.pack_gathers(tl, hl, ml, xc, case["dt"])
        c = case["central"]
        jobs = synth.Jobs(central=np.array([c], np.int32),
                          apert_ptr=np.array([0, gs.ngathers], np.int32),
                          apert_gather=np.arange(gs.ngathers, dtype=np.int32),
                          out_off=np.zeros(1, np.int64), n_out=int(gs.ns[c]))
        grid = synth.Grid(A=np.asarray(case["A"], np.float32), B=np.asarray(case["B"], np.float32),
                          q=np.asarray(case["q"], np.float32))
    return gs, jobs, grid, case["kind"], case["w"]


def brute_panel(kind: str, gs, jobs, grid, w: int):
    """Semblance panel [n_out, n_params], stack panel and contributing counts."""
    hw = (w - 1) // 2
    A = grid.A.astype(np.float64) if kind == "crs" else np.zeros(1)
    B = grid.B.astype(np.float64) if kind == "crs" else np.zeros(1)
    q = grid.q.astype(np.float64)
    npar = A.size * B.size * q.size
    S = np.zeros((jobs.n_out, npar))
    ST = np.zeros((jobs.n_out, npar))
    MM = np.zeros((jobs.n_out, npar), np.int64)
    dt = float(gs.dt)
    for j in range(jobs.njobs):
        c = int(jobs.central[j])
        traces = []
        for gg in jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]:
            gg = int(gg)
            for li in range(int(gs.trace_ptr[gg + 1] - gs.trace_ptr[gg])):
                i = int(gs.trace_ptr[gg]) + li
                dm = float(gs.midpoint[i]) - float(gs.central_x[c]) if kind == "crs" else 0.0
                traces.append((gs.trace(gg, li).astype(np.float64), float(gs.half_offset[i]), dm))
        for s in range(int(gs.ns[c])):
            t0 = s * dt
            row = int(jobs.out_off[j]) + s
            p = 0
            for a_ in A:
                for b_ in B:
                    for q_ in q:
                        rows = []
                        for f, h, dm in traces:
                            T = (t0 + 2 * a_ * dm) ** 2 + 2 * t0 * b_ * dm * dm + q_ * h * h
                            if T < 0:
                                continue
                            tau = math.sqrt(T) / dt
                            first = math.floor(tau) - hw          # first sample read
                            last = first + w                       # last sample read
                            if first < 0 or last > f.size - 1:
                                continue
                            pos = tau - hw + np.arange(w)
                            rows.append(np.interp(pos, np.arange(f.size), f))
                        if rows:
                            V = np.array(rows)
                            D = float((V * V).sum())
                            N = float((V.sum(axis=0) ** 2).sum())
                            S[row, p] = N / (V.shape[0] * D) if D > 0 else 0.0
                            ST[row, p] = float(V.mean())
                            MM[row, p] = V.shape[0]
                        p += 1
    return S, ST, MM


def brute_scan(kind: str, gs, jobs, grid, w: int):
    S, ST, _ = brute_panel(kind, gs, jobs, grid, w)
    best = np.argmax(S, axis=1)
    return best, S[np.arange(S.shape[0]), best], ST[np.arange(S.shape[0]), best], S


def seismic_like(rng: np.random.Generator, fold: int, ns: int, dt: float) -> np.ndarray:
    """Band-limited random traces like the benchmark gathers: white noise
    filtered by a Ricker wavelet of ~10 samples per period, plus white noise
    at a third of its amplitude (an SNR of about 3)."""
    f = 1.0 / (10.0 * dt)
    k = np.arange(-25, 26)
    wav = synth.ricker(k * dt, f)
    x = rng.standard_normal((fold, ns + 50))
    sig = np.stack([np.convolve(r, wav, mode="valid") for r in x])[:, :ns]
    sig /= max(float(np.abs(sig).max()), 1e-30)
    return sig + rng.standard_normal((fold, ns)) * (float(np.sqrt((sig ** 2).mean())) / 3.0)


def random_line(rng: np.random.Generator, ngathers: int, fold_range=(1, 4), ns_range=(12, 40),
                dt=0.004, hmax=300.0, spacing=12.5, zero_trace_prob=0.1, smooth=False):
    """Tiny random gathers on a line (uneven fold and ns, some all-zero traces).
    smooth=False: white Gaussian samples; smooth=True: seismic_like traces."""
    traces, hs, ms = [], [], []
    for g in range(ngathers):
        fold = int(rng.integers(fold_range[0], fold_range[1] + 1))
        ns = int(rng.integers(ns_range[0], ns_range[1] + 1))
        t = (seismic_like(rng, fold, ns, dt) if smooth else rng.standard_normal((fold, ns))).astype(np.float32)
        t[rng.random(fold) < zero_trace_prob] = 0.0
        traces.append(t)
        hs.append(np.sort(rng.uniform(0, hmax, fold)).astype(np.float32))
        ms.append(np.full(fold, spacing * g, np.float32))
    return synth.pack_gathers(traces, hs, ms, [spacing * g for g in range(ngathers)], dt)


def max_dtau_dtheta(gs, jobs, theta) -> np.ndarray:
    """Per output row, the largest |d tau / d theta_k| (samples per unit of A,
    B and q) over the row's aperture traces, from T = (t0 + 2 A dm)^2 +
    2 t0 B dm^2 + q h^2 and tau = sqrt(T) / dt.  Only used to size
    finite-difference steps so that no intersection moves further than a
    chosen fraction of a sample."""
    dt = float(gs.dt)
    out = np.zeros((jobs.n_out, 3))
    for j in range(jobs.njobs):
        c = int(jobs.central[j])
        idx = np.concatenate([np.arange(gs.trace_ptr[g], gs.trace_ptr[g + 1])
                              for g in jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]])
        dm = gs.midpoint[idx].astype(np.float64) - float(gs.central_x[c])
        h = gs.half_offset[idx].astype(np.float64)
        ns = int(gs.ns[c])
        r0 = int(jobs.out_off[j])
        t0 = (np.arange(ns) * dt)[:, None]
        A, B, q = (np.asarray(theta, np.float64)[r0:r0 + ns, k][:, None] for k in range(3))
        T = np.maximum((t0 + 2 * A * dm) ** 2 + 2 * t0 * B * dm * dm + q * h * h, 1e-30)
        den = 2.0 * np.sqrt(T) * dt
        out[r0:r0 + ns, 0] = (np.abs(4 * dm * (t0 + 2 * A * dm)) / den).max(1)
        out[r0:r0 + ns, 1] = (np.abs(2 * t0 * dm * dm) / den).max(1)
        out[r0:r0 + ns, 2] = (h * h / den).max(1)
    return out
