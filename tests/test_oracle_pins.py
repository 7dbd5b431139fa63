"""Pins of the FP64 oracle against things other than itself.

- hand-derived values (tests/golden/hand_cases.json, each with its derivation);
- closed forms at zero moveout and on ramp traces (interpolation of a linear
  function is exact);
- integer-aligned single-event Ricker gathers (S = 1 at the generating
  parameter, which the pick recovers) for CMP and CRS;
- invariants: 0 <= S <= 1, scale and permutation invariance, CRS with
  A = B = 0 equals CMP;
- an independent brute force (tests/helpers.py) on tiny random gathers;
- central finite differences for the analytic gradient;
- and a mutation check: modified copies of the oracle (a dropped term, a sign,
  an index, a transposed operand ...) must each fail at least one pin.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import helpers

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "hand_cases.json")))["cases"]


# --------------------------------------------------------------------------
# pin functions, each returning a list of failure messages (so that the
# mutation check can run them against a modified oracle)
# --------------------------------------------------------------------------
def pin_hand_cases(lib=None):
    bad = []
    for case in CASES:
        gs, jobs, grid, kind, w = helpers.gathers_from_case(case)
        r = oracle.scan(kind, gs, jobs, grid, w, library=lib)
        s = case["s"]
        want = case["S_num"] / case["S_den"]
        if abs(r.s_best[s] - want) > 1e-12:
            bad.append(f"{case['name']}: S {r.s_best[s]!r} != {want!r}")
        if abs(r.stack[s] - case["stack"]) > 1e-12:
            bad.append(f"{case['name']}: stack {r.stack[s]!r} != {case['stack']!r}")
        th = oracle.theta_of(grid, np.zeros(jobs.n_out, np.int64), kind)
        _, _, m, _ = oracle.point(kind, gs, jobs, th, w, library=lib)
        if m[s] != case["M"]:
            bad.append(f"{case['name']}: M {m[s]} != {case['M']}")
    return bad


def pin_zero_moveout_closed_form(lib=None):
    """h = 0: every trace uses the same window; traces alpha_i * g give
    S = (sum alpha)^2 / (M sum alpha^2) and stack = mean(alpha) * mean(window)."""
    bad = []
    rng = np.random.default_rng(5)
    for trial in range(6):
        M = int(rng.integers(1, 7))
        ns, w, dt = 40, [1, 3, 5, 7, 9, 11][trial], 0.004
        g = rng.standard_normal(ns)
        alpha = rng.uniform(-2, 2, M)
        alpha[0] = 1.0 + abs(alpha[0])
        traces = (alpha[:, None] * g[None, :]).astype(np.float32)
        gs = synth.pack_gathers([traces], [np.zeros(M)], [np.zeros(M)], [0.0], dt)
        jobs = synth.cmp_jobs(gs)
        grid = synth.Grid(q=np.array([2e-7], np.float32))
        r = oracle.scan("cmp", gs, jobs, grid, w, library=lib)
        hw = (w - 1) // 2
        a32 = traces[:, 0] / g[0].astype(np.float32)  # the alphas as stored in float32
        for s in range(hw, ns - hw - 1):
            win = traces[:, s - hw:s - hw + w].astype(np.float64)
            if not np.any(win):
                continue
            want = a32.astype(np.float64).sum() ** 2 / (M * (a32.astype(np.float64) ** 2).sum())
            # the float32 storage of alpha_i * g breaks exact proportionality slightly
            if abs(r.s_best[s] - want) > 1e-6:
                bad.append(f"zero moveout trial {trial} s={s}: {r.s_best[s]} vs {want}")
                break
            if abs(r.stack[s] - win.mean()) > 1e-12:
                bad.append(f"zero moveout stack trial {trial} s={s}")
                break
    return bad


def pin_ramp_traces(lib=None):
    """f_i[n] = a_i + b_i n: every window sample is a_i + b_i (tau_i - hw + j)
    exactly, so U, D, S and the stack have closed forms."""
    bad = []
    rng = np.random.default_rng(11)
    ns, w, dt = 200, 7, 0.004
    hw = 3
    M = 5
    a = rng.uniform(-1, 1, M)
    b = rng.uniform(-0.01, 0.01, M)
    traces = (a[:, None] + b[:, None] * np.arange(ns)[None, :]).astype(np.float32)
    h = np.sort(rng.uniform(0, 400, M)).astype(np.float32)
    gs = synth.pack_gathers([traces], [h], [np.zeros(M)], [0.0], dt)
    jobs = synth.cmp_jobs(gs)
    q = synth.velocity_grid(1500, 3000, 4)
    r = oracle.scan("cmp", gs, jobs, synth.Grid(q=q), w, panel=True, library=lib)
    f64 = traces.astype(np.float64)
    for s in range(0, ns, 7):
        for iq, qq in enumerate(q.astype(np.float64)):
            tau = np.sqrt((s * gs.dt) ** 2 + qq * h.astype(np.float64) ** 2) / gs.dt
            k = np.floor(tau)
            ok = (k - hw >= 0) & (k - hw + w <= ns - 1)
            if not ok.any():
                want = 0.0
            else:
                # the stored float32 ramp is a_i' + b_i' n only up to rounding;
                # use the exact line through the two samples around each window
                V = []
                for i in np.nonzero(ok)[0]:
                    pos = tau[i] - hw + np.arange(w)
                    n0 = np.floor(pos).astype(int)
                    lo, hi = f64[i, n0], f64[i, n0 + 1]
                    V.append(lo + (pos - n0) * (hi - lo))
                V = np.array(V)
                want = (V.sum(0) ** 2).sum() / (V.shape[0] * (V * V).sum())
            got = r.panel[s, iq]
            if abs(got - want) > 1e-11:
                bad.append(f"ramp s={s} iq={iq}: {got} vs {want}")
                return bad
    return bad


def _aligned_cmp_gather(v_true, t0e, dt, ns, n_shift, f_peak=25.0, amp=0.8):
    """Traces whose event reaches sample s_e + n_i exactly at q* = 4/v*^2."""
    s_e = int(round(t0e / dt))
    t0e = s_e * dt
    h = (v_true / 2.0) * np.sqrt((t0e + np.asarray(n_shift) * dt) ** 2 - t0e ** 2)
    n = np.arange(ns)
    traces = np.stack([amp * synth.ricker((n - s_e - k) * dt, f_peak) for k in n_shift])
    return traces.astype(np.float32), h.astype(np.float32), s_e


def pin_aligned_ricker_cmp(lib=None):
    bad = []
    dt, ns, w = 0.004, 600, 11
    v_true = 2500.0
    traces, h, s_e = _aligned_cmp_gather(v_true, 1.0, dt, ns, [0, 3, 7, 12, 20, 31, 45, 60])
    gs = synth.pack_gathers([traces], [h], [np.zeros(len(h))], [0.0], dt)
    jobs = synth.cmp_jobs(gs)
    v = np.array([2300, 2400, 2500, 2600, 2700], np.float64)
    q = (4.0 / v ** 2).astype(np.float32)
    r = oracle.scan("cmp", gs, jobs, synth.Grid(q=q), w, panel=True, library=lib)
    if abs(r.panel[s_e, 2] - 1.0) > 1e-6:
        bad.append(f"aligned CMP: S at the true velocity {r.panel[s_e, 2]}")
    if r.best[s_e] != 2:
        bad.append(f"aligned CMP: pick {r.best[s_e]} != 2")
    if not (r.panel[s_e, [0, 1, 3, 4]] < 1.0 - 1e-4).all():
        bad.append("aligned CMP: neighbours not below the true velocity")
    if abs(r.stack[s_e] - traces[0, s_e - 5:s_e + 6].astype(np.float64).mean()) > 1e-6:
        bad.append("aligned CMP: stack is not the windowed mean of the wavelet")
    return bad


def pin_aligned_ricker_crs(lib=None):
    """CRS: traces of 5 gathers (dm = -25..25 m) aligned for (A*, B*, q*)."""
    bad = []
    dt, ns, w = 0.004, 500, 9
    A_t, B_t, v_t = 2e-4, 4e-8, 2500.0
    q_t = 4.0 / v_t ** 2
    s_e = 200
    t0 = s_e * dt
    n = np.arange(ns)
    tl, hl, ml, xc = [], [], [], []
    for g, dm in enumerate([-25.0, -12.5, 0.0, 12.5, 25.0]):
        y = t0 + 2 * A_t * dm
        base = max(2, int(math.ceil((y - t0) / dt)) + 2)
        shifts = np.array([0, 4, 9, 15, 24]) + base + (g % 2)
        # (t0 + n dt)^2 = y^2 + 2 t0 B dm^2 + q h^2  ->  h
        h2 = ((t0 + shifts * dt) ** 2 - y * y - 2 * t0 * B_t * dm * dm) / q_t
        assert (h2 > 0).all()
        h = np.sqrt(h2)
        tl.append(np.stack([0.7 * synth.ricker((n - s_e - k) * dt, 25.0) for k in shifts]).astype(np.float32))
        hl.append(h.astype(np.float32))
        ml.append(np.full(len(h), 100.0 + dm, np.float32))
        xc.append(100.0 + dm)
    gs = synth.pack_gathers(tl, hl, ml, xc, dt)
    jobs = synth.Jobs(central=np.array([2], np.int32), apert_ptr=np.array([0, 5], np.int32),
                      apert_gather=np.arange(5, dtype=np.int32), out_off=np.zeros(1, np.int64),
                      n_out=ns)
    grid = synth.Grid(A=np.array([0.0, 2e-4, 4e-4], np.float32),
                      B=np.array([0.0, 4e-8, 8e-8], np.float32),
                      q=np.array([4.0 / 2300 ** 2, q_t, 4.0 / 2700 ** 2], np.float32))
    r = oracle.scan("crs", gs, jobs, grid, w, panel=True, library=lib)
    true_flat = (1 * 3 + 1) * 3 + 1
    if abs(r.panel[s_e, true_flat] - 1.0) > 1e-5:
        bad.append(f"aligned CRS: S at the true parameters {r.panel[s_e, true_flat]}")
    if r.best[s_e] != true_flat:
        bad.append(f"aligned CRS: pick {r.best[s_e]} != {true_flat}")
    return bad


def pin_tie_break(lib=None):
    """Equal semblance: the smallest flat index wins (duplicated grid values,
    and all-zero data where every S is 0)."""
    bad = []
    rng = np.random.default_rng(3)
    traces = rng.standard_normal((4, 60)).astype(np.float32)
    h = np.array([0, 50, 100, 150], np.float32)
    gs = synth.pack_gathers([traces], [h], [np.zeros(4)], [0.0], 0.004)
    jobs = synth.cmp_jobs(gs)
    q = np.array([1e-6, 1e-6, 1e-6], np.float32)
    r = oracle.scan("cmp", gs, jobs, synth.Grid(q=q), 5, library=lib)
    if (r.best != 0).any():
        bad.append("tie-break: duplicated parameters did not pick index 0")
    gz = synth.pack_gathers([np.zeros((3, 40), np.float32)], [h[:3]], [np.zeros(3)], [0.0], 0.004)
    r = oracle.scan("cmp", gz, synth.cmp_jobs(gz), synth.Grid(q=synth.velocity_grid(1500, 3000, 5)),
                    5, library=lib)
    if (r.best != 0).any() or (r.s_best != 0).any() or (r.stack != 0).any():
        bad.append("all-zero data: expected S = 0, stack = 0 and pick 0")
    return bad


def _tiny_line(seed):
    rng = np.random.default_rng(seed)
    gs = helpers.random_line(rng, 5, fold_range=(1, 3), ns_range=(14, 30), dt=0.004, hmax=200.0,
                             spacing=12.5)
    return gs


def _gap_vs_panel(gap, panel, name):
    """The oracle's gap is the best S minus the second-best S of any other
    parameter (equal values count twice, so a tie gives 0), from a panel the
    brute force computed; infinite with a single parameter."""
    if panel.shape[1] == 1:
        return [] if np.isinf(gap).all() else [f"{name}: gap of a one-parameter grid is not infinite"]
    top = np.sort(panel, axis=1)
    want = top[:, -1] - top[:, -2]
    err = np.abs(gap - want).max(initial=0.0)
    return [f"{name}: gap differs from the brute force's top two by {err}"] if err > 1e-12 else []


def pin_brute_force(lib=None, seeds=(0, 1, 2)):
    bad = []
    for seed in seeds:
        gs = _tiny_line(seed)
        # CMP on every gather
        jobs = synth.cmp_jobs(gs)
        grid = synth.Grid(q=synth.velocity_grid(600, 2400, 5))
        for w in (1, 3, 5):
            r = oracle.scan("cmp", gs, jobs, grid, w, panel=True, library=lib)
            bb, bs, bst, bp = helpers.brute_scan("cmp", gs, jobs, grid, w)
            if np.abs(r.panel - bp).max() > 1e-12:
                bad.append(f"brute CMP seed {seed} w {w}: panel differs by {np.abs(r.panel - bp).max()}")
            bad += _gap_vs_panel(r.gap, bp, f"brute CMP seed {seed} w {w}")
            big = r.gap > 1e-9
            if (r.best[big] != bb[big]).any() or np.abs(r.stack - bst).max() > 1e-12:
                bad.append(f"brute CMP seed {seed} w {w}: pick or stack differs")
        # CRS with a +-1 aperture, parameters that make some T negative
        jobs = synth.line_crs_jobs(gs, [1, 2, 3], 1)
        grid = synth.Grid(A=np.array([-4e-3, 0.0, 3e-3], np.float32),
                          B=np.array([-4e-5, 0.0, 2e-5], np.float32),
                          q=synth.velocity_grid(600, 2400, 3))
        for w in (1, 3):
            r = oracle.scan("crs", gs, jobs, grid, w, panel=True, library=lib)
            bb, bs, bst, bp = helpers.brute_scan("crs", gs, jobs, grid, w)
            if np.abs(r.panel - bp).max() > 1e-12:
                bad.append(f"brute CRS seed {seed} w {w}: panel differs by {np.abs(r.panel - bp).max()}")
            bad += _gap_vs_panel(r.gap, bp, f"brute CRS seed {seed} w {w}")
            big = r.gap > 1e-9
            if (r.best[big] != bb[big]).any() or np.abs(r.stack - bst).max() > 1e-12:
                bad.append(f"brute CRS seed {seed} w {w}: pick or stack differs")
    return bad


def _grad_case():
    """A small CRS case with smooth (band-limited) traces."""
    rng = np.random.default_rng(21)
    dt, ns = 0.004, 300
    n = np.arange(ns)
    tl, hl, ml = [], [], []
    for g in range(3):
        tr = []
        for i in range(4):
            t = 0.05 * rng.standard_normal(ns)  # keeps D away from 0 everywhere
            for _ in range(6):
                t += rng.uniform(-1, 1) * synth.ricker((n - rng.uniform(20, 280)) * dt, 20.0)
            tr.append(t)
        tl.append(np.array(tr, np.float32))
        hl.append(np.sort(rng.uniform(0, 600, 4)).astype(np.float32))
        ml.append(np.full(4, 12.5 * g, np.float32))
    gs = synth.pack_gathers(tl, hl, ml, [12.5 * g for g in range(3)], dt)
    jobs = synth.Jobs(central=np.array([1], np.int32), apert_ptr=np.array([0, 3], np.int32),
                      apert_gather=np.arange(3, dtype=np.int32), out_off=np.zeros(1, np.int64), n_out=ns)
    theta = np.zeros((ns, 3))
    theta[:, 0] = rng.uniform(-3e-4, 3e-4, ns)
    theta[:, 1] = rng.uniform(-6e-8, 6e-8, ns)
    theta[:, 2] = 4.0 / rng.uniform(1800, 3500, ns) ** 2
    return gs, jobs, theta


def pin_gradient_fd(lib=None):
    """Analytic dS/d(A, B, q) and dS/dsample against central differences."""
    bad = []
    gs, jobs, theta = _grad_case()
    w = 9
    ns = jobs.n_out
    g_s = np.random.default_rng(2).uniform(0.5, 1.5, ns)
    gt, gsm, det = oracle.grad("crs", gs, jobs, theta, g_s, w, library=lib, detail=True)
    S0, _, M, _ = oracle.point("crs", gs, jobs, theta, w, library=lib)
    # each row's step in each component moves every one of its intersections
    # by at most 5e-5 samples, inside the oracle's default kink band of 1e-4:
    # only rows it flags as rough can see a kink
    rate = helpers.max_dtau_dtheta(gs, jobs, theta)
    rows = [r for r in range(40, ns - 20, 3) if M[r] > 0 and S0[r] > 0.05 and not det.rough[r]]
    if len(rows) < 60:
        bad.append(f"gradient FD: only {len(rows)} smooth rows to check")
    for k in range(3):
        step = 5e-5 / np.maximum(rate[:, k], 1e-300)
        tp, tm = theta.copy(), theta.copy()
        tp[:, k] += step
        tm[:, k] -= step
        sp, _, mp, _ = oracle.point("crs", gs, jobs, tp, w, library=lib)
        sm, _, mm, _ = oracle.point("crs", gs, jobs, tm, w, library=lib)
        fd = g_s * (sp - sm) / (2 * step)
        nerr = 0
        for r in rows:
            if mp[r] != M[r] or mm[r] != M[r]:
                continue
            scale = abs(fd[r]) + abs(gt[r, k]) + 1e-30
            # FP64 rounding of S (~1e-15) divided by the step bounds the rest
            if abs(fd[r] - gt[r, k]) > 1e-4 * scale + 1e-12 * abs(g_s[r]) / step[r]:
                nerr += 1
        if nerr:
            bad.append(f"gradient FD component {k}: {nerr} of {len(rows)} rows disagree")
    # samples: a handful of single-sample perturbations
    rng = np.random.default_rng(4)
    idx = rng.choice(gs.samples.size, 25, replace=False)
    L0 = float((g_s * S0).sum())
    nerr = 0

    def fd_at(i, eps):
        sp = gs.samples.copy()
        sm = gs.samples.copy()
        sp[i] += np.float32(eps)
        sm[i] -= np.float32(eps)
        d = float(sp[i]) - float(sm[i])  # the exact step after float32 rounding
        gp = synth.Gathers(sp, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset, gs.midpoint,
                           gs.central_x, gs.dt)
        gm = synth.Gathers(sm, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset, gs.midpoint,
                           gs.central_x, gs.dt)
        Lp = float((g_s * oracle.point("crs", gp, jobs, theta, w, library=lib)[0]).sum())
        Lm = float((g_s * oracle.point("crs", gm, jobs, theta, w, library=lib)[0]).sum())
        return (Lp - Lm) / d

    for i in idx:
        # Richardson extrapolation of two central differences (error O(eps^4)):
        # S is a ratio of quadratics in one sample and can curve sharply
        fd = (4.0 * fd_at(i, 5e-5) - fd_at(i, 1e-4)) / 3.0
        if abs(fd - gsm[i]) > 1e-4 * (abs(fd) + abs(gsm[i])) + 1e-7:
            nerr += 1
    if nerr:
        bad.append(f"sample gradient: {nerr} of {idx.size} samples disagree with FD (L0={L0})")
    return bad


def pin_crs_reduces_to_cmp(lib=None):
    """CRS with A = B = 0 over the aperture {c} equals CMP on gather c exactly."""
    bad = []
    gs = _tiny_line(7)
    grid = synth.Grid(A=np.zeros(1, np.float32), B=np.zeros(1, np.float32),
                      q=synth.velocity_grid(600, 2400, 4))
    cm = oracle.scan("cmp", gs, synth.cmp_jobs(gs, [2]), grid, 3, panel=True, library=lib)
    cr = oracle.scan("crs", gs, synth.line_crs_jobs(gs, [2], 0), grid, 3, panel=True, library=lib)
    if not np.array_equal(cm.panel, cr.panel):
        bad.append("CRS(A=B=0) over {c} differs from CMP")
    return bad


def pin_scan_rows(lib=None):
    """oracle_scan_rows on a shuffled subset of rows equals oracle_scan on the
    same rows in every output, for CMP and for CRS with nA != nB != nq (a slip
    in decoding the flat index into (iA, iB, iq) changes the picks)."""
    bad = []
    gs = _tiny_line(5)
    rng = np.random.default_rng(13)
    cases = [("cmp", synth.cmp_jobs(gs), synth.Grid(q=synth.velocity_grid(600, 2400, 7)), 3),
             ("crs", synth.line_crs_jobs(gs, [1, 2, 3], 1),
              synth.Grid(A=np.array([-3e-3, -1e-3, 0.0, 2e-3], np.float32),
                         B=np.array([-3e-5, 1e-5], np.float32),
                         q=synth.velocity_grid(600, 2400, 3)), 5)]
    for kind, jobs, grid, w in cases:
        full = oracle.scan(kind, gs, jobs, grid, w, library=lib)
        rj = np.concatenate([np.full(int(gs.ns[c]), j) for j, c in enumerate(jobs.central)]).astype(np.int32)
        rs = np.concatenate([np.arange(int(gs.ns[c])) for c in jobs.central]).astype(np.int32)
        pick = rng.permutation(rj.size)[: max(1, rj.size * 2 // 3)]
        r = oracle.scan_rows(kind, gs, jobs, grid, w, rj[pick], rs[pick], library=lib)
        rows = jobs.out_off[rj[pick]] + rs[pick]
        for name in ("best", "s_best", "stack", "gap", "fragile", "cond"):
            if not np.array_equal(getattr(r, name), getattr(full, name)[rows]):
                bad.append(f"scan_rows {kind}: {name} differs from the full scan")
    return bad


def pin_condition_number(lib=None):
    """kappa (the oracle's per-cell condition number of S) bounds the
    first-order change of S when every sample moves by a relative delta, and
    for one trace with a one-sample window (S = 1 whenever v != 0) it has the
    closed form 4 (|f[k]| + |f[k+1]|) / |v|."""
    bad = []
    rng = np.random.default_rng(31)
    for w in (1, 5):
        gs = helpers.random_line(rng, 3, fold_range=(2, 4), ns_range=(40, 60), hmax=300.0, smooth=True)
        jobs = synth.line_crs_jobs(gs, [1], 1)
        grid = synth.Grid(A=np.array([-1e-3, 1e-3], np.float32), B=np.zeros(1, np.float32),
                          q=synth.velocity_grid(800, 2400, 3))
        r = oracle.scan("crs", gs, jobs, grid, w, panel=True, library=lib)
        sgn = np.where(rng.random(gs.samples.size) < 0.5, -1.0, 1.0)
        pert = (gs.samples.astype(np.float64) * (1.0 + 1e-6 * sgn)).astype(np.float32)
        nz = gs.samples != 0
        delta = float(np.abs((pert[nz].astype(np.float64) - gs.samples[nz]) / gs.samples[nz]).max())
        gp = synth.Gathers(pert, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset, gs.midpoint,
                           gs.central_x, gs.dt)
        rp = oracle.scan("crs", gp, jobs, grid, w, panel=True, library=lib)
        excess = np.abs(rp.panel - r.panel) - (delta * r.panel_cond * 1.01 + 1e-12)
        if excess.max() > 0:
            bad.append(f"kappa w {w}: a relative {delta:.3g} perturbation moved S beyond delta kappa")
    ns = 30
    f = rng.standard_normal((1, ns)).astype(np.float32)
    g1 = synth.pack_gathers([f], [np.array([40.0], np.float32)], [np.zeros(1)], [0.0], 0.004)
    q = np.array([4.0 / 1900.0 ** 2], np.float32)
    r = oracle.scan("cmp", g1, synth.cmp_jobs(g1), synth.Grid(q=q), 1, library=lib)
    dt1 = float(g1.dt)
    for s in range(ns):
        tau = math.sqrt((s * dt1) ** 2 + float(q[0]) * 40.0 ** 2) / dt1
        k = math.floor(tau)
        if k + 1 > ns - 1:
            continue
        f0, f1 = float(f[0, k]), float(f[0, k + 1])
        v = f0 + (tau - k) * (f1 - f0)
        want = 4.0 * (abs(f0) + abs(f1)) / abs(v)
        if abs(r.cond[s] - want) > 1e-9 * want:
            bad.append(f"kappa of one trace, w = 1, s = {s}: {r.cond[s]} != {want}")
            break
    return bad


def pin_gradient_magnitudes(lib=None):
    """The magnitude sums bound the gradients (|g| <= mag, term by term), and
    the rough flag marks exactly the rows with a contributing intersection
    within the kink band of an integer: one trace at h = 0 has tau = s (every
    row rough); at h > 0 the flag follows the fraction of tau."""
    bad = []
    gs, jobs, theta = _grad_case()
    g_s = np.random.default_rng(6).uniform(-1.5, 1.5, jobs.n_out)
    gt, gsm, d = oracle.grad("crs", gs, jobs, theta, g_s, 9, library=lib, detail=True)
    if (np.abs(gt) > d.g_theta_mag * (1 + 1e-12) + 1e-300).any():
        bad.append("gradient magnitudes: |dL/dtheta| exceeds its magnitude sum")
    if (np.abs(gsm) > d.g_samples_mag * (1 + 1e-12) + 1e-300).any():
        bad.append("gradient magnitudes: |dL/dsample| exceeds its magnitude sum")
    if not (d.g_theta_mag[:, 2] > 0).mean() > 0.9:
        bad.append("gradient magnitudes: dL/dq magnitudes missing")
    rng = np.random.default_rng(8)
    ns, dt = 40, 0.004
    f = rng.standard_normal((3, ns)).astype(np.float32)
    h = np.array([0.0, 0.0, 0.0], np.float32)
    g0 = synth.pack_gathers([f], [h], [np.zeros(3)], [0.0], dt)
    j0 = synth.cmp_jobs(g0)
    th = np.zeros((ns, 3))
    th[:, 2] = 4.0 / 2000.0 ** 2
    _, _, d0 = oracle.grad("cmp", g0, j0, th, np.ones(ns), 3, library=lib, detail=True)
    if not d0.rough[1:ns - 2].all():
        bad.append("rough flag: tau = s exactly (h = 0) not flagged")
    hv = np.float32(900.0)
    g1 = synth.pack_gathers([f[:1]], [np.array([hv])], [np.zeros(1)], [0.0], dt)
    j1 = synth.cmp_jobs(g1)
    for qv, s in ((4.0 / 2000.0 ** 2, 20), (4.0 / 2500.0 ** 2, 25)):
        th = np.zeros((ns, 3))
        th[:, 2] = qv
        _, _, d1 = oracle.grad("cmp", g1, j1, th, np.ones(ns), 1, library=lib, detail=True)
        dtg = float(g1.dt)
        for r in range(ns):
            tau = math.sqrt((r * dtg) ** 2 + qv * float(hv) ** 2) / dtg
            k = math.floor(tau)
            if k + 1 > ns - 1:
                continue
            x = tau - k
            want = x < oracle.KINK_DEFAULT or x > 1.0 - oracle.KINK_DEFAULT
            if bool(d1.rough[r]) != want:
                bad.append(f"rough flag at tau {tau:.9f}: {bool(d1.rough[r])} != {want}")
                break
    # intersections placed 3e-5 below and above an integer (further than the
    # float32 rounding of h can move them) are both kinks
    for c in (-3e-5, 3e-5):
        tau_t = 20.0 + c
        hh = np.float32(math.sqrt(max(tau_t ** 2 - 10.0 ** 2, 0.0)) * dt / math.sqrt(4.0 / 2000.0 ** 2))
        g2 = synth.pack_gathers([f[:1]], [np.array([hh])], [np.zeros(1)], [0.0], dt)
        th = np.zeros((ns, 3))
        th[:, 2] = 4.0 / 2000.0 ** 2
        _, _, d2 = oracle.grad("cmp", g2, synth.cmp_jobs(g2), th, np.ones(ns), 1, library=lib, detail=True)
        dtg = float(g2.dt)
        tau = math.sqrt((10 * dtg) ** 2 + th[10, 2] * float(hh) ** 2) / dtg
        if not (abs(tau - 20.0) < 1e-4 and (tau - 20.0) * c > 0):
            bad.append(f"rough flag case: tau {tau:.9f} not on the intended side of 20")
        elif not d2.rough[10]:
            bad.append(f"rough flag: tau {tau:.9f} next to an integer not flagged")
    return bad


def pin_corrected(lib=None):
    """Gathers corrected along a parameter (oracle.corrected):
    (1) q = 0 (and A = B = 0 for CRS): tau = s, so every trace comes back
        unchanged, except its last sample, which has no successor and reads 0;
    (2) at the true velocity an integer-aligned event lands on its zero-offset
        sample in every trace, so the corrected gather is flat there: every
        trace reads the wavelet's peak amplitude;
    (3) with a one-sample window the point evaluation's stack is the mean of
        the corrected values over the contributing traces."""
    bad = []
    gs = _tiny_line(4)
    for kind, jobs in (("cmp", synth.cmp_jobs(gs)), ("crs", synth.line_crs_jobs(gs, [1, 2, 3], 1))):
        th = np.zeros((jobs.n_out, 3))
        out, off = oracle.corrected(kind, gs, jobs, th, library=lib)
        for j in range(jobs.njobs):
            c = int(jobs.central[j])
            nsc = int(gs.ns[c])
            r = 0
            for g in jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]:
                for li in range(int(gs.trace_ptr[g + 1] - gs.trace_ptr[g])):
                    f = gs.trace(int(g), li).astype(np.float64)
                    want = np.zeros(nsc)
                    m = min(nsc, f.size - 1)
                    want[:m] = f[:m]
                    got = out[off[j] + r * nsc: off[j] + (r + 1) * nsc]
                    if np.abs(got - want).max(initial=0.0) > 1e-12:
                        bad.append(f"corrected identity {kind} job {j} trace {r}")
                    r += 1
    dt, ns = 0.004, 600
    traces, h, s_e = _aligned_cmp_gather(2500.0, 1.0, dt, ns, [0, 3, 7, 12, 20, 31], amp=0.8)
    ag = synth.pack_gathers([traces], [h], [np.zeros(len(h))], [0.0], dt)
    aj = synth.cmp_jobs(ag)
    th = np.zeros((aj.n_out, 3))
    th[:, 2] = float(np.float32(4.0 / 2500.0 ** 2))
    out, off = oracle.corrected("cmp", ag, aj, th, library=lib)
    at = out.reshape(len(h), ns)[:, s_e]
    if np.abs(at - 0.8 * synth.ricker(np.zeros(1), 25.0)[0]).max() > 1e-6:
        bad.append(f"corrected aligned event not flat at its peak: {at}")
    for kind, jobs in (("cmp", synth.cmp_jobs(gs)), ("crs", synth.line_crs_jobs(gs, [1, 2, 3], 1))):
        rng = np.random.default_rng(8)
        th = np.zeros((jobs.n_out, 3))
        th[:, 2] = 4.0 / rng.uniform(600, 2400, jobs.n_out) ** 2
        if kind == "crs":
            th[:, 0] = rng.uniform(-2e-3, 2e-3, jobs.n_out)
            th[:, 1] = rng.uniform(-2e-5, 2e-5, jobs.n_out)
        out, off = oracle.corrected(kind, gs, jobs, th, library=lib)
        _, stack1, m1, _ = oracle.point(kind, gs, jobs, th, 1, library=lib)
        for j in range(jobs.njobs):
            nsc = int(gs.ns[jobs.central[j]])
            ag_ = jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]
            ntr = int(sum(gs.trace_ptr[g + 1] - gs.trace_ptr[g] for g in ag_))
            tot = out[off[j]: off[j] + ntr * nsc].reshape(ntr, nsc).sum(axis=0)
            rows = slice(int(jobs.out_off[j]), int(jobs.out_off[j]) + nsc)
            if np.abs(tot - stack1[rows] * m1[rows]).max(initial=0.0) > 1e-12:
                bad.append(f"corrected {kind} job {j}: sum differs from the w = 1 stack x M")
    return bad


PINS = [pin_hand_cases, pin_zero_moveout_closed_form, pin_ramp_traces, pin_aligned_ricker_cmp,
        pin_aligned_ricker_crs, pin_tie_break, pin_brute_force, pin_gradient_fd,
        pin_crs_reduces_to_cmp, pin_scan_rows, pin_condition_number, pin_gradient_magnitudes,
        pin_corrected]


# --------------------------------------------------------------------------
# the tests
# --------------------------------------------------------------------------
@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    bad = pin()
    assert not bad, "\n".join(bad)


def test_bounds_and_invariances():
    rng = np.random.default_rng(9)
    gs = helpers.random_line(rng, 4, fold_range=(2, 6), ns_range=(60, 90), hmax=400.0)
    jobs = synth.line_crs_jobs(gs, [1, 2], 1)
    grid = synth.Grid(A=np.array([-2e-4, 0.0, 2e-4], np.float32), B=np.array([-5e-8, 5e-8], np.float32),
                      q=synth.velocity_grid(1000, 3000, 5))
    r = oracle.scan("crs", gs, jobs, grid, 5, panel=True)
    assert r.panel.min() >= 0.0 and r.panel.max() <= 1.0 + 1e-12
    # scale invariance of S, linearity of the stack
    g2 = synth.Gathers((gs.samples * np.float32(-4.0)), gs.sample_off, gs.trace_ptr, gs.ns,
                       gs.half_offset, gs.midpoint, gs.central_x, gs.dt)
    r2 = oracle.scan("crs", g2, jobs, grid, 5, panel=True)
    assert np.allclose(r2.panel, r.panel, atol=1e-12, rtol=0)
    assert np.allclose(r2.stack, -4.0 * r.stack, atol=1e-12)
    # permutation of the traces of every gather (with their offsets)
    perm_traces, perm_h, perm_m = [], [], []
    for g in range(gs.ngathers):
        p = rng.permutation(int(gs.trace_ptr[g + 1] - gs.trace_ptr[g]))
        perm_traces.append(gs.gather(g)[p])
        perm_h.append(gs.half_offset[gs.trace_ptr[g]:gs.trace_ptr[g + 1]][p])
        perm_m.append(gs.midpoint[gs.trace_ptr[g]:gs.trace_ptr[g + 1]][p])
    g3 = synth.pack_gathers(perm_traces, perm_h, perm_m, gs.central_x, gs.dt)
    r3 = oracle.scan("crs", g3, jobs, grid, 5, panel=True)
    assert np.allclose(r3.panel, r.panel, atol=1e-12, rtol=0)


def test_crs_zero_dip_equals_cmp_on_union():
    rng = np.random.default_rng(17)
    ns = 50
    gl = [rng.standard_normal((3, ns)).astype(np.float32) for _ in range(3)]
    hl = [np.sort(rng.uniform(0, 300, 3)).astype(np.float32) for _ in range(3)]
    gs = synth.pack_gathers(gl, hl, [np.full(3, 12.5 * g, np.float32) for g in range(3)],
                            [0.0, 12.5, 25.0], 0.004)
    grid = synth.Grid(A=np.zeros(1, np.float32), B=np.zeros(1, np.float32),
                      q=synth.velocity_grid(800, 2400, 6))
    cr = oracle.scan("crs", gs, synth.line_crs_jobs(gs, [1], 1), grid, 5, panel=True)
    union = synth.pack_gathers([np.concatenate(gl)], [np.concatenate(hl)], [np.zeros(9)], [0.0], 0.004)
    cm = oracle.scan("cmp", union, synth.cmp_jobs(union), grid, 5, panel=True)
    assert np.array_equal(cr.panel, cm.panel)


def test_fragile_flag_marks_boundary_windows():
    # one trace, h = 0, tau = s exactly: the upper validity boundary is at
    # tau = ns - 1 - hw, which is hit exactly at s = ns - 1 - hw
    ns, w = 30, 5
    gs = synth.pack_gathers([np.ones((1, ns), np.float32)], [np.zeros(1)], [np.zeros(1)], [0.0], 1.0)
    r = oracle.scan("cmp", gs, synth.cmp_jobs(gs), synth.Grid(q=np.array([1.0], np.float32)), w)
    hw = 2
    assert r.fragile[ns - 1 - hw] and r.fragile[hw]
    assert not r.fragile[10]


def test_invalid_arguments_rejected():
    gs = _tiny_line(0)
    with pytest.raises(ValueError):
        oracle.scan("cmp", gs, synth.cmp_jobs(gs), synth.Grid(q=np.ones(2, np.float32)), 4)


# --------------------------------------------------------------------------
# mutation check: every plausible slip in the oracle must break a pin
# --------------------------------------------------------------------------
MUTATIONS = [
    ("corrected interpolation sign", "v = (double)f[k] + frac * ((double)f[k + 1] - (double)f[k]);",
     "v = (double)f[k] - frac * ((double)f[k + 1] - (double)f[k]);"),
    ("corrected time origin", "traveltime_sq(kind, s * dt, th, dm, h, &mag);",
     "traveltime_sq(kind, (s + 1) * dt, th, dm, h, &mag);"),
    ("corrected displacement", "const double dm = (kind == ORACLE_CRS) ? (double)g.midpoint[i] - xc : 0.0;\n"
     "                double *o", "const double dm = (kind == ORACLE_CRS) ? (double)g.midpoint[i] : 0.0;\n"
     "                double *o"),
    ("interpolation sign", "const double v = f0 + x * (f1 - f0);\n                U[j]",
     "const double v = f0 + x * (f0 - f1);\n                U[j]"),
    ("interpolation index", "const double f0 = f[a + j], f1 = f[a + j + 1];\n            "
     "    const double v", "const double f0 = f[a + j], f1 = f[a + j + 2];\n                const double v"),
    ("window start off by one", "const int64_t a = (int64_t)kf - hw;\n            /* a kink",
     "const int64_t a = (int64_t)kf - hw + 1;\n            /* a kink"),
    ("dropped curvature term", "return y * y + b + c;", "return y * y + c;"),
    ("dip factor", "double y = t0 + 2.0 * th.A * dm;", "double y = t0 + th.A * dm;"),
    ("transposed offset and displacement", "double c = th.q * h * h;", "double c = th.q * dm * dm;"),
    ("CMP traveltime", "return t0 * t0 + th.q * h * h;", "return t0 + th.q * h * h;"),
    ("missing 1/M", "c.N / ((double)c.M * c.D)", "c.N / c.D"),
    ("window edge", "return a >= 0.0 && a + w <= (double)(ns - 1);", "return a >= 0.0 && a + w <= (double)ns;"),
    ("stack normalisation", "c.L / ((double)c.M * (double)w)", "c.L / (double)c.M"),
    ("tie-break", "if (cl.S > s1) {", "if (cl.S >= s1) {"),
    ("dA factor", "4.0 * dm * (t0 + 2.0 * th.A * dm)", "2.0 * dm * (t0 + 2.0 * th.A * dm)"),
    ("dS/dv sign", "2.0 * (Ub[jj] - cl.S * cl.M * v) / MD", "2.0 * (Ub[jj] + cl.S * cl.M * v) / MD"),
    ("sample-gradient weight", "g_samples[base + a + jj] += gs * (1.0 - x) * dS_dv;",
     "g_samples[base + a + jj] += gs * x * dS_dv;"),
    ("dtau/dT", "1.0 / (2.0 * dt * sqrt(T))", "1.0 / (dt * sqrt(T))"),
    ("runner-up dropped", "s2 = s1;\n                        s1 = cl.S;", "s1 = cl.S;"),
    ("scan_rows runner-up dropped", "s2 = s1;\n                s1 = cl.S;", "s1 = cl.S;"),
    ("scan_rows B decode", "            th.B = (kind == ORACLE_CRS) ? (double)B[(p / nq) % nB] : 0.0;",
     "            th.B = (kind == ORACLE_CRS) ? (double)B[(p / nq) % nA] : 0.0;"),
    ("scan_rows A decode", "            th.A = (kind == ORACLE_CRS) ? (double)A[p / ((int64_t)nq * nB)] : 0.0;",
     "            th.A = (kind == ORACLE_CRS) ? (double)A[p / ((int64_t)nq * nA)] : 0.0;"),
    ("kappa energy factor", "kappa += cl.S / cl.D * 2.0 * sqrt(Di)", "kappa += cl.S / cl.D * sqrt(Di)"),
    ("kappa window-sum factor", "kappa += fabs(2.0 * U[j] / MD)", "kappa += fabs(U[j] / MD)"),
    ("gradient magnitude sign", "m_tau += m_dv * fabs(f1 - f0);", "m_tau += m_dv * (f1 - f0);"),
    ("sample magnitude weight", "g_samples_mag[base + a + jj + 1] += fabs(gs) * x * m_dv;",
     "g_samples_mag[base + a + jj + 1] += 0.0 * m_dv;"),
    ("kink band one-sided", "if (x < KINK_TAU || x > 1.0 - KINK_TAU) c.kink = 1;", "if (x < KINK_TAU) c.kink = 1;"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutants_are_caught(name, old, new, tmp_path):
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, f"mutation site for '{name}' not found"
    lib = oracle.compile_variant(src.replace(old, new, 1), str(tmp_path))
    failures = []
    for pin in PINS:
        failures += pin(lib)
        if failures:
            break
    assert failures, f"mutation '{name}' survived every pin"
