"""GPU parity on the degenerate cases of the semblance (Eq. 1) and its scan:

* an all-zero gather: the energy D is 0, so every cell has S = 0 and stack 0,
  and the pick falls to parameter 0;
* identical traces at one offset: every contributing window has S = 1;
* a single-trace gather (M = 1): S = 1 wherever the window has energy;
* a CRS aperture of the maximum 64 gathers, and a CRS job whose whole
  aperture is zero.

Each case is checked against the FP64 oracle and against the exact value the
definition gives."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests import gpu_util as gu
from tests import helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1907_11678_amd as semb
    semb.lib()
    torch.cuda.set_device(0)
    oracle.set_fragility(gu.FRAGILE_TAU, gu.FRAGILE_T_REL)
    yield
    oracle.set_fragility(*oracle.FRAGILE_DEFAULT)


def _say(*a):
    print(*a, flush=True)


def _rows(jobs, j, gs):
    o = int(jobs.out_off[j])
    return slice(o, o + int(gs.ns[int(jobs.central[j])]))


def test_cmp_zero_identical_and_single_trace_gathers():
    rng = np.random.default_rng(11)
    ns, dt = 300, 0.004
    one = helpers.seismic_like(rng, 1, ns, dt).astype(np.float32)
    traces = [np.zeros((4, ns), np.float32),              # D = 0 everywhere
              np.repeat(one, 5, axis=0),                  # five copies of one trace
              one.copy(),                                 # M = 1
              helpers.seismic_like(rng, 6, ns, dt).astype(np.float32)]
    hs = [np.array([0, 200, 400, 800], np.float32), np.full(5, 400.0, np.float32),
          np.array([300.0], np.float32), np.array([0, 150, 300, 450, 600, 750], np.float32)]
    gs = synth.pack_gathers(traces, hs, [np.zeros(len(h)) for h in hs], [0.0, 12.5, 25.0, 37.5], dt)
    jobs = synth.cmp_jobs(gs)
    grid = synth.Grid(q=synth.velocity_grid(1500, 4500, 21))
    w = 9
    gpu = gu.run_scan("cmp", gs, jobs, grid, w, panel=True)
    ref = oracle.scan("cmp", gs, jobs, grid, w, panel=True)
    _say("cmp degenerate", gu.compare("cmp degenerate", gpu, ref, gu.sample_scale(gs, jobs)))
    best, sb, st, pan = gpu

    z = _rows(jobs, 0, gs)
    assert (best[z] == 0).all() and (sb[z] == 0).all() and (st[z] == 0).all() and (pan[z] == 0).all()

    for j in (1, 2):  # identical copies, and a single trace: S = 1 wherever D > 0
        r = _rows(jobs, j, gs)
        on = ref.panel[r] > 0.5
        assert on.sum() > 0.8 * on.size
        assert np.abs(pan[r][on] - 1.0).max() <= 2e-6
        assert (ref.panel[r][~on] == 0).all() and (pan[r][~on] == 0).all()


def test_crs_maximum_aperture_and_zero_aperture():
    """64 gathers of 2 traces around one central (the ABI's aperture limit),
    and a second central whose aperture holds only zero gathers."""
    rng = np.random.default_rng(12)
    ns, dt, G = 200, 0.004, 72
    traces, hs, mids = [], [], []
    for g in range(G):
        live = g < 64
        t = helpers.seismic_like(rng, 2, ns, dt).astype(np.float32) if live else np.zeros((2, ns), np.float32)
        traces.append(t)
        hs.append(rng.uniform(0, 1500, 2).astype(np.float32))
        mids.append(np.full(2, 12.5 * g, np.float32))
    gs = synth.pack_gathers(traces, hs, mids, [12.5 * g for g in range(G)], dt)
    ap0 = list(range(0, 64))       # central 31, 64 gathers
    ap1 = list(range(64, 72))      # central 68, all zero
    jobs = synth.Jobs(central=np.array([31, 68], np.int32),
                      apert_ptr=np.array([0, 64, 72], np.int32),
                      apert_gather=np.array(ap0 + ap1, np.int32),
                      out_off=np.array([0, ns], np.int64), n_out=2 * ns)
    grid = synth.crs_coarse_grid()
    w = 5
    gpu = gu.run_scan("crs", gs, jobs, grid, w, panel=True)
    ref = oracle.scan("crs", gs, jobs, grid, w, panel=True)
    _say("crs 64-gather aperture", gu.compare("crs max aperture", gpu, ref, gu.sample_scale(gs, jobs)))
    best, sb, st, pan = gpu
    z = _rows(jobs, 1, gs)
    assert (best[z] == 0).all() and (sb[z] == 0).all() and (st[z] == 0).all() and (pan[z] == 0).all()
    live = _rows(jobs, 0, gs)
    assert (sb[live] > 0).mean() > 0.9


def test_off_trace_windows_over_a_short_stage_every_shape():
    """Gathers whose windows all lie past the trace end for most output
    samples, so that the first staged chunk holds fewer than w + 1 positions:
    the branch-free tile shapes then read the zeroed block at the start of each
    LDS plane with zero weights.  Every shape must equal the oracle (S = 0,
    stack 0, pick 0 where no window fits) and each other bit for bit."""
    import paper_1907_11678_amd as semb
    rng = np.random.default_rng(41)
    ns, dt, w = 40, 0.004, 31
    q = synth.velocity_grid(1800, 2200, 9)
    # tau(s = 0) = 25 samples at the fastest velocity (and more at the others):
    # every window starts past the last valid start (ns - 1 - w = 8) for every
    # s, and the union range a tile stages, samples 9..39, holds fewer than
    # w + 1 = 32 samples
    h_far = np.float32(25 * dt / np.sqrt(4.0 / 2200.0 ** 2))
    traces = [helpers.seismic_like(rng, 2, ns, dt).astype(np.float32),
              helpers.seismic_like(rng, 3, 200, dt).astype(np.float32)]
    hs = [np.array([h_far, h_far * 1.01], np.float32), np.array([0.0, 100.0, 250.0], np.float32)]
    gs = synth.pack_gathers(traces, hs, [np.zeros(2), np.zeros(3)], [0.0, 12.5], dt)
    jobs = synth.cmp_jobs(gs)
    grid = synth.Grid(q=q)
    dg, dj = gu.device_inputs(gs, jobs)
    ref = oracle.scan("cmp", gs, jobs, grid, w, panel=True)
    base = None
    try:
        for shape in range(semb.SCAN_SHAPES):
            semb.set_scan_shape(0, w, dg, dj, shape)
            got = gu.run_scan("cmp", gs, jobs, grid, w, panel=True, dg=dg, dj=dj)
            gu.compare(f"short stage shape {shape}", got, ref, gu.sample_scale(gs, jobs))
            r0 = _rows(jobs, 0, gs)
            assert (got[3][r0] == 0).all() and (got[1][r0] == 0).all() and (got[0][r0] == 0).all()
            if base is None:
                base = got
            for a, b, what in zip(got, base, ("best", "s_best", "stack", "panel")):
                assert np.array_equal(a, b), f"shape {shape}: {what} differs from shape 0"
    finally:
        semb.set_scan_shape(0, w, dg, dj, -1)


def test_aperture_longer_than_declared_gets_the_marker():
    """A CRS job whose aperture lists more gathers than jobs.max_apert declares
    is not computed by any call: its rows get best = -1, s_best = -1, stack 0
    (panel -1), S = -1 from stack and semb_refine (theta kept), a zero
    gradient, zero corrected gathers; the other jobs are computed as usual and
    match the oracle.  The batched scan does the same."""
    import dataclasses
    import torch
    import paper_1907_11678_amd as semb
    wl = synth.crs_line(centrals=[10, 11], grid=synth.crs_coarse_grid())
    gs = wl.gathers  # gathers renumbered: line gathers 6..15 are 0..9
    c0, c1 = (int(c) for c in wl.jobs.central)
    # job 0: +-4 gathers (9), job 1: +-1 gather (3); declare at most 5
    ap = np.array([0, 9, 12], np.int32)
    ag = np.array(list(wl.jobs.apert_gather[:9]) + [c1 - 1, c1, c1 + 1], np.int32)
    ns = int(gs.ns[c0])
    jobs = synth.Jobs(central=np.array([c0, c1], np.int32), apert_ptr=ap, apert_gather=ag,
                      out_off=np.array([0, ns], np.int64), n_out=2 * ns)
    dg, dj = gu.device_inputs(gs, jobs)
    dj = dataclasses.replace(dj, max_apert=5)
    r0, r1 = slice(0, ns), slice(ns, 2 * ns)
    best, sb, st, pan = gu.run_scan("crs", gs, jobs, wl.grid, wl.w, panel=True, dg=dg, dj=dj)
    assert (best[r0] == -1).all() and (sb[r0] == -1).all() and (st[r0] == 0).all() and (pan[r0] == -1).all()
    one = synth.Jobs(central=jobs.central[1:], apert_ptr=np.array([0, 3], np.int32), apert_gather=ag[9:],
                     out_off=np.zeros(1, np.int64), n_out=ns)
    ref = oracle.scan("crs", gs, one, wl.grid, wl.w, panel=True)
    gu.compare("computed job next to a marked one", (best[r1], sb[r1], st[r1], pan[r1]), ref,
               gu.sample_scale(gs, one))
    th = torch.from_numpy(oracle.theta_of(wl.grid, np.zeros(2 * ns, np.int64), "crs").astype(np.float32)).cuda()
    S = torch.full((2 * ns,), 7.0, device="cuda")
    stk = torch.full((2 * ns,), 7.0, device="cuda")
    semb.stack(dg, dj, 1, th, wl.w, S, stk)
    g_th = torch.full((2 * ns, 3), 7.0, device="cuda")
    semb.semblance_grad(dg, dj, 1, th, torch.ones(2 * ns, device="cuda"), wl.w, g_th, None)
    th_r = th.clone()
    S2 = torch.full((2 * ns,), 7.0, device="cuda")
    st2 = torch.full((2 * ns,), 7.0, device="cuda")
    semb.refine(dg, dj, 1, th_r, wl.w, S2, st2, steps=2)
    off, tot = semb.corrected_offsets(gs.trace_ptr, gs.ns, jobs.central, ap, ag)
    cor = torch.full((tot,), 7.0, device="cuda")
    semb.corrected_gathers(dg, dj, 1, th, torch.from_numpy(off).cuda(), cor)
    torch.cuda.synchronize()
    S, stk, g_th, S2, st2 = (t.cpu().numpy() for t in (S, stk, g_th, S2, st2))
    assert (S[r0] == -1).all() and (stk[r0] == 0).all() and (g_th[r0] == 0).all()
    assert (S2[r0] == -1).all() and (st2[r0] == 0).all()
    assert np.array_equal(th_r.cpu().numpy()[r0], th.cpu().numpy()[r0])
    assert (S[r1] >= 0).all() and (S2[r1] >= 0).all()
    assert (cor.cpu().numpy()[: int(off[1])] == 0).all()
    # the batched scan: both jobs CRS, same declaration
    kind = np.ones(2, np.int32)
    tiles, ng, npart = semb.batch_plan(kind, jobs.central, ap, ag, gs.ns, gs.trace_ptr, 101, wl.grid.n, 64)
    ws = semb.alloc_batch_workspace(dg.nsamples, 9, 9, ng, npart)
    bb = torch.full((2 * ns,), 7, dtype=torch.int32, device="cuda")
    bs = torch.full((2 * ns,), 7.0, device="cuda")
    bt = torch.full((2 * ns,), 7.0, device="cuda")
    qc = torch.from_numpy(synth.velocity_grid(1500, 4500, 101)).cuda()
    A, B, q = (torch.from_numpy(x).cuda() for x in (wl.grid.A, wl.grid.B, wl.grid.q))
    semb.scan_batch(dg, dj, torch.from_numpy(kind).cuda(), qc, 9, A, B, q, 9, torch.from_numpy(tiles).cuda(),
                    ng, npart, bb, bs, bt, ws)
    torch.cuda.synchronize()
    bb, bs, bt = bb.cpu().numpy(), bs.cpu().numpy(), bt.cpu().numpy()
    assert (bb[r0] == -1).all() and (bs[r0] == -1).all() and (bt[r0] == 0).all()
    assert np.array_equal(bb[r1], best[r1]) and np.array_equal(bs[r1], sb[r1].astype(np.float32))
