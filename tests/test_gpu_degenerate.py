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
    _say("crs 64-gather aperture", gu.compare("crs max aperture", gpu, ref, gu.sample_scale(gs, jobs),
                                              s_tol=gu.s_tol(w)))
    best, sb, st, pan = gpu
    z = _rows(jobs, 1, gs)
    assert (best[z] == 0).all() and (sb[z] == 0).all() and (st[z] == 0).all() and (pan[z] == 0).all()
    live = _rows(jobs, 0, gs)
    assert (sb[live] > 0).mean() > 0.9
