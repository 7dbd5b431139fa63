"""GPU parity of the corrected gathers (semb_corrected_gathers) with the FP64
oracle: CMP and CRS, random parameters per output row and the scan's own
picks, uneven fold and trace lengths."""
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


def _run(kind, gs, jobs, theta):
    import torch
    import paper_1907_11678_amd as semb
    dg, dj = gu.device_inputs(gs, jobs)
    off, tot = semb.corrected_offsets(gs.trace_ptr, gs.ns, jobs.central, jobs.apert_ptr, jobs.apert_gather)
    out = torch.full((max(tot, 1),), float("nan"), device="cuda")
    semb.corrected_gathers(dg, dj, 0 if kind == "cmp" else 1, torch.from_numpy(theta.astype(np.float32)).cuda(),
                           torch.from_numpy(off).cuda(), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:tot].astype(np.float64), off


def _compare(kind, gs, jobs, theta):
    got, off = _run(kind, gs, jobs, theta)
    ref, roff = oracle.corrected(kind, gs, jobs, theta.astype(np.float32).astype(np.float64))
    assert np.array_equal(off, roff)
    assert np.isfinite(got).all()
    scale = max(float(np.abs(gs.samples).max()), 1e-30)
    err = np.abs(got - ref).max(initial=0.0) / scale
    assert err <= 2e-6, f"{kind}: max relative error {err:.3g}"
    return err, float((ref != 0).mean())


@pytest.mark.parametrize("kind", ["cmp", "crs"])
def test_random_parameters(kind):
    rng = np.random.default_rng(31)
    gs = helpers.random_line(rng, 8, fold_range=(1, 7), ns_range=(20, 400), hmax=800.0, smooth=True)
    jobs = synth.cmp_jobs(gs) if kind == "cmp" else synth.line_crs_jobs(gs, list(range(8)), 2)
    th = np.zeros((jobs.n_out, 3))
    th[:, 2] = 4.0 / rng.uniform(700, 3000, jobs.n_out) ** 2
    if kind == "crs":
        th[:, 0] = rng.uniform(-3e-3, 3e-3, jobs.n_out)
        th[:, 1] = rng.uniform(-2e-5, 2e-5, jobs.n_out)
    err, filled = _compare(kind, gs, jobs, th)
    print(kind, "corrected: max rel error", err, "non-zero fraction", filled, flush=True)


def test_at_the_scan_picks():
    """The CMP-plain gathers corrected along the scan's picked velocities."""
    import torch
    import paper_1907_11678_amd as semb
    wl = synth.cmp_plain(ids=[3, 4])
    best = gu.run_scan("cmp", wl.gathers, wl.jobs, wl.grid, wl.w)[0]
    th = oracle.theta_of(wl.grid, best, "cmp")
    err, filled = _compare("cmp", wl.gathers, wl.jobs, th)
    assert filled > 0.8
