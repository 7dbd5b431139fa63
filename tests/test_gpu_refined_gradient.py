"""The refinement workload's gradient check: on 4 centrals of the CRS line,
after the coarse 7x7x11 scan and 8 ascent steps, the backward kernel's
dS/d(A, B, q) and dS/dsample at the refined parameters against the oracle's
FP64 gradient (per-row and per-sample bounds of tests/gpu_util.py), and the
oracle's gradient there against central differences of its own S."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests import gpu_util as gu
from tests import helpers
from tests.test_gpu_refine import Refinement

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


def test_gradient_at_the_refined_parameters():
    import torch
    import paper_1907_11678_amd as semb
    wl = synth.crs_line(centrals=[30, 170, 333, 480])
    r = Refinement(wl)  # coarse 7x7x11 + 8 steps
    r.run()
    torch.cuda.synchronize()
    th = r.theta.cpu().numpy()
    n = r.n
    g_s = np.random.default_rng(17).uniform(0.5, 1.5, n).astype(np.float32)
    g_theta = torch.empty((n, 3), device="cuda")
    g_smp = torch.zeros(r.dg.nsamples, device="cuda")
    semb.semblance_grad(r.dg, r.dj, 1, r.theta, torch.from_numpy(g_s).cuda(), wl.w, g_theta, g_smp)
    torch.cuda.synchronize()
    stats = gu.assert_grad_parity("refined theta", "crs", wl.gathers, wl.jobs, th, g_s, wl.w,
                                  g_theta.cpu().numpy().astype(np.float64), g_smp.cpu().numpy().astype(np.float64))
    print("gradient at the refined theta", stats, flush=True)
    # the oracle's gradient at these parameters against central differences of
    # its S, on rows away from kinks (the oracle's default band of 1e-4
    # samples) with S > 0.05.  Each row's step in each component moves every
    # one of its intersections by at most 5e-5 samples, so no difference
    # crosses a kink the flag did not see.
    th64 = th.astype(np.float64)
    gt, _, d = oracle.grad("crs", wl.gathers, wl.jobs, th64, np.ones(n), wl.w, samples_grad=False, detail=True)
    S0, _, M, _ = oracle.point("crs", wl.gathers, wl.jobs, th64, wl.w)
    rows = np.nonzero(~d.rough & (S0 > 0.05) & (M > 0))[0][::3]
    rate = helpers.max_dtau_dtheta(wl.gathers, wl.jobs, th64)  # [n, 3] samples per unit of each component
    bad, checked = 0, 0
    for k in range(3):
        step = 5e-5 / np.maximum(rate[:, k], 1e-300)
        tp, tm = th64.copy(), th64.copy()
        tp[:, k] += step
        tm[:, k] -= step
        sp, _, mp, _ = oracle.point("crs", wl.gathers, wl.jobs, tp, wl.w)
        sm, _, mm, _ = oracle.point("crs", wl.gathers, wl.jobs, tm, wl.w)
        fd = (sp - sm) / (2 * step)
        ok = rows[(mp[rows] == M[rows]) & (mm[rows] == M[rows])]
        err = np.abs(fd[ok] - gt[ok, k])
        lim = 1e-4 * (np.abs(fd[ok]) + np.abs(gt[ok, k])) + 1e-12 / step[ok]
        bad += int((err > lim).sum())
        checked += ok.size
    print(f"finite differences at the refined theta: {checked} row-components, {bad} disagree", flush=True)
    assert rows.size >= 400 and bad == 0

