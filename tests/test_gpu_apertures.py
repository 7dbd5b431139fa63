"""GPU parity of the CRS scan on radius apertures (semb_radius_apertures) over
an irregular line: jittered midpoints give apertures of 2 to 7 gathers and
displacements that are not multiples of the spacing."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests import gpu_util as gu

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


def test_crs_on_radius_apertures():
    import paper_1907_11678_amd as semb
    spec = synth.crs_line_spec()
    ids = list(range(200, 216))
    gs = synth.line_gathers(spec, ids)
    rng = np.random.default_rng(11)
    cx = (gs.central_x.astype(np.float64) + rng.uniform(-5.0, 5.0, gs.ngathers)).astype(np.float32)
    mid = np.repeat(cx, np.diff(gs.trace_ptr))
    gs = dataclasses.replace(gs, central_x=cx, midpoint=mid)
    centrals = np.arange(2, 14, dtype=np.int32)
    ptr, ag, mx = semb.radius_apertures(cx.astype(np.float64), centrals, 40.0)
    assert 2 <= min(np.diff(ptr)) and mx <= 7
    ns = gs.ns[centrals].astype(np.int64)
    out_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    jobs = synth.Jobs(central=centrals, apert_ptr=ptr, apert_gather=ag, out_off=out_off, n_out=int(ns.sum()))
    grid = synth.crs_coarse_grid()
    gpu = gu.run_scan("crs", gs, jobs, grid, 9, panel=True)
    ref = oracle.scan("crs", gs, jobs, grid, 9, panel=True)
    print("radius apertures", np.diff(ptr).tolist(),
          gu.compare("radius crs", gpu, ref, gu.sample_scale(gs, jobs)), flush=True)
