"""GPU test of semb_scan_noalloc, the scan for callers that cannot allocate:
through the C ABI it must give the workspace scans' (cmp_scan / crs_scan)
outputs bit for bit, on two calls in a row, the second on a smaller input
(the per-GPU scratch keeps the first call's contents)."""
from __future__ import annotations

import numpy as np
import pytest

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
    yield


def _outputs(n, npar, panel):
    import torch
    best = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    sb = torch.full((n,), float("nan"), device="cuda")
    st = torch.full((n,), float("nan"), device="cuda")
    pan = torch.full((n, npar), float("nan"), device="cuda") if panel else None
    return best, sb, st, pan


def _both(kind, wl, panel):
    """(workspace scan, no-alloc scan) outputs as numpy arrays."""
    import torch
    import paper_1907_11678_amd as semb
    gs, jobs, grid = wl.gathers, wl.jobs, wl.grid
    dg, dj = gu.device_inputs(gs, jobs)
    assert semb.workspace_bytes(dg.nsamples) <= semb.NOALLOC_SCRATCH_BYTES
    npar = grid.n if kind == "crs" else grid.q.size
    q = torch.from_numpy(grid.q).cuda()
    A = torch.from_numpy(grid.A).cuda() if kind == "crs" else None
    B = torch.from_numpy(grid.B).cuda() if kind == "crs" else None
    ref = _outputs(jobs.n_out, npar, panel)
    ws = semb.alloc_workspace(dg.nsamples)
    if kind == "cmp":
        semb.cmp_scan(dg, dj, q, wl.w, *ref[:3], ws, panel=ref[3])
    else:
        semb.crs_scan(dg, dj, A, B, q, wl.w, *ref[:3], ws, panel=ref[3])
    got = _outputs(jobs.n_out, npar, panel)
    semb.scan_noalloc(0 if kind == "cmp" else 1, dg, dj, q, wl.w, *got[:3], A=A, B=B, panel=got[3])
    torch.cuda.synchronize()
    to = lambda t: None if t is None else t.cpu().numpy()
    return [to(t) for t in ref], [to(t) for t in got]


@pytest.mark.parametrize("kind", ["cmp", "crs"])
def test_noalloc_equals_the_workspace_scan(kind):
    if kind == "cmp":
        big, small = synth.cmp_plain(), synth.cmp_plain(ids=[3, 9, 40])
    else:
        g = synth.crs_coarse_grid()
        big, small = synth.crs_line(centrals=[30, 31, 200], grid=g), synth.crs_line(centrals=[77], grid=g)
    assert small.gathers.samples.size < big.gathers.samples.size
    for name, wl, panel in (("first", big, True), ("second, smaller", small, False)):
        ref, got = _both(kind, wl, panel)
        for a, b, what in zip(got, ref, ("best", "s_best", "stack", "panel")):
            if a is None:
                continue
            assert np.array_equal(a, b), f"{kind} {name} call: {what} differs from the workspace scan"
        assert (ref[0] >= 0).all() and np.isfinite(ref[1]).all()
        print(kind, name, "rows", ref[0].size, "identical", flush=True)

