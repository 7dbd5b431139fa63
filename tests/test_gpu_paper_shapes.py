"""GPU parity on the paper's dataset shapes (Table 1): fold 1000 apertures
(more traces than the tile keeps metadata for at once, so the trace metadata
is loaded in parts), 1650-sample traces, and the 17- and 19-sample windows."""
from __future__ import annotations

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


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dataset,ids", [(7, [3]), (4, [0, 1, 2])])
def test_cmp_paper_shape_full_oracle(dataset, ids):
    """Every row of fold-1000 x 1650 (w 19) and fold-60 x 1650 (w 17) gathers."""
    wl = synth.paper_shape(dataset, 8, centrals=ids)
    gpu = gu.run_scan("cmp", wl.gathers, wl.jobs, wl.grid, wl.w)
    ref = oracle.scan("cmp", wl.gathers, wl.jobs, wl.grid, wl.w)
    _say(f"data{dataset} cmp", gu.compare(f"data{dataset}", gpu, ref, gu.sample_scale(wl.gathers, wl.jobs)))


@pytest.mark.parametrize("dataset", [5, 8])
def test_crs_paper_shape_sampled_rows(dataset):
    """CRS over +-1 gathers of fold 1000 (3000 traces per aperture), coarse grid."""
    wl = synth.paper_shape(dataset, 12, kind="crs", half_aperture=1, centrals=[5, 6])
    gpu = gu.run_scan("crs", wl.gathers, wl.jobs, wl.grid, wl.w)
    rng = np.random.default_rng(dataset)
    ns = int(wl.gathers.ns[0])
    rj = rng.integers(0, wl.jobs.njobs, 24).astype(np.int32)
    rs = rng.integers(0, ns, 24).astype(np.int32)
    ref = oracle.scan_rows("crs", wl.gathers, wl.jobs, wl.grid, wl.w, rj, rs)
    rows = wl.jobs.out_off[rj] + rs
    _say(f"data{dataset} crs", gu.compare(f"data{dataset} crs", gpu, ref,
                                          gu.sample_scale(wl.gathers, wl.jobs), rows))
