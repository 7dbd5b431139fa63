"""Host tests of the radius aperture search (semb_radius_apertures): equal to
a brute-force distance test on random 2D midpoints (duplicates, radius 0),
and on a regular line equal to the +-k gather apertures the CRS workloads use."""
from __future__ import annotations

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def semb():
    import paper_1907_11678_amd as pkg
    import os
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1907_11678_amd import build
        build.build()
    pkg.lib()
    return pkg


def _brute(x, y, centrals, r):
    out = []
    for c in centrals:
        d2 = (x - x[c]) ** 2 + ((y - y[c]) ** 2 if y is not None else 0.0)
        out.append(np.nonzero(d2 <= r * r)[0])
    return out


@pytest.mark.parametrize("seed,r,planar", [(0, 30.0, True), (1, 0.0, True), (2, 75.0, False), (3, 1e4, True)])
def test_matches_brute_force(semb, seed, r, planar):
    rng = np.random.default_rng(seed)
    n = 500
    x = rng.uniform(-300, 300, n).round(1)
    y = rng.uniform(-300, 300, n).round(1) if planar else None
    x[:20] = x[20:40]  # coinciding midpoints
    if planar:
        y[:20] = y[20:40]
    centrals = rng.integers(0, n, 120).astype(np.int32)
    ptr, ag, mx = semb.radius_apertures(x, centrals, r, y=y)
    ref = _brute(x, y, centrals, r)
    assert ptr[0] == 0 and ptr.size == centrals.size + 1
    for i, want in enumerate(ref):
        got = ag[ptr[i]:ptr[i + 1]]
        assert np.array_equal(got, want), i
        assert centrals[i] in got
    assert mx == max(len(w) for w in ref)


def test_line_radius_equals_k_gathers(semb):
    """On the 12.5 m line, radius 4 x 12.5 m (+ rounding room) is the +-4 aperture."""
    spec = synth.crs_line_spec()
    gs = synth.line_gathers(spec, list(range(40)))
    x = gs.central_x.astype(np.float64)
    centrals = np.arange(40, dtype=np.int32)
    ptr, ag, mx = semb.radius_apertures(x, centrals, 4 * 12.5 + 1e-6)
    jobs = synth.line_crs_jobs(gs, centrals, 4)
    assert np.array_equal(ptr, jobs.apert_ptr) and np.array_equal(ag, jobs.apert_gather) and mx == 9


def test_rejects_bad_input(semb):
    from paper_1907_11678_amd import SembError
    with pytest.raises(SembError):
        semb.radius_apertures(np.zeros(3), np.array([3], np.int32), 1.0)
    with pytest.raises(SembError):
        semb.radius_apertures(np.zeros(3), np.array([0], np.int32), -1.0)
    with pytest.raises(SembError):
        semb.radius_apertures(np.array([0.0, np.nan]), np.array([0], np.int32), 1.0)
