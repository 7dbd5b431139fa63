"""Property-based search (hypothesis) over tiny random cases: the FP64 oracle
must equal the independent brute-force evaluation of Eq. (1) in
tests/helpers.py on every panel cell (and in the top-two gap), whatever the fold, trace lengths,
windows, offsets, CRS dips and curvatures (negative radicands included),
all-zero traces and window positions at the trace ends."""
from __future__ import annotations

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import synth
from tests import helpers


@st.composite
def tiny_case(draw):
    ng = draw(st.integers(1, 4))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    traces, hs, ms = [], [], []
    for g in range(ng):
        fold = draw(st.integers(1, 3))
        ns = draw(st.integers(1, 30))
        t = rng.standard_normal((fold, ns)).astype(np.float32)
        if draw(st.booleans()):
            t[0] = 0.0
        traces.append(t)
        hs.append(np.sort(rng.uniform(0, draw(st.sampled_from([0.0, 50.0, 400.0])), fold)).astype(np.float32))
        ms.append(np.full(fold, 12.5 * g, np.float32))
    gs = synth.pack_gathers(traces, hs, ms, [12.5 * g for g in range(ng)], 0.004)
    w = draw(st.sampled_from([1, 3, 5, 7]))
    kind = draw(st.sampled_from(["cmp", "crs"]))
    if kind == "cmp":
        jobs = synth.cmp_jobs(gs)
        grid = synth.Grid(q=synth.velocity_grid(500.0, 3000.0, draw(st.integers(1, 4))))
    else:
        k = draw(st.integers(0, 2))
        jobs = synth.line_crs_jobs(gs, list(range(ng)), k)
        grid = synth.Grid(A=np.array(draw(st.lists(st.sampled_from([-5e-3, -1e-4, 0.0, 2e-3]), min_size=1,
                                                   max_size=2, unique=True)), np.float32),
                          B=np.array(draw(st.lists(st.sampled_from([-5e-5, 0.0, 3e-5]), min_size=1, max_size=2,
                                                   unique=True)), np.float32),
                          q=synth.velocity_grid(500.0, 3000.0, draw(st.integers(1, 3))))
    return kind, gs, jobs, grid, w


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_case())
def test_oracle_equals_brute_force(case):
    kind, gs, jobs, grid, w = case
    r = oracle.scan(kind, gs, jobs, grid, w, panel=True)
    S, ST, M = helpers.brute_panel(kind, gs, jobs, grid, w)
    assert np.abs(r.panel - S).max(initial=0.0) <= 1e-12
    assert (r.s_best >= -1e-15).all() and (r.s_best <= 1.0 + 1e-12).all()
    if S.size:
        rows = np.arange(S.shape[0])
        # the pick maximises the brute force's S, and is the first maximiser of
        # the oracle's own panel (ties go to the smallest index)
        assert (S[rows, r.best] >= S.max(axis=1) - 1e-12).all()
        assert np.array_equal(r.best, np.argmax(r.panel, axis=1))
        assert np.abs(r.stack - ST[rows, r.best]).max() <= 1e-12
        # gap: best minus second-best S over the brute force's panel
        if S.shape[1] > 1:
            top = np.sort(S, axis=1)
            assert np.abs(r.gap - (top[:, -1] - top[:, -2])).max() <= 1e-12
        else:
            assert np.isinf(r.gap).all()
        # the row-subset scan reproduces the full scan on every row it is given
        rj = np.concatenate([np.full(int(gs.ns[c]), j) for j, c in enumerate(jobs.central)]).astype(np.int32)
        rs = np.concatenate([np.arange(int(gs.ns[c])) for c in jobs.central]).astype(np.int32)
        rr = oracle.scan_rows(kind, gs, jobs, grid, w, rj[::-1], rs[::-1])
        out = jobs.out_off[rj[::-1]] + rs[::-1]
        for name in ("best", "s_best", "stack", "gap", "fragile"):
            assert np.array_equal(getattr(rr, name), getattr(r, name)[out]), name
