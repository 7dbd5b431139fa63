"""GPU tests of the batched scan (mixed CMP/CRS jobs, uneven fold and length,
one persistent launch): it must equal the per-kind scans, match the oracle on
sampled rows, and replay identically from a captured HIP graph."""
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


class Batch:
    """A batch on the device, with its plan, workspace and outputs."""

    def __init__(self, bw: synth.BatchWorkload, split_params: int = 256):
        import torch
        import paper_1907_11678_amd as semb
        self.bw = bw
        gs, jobs = bw.gathers, bw.jobs
        self.dg, self.dj = gu.device_inputs(gs, jobs)
        self.kind = torch.from_numpy(bw.kind).cuda()
        tiles, self.ng, self.np = semb.batch_plan(bw.kind, jobs.central, jobs.apert_ptr, jobs.apert_gather,
                                                  gs.ns, gs.trace_ptr, bw.grid_cmp.n, bw.grid_crs.n,
                                                  split_params)
        self.ntiles = tiles.shape[0]
        self.tiles = torch.from_numpy(tiles).cuda()
        self.ws = semb.alloc_batch_workspace(self.dg.nsamples, bw.w_cmp, bw.w_crs, self.ng, self.np)
        self.qc = torch.from_numpy(bw.grid_cmp.q).cuda()
        self.A, self.B, self.qr = (torch.from_numpy(x).cuda() for x in (bw.grid_crs.A, bw.grid_crs.B,
                                                                           bw.grid_crs.q))
        n = jobs.n_out
        self.best = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        self.sb = torch.full((n,), float("nan"), device="cuda")
        self.st = torch.full((n,), float("nan"), device="cuda")

    def run(self, stream=None):
        import paper_1907_11678_amd as semb
        semb.scan_batch(self.dg, self.dj, self.kind, self.qc, self.bw.w_cmp, self.A, self.B, self.qr,
                        self.bw.w_crs, self.tiles, self.ng, self.np, self.best, self.sb, self.st, self.ws,
                        stream=stream)

    def outputs(self):
        return (self.best.cpu().numpy(), self.sb.cpu().numpy().astype(np.float64),
                self.st.cpu().numpy().astype(np.float64))


def _kind_rows(bw, kind):
    rows = []
    for j in np.nonzero(bw.kind == kind)[0]:
        o = int(bw.jobs.out_off[j])
        rows.append(np.arange(o, o + int(bw.gathers.ns[bw.jobs.central[j]])))
    return np.concatenate(rows) if rows else np.zeros(0, np.int64)


@pytest.mark.parametrize("split,w_cmp,w_crs", [(256, 11, 9), (4096, 11, 9), (256, 15, 15), (256, 9, 11)])
def test_batch_equals_per_kind_scans(split, w_cmp, w_crs):
    """A 40-gather stretch of the batched line (uneven fold 8..120 and length
    500..2000): the batch must reproduce cmp_scan on its CMP jobs and crs_scan
    on its CRS jobs exactly (same per-cell sums in the same order), in every
    batch tile shape and for every window the batch kernel is built for (CRS
    tiles hold 4 parameters per wave at w 9 and 2 above)."""
    import dataclasses
    import torch
    import paper_1907_11678_amd as semb
    bw = dataclasses.replace(synth.batched_line(ids=range(2000, 2040)), w_cmp=w_cmp, w_crs=w_crs)
    b = Batch(bw, split)
    refs = {}
    for kind, grid, w in ((0, bw.grid_cmp, bw.w_cmp), (1, bw.grid_crs, bw.w_crs)):
        sub = bw.subset(kind)
        refs[kind] = gu.run_scan("cmp" if kind == 0 else "crs", bw.gathers, sub, grid, w, dg=b.dg,
                                 dj=gu.device_inputs(bw.gathers, sub)[1])
    try:
        for shape in range(semb.BATCH_SHAPES):
            semb.set_batch_choice(bw.w_cmp, bw.w_crs, b.dg, b.dj, shape, split)
            assert semb.batch_choice(bw.w_cmp, bw.w_crs, b.dg, b.dj) == (shape, split)
            b.best.fill_(-7)
            b.run()
            torch.cuda.synchronize()
            best, sb, st = b.outputs()
            for kind in (0, 1):
                ref = refs[kind]
                rows = _kind_rows(bw, kind)
                assert np.array_equal(best[rows], ref[0][rows]), (shape, kind)
                assert np.array_equal(sb[rows], ref[1][rows]), (shape, kind)
                assert np.array_equal(st[rows], ref[2][rows]), (shape, kind)
    finally:
        semb.set_batch_choice(bw.w_cmp, bw.w_crs, b.dg, b.dj, -1)
    _say("batch == per-kind scans in every shape", b.ntiles, "tiles", b.ng, "groups")


def test_batch_tuner_records_a_bit_identical_choice():
    """tune_batch times every batch shape over two splits on a 200-gather
    stretch, excludes none (they are bit-identical), records the fastest
    (shape, split), and the scan with the recorded choice still equals the
    per-kind scans."""
    import torch
    import paper_1907_11678_amd as semb
    bw = synth.batched_line(ids=range(1000, 1200))
    b = Batch(bw, 256)
    jobs, gs = bw.jobs, bw.gathers
    shape, split, times = semb.tune_batch(b.dg, b.dj, bw.kind, b.kind, b.qc, bw.w_cmp, b.A, b.B, b.qr, bw.w_crs,
                                          jobs.central, jobs.apert_ptr, jobs.apert_gather, gs.ns, gs.trace_ptr,
                                          b.best, b.sb, b.st, splits=(256, 1024), reps=1, sample_jobs=120)
    try:
        _say("batch tuner:", shape, split, times)
        assert set(times) == {256, 1024}
        assert all(m >= 0 for ms in times.values() for m in ms)
        assert semb.batch_choice(bw.w_cmp, bw.w_crs, b.dg, b.dj) == (shape, split)
        faster = {(s, sp): ms[s] for sp, ms in times.items() for s in range(semb.BATCH_SHAPES)}
        assert faster[(shape, split)] == min(faster[(s, split)] for s in range(semb.BATCH_SHAPES)
                                             if s == 0 or faster[(s, split)] < 0.98 * faster[(0, split)])
        b2 = Batch(bw, split)
        b2.run()
        torch.cuda.synchronize()
        best, sb, st = b2.outputs()
        for kind, grid, w in ((0, bw.grid_cmp, bw.w_cmp), (1, bw.grid_crs, bw.w_crs)):
            sub = bw.subset(kind)
            ref = gu.run_scan("cmp" if kind == 0 else "crs", gs, sub, grid, w, dg=b.dg,
                              dj=gu.device_inputs(gs, sub)[1])
            rows = _kind_rows(bw, kind)
            assert np.array_equal(best[rows], ref[0][rows]) and np.array_equal(sb[rows], ref[1][rows])
    finally:
        semb.clear_tuning()


def test_tiles_outside_the_given_plan_sizes_are_skipped():
    """Called with ngroups = nparts = 0 for a plan whose CRS tiles are split
    into groups, the kernel skips every split tile (their rows stay unwritten)
    and still computes the unsplit CMP tiles exactly.  The workspace is sized
    for the real plan, so every address the call could form stays inside it."""
    import torch
    import paper_1907_11678_amd as semb
    bw = synth.batched_line(ids=range(2000, 2012))
    b = Batch(bw, 256)
    assert b.ng > 0 and b.np > 0
    semb.scan_batch(b.dg, b.dj, b.kind, b.qc, bw.w_cmp, b.A, b.B, b.qr, bw.w_crs, b.tiles, 0, 0,
                    b.best, b.sb, b.st, b.ws)
    torch.cuda.synchronize()
    best, sb, st = b.outputs()
    crs_rows, cmp_rows = _kind_rows(bw, 1), _kind_rows(bw, 0)
    assert (best[crs_rows] == -7).all() and np.isnan(sb[crs_rows]).all()
    sub = bw.subset(0)
    ref = gu.run_scan("cmp", bw.gathers, sub, bw.grid_cmp, bw.w_cmp, dg=b.dg,
                      dj=gu.device_inputs(bw.gathers, sub)[1])
    assert np.array_equal(best[cmp_rows], ref[0][cmp_rows])
    assert np.array_equal(sb[cmp_rows], ref[1][cmp_rows])
    _say("skipped", len(crs_rows), "CRS rows of split tiles; CMP rows equal the per-kind scan")


def test_batch_matches_oracle_on_sampled_rows():
    import torch
    bw = synth.batched_line(ids=range(600, 624))
    b = Batch(bw)
    b.run()
    torch.cuda.synchronize()
    best, sb, st = b.outputs()
    rng = np.random.default_rng(4)
    for kind, grid, w, nrow in ((0, bw.grid_cmp, bw.w_cmp, 48), (1, bw.grid_crs, bw.w_crs, 16)):
        sub = bw.subset(kind)
        pick = rng.integers(0, sub.njobs, nrow)
        rj = pick.astype(np.int32)
        rs = np.array([rng.integers(0, int(bw.gathers.ns[sub.central[j]])) for j in pick], np.int32)
        ref = oracle.scan_rows("cmp" if kind == 0 else "crs", bw.gathers, sub, grid, w, rj, rs)
        rows = sub.out_off[rj] + rs
        _say("batch vs oracle", kind, gu.compare(f"batch kind {kind}", (best, sb, st, None), ref,
                                                 gu.sample_scale(bw.gathers, sub), rows))


def test_batch_graph_replay():
    """Capture the batch (energy planes, counter reset, persistent kernel) in a
    HIP graph; replay it three times with eager work in between and check
    every replay against the eager result."""
    import torch
    bw = synth.batched_line(ids=range(3000, 3030))
    b = Batch(bw)
    b.run()
    torch.cuda.synchronize()
    eager = b.outputs()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(stream=s)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    for k in range(3):
        b.best.fill_(-7)
        b.sb.fill_(float("nan"))
        b.st.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = b.outputs()
        for a_, e_ in zip(got, eager):
            assert np.array_equal(a_, e_), f"replay {k} differs"
        del junk


def test_batch_full_size_sampled():
    """The whole 4096-gather batched line in the bench's configuration (split
    256, one persistent launch); the oracle checks sampled rows of both kinds."""
    import torch
    bw = synth.batched_line()
    _say("batched line generated")
    b = Batch(bw, 256)
    b.run()
    torch.cuda.synchronize()
    best, sb, st = b.outputs()
    rng = np.random.default_rng(12)
    for kind, grid, w, nrow in ((0, bw.grid_cmp, bw.w_cmp, 32), (1, bw.grid_crs, bw.w_crs, 12)):
        sub = bw.subset(kind)
        pick = rng.integers(0, sub.njobs, nrow)
        rj = pick.astype(np.int32)
        rs = np.array([rng.integers(0, int(bw.gathers.ns[sub.central[j]])) for j in pick], np.int32)
        ref = oracle.scan_rows("cmp" if kind == 0 else "crs", bw.gathers, sub, grid, w, rj, rs)
        rows = sub.out_off[rj] + rs
        _say("full batch vs oracle", kind, gu.compare(f"full batch kind {kind}", (best, sb, st, None), ref,
                                                      gu.sample_scale(bw.gathers, sub), rows))
