"""Host-side checks of the C ABI (no GPU needed, nothing is launched):
the library loads, exports every function include/semb.h declares, and
rejects invalid arguments before enqueueing anything."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semb.h")


@pytest.fixture(scope="module")
def semb():
    import paper_1907_11678_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1907_11678_amd import build
        build.build()
    pkg.lib()
    return pkg


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("cmp_scan", "crs_scan", "stack", "semblance_grad", "semb_workspace_bytes",
              "semb_last_error", "semb_version"):
        assert n in names, names


def test_library_exports_every_declared_function(semb):
    out = subprocess.check_output(["nm", "-D", "--defined-only", semb.LIB_PATH]).decode()
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = C.CDLL(semb.LIB_PATH)
    for n in declared_functions():
        getattr(L, n)


def test_library_targets_gfx950(semb):
    blob = open(semb.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def _gathers(semb, **kw):
    fake = 0x1000  # never dereferenced: validation fails before any device access
    g = semb.CGathers(fake, fake, fake, fake, fake, fake, fake, 1, 1, 64, 64, 0.004)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def _jobs(semb, **kw):
    fake = 0x2000
    j = semb.CJobs(fake, fake, fake, fake, 1, 1, 64)
    for k, v in kw.items():
        setattr(j, k, v)
    return j


def _outs(semb):
    fake = 0x3000
    return semb.COutputs(fake, fake, fake, None)


@pytest.mark.parametrize("bad", [
    dict(g=dict(dt=0.0)), dict(g=dict(dt=float("nan"))), dict(g=dict(ns_max=0)),
    dict(g=dict(ns_max=5000)), dict(g=dict(samples=None)), dict(g=dict(ngathers=0)),
    dict(j=dict(njobs=-1)), dict(j=dict(max_apert=0)), dict(j=dict(central=None)),
    dict(w=4), dict(w=0), dict(w=33), dict(nq=0),
])
def test_invalid_arguments_return_einval(semb, bad):
    L = semb.lib()
    g = _gathers(semb, **bad.get("g", {}))
    j = _jobs(semb, **bad.get("j", {}))
    out = _outs(semb)
    st = L.cmp_scan(C.byref(g), C.byref(j), C.c_void_p(0x4000), bad.get("nq", 8), bad.get("w", 11),
                    C.byref(out), C.c_void_p(0x10000), 1 << 20, None)
    assert st == 1, semb.last_error()
    assert semb.last_error()


def test_crs_requires_midpoints_and_aperture(semb):
    L = semb.lib()
    g = _gathers(semb, midpoint=None)
    j = _jobs(semb)
    out = _outs(semb)
    P = C.c_void_p(0x4000)
    assert L.crs_scan(C.byref(g), C.byref(j), P, 2, P, 2, P, 2, 9, C.byref(out), C.c_void_p(0x10000),
                      1 << 20, None) == 1
    g = _gathers(semb)
    j = _jobs(semb, apert_ptr=None)
    assert L.crs_scan(C.byref(g), C.byref(j), P, 2, P, 2, P, 2, 9, C.byref(out), C.c_void_p(0x10000),
                      1 << 20, None) == 1


def test_small_or_misaligned_workspace(semb):
    L = semb.lib()
    g = _gathers(semb, nsamples=1000)
    j = _jobs(semb)
    out = _outs(semb)
    need = semb.workspace_bytes(1000)
    assert need >= 3 * 1000 * 4
    P = C.c_void_p(0x4000)
    assert L.cmp_scan(C.byref(g), C.byref(j), P, 8, 11, C.byref(out), C.c_void_p(0x10000), need - 1,
                      None) == 2
    assert L.cmp_scan(C.byref(g), C.byref(j), P, 8, 11, C.byref(out), C.c_void_p(0x10004), need,
                      None) == 2
    assert L.cmp_scan(C.byref(g), C.byref(j), P, 8, 11, C.byref(out), None, need, None) == 2


def test_noalloc_scan_validates(semb):
    """semb_scan_noalloc rejects gathers larger than its static scratch, and
    every argument cmp_scan / crs_scan reject, before touching the device."""
    L = semb.lib()
    out = _outs(semb)
    P = C.c_void_p(0x4000)
    limit = semb.NOALLOC_SCRATCH_BYTES
    assert semb.workspace_bytes(limit // 12 - 4096) <= limit < semb.workspace_bytes(limit // 12 + 4096)
    g = _gathers(semb, nsamples=limit // 12 + 4096)
    assert L.semb_scan_noalloc(0, C.byref(g), C.byref(_jobs(semb)), None, 1, None, 1, P, 8, 11, C.byref(out),
                               None) == 1
    assert "scratch" in semb.last_error()
    g = _gathers(semb, nsamples=1000)
    assert L.semb_scan_noalloc(0, C.byref(g), C.byref(_jobs(semb)), None, 1, None, 1, P, 8, 4, C.byref(out),
                               None) == 1  # even w
    assert L.semb_scan_noalloc(2, C.byref(g), C.byref(_jobs(semb)), None, 1, None, 1, P, 8, 11, C.byref(out),
                               None) == 1  # bad kind
    assert L.semb_scan_noalloc(1, C.byref(g), C.byref(_jobs(semb)), None, 1, None, 1, P, 8, 9, C.byref(out),
                               None) == 1  # CRS without A, B


def test_theta_shift_validates(semb):
    """semb_theta_shift rejects a negative n, missing arrays, lo > hi and a
    non-finite shift before it touches the device; n = 0 is a no-op."""
    L = semb.lib()
    f3 = C.c_float * 3
    P = C.c_void_p(0x4000)
    ok = (f3(0, 0, 1), f3(-1, -1, -1), f3(1, 1, 1))
    assert L.semb_theta_shift(P, 0, *ok, None) == 0
    assert L.semb_theta_shift(P, -1, *ok, None) == 1
    assert L.semb_theta_shift(None, 4, *ok, None) == 1
    assert L.semb_theta_shift(P, 4, f3(0, 0, 1), f3(-1, 2, -1), f3(1, 1, 1), None) == 1
    assert L.semb_theta_shift(P, 4, f3(0, float("nan"), 1), f3(-1, -1, -1), f3(1, 1, 1), None) == 1
    assert L.semb_theta_shift(P, 4, None, f3(-1, -1, -1), f3(1, 1, 1), None) == 1


def test_multistart_requires_the_unshifted_start_first(semb):
    """refine_multistart refuses offsets whose first entry is not zero (start 0
    must be the scan's own pick) before it touches the device."""
    with pytest.raises(ValueError):
        semb.refine_multistart(None, None, 1, None, None, None, None, 9, 2, None, None, None, None, None, None,
                               None, None, offsets=((0.0, 0.0, 0.3), (0.0, 0.0, 0.0)))
    with pytest.raises(ValueError):  # a peak the panel search does not return
        semb.refine_multistart(None, None, 1, None, None, None, None, 9, 2, None, None, None, None, None, None,
                               None, None, starts=((0, (0, 0, 0)), (2, (0, 0, 0))))
    k0, o0 = semb.MULTISTART_STARTS[0]
    assert k0 == 0 and all(v == 0.0 for v in o0)
    assert max(k for k, _ in semb.MULTISTART_STARTS) < semb.MULTISTART_PEAKS


def test_probe_validates(semb):
    """semb_probe rejects unknown probes, reps outside 1..100 and missing
    outputs before it touches the device."""
    L = semb.lib()
    r, m = C.c_double(), C.c_double()
    assert L.semb_probe(5, 5, C.byref(r), C.byref(m)) == 1
    assert L.semb_probe(-1, 5, C.byref(r), C.byref(m)) == 1
    assert L.semb_probe(0, 0, C.byref(r), C.byref(m)) == 1
    assert L.semb_probe(0, 101, C.byref(r), C.byref(m)) == 1
    assert L.semb_probe(0, 5, None, C.byref(m)) == 1
    assert set(semb.PROBES) == {"fma_f32", "fma_f64", "rsq_f64", "lds_read", "lds_read2"}


def test_point_calls_validate(semb):
    L = semb.lib()
    g = _gathers(semb)
    j = _jobs(semb)
    P = C.c_void_p(0x4000)
    assert L.stack(C.byref(g), C.byref(j), 7, P, 11, P, P, None) == 1          # bad kind
    assert L.stack(C.byref(g), C.byref(j), 0, None, 11, P, P, None) == 1       # no theta
    assert L.semblance_grad(C.byref(g), C.byref(j), 0, P, None, 11, P, None, None) == 1  # no g_s
    assert L.semblance_grad(C.byref(g), C.byref(j), 1, P, P, 10, P, None, None) == 1    # even w


def test_refinement_peaks_best_of_and_corrected_gathers_validate(semb):
    """Host-side checks of the point-path helpers: each bad argument is
    rejected with SEMB_EINVAL before anything touches the (fake) device
    pointers."""
    L = semb.lib()
    g = _gathers(semb)
    j = _jobs(semb)
    P = C.c_void_p(0x4000)

    def opts(**kw):
        o = semb.CRefineOpts(8, 0.5, 1.25, (C.c_float * 3)(1e-4, 1e-8, 1e-7), (C.c_float * 3)(-1, -1, 0),
                             (C.c_float * 3)(1, 1, 1))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    assert L.semb_refine(C.byref(g), C.byref(j), 7, P, C.byref(opts()), 11, P, P, None) == 1   # kind
    assert L.semb_refine(C.byref(g), C.byref(j), 0, P, None, 11, P, P, None) == 1             # no options
    for bad in (dict(steps=-1), dict(grow=0.5), dict(eta0=float("nan")), dict(eta0=-1.0),
                dict(lo=(C.c_float * 3)(0, 0, 2)), dict(scale=(C.c_float * 3)(1, float("inf"), 1))):
        assert L.semb_refine(C.byref(g), C.byref(j), 0, P, C.byref(opts(**bad)), 11, P, P, None) == 1, bad
    assert L.semb_refine(C.byref(g), C.byref(j), 0, None, C.byref(opts()), 11, P, P, None) == 1  # no theta

    assert L.semb_theta_from_best(P, -1, None, 0, None, 0, P, 4, P, None) == 1                # n_out
    assert L.semb_theta_from_best(P, 10, None, 0, None, 0, None, 4, P, None) == 1             # no q
    assert L.semb_theta_from_best(P, 10, None, 0, None, 0, P, 0, P, None) == 1                # nq
    assert L.semb_theta_from_best(P, 10, P, 0, P, 2, P, 4, P, None) == 1                      # nA with A
    assert L.semb_theta_from_best(P, 10, P, 70000, P, 70000, P, 4, P, None) == 1              # grid size

    assert L.semb_corrected_gathers(C.byref(g), C.byref(j), 5, P, P, P, None) == 1            # kind
    assert L.semb_corrected_gathers(C.byref(g), C.byref(j), 0, None, P, P, None) == 1         # no theta
    assert L.semb_corrected_gathers(C.byref(g), C.byref(j), 0, P, None, P, None) == 1         # no offsets

    for n, nA, nB, nq, K in ((-1, 1, 1, 5, 2), (4, 0, 1, 5, 2), (4, 1, 1, 0, 2), (4, 1, 1, 5, 0),
                             (4, 1, 1, 5, 9), (4, 70000, 70000, 5, 2)):
        assert L.semb_panel_peaks(P, n, nA, nB, nq, K, P, P, None) == 1, (n, nA, nB, nq, K)
    assert L.semb_panel_peaks(None, 4, 1, 1, 5, 2, P, P, None) == 1

    assert L.semb_best_of(0, 4, P, P, P, P, P, P, None) == 1
    assert L.semb_best_of(2, -1, P, P, P, P, P, P, None) == 1
    assert L.semb_best_of(2, 4, P, None, P, P, P, P, None) == 1
    assert semb.last_error()


def test_scan_batch_validates(semb):
    L = semb.lib()
    g = _gathers(semb, nsamples=1000)
    j = _jobs(semb)
    P = C.c_void_p(0x4000)

    def batch(**kw):
        b = semb.CBatch(P, P, 101, 11, P, 11, P, 11, P, 21, 9)
        for k, v in kw.items():
            setattr(b, k, v)
        return b

    need = semb.batch_workspace_bytes(1000, 11, 9, 0, 0)
    ws = C.c_void_p(0x100000)
    out = _outs(semb)
    tiles = C.c_void_p(0x5000)
    assert L.scan_batch(C.byref(g), C.byref(j), C.byref(batch(w_cmp=13)), tiles, 1, 0, 0, C.byref(out), ws, need,
                        None) == 1                                                           # window
    assert L.scan_batch(C.byref(g), C.byref(j), C.byref(batch(nq_cmp=0)), tiles, 1, 0, 0, C.byref(out), ws, need,
                        None) == 1                                                           # no CMP grid
    assert L.scan_batch(C.byref(g), C.byref(j), C.byref(batch()), tiles, -1, 0, 0, C.byref(out), ws, need,
                        None) == 1                                                           # plan sizes
    assert L.scan_batch(C.byref(g), C.byref(j), C.byref(batch()), None, 4, 0, 0, C.byref(out), ws, need,
                        None) == 1                                                           # no tiles
    with_panel = semb.COutputs(0x3000, 0x3000, 0x3000, 0x3000, None)
    assert L.scan_batch(C.byref(g), C.byref(j), C.byref(batch()), tiles, 1, 0, 0, C.byref(with_panel), ws, need,
                        None) == 1                                                           # panel
    assert L.scan_batch(C.byref(g), C.byref(j), C.byref(batch()), tiles, 1, 0, 0, C.byref(out), ws, need - 1,
                        None) == 2                                                           # workspace size
    assert L.scan_batch(C.byref(g), C.byref(j), C.byref(batch()), tiles, 1, 0, 0, C.byref(out),
                        C.c_void_p(0x100004), need, None) == 2                               # alignment


def test_version(semb):
    assert "gfx950" in semb.version()


def test_batch_plan_host_only(semb):
    """The planner is host code: tiles cover every (job, sample block,
    parameter) once, longest first, with consistent groups."""
    import numpy as np
    kind = np.array([0, 1, 1, 0], np.int32)
    central = np.arange(4, dtype=np.int32)
    apert_ptr = np.array([0, 1, 4, 6, 7], np.int32)
    apert_gather = np.array([0, 0, 1, 2, 2, 3, 3], np.int32)
    ns = np.array([100, 64, 300, 1], np.int32)
    trace_ptr = np.array([0, 5, 7, 20, 22], np.int32)
    tiles, ng, npart = semb.batch_plan(kind, central, apert_ptr, apert_gather, ns, trace_ptr, 101, 2541, 256)
    cover = {}
    for t in tiles:
        cover.setdefault((int(t[0]), int(t[1])), []).append((int(t[2]), int(t[3]), int(t[4]), int(t[5]),
                                                             int(t[6]), int(t[7])))
    assert set(cover) == {(0, 0), (0, 1), (1, 0), (2, 0), (2, 1), (2, 2), (2, 3), (2, 4), (3, 0)}
    for (j, sb), parts in cover.items():
        parts.sort()
        npar = 2541 if kind[j] else 101
        assert parts[0][0] == 0 and parts[-1][1] == npar
        assert all(parts[i][1] == parts[i + 1][0] for i in range(len(parts) - 1))
        assert all(p[4] == len(parts) for p in parts)
        assert sorted(p[3] for p in parts) == list(range(len(parts)))
        if len(parts) > 1:
            assert len({p[2] for p in parts}) == 1 and parts[0][2] >= 0
    assert ng == 1 * 5 + 1 * 1 and npart == 6 * 10
    # the CRS tiles (cost ~ 64 x 256 x traces) come before the CMP ones
    assert tiles[0][0] in (1, 2)


def test_batch_plan_rounds_the_split_to_whole_blocks(semb):
    """A requested split is rounded up to whole 32-parameter blocks (8 waves x
    4 parameters of a CRS tile)."""
    import numpy as np
    kind = np.array([1, 0], np.int32)
    tiles, ng, npart = semb.batch_plan(kind, np.array([0, 1], np.int32), np.array([0, 2, 3], np.int32),
                                       np.array([0, 1, 1], np.int32), np.array([64, 64], np.int32),
                                       np.array([0, 3, 6], np.int32), 101, 2541, 40)
    spans = sorted((int(t[2]), int(t[3])) for t in tiles if t[0] == 0)
    assert spans[0] == (0, 64) and spans[-1] == (2496, 2541)
    assert all(b - a == 64 for a, b in spans[:-1]) and len(spans) == 40


def test_batch_plan_never_splits_at_int32_max(semb):
    import numpy as np
    kind = np.array([1, 0], np.int32)
    tiles, ng, npart = semb.batch_plan(kind, np.array([0, 1], np.int32), np.array([0, 2, 3], np.int32),
                                       np.array([0, 1, 1], np.int32), np.array([130, 64], np.int32),
                                       np.array([0, 3, 6], np.int32), 101, 2541, 2 ** 31 - 1)
    assert len(tiles) == 3 + 1 and ng == 0 and npart == 0
    assert all(int(t[2]) == 0 and int(t[6]) == 1 for t in tiles)


def test_batch_plan_rejects_bad_input(semb):
    import numpy as np
    with pytest.raises(semb.SembError):
        semb.batch_plan(np.array([2], np.int32), np.array([0], np.int32), np.array([0, 1], np.int32),
                        np.array([0], np.int32), np.array([10], np.int32), np.array([0, 1], np.int32), 5, 5)
    with pytest.raises(semb.SembError):
        semb.batch_plan(np.array([0], np.int32), np.array([3], np.int32), np.array([0, 1], np.int32),
                        np.array([0], np.int32), np.array([10], np.int32), np.array([0, 1], np.int32), 5, 5)
    # a CRS aperture of more than SEMB_APERT_LIMIT (64) gathers cannot be scanned
    ng = 70
    ok = dict(ns=np.full(ng, 10, np.int32), trace_ptr=np.arange(ng + 1, dtype=np.int32))
    semb.batch_plan(np.array([1], np.int32), np.array([30], np.int32), np.array([0, 64], np.int32),
                    np.arange(64, dtype=np.int32), ok["ns"], ok["trace_ptr"], 5, 5)
    with pytest.raises(semb.SembError, match="aperture"):
        semb.batch_plan(np.array([1], np.int32), np.array([30], np.int32), np.array([0, 65], np.int32),
                        np.arange(65, dtype=np.int32), ok["ns"], ok["trace_ptr"], 5, 5)


def test_shape_names_and_host_side_table(semb):
    L = semb.lib()
    for s in range(semb.SCAN_SHAPES):
        assert semb.shape_name(s)
    assert semb.shape_name(semb.SCAN_SHAPES) is None and semb.shape_name(-1) is None
    g = _gathers(semb, ntraces=600, ngathers=20, ns_max=1000)
    j = _jobs(semb, max_apert=9)
    L.semb_clear_tuning()
    assert L.semb_scan_shape(0, 11, C.byref(g), C.byref(j)) == 0
    assert L.semb_scan_shape(1, 11, C.byref(g), C.byref(j)) == 2   # the CRS default
    assert L.semb_set_scan_shape(1, 11, C.byref(g), C.byref(j), 3) == 0
    assert L.semb_scan_shape(1, 11, C.byref(g), C.byref(j)) == 3
    g2 = _gathers(semb, ntraces=600, ngathers=20, ns_max=1900)  # another ns bucket
    assert L.semb_scan_shape(1, 11, C.byref(g2), C.byref(j)) == 2
    assert L.semb_scan_shape(1, 9, C.byref(g), C.byref(j)) == 2   # other window
    assert L.semb_set_scan_shape(1, 11, C.byref(g), C.byref(j), semb.SCAN_SHAPES) == 1
    assert L.semb_set_scan_shape(2, 11, C.byref(g), C.byref(j), 0) == 1
    assert L.semb_set_scan_shape(1, 11, C.byref(g), C.byref(j), -1) == 0
    assert L.semb_scan_shape(1, 11, C.byref(g), C.byref(j)) == 2
    L.semb_clear_tuning()


def test_tuner_rejects_bad_arguments(semb):
    L = semb.lib()
    g, j, out = _gathers(semb), _jobs(semb), _outs(semb)
    shape = C.c_int32(0)
    P = C.c_void_p(0x4000)
    assert L.semb_tune_scan(C.byref(g), C.byref(j), 0, None, 1, None, 1, P, 8, 11, 0, 1, C.byref(out),
                            C.c_void_p(0x10000), 1 << 20, C.byref(shape), None, None) == 1
    assert L.semb_tune_scan(C.byref(g), C.byref(j), 0, None, 1, None, 1, P, 8, 11, 4, 1, C.byref(out),
                            C.c_void_p(0x10000), 1 << 20, None, None, None) == 1
    assert L.semb_tune_scan(C.byref(g), C.byref(j), 5, None, 1, None, 1, P, 8, 11, 4, 1, C.byref(out),
                            C.c_void_p(0x10000), 1 << 20, C.byref(shape), None, None) == 1


def test_tuning_table_round_trip(semb, tmp_path):
    """Scan and batch choices written with semb_tuning_save come back after a
    clear with semb_tuning_load; a file with a line that is not an entry is
    refused and leaves the table as it was."""
    L = semb.lib()
    L.semb_clear_tuning()
    g1, g2 = _gathers(semb, ntraces=30, ngathers=1, ns_max=1000), _gathers(semb, ntraces=60, ngathers=1, ns_max=2000)
    j1 = _jobs(semb, max_apert=9)
    assert L.semb_set_scan_shape(0, 15, C.byref(g2), C.byref(j1), 3) == 0
    assert L.semb_set_scan_shape(1, 9, C.byref(g1), C.byref(j1), 4) == 0
    assert L.semb_set_batch_choice(11, 9, C.byref(g1), C.byref(j1), 2, 1024) == 0
    path = str(tmp_path / "tuning.txt")
    assert semb.save_tuning(path) == 3
    L.semb_clear_tuning()
    assert semb.lib().semb_scan_shape(0, 15, C.byref(g2), C.byref(j1)) == 0
    sh, sp = C.c_int32(-1), C.c_int32(-1)
    L.semb_batch_choice(11, 9, C.byref(g1), C.byref(j1), C.byref(sh), C.byref(sp))
    assert (sh.value, sp.value) == (0, 256)
    assert semb.load_tuning(path) == 3
    assert L.semb_scan_shape(0, 15, C.byref(g2), C.byref(j1)) == 3
    assert L.semb_scan_shape(1, 9, C.byref(g1), C.byref(j1)) == 4
    L.semb_batch_choice(11, 9, C.byref(g1), C.byref(j1), C.byref(sh), C.byref(sp))
    assert (sh.value, sp.value) == (2, 1024)
    bad = tmp_path / "bad.txt"
    bad.write_text("scan 0 15 6 11 1\nnot an entry\n")
    with pytest.raises(semb.SembError):
        semb.load_tuning(str(bad))
    assert L.semb_scan_shape(0, 15, C.byref(g2), C.byref(j1)) == 3  # unchanged
    for text in ("batch 11 9 5 10 7 256\n",        # shape out of range
                 "scan 0 15 6 11 1 extra\n",       # trailing words
                 "scan 0 14 6 11 1\n",             # an even window
                 "batch 11 9 -1 10 0 256\n",       # a negative bucket
                 "scan 0 15 6 11 1" + " " * 300 + "\n"):  # longer than any entry
        bad.write_text(text)
        with pytest.raises(semb.SembError):
            semb.load_tuning(str(bad))
    assert L.semb_scan_shape(0, 15, C.byref(g2), C.byref(j1)) == 3  # still unchanged
    ok = tmp_path / "ok.txt"
    ok.write_text("# a comment\n\n   \n  scan 0 15 6 11 2  \r\n")  # blank lines, spaces, CRLF
    assert semb.load_tuning(str(ok)) == 1
    with pytest.raises(semb.SembError):
        semb.load_tuning(str(tmp_path / "missing.txt"))
    L.semb_clear_tuning()


def test_shape_count_matches_the_header(semb):
    text = open(HEADER).read()
    assert f"#define SEMB_SCAN_SHAPES {semb.SCAN_SHAPES}" in text
    assert f"#define SEMB_BATCH_SHAPES {semb.BATCH_SHAPES}" in text
    assert all(semb.batch_shape_name(s) for s in range(semb.BATCH_SHAPES))
    assert semb.batch_shape_name(semb.BATCH_SHAPES) is None


def test_shape_table_under_concurrent_threads(semb):
    """The tuner's process-wide table is guarded by a mutex: threads that set,
    read and clear their own keys concurrently (ctypes releases the GIL during
    the calls) each see their own entries."""
    import threading
    L = semb.lib()
    L.semb_clear_tuning()
    errors = []

    def worker(k):
        g = _gathers(semb, ntraces=600, ngathers=20, ns_max=64 << (k % 4))
        j = _jobs(semb, max_apert=9)
        w = 2 * k + 1
        try:
            for it in range(2000):
                shape = (k + it) % semb.SCAN_SHAPES
                assert L.semb_set_scan_shape(k % 2, w, C.byref(g), C.byref(j), shape) == 0
                got = L.semb_scan_shape(k % 2, w, C.byref(g), C.byref(j))
                assert got == shape, (k, it, got, shape)
            assert L.semb_set_scan_shape(k % 2, w, C.byref(g), C.byref(j), -1) == 0
        except AssertionError as e:  # pragma: no cover - reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors[:3]
    L.semb_clear_tuning()
