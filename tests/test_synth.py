"""The seeded input generator: determinism, subsets, shapes and counts."""
import numpy as np

import synth


def test_cmp_subset_regenerates_bit_identically():
    full = synth.cmp_plain()
    sub = synth.cmp_plain(ids=[3, 17, 63])
    for k, g in enumerate([3, 17, 63]):
        assert np.array_equal(full.gathers.gather(g), sub.gathers.gather(k))
        a, b = full.gathers.trace_ptr[g], full.gathers.trace_ptr[g + 1]
        assert np.array_equal(full.gathers.half_offset[a:b], sub.gathers.half_offset[24 * k:24 * (k + 1)])


def test_cmp_plain_shape_and_eval_count():
    w = synth.cmp_plain(ids=[0, 1])
    assert w.gathers.gather(0).shape == (24, 1000)
    assert w.gathers.dt == float(np.float32(0.004))
    h = w.gathers.half_offset
    assert (h >= 0).all() and (h <= 1500).all()
    assert np.all(np.diff(h[:24]) >= 0)
    full = synth.cmp_plain()
    assert synth.count_evals(full.gathers, full.jobs, full.grid) == 64 * 24 * 1000 * 101


def test_velocity_grid_is_four_over_v_squared():
    q = synth.velocity_grid(1500.0, 4500.0, 101)
    v = 1500.0 + 30.0 * np.arange(101)
    assert np.allclose(q, 4.0 / v ** 2, rtol=1e-7, atol=0)
    assert q.dtype == np.float32


def test_crs_line_subset_matches_full_line_gathers():
    spec = synth.crs_line_spec()
    wl = synth.crs_line(centrals=[10, 11])
    direct = synth.line_gathers(spec, ids=list(range(6, 16)))
    assert wl.gathers.ngathers == 10
    assert np.array_equal(wl.gathers.samples, direct.samples)
    assert list(wl.jobs.apert_ptr) == [0, 9, 18]
    assert wl.grid.n == 21 * 21 * 41
    assert np.allclose(wl.gathers.central_x, 12.5 * np.arange(6, 16))


def test_cmp_fill_matches_per_gather_generation():
    spec = synth.cmp_large_spec()
    spec.ngathers = 3
    out = np.empty(3 * spec.fold * spec.ns, np.float32)
    h = np.empty(3 * spec.fold, np.float32)
    synth.cmp_fill(spec, out, h, threads=2)
    tr, hh = synth.cmp_gather(spec, 2)
    assert np.array_equal(out[2 * spec.fold * spec.ns:], tr.ravel())
    assert np.array_equal(h[2 * spec.fold:], hh)


def test_batched_line_shapes_and_kinds():
    spec = synth.batched_line_spec()
    folds, nss = zip(*[synth._line_shape(spec, g) for g in range(200)])
    assert min(folds) >= 8 and max(folds) <= 120 and min(nss) >= 500 and max(nss) <= 2000
    kinds = synth.batched_kinds()
    assert kinds.size == 4096 and int((kinds == 0).sum()) == 2867


def test_noise_level_follows_snr():
    spec = synth.cmp_plain_spec()
    spec.snr = 1e12
    clean, _ = synth.cmp_gather(spec, 0)
    spec2 = synth.cmp_plain_spec()
    noisy, _ = synth.cmp_gather(spec2, 0)
    rms = np.sqrt(np.mean(clean.astype(np.float64) ** 2))
    noise = noisy.astype(np.float64) - clean
    assert abs(np.sqrt(np.mean(noise ** 2)) / rms - 1.0 / spec2.snr) < 0.01


def test_paper_shapes():
    assert synth.paper_window(220) == 19 and synth.paper_window(240) == 17
    for d, (fold, ns, _) in synth.PAPER_DATASETS.items():
        spec = synth.paper_shape_spec(d, 10)
        assert spec.fold == fold and spec.ns == ns
    wl = synth.paper_shape(5, 3)
    assert wl.gathers.ngathers == 3 and int(wl.gathers.trace_ptr[-1]) == 3000
    assert (wl.gathers.ns == 550).all() and wl.w == 19 and wl.grid.q.size == 101
    sub = synth.paper_shape(5, 3, centrals=[2])
    assert np.array_equal(sub.gathers.gather(0), wl.gathers.gather(2))
    crs = synth.paper_shape(2, 9, kind="crs", half_aperture=1, centrals=[4])
    assert crs.jobs.njobs == 1 and crs.gathers.ngathers == 3 and crs.w == 17
    assert crs.grid.n == 7 * 7 * 11
