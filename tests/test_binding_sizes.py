"""The Python binding refuses tensors smaller than what a call reads or
writes, before anything reaches the library (the C ABI sees only pointers).
CPU-only: the size checks run before any device pointer is taken."""
from __future__ import annotations

import pytest

torch = pytest.importorskip("torch")
semb = pytest.importorskip("paper_1907_11678_amd")


def _inputs(n_out=100, njobs=2):
    g = semb.DeviceGathers(samples=torch.zeros(1000), sample_off=torch.zeros(2, dtype=torch.int64),
                           trace_ptr=torch.zeros(3, dtype=torch.int32), ns=torch.zeros(2, dtype=torch.int32),
                           half_offset=torch.zeros(10), midpoint=torch.zeros(10), central_x=torch.zeros(2),
                           ns_max=50, dt=0.004)
    j = semb.DeviceJobs(central=torch.zeros(njobs, dtype=torch.int32), apert_ptr=None, apert_gather=None,
                        out_off=torch.zeros(njobs, dtype=torch.int64), max_apert=1, n_out=n_out)
    return g, j


def test_scan_outputs_must_hold_every_row_and_panel_cell():
    g, j = _inputs()
    q = torch.zeros(7)
    ok = torch.zeros(100)
    with pytest.raises(ValueError, match="best"):
        semb.cmp_scan(g, j, q, 11, torch.zeros(99, dtype=torch.int32), ok, ok, torch.zeros(16))
    with pytest.raises(ValueError, match="stack_out"):
        semb.cmp_scan(g, j, q, 11, torch.zeros(100, dtype=torch.int32), ok, torch.zeros(3), torch.zeros(16))
    with pytest.raises(ValueError, match="panel"):
        semb.cmp_scan(g, j, q, 11, torch.zeros(100, dtype=torch.int32), ok, ok, torch.zeros(16),
                      panel=torch.zeros(100 * 7 - 1))
    A, B = torch.zeros(3), torch.zeros(2)
    with pytest.raises(ValueError, match="panel_f16"):
        semb.crs_scan(g, j, A, B, q, 9, torch.zeros(100, dtype=torch.int32), ok, ok, torch.zeros(16),
                      panel_f16=torch.zeros(100 * 42 - 1, dtype=torch.float16))


def test_point_calls_need_three_parameters_per_row():
    g, j = _inputs()
    with pytest.raises(ValueError, match="theta"):
        semb.stack(g, j, 0, torch.zeros(299), 11, torch.zeros(100), torch.zeros(100))
    with pytest.raises(ValueError, match="g_theta"):
        semb.semblance_grad(g, j, 0, torch.zeros(300), torch.zeros(100), 11, torch.zeros(10))
    with pytest.raises(ValueError, match="g_samples"):
        semb.semblance_grad(g, j, 0, torch.zeros(300), torch.zeros(100), 11, torch.zeros(300),
                            g_samples=torch.zeros(999))
    with pytest.raises(ValueError, match="s_out"):
        semb.refine(g, j, 0, torch.zeros(300), 11, torch.zeros(5), torch.zeros(100))
    with pytest.raises(ValueError, match="theta"):
        semb.theta_from_best(torch.zeros(10, dtype=torch.int32), torch.zeros(4), torch.zeros(29))


def test_multistart_helpers_check_their_shapes():
    with pytest.raises(ValueError, match="best_k"):
        semb.panel_peaks(torch.zeros(10, 60), 3, 4, 5, 2, torch.zeros(19, dtype=torch.int32), torch.zeros(20))
    with pytest.raises(ValueError, match="theta_out"):
        semb.best_of(torch.zeros(2, 10), torch.zeros(2, 10), torch.zeros(2, 10, 3), torch.zeros(10),
                     torch.zeros(10), torch.zeros(29))


def test_no_jobs_needs_no_outputs():
    """With no jobs nothing is written, so empty outputs pass the size checks
    (the call then fails only on the CPU tensors, which this test expects)."""
    g, j = _inputs(n_out=0, njobs=0)
    with pytest.raises(ValueError, match="GPU"):
        semb.cmp_scan(g, j, torch.zeros(7), 11, torch.zeros(0, dtype=torch.int32), torch.zeros(0),
                      torch.zeros(0), torch.zeros(16))


def test_gathers_and_jobs_arrays_must_agree_in_length():
    g, j = _inputs()
    g.trace_ptr = torch.zeros(2, dtype=torch.int32)  # 2 gathers need 3 entries
    with pytest.raises(ValueError, match="trace_ptr"):
        g.cstruct()
    g, j = _inputs()
    g.midpoint = torch.zeros(9)  # 10 traces
    with pytest.raises(ValueError, match="midpoint"):
        g.cstruct()
    g, j = _inputs()
    j.out_off = torch.zeros(3, dtype=torch.int64)  # 2 jobs
    with pytest.raises(ValueError, match="out_off"):
        j.cstruct()
    j = semb.DeviceJobs(central=torch.zeros(2, dtype=torch.int32), apert_ptr=torch.zeros(2, dtype=torch.int32),
                        apert_gather=torch.zeros(2, dtype=torch.int32), out_off=torch.zeros(2, dtype=torch.int64),
                        max_apert=1, n_out=10)
    with pytest.raises(ValueError, match="apert_ptr"):
        j.cstruct()
