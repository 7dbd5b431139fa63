"""FP64 CPU oracle of the semblance scan -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
import this module.  It wraps ``oracle.c`` (plain C, FP64, OpenMP over output
rows) through ctypes.  It shares no code with the HIP path; the only thing the
two sides have in common is the seeded input generator in ``synth``.

Every function takes a ``synth.Gathers``/``synth.Jobs``/``synth.Grid`` triple
(plain numpy arrays) and returns numpy arrays in FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CMP, CRS = 0, 1
_KIND = {"cmp": CMP, "crs": CRS}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Library:
    """ctypes view of one build of oracle.c (the default build, or a variant
    compiled by a test from a modified copy of the source)."""

    def __init__(self, path: str):
        L = C.CDLL(path)
        P = C.c_void_p
        i32, f64 = C.c_int32, C.c_double
        common = [C.c_int, P, P, P, P, P, P, P, f64, i32, P, P, P, P]
        L.oracle_scan.argtypes = common + [P, i32, P, i32, P, i32, i32, P, P, P, P, P, P, P, P, C.c_int]
        L.oracle_point.argtypes = common + [P, i32, P, P, P, P, C.c_int]
        L.oracle_grad.argtypes = common + [P, P, i32, P, P, P, P, P, P, C.c_int]
        L.oracle_corrected.argtypes = common + [P, P, P, C.c_int]
        L.oracle_corrected.restype = C.c_int
        L.oracle_scan_rows.argtypes = [C.c_int, P, P, P, P, P, P, P, f64, i32, P, P, P, P, P,
                                       P, i32, P, i32, P, i32, i32, P, P, P, P, P, P, C.c_int]
        for f in (L.oracle_scan, L.oracle_point, L.oracle_grad, L.oracle_scan_rows):
            f.restype = C.c_int
        L.oracle_max_threads.restype = C.c_int
        L.oracle_set_fragility.argtypes = [C.c_double, C.c_double]
        L.oracle_set_fragility.restype = None
        L.oracle_set_kink.argtypes = [C.c_double]
        L.oracle_set_kink.restype = None
        self.L = L
        self.path = path


_lib = None


def lib() -> Library:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = Library(LIB)
    return _lib


def compile_variant(src_text: str, out_dir: str) -> Library:
    """Compile a (modified) copy of the oracle source into out_dir and load it."""
    src = os.path.join(out_dir, "oracle_variant.c")
    so = os.path.join(out_dir, "liboracle_variant.so")
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so,
                           src, "-lm"])
    return Library(so)


FRAGILE_DEFAULT = (1e-3, 1e-6)


def set_fragility(tau_samples: float, t_rel: float, library: Library | None = None):
    """Set the perturbations that flag a cell as fragile (see oracle.c)."""
    (library or lib()).L.oracle_set_fragility(float(tau_samples), float(t_rel))


KINK_DEFAULT = 1e-4


def set_kink(tau_samples: float, library: Library | None = None):
    """Set the distance (samples) of a contributing intersection from an
    integer that flags its cell as a kink of the gradient (see oracle.c)."""
    (library or lib()).L.oracle_set_kink(float(tau_samples))


def max_threads() -> int:
    return int(lib().L.oracle_max_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class _Args:
    """Keeps contiguous copies alive for the duration of a call."""

    def __init__(self, kind, gs, jobs):
        self.kind = _KIND[kind] if isinstance(kind, str) else int(kind)
        self.keep = [
            _c(gs.samples, np.float32), _c(gs.sample_off, np.int64), _c(gs.trace_ptr, np.int32),
            _c(gs.ns, np.int32), _c(gs.half_offset, np.float32), _c(gs.midpoint, np.float32),
            _c(gs.central_x, np.float32),
        ]
        self.jobs = [_c(jobs.central, np.int32), _c(jobs.apert_ptr, np.int32),
                     _c(jobs.apert_gather, np.int32), _c(jobs.out_off, np.int64)]
        self.dt = float(gs.dt)
        self.njobs = int(jobs.central.shape[0])

    def head(self):
        k = self.keep
        j = self.jobs
        return [self.kind, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]), _p(k[5]), _p(k[6]),
                self.dt, self.njobs, _p(j[0]), _p(j[1]), _p(j[2]), _p(j[3])]


@dataclass
class ScanResult:
    best: np.ndarray     # int32 [n_out] flat parameter index
    s_best: np.ndarray   # float64 [n_out]
    stack: np.ndarray    # float64 [n_out]
    gap: np.ndarray      # float64 [n_out] best S minus runner-up S
    fragile: np.ndarray  # bool [n_out]
    panel: np.ndarray | None  # float64 [n_out, n_params]
    cond: np.ndarray | None = None  # float64 [n_out] condition number of S at the pick
    panel_cond: np.ndarray | None = None  # float64 [n_out, n_params] of every cell (with panel)


def _n_out(jobs) -> int:
    return int(jobs.n_out)


def scan(kind, gs, jobs, grid, w: int, panel: bool = False, nthreads: int | None = None,
         library: Library | None = None) -> ScanResult:
    """Exhaustive semblance scan in FP64 (section 3.2's grid search)."""
    a = _Args(kind, gs, jobs)
    n = _n_out(jobs)
    A, B, q = _c(grid.A, np.float32), _c(grid.B, np.float32), _c(grid.q, np.float32)
    npar = (A.size * B.size if a.kind == CRS else 1) * q.size
    best = np.zeros(n, np.int32)
    sb = np.zeros(n, np.float64)
    st = np.zeros(n, np.float64)
    gap = np.zeros(n, np.float64)
    fr = np.zeros(n, np.uint8)
    cond = np.zeros(n, np.float64)
    pan = np.zeros((n, npar), np.float64) if panel else None
    pcond = np.zeros((n, npar), np.float64) if panel else None
    rc = (library or lib()).L.oracle_scan(*a.head(), _p(A), A.size, _p(B), B.size, _p(q), q.size, int(w),
                           _p(best), _p(sb), _p(st), _p(pan), _p(gap), _p(fr), _p(cond), _p(pcond),
                           int(nthreads or max_threads()))
    if rc != 0:
        raise ValueError("oracle_scan: invalid arguments")
    return ScanResult(best, sb, st, gap, fr.astype(bool), pan, cond, pcond)


def scan_rows(kind, gs, jobs, grid, w: int, row_job, row_s, nthreads: int | None = None,
              library: Library | None = None) -> ScanResult:
    """The exhaustive scan for selected output rows (row r = sample row_s[r] of
    job row_job[r]); results are indexed by r (panel is None)."""
    a = _Args(kind, gs, jobs)
    rj = _c(row_job, np.int32)
    rs = _c(row_s, np.int32)
    n = rj.size
    A, B, q = _c(grid.A, np.float32), _c(grid.B, np.float32), _c(grid.q, np.float32)
    best = np.zeros(n, np.int32)
    sb = np.zeros(n, np.float64)
    st = np.zeros(n, np.float64)
    gap = np.zeros(n, np.float64)
    fr = np.zeros(n, np.uint8)
    cond = np.zeros(n, np.float64)
    k = a.keep
    j = a.jobs
    rc = (library or lib()).L.oracle_scan_rows(
        a.kind, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]), _p(k[5]), _p(k[6]), a.dt, n,
        _p(rj), _p(rs), _p(j[0]), _p(j[1]), _p(j[2]), _p(A), A.size, _p(B), B.size, _p(q), q.size,
        int(w), _p(best), _p(sb), _p(st), _p(gap), _p(fr), _p(cond), int(nthreads or max_threads()))
    if rc != 0:
        raise ValueError("oracle_scan_rows: invalid arguments")
    return ScanResult(best, sb, st, gap, fr.astype(bool), None, cond)


def point(kind, gs, jobs, theta: np.ndarray, w: int, nthreads: int | None = None,
          library: Library | None = None):
    """Semblance, stack, contributing-trace count and fragility per output row
    at theta[row] = (A, B, q)."""
    a = _Args(kind, gs, jobs)
    n = _n_out(jobs)
    th = _c(theta, np.float64).reshape(n, 3)
    s = np.zeros(n, np.float64)
    st = np.zeros(n, np.float64)
    m = np.zeros(n, np.int32)
    fr = np.zeros(n, np.uint8)
    rc = (library or lib()).L.oracle_point(*a.head(), _p(th), int(w), _p(s), _p(st), _p(m), _p(fr),
                            int(nthreads or max_threads()))
    if rc != 0:
        raise ValueError("oracle_point: invalid arguments")
    return s, st, m, fr.astype(bool)


@dataclass
class GradDetail:
    """Sizes and flags that go with a gradient (see oracle_grad)."""
    g_theta_mag: np.ndarray      # [n_out, 3] the gradient's terms summed by magnitude
    g_samples_mag: np.ndarray    # [n_samples] same for the sample gradient
    rough: np.ndarray            # bool [n_out] kink or fragile row
    samples_rough: np.ndarray    # bool [n_samples] read by a rough row's windows


def grad(kind, gs, jobs, theta: np.ndarray, g_s: np.ndarray, w: int, samples_grad: bool = True,
         nthreads: int | None = None, library: Library | None = None, detail: bool = False):
    """dL/dtheta [n_out, 3] and dL/dsamples (or None) for L = sum g_s * S(theta);
    with detail=True also a GradDetail."""
    a = _Args(kind, gs, jobs)
    n = _n_out(jobs)
    th = _c(theta, np.float64).reshape(n, 3)
    gsv = _c(g_s, np.float64).reshape(n)
    gt = np.zeros((n, 3), np.float64)
    nsm = gs.samples.shape[0]
    gsm = np.zeros(nsm, np.float64) if samples_grad else None
    d = GradDetail(np.zeros((n, 3)), np.zeros(nsm), np.zeros(n, np.uint8), np.zeros(nsm, np.uint8)) \
        if detail else None
    rc = (library or lib()).L.oracle_grad(
        *a.head(), _p(th), _p(gsv), int(w), _p(gt), _p(gsm),
        _p(d.g_theta_mag) if d else None, _p(d.g_samples_mag) if d else None,
        _p(d.rough) if d else None, _p(d.samples_rough) if d else None,
        int(nthreads or max_threads()))
    if rc != 0:
        raise ValueError("oracle_grad: invalid arguments")
    if d is None:
        return gt, gsm
    d.rough = d.rough.astype(bool)
    d.samples_rough = d.samples_rough.astype(bool)
    return gt, gsm, d


def corrected_offsets(gs, jobs) -> tuple[np.ndarray, int]:
    """(corr_off [njobs], total): job j's corrected traces start at corr_off[j]
    and hold (aperture traces) x (samples of its central gather) values."""
    tp = np.asarray(gs.trace_ptr, np.int64)
    off = np.zeros(jobs.njobs, np.int64)
    tot = 0
    for j in range(jobs.njobs):
        ag = jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]
        ntr = int((tp[ag + 1] - tp[ag]).sum())
        off[j] = tot
        tot += ntr * int(gs.ns[jobs.central[j]])
    return off, tot


def corrected(kind, gs, jobs, theta: np.ndarray, nthreads: int | None = None,
              library: Library | None = None):
    """The aperture traces of every job read along theta[row] (see
    oracle_corrected); returns (values [total], corr_off [njobs])."""
    a = _Args(kind, gs, jobs)
    n = _n_out(jobs)
    th = _c(theta, np.float64).reshape(n, 3)
    off, tot = corrected_offsets(gs, jobs)
    out = np.zeros(max(tot, 1), np.float64)
    rc = (library or lib()).L.oracle_corrected(*a.head(), _p(th), _p(off), _p(out), int(nthreads or max_threads()))
    if rc != 0:
        raise ValueError("oracle_corrected: invalid arguments")
    return out[:tot], off


def theta_of(grid, flat: np.ndarray, kind) -> np.ndarray:
    """(A, B, q) [n, 3] of flat parameter indices (flat = (iA*nB + iB)*nq + iq)."""
    flat = np.asarray(flat, np.int64)
    nq, nB = grid.q.size, grid.B.size
    out = np.zeros((flat.size, 3), np.float64)
    out[:, 2] = grid.q[flat % nq]
    if (_KIND[kind] if isinstance(kind, str) else kind) == CRS:
        out[:, 1] = grid.B[(flat // nq) % nB]
        out[:, 0] = grid.A[flat // (nq * nB)]
    return out
