"""MI355X-native semblance parameter scan (CMP and 2D CRS).

Thin Python binding of ``libsemb.so`` (HIP kernels for gfx950 behind the C
ABI in ``include/semb.h``).  Every step of the computation runs in those
kernels; this module only marshals arguments: torch tensors provide device
memory and the current HIP stream, and their pointers are handed to the C
functions of the same names (``cmp_scan``, ``crs_scan``, ``stack``,
``semblance_grad``).  There is no CPU fallback: if the library is missing
or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsemb.so")

KIND_CMP, KIND_CRS = 0, 1
W_MAX = 31
NS_LIMIT = 2048
APERT_LIMIT = 64
_STATUS = {0: "SEMB_OK", 1: "SEMB_EINVAL", 2: "SEMB_EWORKSPACE", 3: "SEMB_EHIP"}


class SembError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


# ---------------------------------------------------------------------------
# C structs (mirror include/semb.h)
# ---------------------------------------------------------------------------
class CGathers(C.Structure):
    _fields_ = [("samples", C.c_void_p), ("sample_off", C.c_void_p), ("trace_ptr", C.c_void_p),
                ("ns", C.c_void_p), ("half_offset", C.c_void_p), ("midpoint", C.c_void_p),
                ("central_x", C.c_void_p), ("ngathers", C.c_int32), ("ntraces", C.c_int32),
                ("ns_max", C.c_int32), ("nsamples", C.c_int64), ("dt", C.c_float)]


class CJobs(C.Structure):
    _fields_ = [("central", C.c_void_p), ("apert_ptr", C.c_void_p), ("apert_gather", C.c_void_p),
                ("out_off", C.c_void_p), ("njobs", C.c_int32), ("max_apert", C.c_int32),
                ("n_out", C.c_int64)]


class COutputs(C.Structure):
    _fields_ = [("best", C.c_void_p), ("s_best", C.c_void_p), ("stack", C.c_void_p),
                ("panel", C.c_void_p), ("panel_f16", C.c_void_p)]


class CRefineOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("eta0", C.c_float), ("grow", C.c_float), ("scale", C.c_float * 3), ("lo", C.c_float * 3),
                ("hi", C.c_float * 3)]


class CTile(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("job", "sblk", "p_begin", "p_end", "group", "split", "nsplit",
                                          "part_base")]


class CBatchHost(C.Structure):
    _fields_ = [("njobs", C.c_int32), ("kind", C.c_void_p), ("central", C.c_void_p),
                ("apert_ptr", C.c_void_p), ("apert_gather", C.c_void_p), ("ngathers", C.c_int32),
                ("ns", C.c_void_p), ("trace_ptr", C.c_void_p), ("npar_cmp", C.c_int32),
                ("npar_crs", C.c_int32)]


class CBatch(C.Structure):
    _fields_ = [("kind", C.c_void_p), ("q_cmp", C.c_void_p), ("nq_cmp", C.c_int32), ("w_cmp", C.c_int32),
                ("A", C.c_void_p), ("nA", C.c_int32), ("B", C.c_void_p), ("nB", C.c_int32),
                ("q_crs", C.c_void_p), ("nq_crs", C.c_int32), ("w_crs", C.c_int32)]


_lib = None


def lib():
    """The loaded libsemb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_1907_11678_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.semb_workspace_bytes.argtypes = [i64]
        L.semb_workspace_bytes.restype = C.c_size_t
        L.cmp_scan.argtypes = [P, P, P, i32, i32, P, P, C.c_size_t, P]
        L.semb_scan_noalloc.argtypes = [i32, P, P, P, i32, P, i32, P, i32, i32, P, P]
        L.crs_scan.argtypes = [P, P, P, i32, P, i32, P, i32, i32, P, P, C.c_size_t, P]
        L.stack.argtypes = [P, P, i32, P, i32, P, P, P]
        L.semblance_grad.argtypes = [P, P, i32, P, P, i32, P, P, P]
        for f in (L.cmp_scan, L.crs_scan, L.stack, L.semblance_grad):
            f.restype = C.c_int
        L.semb_batch_plan.argtypes = [P, i32, P, i64, P, P]
        L.semb_batch_plan.restype = i64
        L.semb_batch_workspace_bytes.argtypes = [i64, i32, i32, i32, i32]
        L.semb_batch_workspace_bytes.restype = C.c_size_t
        L.scan_batch.argtypes = [P, P, P, P, i64, i32, i32, P, P, C.c_size_t, P]
        L.scan_batch.restype = C.c_int
        L.semb_refine.argtypes = [P, P, i32, P, P, i32, P, P, P]
        L.semb_refine.restype = C.c_int
        L.semb_theta_from_best.argtypes = [P, i64, P, i32, P, i32, P, i32, P, P]
        L.semb_theta_from_best.restype = C.c_int
        L.semb_shape_name.argtypes = [i32]
        L.semb_shape_name.restype = C.c_char_p
        L.semb_tune_scan.argtypes = [P, P, i32, P, i32, P, i32, P, i32, i32, i32, i32, P, P, C.c_size_t, P, P, P]
        L.semb_tune_scan.restype = C.c_int
        L.semb_set_scan_shape.argtypes = [i32, i32, P, P, i32]
        L.semb_set_scan_shape.restype = C.c_int
        L.semb_scan_shape.argtypes = [i32, i32, P, P]
        L.semb_scan_shape.restype = i32
        L.semb_clear_tuning.argtypes = []
        L.semb_clear_tuning.restype = None
        L.semb_corrected_gathers.argtypes = [P, P, i32, P, P, P, P]
        L.semb_corrected_gathers.restype = C.c_int
        L.semb_panel_peaks.argtypes = [P, i64, i32, i32, i32, i32, P, P, P]
        L.semb_panel_peaks.restype = C.c_int
        L.semb_best_of.argtypes = [i32, i64, P, P, P, P, P, P, P]
        L.semb_best_of.restype = C.c_int
        L.semb_batch_shape_name.argtypes = [i32]
        L.semb_batch_shape_name.restype = C.c_char_p
        L.semb_set_batch_choice.argtypes = [i32, i32, P, P, i32, i32]
        L.semb_set_batch_choice.restype = C.c_int
        L.semb_batch_choice.argtypes = [i32, i32, P, P, P, P]
        L.semb_batch_choice.restype = None
        L.semb_tune_batch.argtypes = [P, P, P, P, i64, i32, i32, i32, i32, P, P, C.c_size_t, P, P, P]
        L.semb_tune_batch.restype = C.c_int
        L.semb_tuning_save.argtypes = [C.c_char_p]
        L.semb_tuning_save.restype = C.c_int32
        L.semb_tuning_load.argtypes = [C.c_char_p]
        L.semb_tuning_load.restype = C.c_int32
        L.semb_radius_apertures.argtypes = [P, P, i32, P, i32, C.c_double, P, P, P]
        L.semb_radius_apertures.restype = i64
        L.semb_kernel_timer_start.argtypes = [i32]
        L.semb_kernel_timer_start.restype = C.c_int
        L.semb_kernel_timer_stop.argtypes = [P, P, i32]
        L.semb_kernel_timer_stop.restype = C.c_int
        L.semb_theta_shift.argtypes = [P, i64, P, P, P, P]
        L.semb_theta_shift.restype = C.c_int
        L.semb_probe.argtypes = [i32, i32, P, P]
        L.semb_probe.restype = C.c_int
        L.semb_last_error.restype = C.c_char_p
        L.semb_version.restype = C.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().semb_last_error().decode()


def version() -> str:
    return lib().semb_version().decode()


PROBES = {"fma_f32": 0, "fma_f64": 1, "rsq_f64": 2, "lds_read": 3, "lds_read2": 4}


def probe(name: str, reps: int = 5) -> tuple[float, float]:
    """One microbenchmark on the current device: (rate, ms per launch).
    fma_f32 / fma_f64: flops/s of plain FMAs; rsq_f64: v_rsq_f64 lane
    results/s; lds_read: LDS bytes read/s with 16-byte reads; lds_read2: the
    same with the paired 4-byte reads of a scan window."""
    rate, ms = C.c_double(0.0), C.c_double(0.0)
    _check(lib().semb_probe(PROBES[name], int(reps), C.byref(rate), C.byref(ms)))
    return float(rate.value), float(ms.value)


def workspace_bytes(nsamples: int) -> int:
    return int(lib().semb_workspace_bytes(int(nsamples)))


class KernelTimer:
    """Context manager around semb_kernel_timer_start / _stop: collects the
    durations (ms) of the main-kernel launches this thread makes inside the
    block, in launch order, into `.ms` on exit."""

    def __init__(self, capacity: int = 256):
        self.capacity = int(capacity)
        self.ms: list[float] = []

    def __enter__(self):
        _check(lib().semb_kernel_timer_start(self.capacity))
        return self

    def __exit__(self, *exc):
        n = C.c_int32(0)
        buf = (C.c_float * self.capacity)()
        _check(lib().semb_kernel_timer_stop(C.byref(n), buf, self.capacity))
        self.ms = [float(buf[i]) for i in range(min(n.value, self.capacity))]
        return False


def _check(status: int):
    if status != 0:
        raise SembError(status, last_error())


def _ptr(t) -> int | None:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _typed(t, dtype, name):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return _ptr(t)


def _need(t, n: int, name: str):
    """The library writes or reads n elements of t: refuse a smaller tensor
    before anything is enqueued (the C ABI sees only the pointer)."""
    if t is not None and int(t.numel()) < int(n):
        raise ValueError(f"{name} has {int(t.numel())} elements; the call needs {int(n)}")


def _scan_outputs(jobs: "DeviceJobs", npar: int, best, s_best, stack_out, panel=None, panel_f16=None):
    n = jobs.n_out if jobs.njobs > 0 else 0
    for t, name in ((best, "best"), (s_best, "s_best"), (stack_out, "stack_out")):
        _need(t, n, name)
    _need(panel, n * npar, "panel")
    _need(panel_f16, n * npar, "panel_f16")


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# device-resident inputs
# ---------------------------------------------------------------------------
@dataclass
class DeviceGathers:
    """Gathers resident in device memory (see ``include/semb.h``)."""
    samples: object
    sample_off: object
    trace_ptr: object
    ns: object
    half_offset: object
    midpoint: object
    central_x: object
    ns_max: int
    dt: float

    @property
    def ngathers(self) -> int:
        return int(self.ns.numel())

    @property
    def ntraces(self) -> int:
        return int(self.half_offset.numel())

    @property
    def nsamples(self) -> int:
        return int(self.samples.numel())

    def cstruct(self) -> CGathers:
        import torch
        ng, nt = self.ngathers, self.ntraces
        for t, n, name in ((self.sample_off, ng, "sample_off"), (self.trace_ptr, ng + 1, "trace_ptr"),
                           (self.central_x, ng, "central_x"), (self.midpoint, nt, "midpoint")):
            if t is not None and int(t.numel()) != n:
                raise ValueError(f"gathers.{name} has {int(t.numel())} elements; {n} expected "
                                 f"({ng} gathers, {nt} traces)")
        return CGathers(_typed(self.samples, torch.float32, "samples"),
                        _typed(self.sample_off, torch.int64, "sample_off"),
                        _typed(self.trace_ptr, torch.int32, "trace_ptr"),
                        _typed(self.ns, torch.int32, "ns"),
                        _typed(self.half_offset, torch.float32, "half_offset"),
                        _typed(self.midpoint, torch.float32, "midpoint"),
                        _typed(self.central_x, torch.float32, "central_x"),
                        self.ngathers, self.ntraces, int(self.ns_max), self.nsamples, float(self.dt))


@dataclass
class DeviceJobs:
    central: object
    apert_ptr: object
    apert_gather: object
    out_off: object
    max_apert: int
    n_out: int

    @property
    def njobs(self) -> int:
        return int(self.central.numel())

    def cstruct(self) -> CJobs:
        import torch
        nj = self.njobs
        for t, n, name in ((self.out_off, nj, "out_off"), (self.apert_ptr, nj + 1, "apert_ptr")):
            if t is not None and int(t.numel()) != n:
                raise ValueError(f"jobs.{name} has {int(t.numel())} elements; {n} expected ({nj} jobs)")
        return CJobs(_typed(self.central, torch.int32, "central"),
                     _typed(self.apert_ptr, torch.int32, "apert_ptr"),
                     _typed(self.apert_gather, torch.int32, "apert_gather"),
                     _typed(self.out_off, torch.int64, "out_off"),
                     self.njobs, int(self.max_apert), int(self.n_out))


def upload_gathers(samples, sample_off, trace_ptr, ns, half_offset, midpoint, central_x, dt,
                   device="cuda") -> DeviceGathers:
    """Copy host arrays (numpy or torch) to the device with the ABI's dtypes."""
    import torch

    def t(a, dt_):
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            return a.to(device=device, dtype=dt_).contiguous()
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt_)

    ns_host = np.asarray(ns.cpu() if isinstance(ns, torch.Tensor) else ns)
    return DeviceGathers(t(samples, torch.float32), t(sample_off, torch.int64),
                         t(trace_ptr, torch.int32), t(ns, torch.int32),
                         t(half_offset, torch.float32), t(midpoint, torch.float32),
                         t(central_x, torch.float32), int(ns_host.max()) if ns_host.size else 1,
                         float(np.float32(dt)))


def upload_jobs(central, apert_ptr, apert_gather, out_off, n_out, device="cuda") -> DeviceJobs:
    import torch

    def t(a, dt_):
        if a is None:
            return None
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt_)

    ap = None if apert_ptr is None else np.asarray(apert_ptr)
    max_apert = int(np.diff(ap).max()) if ap is not None and ap.size > 1 else 1
    return DeviceJobs(t(central, torch.int32), t(apert_ptr, torch.int32),
                      t(apert_gather, torch.int32), t(out_off, torch.int64), max(1, max_apert),
                      int(n_out))


# ---------------------------------------------------------------------------
# the four calls
# ---------------------------------------------------------------------------
def _outputs(best, s_best, stack_out, panel, panel_f16=None) -> COutputs:
    import torch
    return COutputs(_typed(best, torch.int32, "best"), _typed(s_best, torch.float32, "s_best"),
                    _typed(stack_out, torch.float32, "stack"), _typed(panel, torch.float32, "panel"),
                    _typed(panel_f16, torch.float16, "panel_f16"))


def cmp_scan(g: DeviceGathers, jobs: DeviceJobs, q, w: int, best, s_best, stack_out, ws,
             panel=None, stream=None, panel_f16=None):
    """Enqueue the CMP scan; results land in best / s_best / stack_out (/ panel,
    panel_f16)."""
    import torch
    _scan_outputs(jobs, int(q.numel()), best, s_best, stack_out, panel, panel_f16)
    gs, js, out = g.cstruct(), jobs.cstruct(), _outputs(best, s_best, stack_out, panel, panel_f16)
    _check(lib().cmp_scan(C.byref(gs), C.byref(js), _typed(q, torch.float32, "q"), int(q.numel()),
                          int(w), C.byref(out), _ptr(ws), int(ws.numel() * ws.element_size()),
                          _stream(stream)))


def crs_scan(g: DeviceGathers, jobs: DeviceJobs, A, B, q, w: int, best, s_best, stack_out, ws,
             panel=None, stream=None, panel_f16=None):
    """Enqueue the 2D CRS scan (flat parameter index (iA*nB + iB)*nq + iq)."""
    import torch
    _scan_outputs(jobs, int(A.numel()) * int(B.numel()) * int(q.numel()), best, s_best, stack_out, panel, panel_f16)
    gs, js, out = g.cstruct(), jobs.cstruct(), _outputs(best, s_best, stack_out, panel, panel_f16)
    _check(lib().crs_scan(C.byref(gs), C.byref(js), _typed(A, torch.float32, "A"), int(A.numel()),
                          _typed(B, torch.float32, "B"), int(B.numel()),
                          _typed(q, torch.float32, "q"), int(q.numel()), int(w), C.byref(out),
                          _ptr(ws), int(ws.numel() * ws.element_size()), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # SEMB_NOALLOC_SCRATCH_BYTES


def scan_noalloc(kind: int, g: DeviceGathers, jobs: DeviceJobs, q, w: int, best, s_best, stack_out, A=None,
                 B=None, panel=None, stream=None, panel_f16=None):
    """The CMP (kind 0) or CRS (kind 1) scan without a workspace: the library's
    per-GPU static scratch holds the window-energy planes (semb_scan_noalloc)."""
    import torch
    crs = int(kind) == 1
    npar = (int(A.numel()) * int(B.numel()) if crs else 1) * int(q.numel())
    _scan_outputs(jobs, npar, best, s_best, stack_out, panel, panel_f16)
    gs, js, out = g.cstruct(), jobs.cstruct(), _outputs(best, s_best, stack_out, panel, panel_f16)
    _check(lib().semb_scan_noalloc(int(kind), C.byref(gs), C.byref(js),
                                   _typed(A, torch.float32, "A") if crs else None,
                                   int(A.numel()) if crs else 1,
                                   _typed(B, torch.float32, "B") if crs else None,
                                   int(B.numel()) if crs else 1,
                                   _typed(q, torch.float32, "q"), int(q.numel()), int(w), C.byref(out),
                                   _stream(stream)))


def stack(g: DeviceGathers, jobs: DeviceJobs, kind: int, theta, w: int, s_out, stack_out, stream=None):
    """Semblance and stack at theta[row] = (A, B, q) for every output row."""
    import torch
    n = jobs.n_out if jobs.njobs > 0 else 0
    _need(theta, 3 * n, "theta")
    _need(s_out, n, "s_out")
    _need(stack_out, n, "stack_out")
    gs, js = g.cstruct(), jobs.cstruct()
    _check(lib().stack(C.byref(gs), C.byref(js), int(kind), _typed(theta, torch.float32, "theta"),
                       int(w), _typed(s_out, torch.float32, "s_out"),
                       _typed(stack_out, torch.float32, "stack_out"), _stream(stream)))


def semblance_grad(g: DeviceGathers, jobs: DeviceJobs, kind: int, theta, g_s, w: int, g_theta,
                   g_samples=None, stream=None):
    """dL/dtheta (overwritten) and dL/dsamples (accumulated) for L = sum g_s * S."""
    import torch
    n = jobs.n_out if jobs.njobs > 0 else 0
    _need(theta, 3 * n, "theta")
    _need(g_s, n, "g_s")
    _need(g_theta, 3 * n, "g_theta")
    _need(g_samples, g.nsamples, "g_samples")
    gs, js = g.cstruct(), jobs.cstruct()
    _check(lib().semblance_grad(C.byref(gs), C.byref(js), int(kind),
                                _typed(theta, torch.float32, "theta"),
                                _typed(g_s, torch.float32, "g_s"), int(w),
                                _typed(g_theta, torch.float32, "g_theta"),
                                _typed(g_samples, torch.float32, "g_samples"), _stream(stream)))


def alloc_workspace(nsamples: int, device="cuda"):
    """A workspace tensor of the size cmp_scan / crs_scan need (256-byte aligned)."""
    import torch
    nbytes = workspace_bytes(nsamples)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


# ---------------------------------------------------------------------------
# CRS apertures by radius (host)
# ---------------------------------------------------------------------------
def radius_apertures(x, centrals, radius: float, y=None):
    """(apert_ptr, apert_gather, max_apert) of the gathers within `radius` of
    each central's midpoint (x[, y] per gather, metres).  crs_scan's
    traveltime is the 2D CRS one: it measures dm along the one coordinate the
    gathers' midpoint / central_x hold, whatever y did to the apertures."""
    import numpy as np
    x = np.ascontiguousarray(x, np.float64)
    yv = None if y is None else np.ascontiguousarray(y, np.float64)
    cen = np.ascontiguousarray(centrals, np.int32)
    ptr = np.zeros(cen.size + 1, np.int32)
    mx = C.c_int32(0)
    L = lib()
    args = (x.ctypes.data, None if yv is None else yv.ctypes.data, int(x.size), cen.ctypes.data, int(cen.size),
            float(radius))
    n = L.semb_radius_apertures(*args, ptr.ctypes.data, None, C.byref(mx))
    if n < 0:
        raise SembError(1, last_error())
    ag = np.zeros(max(int(n), 1), np.int32)
    n2 = L.semb_radius_apertures(*args, ptr.ctypes.data, ag.ctypes.data, C.byref(mx))
    if n2 != n:
        raise SembError(1, last_error())
    return ptr, ag[:n], int(mx.value)


# ---------------------------------------------------------------------------
# tile shapes of the exhaustive scan and their tuner
# ---------------------------------------------------------------------------
SCAN_SHAPES = 6


def shape_name(shape: int) -> str | None:
    r = lib().semb_shape_name(int(shape))
    return None if r is None else r.decode()


def tune_scan(kind: int, g: DeviceGathers, jobs: DeviceJobs, q, w: int, best, s_best, stack_out, ws,
              A=None, B=None, sample_jobs: int = 256, reps: int = 2, stream=None):
    """Time every tile shape on the first `sample_jobs` jobs, record the fastest
    whose outputs equal the default shape's, and return (shape, [ms per shape]
    with -1 for excluded shapes).  Synchronizes the stream."""
    import torch
    nA = int(A.numel()) if A is not None else 1
    nB = int(B.numel()) if B is not None else 1
    _scan_outputs(jobs, (nA * nB if kind == KIND_CRS else 1) * int(q.numel()), best, s_best, stack_out)
    gs, js, out = g.cstruct(), jobs.cstruct(), _outputs(best, s_best, stack_out, None)
    shape = C.c_int32(-1)
    ms = (C.c_float * SCAN_SHAPES)()
    _check(lib().semb_tune_scan(C.byref(gs), C.byref(js), int(kind),
                                _typed(A, torch.float32, "A") if A is not None else None, nA,
                                _typed(B, torch.float32, "B") if B is not None else None, nB,
                                _typed(q, torch.float32, "q"), int(q.numel()), int(w), int(sample_jobs),
                                int(reps), C.byref(out), _ptr(ws), int(ws.numel() * ws.element_size()),
                                C.byref(shape), ms, _stream(stream)))
    return int(shape.value), [float(x) for x in ms]


def set_scan_shape(kind: int, w: int, g: DeviceGathers, jobs: DeviceJobs, shape: int):
    """Use `shape` (-1: back to the tuned/default choice) for scans with this key."""
    gs, js = g.cstruct(), jobs.cstruct()
    _check(lib().semb_set_scan_shape(int(kind), int(w), C.byref(gs), C.byref(js), int(shape)))


def scan_shape(kind: int, w: int, g: DeviceGathers, jobs: DeviceJobs) -> int:
    gs, js = g.cstruct(), jobs.cstruct()
    return int(lib().semb_scan_shape(int(kind), int(w), C.byref(gs), C.byref(js)))


def clear_tuning():
    lib().semb_clear_tuning()


def save_tuning(path: str) -> int:
    """Write the tuning table (scan and batch choices) to `path`; returns the
    number of entries."""
    n = int(lib().semb_tuning_save(os.fsencode(path)))
    if n < 0:
        raise SembError(1, last_error())
    return n


def load_tuning(path: str) -> int:
    """Merge the entries of a saved tuning table into the process's table."""
    n = int(lib().semb_tuning_load(os.fsencode(path)))
    if n < 0:
        raise SembError(1, last_error())
    return n


# ---------------------------------------------------------------------------
# batched scan (mixed CMP / CRS jobs, one persistent launch)
# ---------------------------------------------------------------------------
def batch_plan(kind, central, apert_ptr, apert_gather, ns, trace_ptr, npar_cmp: int, npar_crs: int,
               split_params: int = 256):
    """Tile list of a batch (host arrays in, numpy int32 [ntiles, 8] out), plus
    (ngroups, nparts) for the workspace."""
    arr = [np.ascontiguousarray(a, np.int32) for a in (kind, central, apert_ptr, apert_gather, ns, trace_ptr)]
    p = [a.ctypes.data_as(C.c_void_p) for a in arr]
    h = CBatchHost(int(arr[0].size), p[0], p[1], p[2], p[3], int(arr[4].size), p[4], p[5],
                   int(npar_cmp), int(npar_crs))
    ng, npart = C.c_int32(0), C.c_int32(0)
    n = lib().semb_batch_plan(C.byref(h), int(split_params), None, 0, C.byref(ng), C.byref(npart))
    if n < 0:
        raise SembError(1, last_error())
    tiles = np.zeros((max(n, 1), 8), np.int32)
    n2 = lib().semb_batch_plan(C.byref(h), int(split_params), tiles.ctypes.data_as(C.c_void_p), int(n),
                               C.byref(ng), C.byref(npart))
    if n2 != n:
        raise SembError(1, last_error())
    return tiles[:n], int(ng.value), int(npart.value)


BATCH_SHAPES = 3  # SEMB_BATCH_SHAPES


def batch_shape_name(shape: int) -> str | None:
    r = lib().semb_batch_shape_name(int(shape))
    return r.decode() if r else None


def set_batch_choice(w_cmp: int, w_crs: int, g: DeviceGathers, jobs: DeviceJobs, shape: int, split_params: int = 256):
    gs, js = g.cstruct(), jobs.cstruct()
    _check(lib().semb_set_batch_choice(int(w_cmp), int(w_crs), C.byref(gs), C.byref(js), int(shape),
                                       int(split_params)))


def batch_choice(w_cmp: int, w_crs: int, g: DeviceGathers, jobs: DeviceJobs) -> tuple[int, int]:
    """(batch shape, split_params) recorded for this key (defaults 0, 256)."""
    gs, js = g.cstruct(), jobs.cstruct()
    sh, sp = C.c_int32(0), C.c_int32(0)
    lib().semb_batch_choice(int(w_cmp), int(w_crs), C.byref(gs), C.byref(js), C.byref(sh), C.byref(sp))
    return int(sh.value), int(sp.value)


def tune_batch(g: DeviceGathers, jobs: DeviceJobs, kind_host, kind, q_cmp, w_cmp: int, A, B, q_crs, w_crs: int,
               central, apert_ptr, apert_gather, ns, trace_ptr, best, s_best, stack_out, splits=(256, 1024),
               reps: int = 1, sample_jobs: int | None = None, stream=None):
    """Choose the batch tile shape and parameter split: for each split, plan the
    first `sample_jobs` jobs (all by default; host arrays), time every shape
    with semb_tune_batch (shapes whose outputs differ from shape 0's are
    excluded), and require the outputs of every split to equal the first
    split's bit for bit; record the fastest (shape, split) for the key of the
    whole batch (g, jobs) and return (shape, split, {split: [ms per shape]}).
    Synchronizes the stream."""
    import torch
    nj = len(central) if sample_jobs is None else min(int(sample_jobs), len(central))
    kind_host, central = np.asarray(kind_host)[:nj], np.asarray(central)[:nj]
    apert_ptr = np.asarray(apert_ptr)[:nj + 1]
    nA, nB = int(A.numel()), int(B.numel())
    gs, js = g.cstruct(), jobs.cstruct()
    b = CBatch(_typed(kind, torch.int32, "kind"), _typed(q_cmp, torch.float32, "q_cmp"), int(q_cmp.numel()),
               int(w_cmp), _typed(A, torch.float32, "A"), nA, _typed(B, torch.float32, "B"), nB,
               _typed(q_crs, torch.float32, "q_crs"), int(q_crs.numel()), int(w_crs))
    out = _outputs(best, s_best, stack_out, None)
    times, ref, choice = {}, None, None
    for split in splits:
        tiles, ng, npart = batch_plan(kind_host, central, apert_ptr, apert_gather, ns, trace_ptr,
                                      int(q_cmp.numel()), nA * nB * int(q_crs.numel()), split)
        dt = torch.from_numpy(tiles).to(best.device)
        ws = alloc_batch_workspace(g.nsamples, w_cmp, w_crs, ng, npart, device=best.device)
        shape = C.c_int32(-1)
        ms = (C.c_float * BATCH_SHAPES)()
        _check(lib().semb_tune_batch(C.byref(gs), C.byref(js), C.byref(b), _typed(dt, torch.int32, "tiles"),
                                     int(tiles.shape[0]), ng, npart, int(split), int(reps), C.byref(out), _ptr(ws),
                                     int(ws.numel() * ws.element_size()), C.byref(shape), ms, _stream(stream)))
        # the outputs of the shape just recorded (the last shape timed may have been excluded)
        scan_batch(g, jobs, kind, q_cmp, w_cmp, A, B, q_crs, w_crs, dt, ng, npart, best, s_best, stack_out, ws,
                   stream=stream)
        torch.cuda.synchronize()
        # bit patterns, so that rows no sampled job writes (whatever they hold, NaN included) compare equal
        got = tuple(t.view(torch.int32).clone() for t in (best, s_best, stack_out))
        if ref is None:
            ref = got
        elif not all(torch.equal(x, y) for x, y in zip(got, ref)):
            continue  # a split whose outputs differ is never chosen
        times[split] = [float(x) for x in ms]
        t = times[split][int(shape.value)]
        if choice is None or t < choice[2]:
            choice = (int(shape.value), int(split), t)
    set_batch_choice(w_cmp, w_crs, g, jobs, choice[0], choice[1])
    return choice[0], choice[1], times


def batch_workspace_bytes(nsamples: int, w_cmp: int, w_crs: int, ngroups: int, nparts: int) -> int:
    return int(lib().semb_batch_workspace_bytes(int(nsamples), int(w_cmp), int(w_crs), int(ngroups),
                                                int(nparts)))


def alloc_batch_workspace(nsamples, w_cmp, w_crs, ngroups, nparts, device="cuda"):
    import torch
    nbytes = batch_workspace_bytes(nsamples, w_cmp, w_crs, ngroups, nparts)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def scan_batch(g: DeviceGathers, jobs: DeviceJobs, kind, q_cmp, w_cmp: int, A, B, q_crs, w_crs: int, tiles,
               ngroups: int, nparts: int, best, s_best, stack_out, ws, stream=None):
    """Enqueue the batched scan; tiles: device int32 [ntiles, 8] from batch_plan."""
    import torch
    _scan_outputs(jobs, 0, best, s_best, stack_out)
    _need(kind, jobs.njobs, "kind")
    if tiles.dim() != 2 or int(tiles.shape[1]) != 8:
        raise ValueError("tiles must be [ntiles, 8] as batch_plan returns them")
    gs, js = g.cstruct(), jobs.cstruct()
    b = CBatch(_typed(kind, torch.int32, "kind"), _typed(q_cmp, torch.float32, "q_cmp"), int(q_cmp.numel()),
               int(w_cmp), _typed(A, torch.float32, "A"), int(A.numel()), _typed(B, torch.float32, "B"),
               int(B.numel()), _typed(q_crs, torch.float32, "q_crs"), int(q_crs.numel()), int(w_crs))
    out = _outputs(best, s_best, stack_out, None)
    _check(lib().scan_batch(C.byref(gs), C.byref(js), C.byref(b), _typed(tiles, torch.int32, "tiles"),
                            int(tiles.shape[0]), int(ngroups), int(nparts), C.byref(out), _ptr(ws),
                            int(ws.numel() * ws.element_size()), _stream(stream)))


# ---------------------------------------------------------------------------
# refinement and autograd
# ---------------------------------------------------------------------------
def theta_from_best(best, q, theta, A=None, B=None, stream=None):
    """theta[row] = grid parameter (A, B, q) of the flat index best[row]."""
    import torch
    _need(theta, 3 * int(best.numel()), "theta")
    _check(lib().semb_theta_from_best(_typed(best, torch.int32, "best"), int(best.numel()),
                                      _typed(A, torch.float32, "A"), int(A.numel()) if A is not None else 1,
                                      _typed(B, torch.float32, "B"), int(B.numel()) if B is not None else 1,
                                      _typed(q, torch.float32, "q"), int(q.numel()),
                                      _typed(theta, torch.float32, "theta"), _stream(stream)))


def theta_shift(theta, d, lo=(-1e30, -1e30, -1e30), hi=(1e30, 1e30, 1e30), stream=None):
    """theta [n, 3] += d, clamped to [lo, hi] per component (see semb_theta_shift)."""
    import torch
    n = int(theta.numel()) // 3
    f3 = C.c_float * 3
    _check(lib().semb_theta_shift(_typed(theta, torch.float32, "theta"), n, f3(*d), f3(*lo), f3(*hi),
                                  _stream(stream)))


def refine(g: DeviceGathers, jobs: DeviceJobs, kind: int, theta, w: int, s_out, stack_out, steps: int = 8,
           eta0: float = 0.5, scale=(1.0, 1.0, 1.0), lo=(-1e30, -1e30, -1e30), hi=(1e30, 1e30, 1e30),
           stream=None, grow: float = 1.2):
    """Gradient-ascent refinement of theta [n_out, 3] in place (see semb_refine)."""
    import torch
    n = jobs.n_out if jobs.njobs > 0 else 0
    _need(theta, 3 * n, "theta")
    _need(s_out, n, "s_out")
    _need(stack_out, n, "stack_out")
    gs, js = g.cstruct(), jobs.cstruct()
    o = CRefineOpts(int(steps), float(eta0), float(grow), (C.c_float * 3)(*scale), (C.c_float * 3)(*lo),
                    (C.c_float * 3)(*hi))
    _check(lib().semb_refine(C.byref(gs), C.byref(js), int(kind), _typed(theta, torch.float32, "theta"),
                             C.byref(o), int(w), _typed(s_out, torch.float32, "s_out"),
                             _typed(stack_out, torch.float32, "stack_out"), _stream(stream)))


def corrected_offsets(trace_ptr, ns, central, apert_ptr=None, apert_gather=None):
    """(corr_off [njobs] int64, total) for semb_corrected_gathers: job j's
    corrected traces take (aperture traces) x ns[central[j]] values.  Host
    arrays (numpy)."""
    import numpy as np
    tp = np.asarray(trace_ptr, np.int64)
    ns = np.asarray(ns, np.int64)
    central = np.asarray(central, np.int64)
    if apert_ptr is None:
        ntr = tp[central + 1] - tp[central]
    else:
        ap = np.asarray(apert_ptr, np.int64)
        ag = np.asarray(apert_gather, np.int64)
        per = tp[ag + 1] - tp[ag]
        csum = np.concatenate([[0], np.cumsum(per)])
        ntr = csum[ap[1:]] - csum[ap[:-1]]
    sizes = ntr * ns[central]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return off, int(sizes.sum())


def corrected_gathers(g: DeviceGathers, jobs: DeviceJobs, kind: int, theta, corr_off, out, stream=None):
    """Every job's aperture traces read along theta[row] (see semb_corrected_gathers);
    out must hold the total that corrected_offsets returns."""
    import torch
    _need(theta, 3 * (jobs.n_out if jobs.njobs > 0 else 0), "theta")
    _need(corr_off, jobs.njobs, "corr_off")
    gs, js = g.cstruct(), jobs.cstruct()
    _check(lib().semb_corrected_gathers(C.byref(gs), C.byref(js), int(kind), _typed(theta, torch.float32, "theta"),
                                        _typed(corr_off, torch.int64, "corr_off"), _typed(out, torch.float32, "out"),
                                        _stream(stream)))


def panel_peaks(panel, nA: int, nB: int, nq: int, K: int, best_k, s_k, stream=None):
    """The K best local maxima of each panel row (panel [n_rows, nA*nB*nq]);
    best_k, s_k: [K, n_rows]."""
    import torch
    n = int(panel.shape[0])
    _need(panel, n * int(nA) * int(nB) * int(nq), "panel")
    _need(best_k, int(K) * n, "best_k")
    _need(s_k, int(K) * n, "s_k")
    _check(lib().semb_panel_peaks(_typed(panel, torch.float32, "panel"), n, int(nA), int(nB), int(nq), int(K),
                                  _typed(best_k, torch.int32, "best_k"), _typed(s_k, torch.float32, "s_k"),
                                  _stream(stream)))


def best_of(s_k, stack_k, theta_k, s_out, stack_out, theta_out, stream=None):
    """Per row, the candidate with the largest S among K: s_k, stack_k [K, n],
    theta_k [K, n, 3] -> s_out, stack_out [n], theta_out [n, 3]."""
    import torch
    K, n = int(s_k.shape[0]), int(s_k.shape[1])
    _need(stack_k, K * n, "stack_k")
    _need(theta_k, 3 * K * n, "theta_k")
    _need(s_out, n, "s_out")
    _need(stack_out, n, "stack_out")
    _need(theta_out, 3 * n, "theta_out")
    _check(lib().semb_best_of(K, n, _typed(s_k, torch.float32, "s_k"), _typed(stack_k, torch.float32, "stack_k"),
                              _typed(theta_k, torch.float32, "theta_k"), _typed(s_out, torch.float32, "s_out"),
                              _typed(stack_out, torch.float32, "stack_out"),
                              _typed(theta_out, torch.float32, "theta_out"), _stream(stream)))


# The multi-start rule the bench and the tests use: the 4 best local maxima
# of the coarse panel; the best two each also shifted by -0.3, +0.3, -0.6 and
# +0.6 coarse cells in q; 16 sign steps from each of the 12 starts.  Chosen on
# the CPU with the FP64 oracle on 4 CRS-line centrals (40, 140, 260, 380):
# 94.3% of the rows end within 1e-4 of the fine grid's S (5th percentile of
# the gap -0.0003), against 88.7% (-0.038) for the 4 best peaks with 32 steps
# each, for 192 instead of 128 start-steps.  Shifts along q reach the side
# lobes of the wavelet that share a coarse cell with the main lobe; the third
# and fourth peaks reach basins the best two miss.
MULTISTART_PEAKS = 4
_Q_SHIFTS = ((0.0, 0.0, 0.0), (0.0, 0.0, -0.3), (0.0, 0.0, 0.3), (0.0, 0.0, -0.6), (0.0, 0.0, 0.6))
MULTISTART_STARTS = tuple((k, o) for k in (0, 1) for o in _Q_SHIFTS) + ((2, _Q_SHIFTS[0]), (3, _Q_SHIFTS[0]))
MULTISTART_STEPS = 16


def refine_multistart(g: DeviceGathers, jobs: DeviceJobs, kind: int, panel, A, B, q, w: int, K: int, theta_k,
                      s_k, stack_k, best_k, peak_s, s_out, stack_out, theta_out, steps: int = 8,
                      eta0: float = 0.5, scale=(1.0, 1.0, 1.0), lo=(-1e30, -1e30, -1e30), hi=(1e30, 1e30, 1e30),
                      grow: float = 1.2, stream=None, offsets=((0.0, 0.0, 0.0),), starts=None):
    """Refinement from the K best local maxima of a coarse scan's panel:
    peaks, then one ascent from each start, then the best of them.  A start
    is (peak index < K, offset): the peak's grid parameters shifted by offset
    (in units of `scale`, clamped to [lo, hi]).  `starts` lists them; by
    default every peak with every one of `offsets`.  The first start must be
    (0, zero), the scan's own pick, so the result is never worse than a
    single start.  Scratch tensors: theta_k [len(starts), n, 3], s_k, stack_k
    [len(starts), n] (FP32), best_k [K, n] (int32), peak_s [K, n] (FP32)."""
    if starts is None:
        starts = [(k, o) for k in range(K) for o in offsets]
    starts = [(int(k), tuple(float(v) for v in o)) for k, o in starts]
    if not starts or starts[0][0] != 0 or any(v != 0.0 for v in starts[0][1]):
        raise ValueError("the first start must be peak 0 unshifted")
    if any(k < 0 or k >= K for k, _ in starts):
        raise ValueError(f"a start names a peak outside 0..{K - 1}")
    ns = len(starts)
    if int(theta_k.shape[0]) < ns or int(s_k.shape[0]) < ns or int(stack_k.shape[0]) < ns:
        raise ValueError(f"theta_k, s_k and stack_k need {ns} starts")
    nA = int(A.numel()) if A is not None else 1
    nB = int(B.numel()) if B is not None else 1
    panel_peaks(panel, nA, nB, int(q.numel()), K, best_k, peak_s, stream=stream)
    for i, (k, off) in enumerate(starts):
        theta_from_best(best_k[k], q, theta_k[i], A=A, B=B, stream=stream)
        if any(v != 0.0 for v in off):
            theta_shift(theta_k[i], [off[c] * float(scale[c]) for c in range(3)], lo, hi, stream=stream)
        refine(g, jobs, kind, theta_k[i], w, s_k[i], stack_k[i], steps=steps, eta0=eta0, scale=scale, lo=lo,
               hi=hi, grow=grow, stream=stream)
    best_of(s_k[:ns], stack_k[:ns], theta_k[:ns], s_out, stack_out, theta_out, stream=stream)


def _semblance_at_class():
    import torch

    class SemblanceAt(torch.autograd.Function):
        """S(theta) per output row: forward = `stack`, backward = `semblance_grad`.

        Inputs: samples (the tensor g.samples holds, so its gradient can be
        requested), theta [n_out, 3]; g, jobs, kind and w are constants."""

        @staticmethod
        def forward(ctx, samples, theta, g, jobs, kind, w):
            if samples.data_ptr() != g.samples.data_ptr():
                raise ValueError("samples must be the tensor the gathers were uploaded with")
            theta = theta.contiguous()
            # zeros: rows that no job covers (gaps between out_off ranges) stay 0
            S = torch.zeros(jobs.n_out, dtype=torch.float32, device=theta.device)
            st = torch.zeros_like(S)
            stack(g, jobs, kind, theta, w, S, st)
            ctx.save_for_backward(theta)
            ctx.g, ctx.jobs, ctx.kind, ctx.w = g, jobs, kind, w
            ctx.mark_non_differentiable(st)
            return S, st

        @staticmethod
        def backward(ctx, gS, _gst):
            (theta,) = ctx.saved_tensors
            g_theta = torch.zeros_like(theta)
            g_samples = torch.zeros_like(ctx.g.samples) if ctx.needs_input_grad[0] else None
            semblance_grad(ctx.g, ctx.jobs, ctx.kind, theta, gS.contiguous().float(), ctx.w, g_theta, g_samples)
            return g_samples, g_theta, None, None, None, None

    return SemblanceAt


_SemblanceAt = None


def semblance_at(samples, theta, g: DeviceGathers, jobs: DeviceJobs, kind: int, w: int):
    """Differentiable S (and non-differentiable stack) at theta; see SemblanceAt."""
    global _SemblanceAt
    if _SemblanceAt is None:
        _SemblanceAt = _semblance_at_class()
    return _SemblanceAt.apply(samples, theta, g, jobs, kind, w)
