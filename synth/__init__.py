"""Seeded synthetic seismic gathers for the semblance scan.

This module is shared by the tests, the benchmark and the FP64 oracle's
drivers.  It only *models data*: Ricker wavelets placed on reflection
traveltime curves plus Gaussian noise, and the candidate parameter grids of
each workload.  It contains none of the scan's arithmetic (no interpolation
at an intersection, no semblance, no pick), so neither the oracle nor the
HIP path borrows anything from it beyond its arrays.

Layout of a gather set (the paper's CDP data structure, section 3.2, Fig. 5a):
every gather g owns the traces ``trace_ptr[g] .. trace_ptr[g+1]-1``; those
traces are stored one after another starting at element ``sample_off[g]`` of
``samples``, each ``ns[g]`` samples long, sample n at time n*dt (t=0 first).

Randomness: numpy ``Generator(PCG64)``.  Every gather draws from its own
child stream ``SeedSequence(seed, spawn_key=(0, g))`` and every line-global
event from ``SeedSequence(seed, spawn_key=(1, e))``, so any subset of gathers
regenerates bit-identically without generating the rest.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 1907116780
MIDPOINT_SPACING = 12.5  # m, distance between neighbouring CMP positions on a line


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class Gathers:
    """A set of gathers in the trace-contiguous FP32 layout described above."""

    samples: np.ndarray      # float32 [total samples]
    sample_off: np.ndarray   # int64  [ngathers]
    trace_ptr: np.ndarray    # int32  [ngathers + 1]
    ns: np.ndarray           # int32  [ngathers]
    half_offset: np.ndarray  # float32 [ntraces], metres
    midpoint: np.ndarray     # float32 [ntraces], metres along the line
    central_x: np.ndarray    # float32 [ngathers], metres
    dt: float                # seconds; always a value exactly representable in float32

    @property
    def ngathers(self) -> int:
        return int(self.ns.shape[0])

    @property
    def ntraces(self) -> int:
        return int(self.half_offset.shape[0])

    def trace(self, g: int, i: int) -> np.ndarray:
        """Samples of the i-th trace (local index) of gather g."""
        n = int(self.ns[g])
        o = int(self.sample_off[g]) + i * n
        return self.samples[o:o + n]

    def gather(self, g: int) -> np.ndarray:
        n = int(self.ns[g])
        m = int(self.trace_ptr[g + 1] - self.trace_ptr[g])
        o = int(self.sample_off[g])
        return self.samples[o:o + m * n].reshape(m, n)


@dataclass
class Jobs:
    """Scan jobs: job j stacks at gather ``central[j]`` using the traces of the
    gathers ``apert_gather[apert_ptr[j]:apert_ptr[j+1]]`` (for CMP just the
    central gather).  ``out_off[j]`` is the first output row of job j."""

    central: np.ndarray      # int32 [njobs]
    apert_ptr: np.ndarray    # int32 [njobs + 1]
    apert_gather: np.ndarray  # int32 [sum of aperture sizes]
    out_off: np.ndarray      # int64 [njobs]
    n_out: int               # total output rows

    @property
    def njobs(self) -> int:
        return int(self.central.shape[0])


@dataclass
class Grid:
    """Candidate parameters.  CMP uses q only (A = B = [0]); CRS uses all three.
    Flat parameter index = (iA * nB + iB) * nq + iq."""

    q: np.ndarray                                   # float32, s^2/m^2 (q = 4/v^2)
    A: np.ndarray = field(default_factory=lambda: np.zeros(1, np.float32))  # s/m
    B: np.ndarray = field(default_factory=lambda: np.zeros(1, np.float32))  # s/m^2

    @property
    def n(self) -> int:
        return int(self.A.size * self.B.size * self.q.size)


@dataclass
class Workload:
    name: str
    kind: str        # "cmp" or "crs"
    gathers: Gathers
    jobs: Jobs
    grid: Grid
    w: int           # semblance window length in samples (odd)


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------
def ricker(t: np.ndarray, f: float) -> np.ndarray:
    """Ricker wavelet of peak frequency f (Hz), centred at t=0, peak value 1."""
    a = (math.pi * f * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=key)))


def velocity_grid(v_lo: float, v_hi: float, n: int) -> np.ndarray:
    """n velocities uniformly spaced in [v_lo, v_hi] (FP64) -> q = 4/v^2 in FP32."""
    v = np.linspace(v_lo, v_hi, n, dtype=np.float64)
    return (4.0 / (v * v)).astype(np.float32)


def uniform_grid(lo: float, hi: float, n: int) -> np.ndarray:
    return np.linspace(lo, hi, n, dtype=np.float64).astype(np.float32)


def pack_gathers(traces: list, half_offsets: list, midpoints: list,
                 central_x, dt: float) -> Gathers:
    """Pack per-gather [fold, ns] arrays into the contiguous layout."""
    ns = np.array([t.shape[1] for t in traces], np.int32)
    fold = np.array([t.shape[0] for t in traces], np.int64)
    trace_ptr = np.zeros(len(traces) + 1, np.int32)
    trace_ptr[1:] = np.cumsum(fold)
    sizes = fold * ns.astype(np.int64)
    sample_off = np.zeros(len(traces), np.int64)
    if len(traces) > 1:
        sample_off[1:] = np.cumsum(sizes)[:-1]
    samples = np.empty(int(sizes.sum()), np.float32)
    for g, t in enumerate(traces):
        samples[sample_off[g]:sample_off[g] + sizes[g]] = np.asarray(t, np.float32).ravel()
    return Gathers(samples=samples, sample_off=sample_off, trace_ptr=trace_ptr, ns=ns,
                   half_offset=np.concatenate([np.asarray(h, np.float32) for h in half_offsets])
                   if traces else np.zeros(0, np.float32),
                   midpoint=np.concatenate([np.asarray(m, np.float32) for m in midpoints])
                   if traces else np.zeros(0, np.float32),
                   central_x=np.asarray(central_x, np.float32),
                   dt=float(np.float32(dt)))


def cmp_jobs(gathers: Gathers, ids=None) -> Jobs:
    """One CMP job per gather in ``ids`` (default: all), outputs packed in order."""
    ids = np.arange(gathers.ngathers, dtype=np.int32) if ids is None else np.asarray(ids, np.int32)
    ns = gathers.ns[ids].astype(np.int64)
    out_off = np.zeros(ids.size, np.int64)
    if ids.size > 1:
        out_off[1:] = np.cumsum(ns)[:-1]
    return Jobs(central=ids.copy(), apert_ptr=np.arange(ids.size + 1, dtype=np.int32),
                apert_gather=ids.copy(), out_off=out_off, n_out=int(ns.sum()))


def line_crs_jobs(gathers: Gathers, centrals, half_aperture: int) -> Jobs:
    """CRS jobs on a line: central c uses gathers c-k..c+k (truncated at the ends)."""
    centrals = np.asarray(centrals, np.int32)
    G = gathers.ngathers
    ptr = [0]
    ag = []
    for c in centrals:
        lo, hi = max(0, int(c) - half_aperture), min(G - 1, int(c) + half_aperture)
        ag.extend(range(lo, hi + 1))
        ptr.append(len(ag))
    ns = gathers.ns[centrals].astype(np.int64)
    out_off = np.zeros(centrals.size, np.int64)
    if centrals.size > 1:
        out_off[1:] = np.cumsum(ns)[:-1]
    return Jobs(central=centrals.copy(), apert_ptr=np.asarray(ptr, np.int32),
                apert_gather=np.asarray(ag, np.int32), out_off=out_off, n_out=int(ns.sum()))


def count_evals(gathers: Gathers, jobs: Jobs, grid: Grid) -> int:
    """Nominal evaluations = sum over jobs of ns(central) * n_params * aperture traces."""
    tot = 0
    tp = gathers.trace_ptr.astype(np.int64)
    for j in range(jobs.njobs):
        gs = jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]
        m = int((tp[gs + 1] - tp[gs]).sum())
        tot += int(gathers.ns[jobs.central[j]]) * grid.n * m
    return tot


# --------------------------------------------------------------------------
# CMP gathers: independent hyperbolic events per gather
# --------------------------------------------------------------------------
@dataclass
class CmpSpec:
    ngathers: int
    fold: int
    ns: int
    dt: float
    h_max: float
    nevents: int
    f_peak: float
    t0_range: tuple
    v_range: tuple
    amp_range: tuple
    random_polarity: bool
    snr: float
    seed: int


def cmp_gather(spec: CmpSpec, g: int):
    """Gather g of a CMP workload: (traces [fold, ns] float32, h [fold] float32).

    Each event has zero-offset time t0, velocity v and amplitude a; on a trace
    with half-offset h it arrives at t = sqrt(t0^2 + (2h/v)^2) and adds
    a * ricker(t_n - t).  Gaussian noise of standard deviation
    RMS(noise-free gather)/SNR is then added.
    """
    rng = _rng(spec.seed, 0, g)
    h = np.sort(rng.uniform(0.0, spec.h_max, spec.fold))
    h32 = h.astype(np.float32)
    t0 = rng.uniform(*spec.t0_range, spec.nevents)
    v = rng.uniform(*spec.v_range, spec.nevents)
    amp = rng.uniform(*spec.amp_range, spec.nevents)
    if spec.random_polarity:
        amp = amp * np.where(rng.random(spec.nevents) < 0.5, -1.0, 1.0)
    noise = rng.standard_normal((spec.fold, spec.ns), dtype=np.float32)
    clean = np.zeros((spec.fold, spec.ns), np.float64)
    hh = h32.astype(np.float64)
    for e in range(spec.nevents):
        t = np.sqrt(t0[e] ** 2 + (2.0 * hh / v[e]) ** 2)
        _add_wavelets(clean, t, amp[e] * np.ones_like(t), spec.dt, spec.f_peak)
    rms = math.sqrt(float(np.mean(clean * clean)))
    out = clean + (rms / spec.snr) * noise.astype(np.float64)
    return out.astype(np.float32), h32


def _add_wavelets(dst: np.ndarray, t: np.ndarray, amp: np.ndarray, dt: float, f: float):
    """dst[i, n] += amp[i] * ricker(n*dt - t[i]) for samples within 2/f of t[i]."""
    ntr, ns = dst.shape
    half = int(math.ceil(2.0 / (f * dt))) + 1
    k = np.arange(-half, half + 1)
    centre = np.floor(t / dt).astype(np.int64)
    idx = centre[:, None] + k[None, :]
    ok = (idx >= 0) & (idx < ns) & np.isfinite(t)[:, None] & (amp != 0)[:, None]
    vals = amp[:, None] * ricker(idx * dt - t[:, None], f)
    rows = np.broadcast_to(np.arange(ntr)[:, None], idx.shape)
    dst[rows[ok], idx[ok]] += vals[ok]


def cmp_workload(spec: CmpSpec, q: np.ndarray, w: int, name: str, ids=None,
                 threads: int | None = None) -> Workload:
    """Generate gathers ``ids`` (default all) of a CMP workload."""
    ids = list(range(spec.ngathers)) if ids is None else list(ids)
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda g: cmp_gather(spec, g), ids))
    gs = pack_gathers([r[0] for r in res], [r[1] for r in res],
                      [np.full(spec.fold, MIDPOINT_SPACING * g, np.float32) for g in ids],
                      [MIDPOINT_SPACING * g for g in ids], spec.dt)
    return Workload(name=name, kind="cmp", gathers=gs, jobs=cmp_jobs(gs), grid=Grid(q=q), w=w)


def cmp_fill(spec: CmpSpec, out: np.ndarray, h_out: np.ndarray, threads: int | None = None):
    """Fill preallocated arrays with ALL gathers of a uniform CMP workload.

    out: float32 [ngathers * fold * ns] (e.g. a pinned host buffer viewed as
    numpy); h_out: float32 [ngathers * fold].  Used for workloads too large to
    build through lists.
    """
    threads = threads or min(16, os.cpu_count() or 1)
    per = spec.fold * spec.ns

    def work(g):
        tr, h = cmp_gather(spec, g)
        out[g * per:(g + 1) * per] = tr.ravel()
        h_out[g * spec.fold:(g + 1) * spec.fold] = h

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(spec.ngathers)))


def uniform_cmp_layout(spec: CmpSpec, samples: np.ndarray, half_offset: np.ndarray) -> Gathers:
    G = spec.ngathers
    return Gathers(samples=samples,
                   sample_off=np.arange(G, dtype=np.int64) * (spec.fold * spec.ns),
                   trace_ptr=(np.arange(G + 1, dtype=np.int64) * spec.fold).astype(np.int32),
                   ns=np.full(G, spec.ns, np.int32), half_offset=half_offset,
                   midpoint=np.repeat((np.arange(G) * MIDPOINT_SPACING).astype(np.float32), spec.fold),
                   central_x=(np.arange(G) * MIDPOINT_SPACING).astype(np.float32),
                   dt=float(np.float32(spec.dt)))


# --------------------------------------------------------------------------
# CRS line: line-global events on reflection surfaces
# --------------------------------------------------------------------------
@dataclass
class LineSpec:
    ngathers: int
    fold: object          # int, or (lo, hi) inclusive for a uniform integer fold
    ns: object            # int, or (lo, hi) inclusive
    dt: float
    h_max: float
    nevents: int
    f_peak: float
    t0_range: tuple
    A_range: tuple
    B_range: tuple
    v_range: tuple
    amp_range: tuple
    taper_halfwidth: float
    snr: float
    seed: int


def line_events(spec: LineSpec):
    """Line-global events: arrays x_e, t0, A, B, v, amp (with polarity)."""
    L = MIDPOINT_SPACING * (spec.ngathers - 1)
    ev = np.empty((spec.nevents, 6), np.float64)
    for e in range(spec.nevents):
        r = _rng(spec.seed, 1, e)
        x = r.uniform(0.0, L)
        t0 = r.uniform(*spec.t0_range)
        A = r.uniform(*spec.A_range)
        B = r.uniform(*spec.B_range)
        v = r.uniform(*spec.v_range)
        a = r.uniform(*spec.amp_range) * (-1.0 if r.random() < 0.5 else 1.0)
        ev[e] = (x, t0, A, B, v, a)
    return ev


def _line_shape(spec: LineSpec, g: int):
    """(fold, ns) of gather g; uneven shapes come from the gather's own stream."""
    r = _rng(spec.seed, 2, g)
    fold = spec.fold if isinstance(spec.fold, int) else int(r.integers(spec.fold[0], spec.fold[1] + 1))
    ns = spec.ns if isinstance(spec.ns, int) else int(r.integers(spec.ns[0], spec.ns[1] + 1))
    return fold, ns


def line_gather(spec: LineSpec, g: int, events: np.ndarray):
    """Gather g of a line: midpoint x_g = 12.5 g m for all its traces.

    An event (x_e, t0, A, B, v, a) reaches a trace with midpoint displacement
    d = x_g - x_e and half-offset h at t = sqrt((t0 + 2 A d)^2 + 2 t0 B d^2
    + (4/v^2) h^2) (skipped where the radicand is negative), with amplitude
    a * cos^2(pi d / (2 W)) for |d| < W (W = taper half-width).
    """
    fold, ns = _line_shape(spec, g)
    rng = _rng(spec.seed, 0, g)
    h = np.sort(rng.uniform(0.0, spec.h_max, fold)).astype(np.float32)
    noise = rng.standard_normal((fold, ns), dtype=np.float32)
    xg = float(np.float32(MIDPOINT_SPACING * g))
    clean = np.zeros((fold, ns), np.float64)
    hh = h.astype(np.float64)
    W = spec.taper_halfwidth
    near = np.nonzero(np.abs(xg - events[:, 0]) < W)[0]
    for e in near:
        x, t0, A, B, v, a = events[e]
        d = xg - x
        taper = math.cos(math.pi * d / (2.0 * W)) ** 2
        T = (t0 + 2.0 * A * d) ** 2 + 2.0 * t0 * B * d * d + (4.0 / (v * v)) * hh * hh
        t = np.where(T >= 0.0, np.sqrt(np.maximum(T, 0.0)), np.nan)
        _add_wavelets(clean, t, np.full(fold, a * taper), spec.dt, spec.f_peak)
    rms = math.sqrt(float(np.mean(clean * clean))) if clean.size else 0.0
    out = clean + (rms / spec.snr) * noise.astype(np.float64)
    return out.astype(np.float32), h, xg


def line_gathers(spec: LineSpec, ids=None, threads: int | None = None) -> Gathers:
    """Gathers ``ids`` (default: the whole line) of a line workload."""
    ids = list(range(spec.ngathers)) if ids is None else list(ids)
    events = line_events(spec)
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda g: line_gather(spec, g, events), ids))
    return pack_gathers([r[0] for r in res], [r[1] for r in res],
                        [np.full(r[0].shape[0], r[2], np.float32) for r in res],
                        [r[2] for r in res], spec.dt)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def cmp_plain_spec() -> CmpSpec:
    """64 midpoints x fold 24 x 1000 samples at 4 ms, 5 Ricker(25 Hz) events, SNR 4."""
    return CmpSpec(ngathers=64, fold=24, ns=1000, dt=0.004, h_max=1500.0, nevents=5,
                   f_peak=25.0, t0_range=(0.2, 3.8), v_range=(1800.0, 4000.0),
                   amp_range=(0.5, 1.0), random_polarity=False, snr=4.0, seed=ROOT_SEED + 0)


def cmp_plain(ids=None) -> Workload:
    """CMP plain: 101 velocities 1500..4500 m/s, window 11."""
    return cmp_workload(cmp_plain_spec(), velocity_grid(1500.0, 4500.0, 101), 11, "cmp_plain", ids)


def cmp_large_spec() -> CmpSpec:
    """20000 midpoints x fold 60 x 2000 samples at 2 ms, 8 Ricker(30 Hz) events of
    random polarity, SNR 2."""
    return CmpSpec(ngathers=20000, fold=60, ns=2000, dt=0.002, h_max=3000.0, nevents=8,
                   f_peak=30.0, t0_range=(0.2, 3.8), v_range=(1500.0, 4800.0),
                   amp_range=(0.5, 1.0), random_polarity=True, snr=2.0, seed=ROOT_SEED + 1)


def cmp_large_grid() -> np.ndarray:
    """201 velocities 1400..5000 m/s (18 m/s apart)."""
    return velocity_grid(1400.0, 5000.0, 201)


def cmp_large(ids=None) -> Workload:
    """A subset (default: the first 16 gathers) of the CMP large workload."""
    ids = list(range(16)) if ids is None else ids
    return cmp_workload(cmp_large_spec(), cmp_large_grid(), 15, "cmp_large", ids)


def crs_line_spec() -> LineSpec:
    """A 520-gather line (12.5 m apart), fold 30, 1000 samples at 4 ms, 300 events,
    Ricker 25 Hz, SNR 3."""
    return LineSpec(ngathers=520, fold=30, ns=1000, dt=0.004, h_max=1500.0, nevents=300,
                    f_peak=25.0, t0_range=(0.2, 3.8), A_range=(-4e-4, 4e-4),
                    B_range=(-8e-8, 8e-8), v_range=(1800.0, 4000.0), amp_range=(0.5, 1.0),
                    taper_halfwidth=100.0, snr=3.0, seed=ROOT_SEED + 2)


def crs_grid() -> Grid:
    """A 21 x B 21 x v 41 (1500..4500 m/s)."""
    return Grid(A=uniform_grid(-5e-4, 5e-4, 21), B=uniform_grid(-1e-7, 1e-7, 21),
                q=velocity_grid(1500.0, 4500.0, 41))


def crs_coarse_grid() -> Grid:
    """A 7 x B 7 x v 11 over the same ranges."""
    return Grid(A=uniform_grid(-5e-4, 5e-4, 7), B=uniform_grid(-1e-7, 1e-7, 7),
                q=velocity_grid(1500.0, 4500.0, 11))


CRS_HALF_APERTURE = 4


def crs_line(centrals=None, grid: Grid | None = None) -> Workload:
    """2D CRS: centrals 4..515 with a +-4 gather aperture (default: all 512).

    Only the gathers the chosen centrals need are generated; gather indices in
    the returned set are renumbered, the midpoints keep their line positions.
    """
    spec = crs_line_spec()
    k = CRS_HALF_APERTURE
    centrals = list(range(k, spec.ngathers - k)) if centrals is None else list(centrals)
    need = sorted({g for c in centrals for g in range(max(0, c - k), min(spec.ngathers, c + k + 1))})
    gs = line_gathers(spec, need)
    pos = {g: i for i, g in enumerate(need)}
    ptr, ag = [0], []
    for c in centrals:
        ag.extend(pos[g] for g in range(max(0, c - k), min(spec.ngathers, c + k + 1)))
        ptr.append(len(ag))
    cen = np.array([pos[c] for c in centrals], np.int32)
    ns = gs.ns[cen].astype(np.int64)
    out_off = np.zeros(cen.size, np.int64)
    if cen.size > 1:
        out_off[1:] = np.cumsum(ns)[:-1]
    jobs = Jobs(central=cen, apert_ptr=np.asarray(ptr, np.int32),
                apert_gather=np.asarray(ag, np.int32), out_off=out_off, n_out=int(ns.sum()))
    return Workload(name="crs_line", kind="crs", gathers=gs, jobs=jobs,
                    grid=grid if grid is not None else crs_grid(), w=9)


def batched_line_spec() -> LineSpec:
    """4096 gathers, fold U{8..120}, 500..2000 samples at 4 ms, the CRS line event
    model (events scaled to the line length), SNR 3."""
    return LineSpec(ngathers=4096, fold=(8, 120), ns=(500, 2000), dt=0.004, h_max=1500.0,
                    nevents=2363, f_peak=25.0, t0_range=(0.2, 3.8), A_range=(-4e-4, 4e-4),
                    B_range=(-8e-8, 8e-8), v_range=(1800.0, 4000.0), amp_range=(0.5, 1.0),
                    taper_halfwidth=100.0, snr=3.0, seed=ROOT_SEED + 3)


def batched_kinds(n: int = 4096, n_cmp: int = 2867, seed: int = ROOT_SEED + 3) -> np.ndarray:
    """Seeded choice of exactly n_cmp CMP jobs (0) and the rest CRS (1)."""
    kinds = np.ones(n, np.int32)
    kinds[_rng(seed, 3, 0).permutation(n)[:n_cmp]] = 0
    return kinds


@dataclass
class BatchWorkload:
    """Mixed CMP/CRS jobs on one line of uneven gathers (one job per gather)."""
    gathers: Gathers
    jobs: Jobs                 # aperture CSR: the central alone for CMP jobs
    kind: np.ndarray           # int32 [njobs], 0 = CMP, 1 = CRS
    grid_cmp: Grid
    grid_crs: Grid
    w_cmp: int
    w_crs: int

    def subset(self, kind: int) -> Jobs:
        """The jobs of one kind (same output rows as in the batch)."""
        sel = np.nonzero(self.kind == kind)[0]
        ptr, ag = [0], []
        for j in sel:
            ag.extend(self.jobs.apert_gather[self.jobs.apert_ptr[j]:self.jobs.apert_ptr[j + 1]])
            ptr.append(len(ag))
        return Jobs(central=self.jobs.central[sel].copy(), apert_ptr=np.asarray(ptr, np.int32),
                    apert_gather=np.asarray(ag, np.int32), out_off=self.jobs.out_off[sel].copy(),
                    n_out=self.jobs.n_out)


def batched_line(ids=None, half_aperture: int = 2) -> BatchWorkload:
    """The batched workload: 4096 gathers of uneven fold (8..120) and length
    (500..2000 samples at 4 ms); 2867 CMP jobs (101 velocities 1500..4500 m/s,
    window 11) and 1229 CRS jobs (A 11 x B 11 x v 21 over the CRS line's ranges,
    +-2 neighbouring gathers truncated at the line ends, window 9).

    ids: optional subset of gathers (e.g. a contiguous stretch); every job is
    then restricted to gathers inside the subset."""
    spec = batched_line_spec()
    kinds_all = batched_kinds(spec.ngathers)
    ids = list(range(spec.ngathers)) if ids is None else list(ids)
    gs = line_gathers(spec, ids)
    pos = {g: i for i, g in enumerate(ids)}
    kind = np.array([kinds_all[g] for g in ids], np.int32)
    ptr, ag = [0], []
    for g, k in zip(ids, kind):
        if k == 0:
            ag.append(pos[g])
        else:
            ag.extend(pos[x] for x in range(g - half_aperture, g + half_aperture + 1) if x in pos)
        ptr.append(len(ag))
    central = np.arange(len(ids), dtype=np.int32)
    ns = gs.ns.astype(np.int64)
    out_off = np.zeros(len(ids), np.int64)
    if len(ids) > 1:
        out_off[1:] = np.cumsum(ns)[:-1]
    jobs = Jobs(central=central, apert_ptr=np.asarray(ptr, np.int32), apert_gather=np.asarray(ag, np.int32),
                out_off=out_off, n_out=int(ns.sum()))
    return BatchWorkload(gathers=gs, jobs=jobs, kind=kind,
                         grid_cmp=Grid(q=velocity_grid(1500.0, 4500.0, 101)),
                         grid_crs=Grid(A=uniform_grid(-5e-4, 5e-4, 11), B=uniform_grid(-1e-7, 1e-7, 11),
                                       q=velocity_grid(1500.0, 4500.0, 21)),
                         w_cmp=11, w_crs=9)


# --------------------------------------------------------------------------
# the paper's dataset shapes (Table 1): fold, samples per trace, and the
# "dt" column, which sets how many samples one window access reads
# --------------------------------------------------------------------------
PAPER_DATASETS = {1: (60, 550, 220), 2: (60, 550, 240), 3: (60, 1650, 220), 4: (60, 1650, 240),
                  5: (1000, 550, 220), 6: (1000, 550, 240), 7: (1000, 1650, 220), 8: (1000, 1650, 240)}


def paper_window(dt_column: int) -> int:
    """Window length read from Table 1's "dt" column taken as microseconds per
    sample under a fixed +-2 ms window: 2 * floor(2000 / dt) + 1 samples (19 for
    220, 17 for 240; the 19-sample window is 76 B of FP32, the largest access
    the paper quotes)."""
    return 2 * (2000 // int(dt_column)) + 1


def paper_shape_spec(dataset: int, ngathers: int) -> LineSpec:
    """A line of ``ngathers`` gathers with dataset ``dataset``'s fold and trace
    length, sampled at 4 ms (the sampling interval itself is not given), the CRS
    line's event model scaled to the line and to the trace length, SNR 3.  The
    datasets that differ only in the "dt" column share their data."""
    fold, ns, _ = PAPER_DATASETS[dataset]
    t_end = 0.9 * ns * 0.004
    return LineSpec(ngathers=ngathers, fold=fold, ns=ns, dt=0.004, h_max=1500.0,
                    nevents=max(1, int(math.ceil(0.58 * ngathers))), f_peak=25.0, t0_range=(0.2, t_end),
                    A_range=(-4e-4, 4e-4), B_range=(-8e-8, 8e-8), v_range=(1800.0, 4000.0),
                    amp_range=(0.5, 1.0), taper_halfwidth=100.0, snr=3.0,
                    seed=ROOT_SEED + 10 + (dataset - 1) // 2)  # datasets 2k-1 and 2k share fold and ns


def paper_shape(dataset: int, ngathers: int, kind: str = "cmp", half_aperture: int = 2,
                centrals=None) -> Workload:
    """Dataset ``dataset`` of Table 1 at a chosen number of gathers.  CMP: one
    job per gather, 101 velocities 1500..4500 m/s.  CRS: centrals (default: all
    with a full aperture) with +-``half_aperture`` gathers and the coarse
    7 x 7 x 11 grid.  The window follows ``paper_window``."""
    fold, ns, dtc = PAPER_DATASETS[dataset]
    spec = paper_shape_spec(dataset, ngathers)
    w = paper_window(dtc)
    if kind == "cmp":
        ids = list(range(ngathers)) if centrals is None else list(centrals)
        gs = line_gathers(spec, ids)
        return Workload(name=f"paper_data{dataset}", kind="cmp", gathers=gs, jobs=cmp_jobs(gs),
                        grid=Grid(q=velocity_grid(1500.0, 4500.0, 101)), w=w)
    k = half_aperture
    centrals = list(range(k, ngathers - k)) if centrals is None else list(centrals)
    need = sorted({g for c in centrals for g in range(max(0, c - k), min(ngathers, c + k + 1))})
    gs = line_gathers(spec, need)
    pos = {g: i for i, g in enumerate(need)}
    ptr, ag = [0], []
    for c in centrals:
        ag.extend(pos[g] for g in range(max(0, c - k), min(ngathers, c + k + 1)))
        ptr.append(len(ag))
    cen = np.array([pos[c] for c in centrals], np.int32)
    nsv = gs.ns[cen].astype(np.int64)
    out_off = np.zeros(cen.size, np.int64)
    if cen.size > 1:
        out_off[1:] = np.cumsum(nsv)[:-1]
    jobs = Jobs(central=cen, apert_ptr=np.asarray(ptr, np.int32), apert_gather=np.asarray(ag, np.int32),
                out_off=out_off, n_out=int(nsv.sum()))
    return Workload(name=f"paper_data{dataset}_crs", kind="crs", gathers=gs, jobs=jobs,
                    grid=crs_coarse_grid(), w=w)
