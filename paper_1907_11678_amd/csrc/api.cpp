// api.cpp -- host side of the C ABI declared in include/semb.h: argument
// validation, workspace carving, launch configuration and error reporting.
// Apart from the tuners and the probes, nothing here allocates device memory
// or synchronises a stream.

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace semb {
int run_probe(int probe, int reps, double *rate, double *ms);  // probe.hip
hipError_t launch_theta_shift(float *theta, int64_t n, const float *d, const float *lo, const float *hi,
                              hipStream_t stream);  // point.hip
}

namespace {

thread_local std::string g_last_error;

semb_status fail(semb_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

semb_status fail(semb_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

semb_status hip_status(hipError_t e, const char *what)
{
    if (e == hipSuccess) return SEMB_OK;
    return fail(SEMB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Per-thread kernel timer: event pairs recorded around main-kernel launches.
struct KernelTimer {
    std::vector<hipEvent_t> start, stop;
    int used = 0;
    bool on = false;

    void release()
    {
        for (hipEvent_t e : start)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : stop)
            if (e) (void)hipEventDestroy(e);
        start.clear();
        stop.clear();
        used = 0;
        on = false;
    }
};

thread_local KernelTimer g_timer;

// Run `launch` (which enqueues one kernel on `stream`); bracket it with this
// thread's next event pair when the timer is on and the stream is not being
// captured.
template <class F>
hipError_t timed(hipStream_t stream, F launch)
{
    KernelTimer &t = g_timer;
    bool rec = false;
    if (t.on && t.used < (int)t.start.size()) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        rec = hipStreamIsCapturing(stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
    }
    if (rec) {
        const hipError_t e = hipEventRecord(t.start[t.used], stream);
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch();
    if (rec && e == hipSuccess) {
        e = hipEventRecord(t.stop[t.used], stream);
        if (e == hipSuccess) ++t.used;
    }
    return e;
}

constexpr size_t kAlign = 256;
constexpr int kScanCap = 2048;  // LDS positions per stage in the scan kernel (>= ns_max)

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

semb_status check_gathers(const semb_gathers *g, bool crs)
{
    if (!g) return fail(SEMB_EINVAL, "gathers is NULL");
    if (g->ngathers < 1 || g->ntraces < 0) return fail(SEMB_EINVAL, "ngathers must be >= 1 and ntraces >= 0");
    if (!g->samples || !g->sample_off || !g->trace_ptr || !g->ns || !g->half_offset)
        return fail(SEMB_EINVAL, "a required gathers array is NULL");
    if (crs && (!g->midpoint || !g->central_x))
        return fail(SEMB_EINVAL, "CRS needs midpoint and central_x");
    if (!(g->dt > 0.f) || !isfinite(g->dt)) return fail(SEMB_EINVAL, "dt must be finite and > 0");
    if (g->ns_max < 1 || g->ns_max > SEMB_NS_LIMIT)
        return fail(SEMB_EINVAL, "ns_max must lie in 1..%d", SEMB_NS_LIMIT);
    if (g->nsamples < 0) return fail(SEMB_EINVAL, "nsamples must be >= 0");
    return SEMB_OK;
}

semb_status check_jobs(const semb_jobs *j, bool crs, const semb_gathers *g)
{
    if (!j) return fail(SEMB_EINVAL, "jobs is NULL");
    if (j->njobs < 0) return fail(SEMB_EINVAL, "njobs must be >= 0");
    if (j->njobs == 0) return SEMB_OK;
    if (!j->central || !j->out_off) return fail(SEMB_EINVAL, "jobs.central and jobs.out_off are required");
    if (crs && (!j->apert_ptr || !j->apert_gather))
        return fail(SEMB_EINVAL, "CRS jobs need apert_ptr and apert_gather");
    if (j->max_apert < 1 || j->max_apert > SEMB_APERT_LIMIT)
        return fail(SEMB_EINVAL, "max_apert must lie in 1..%d", SEMB_APERT_LIMIT);
    if (j->n_out < 0) return fail(SEMB_EINVAL, "n_out must be >= 0");
    const long long nblk = (long long)j->njobs * ((g->ns_max + 63) / 64);
    if (nblk > 0x7fffffffLL) return fail(SEMB_EINVAL, "too many jobs for one launch");
    return SEMB_OK;
}

semb_status check_w(int32_t w)
{
    if (w < 1 || w > SEMB_W_MAX || (w % 2) == 0)
        return fail(SEMB_EINVAL, "w must be odd and lie in 1..%d (got %d)", SEMB_W_MAX, w);
    return SEMB_OK;
}

#define TRY(x)                               \
    do {                                     \
        semb_status _st = (x);               \
        if (_st != SEMB_OK) return _st;      \
    } while (0)

semb::GatherView gather_view(const semb_gathers *g)
{
    semb::GatherView v{};
    v.samples = g->samples;
    v.sample_off = g->sample_off;
    v.trace_ptr = g->trace_ptr;
    v.ns = g->ns;
    v.half_offset = g->half_offset;
    v.midpoint = g->midpoint;
    v.central_x = g->central_x;
    v.dt = g->dt;
    return v;
}

semb::JobView job_view(const semb_jobs *jobs, const semb_gathers *g, bool crs)
{
    semb::JobView v{};
    v.central = jobs->central;
    v.apert_ptr = crs ? jobs->apert_ptr : nullptr;
    v.apert_gather = crs ? jobs->apert_gather : nullptr;
    v.out_off = jobs->out_off;
    v.njobs = jobs->njobs;
    v.n_sblk = (g->ns_max + 63) / 64;
    v.max_apert = jobs->max_apert;
    return v;
}

// ---- tile shapes of the exhaustive scan and the tuner's choices ------------
// The choice is kept per (kind, window, traces per job, samples per trace),
// the two sizes as powers-of-two buckets computed from host-side fields.
struct ShapeKey {
    int kind, w, traces, ns;
    bool operator<(const ShapeKey &o) const
    {
        return std::tie(kind, w, traces, ns) < std::tie(o.kind, o.w, o.traces, o.ns);
    }
};

std::mutex g_shape_mu;
std::map<ShapeKey, int> g_shapes;

int log2_bucket(double v)
{
    int b = 0;
    while (b < 40 && (double)(1LL << b) < v) ++b;
    return b;
}

ShapeKey shape_key(int kind, int w, const semb_gathers *g, const semb_jobs *jobs)
{
    const double fold = g->ngathers > 0 ? (double)g->ntraces / g->ngathers : 0.0;
    const double apert = kind == SEMB_KIND_CRS ? (double)std::max(1, jobs->max_apert) : 1.0;
    return ShapeKey{kind, w, log2_bucket(fold * apert), log2_bucket(g->ns_max)};
}

int default_shape(int kind) { return kind == SEMB_KIND_CRS ? 2 : 0; }

// The batched scan's choices: tile shape and parameter split per (w_cmp, w_crs,
// traces per job, samples per trace), the sizes as in ShapeKey.
struct BatchKey {
    int wc, wr, traces, ns;
    bool operator<(const BatchKey &o) const { return std::tie(wc, wr, traces, ns) < std::tie(o.wc, o.wr, o.traces, o.ns); }
};
struct BatchChoice {
    int shape, split;
};
constexpr int kDefaultBatchShape = 0;
constexpr int kDefaultBatchSplit = 256;
std::map<BatchKey, BatchChoice> g_batch;  // guarded by g_shape_mu

BatchKey batch_key(int wc, int wr, const semb_gathers *g, const semb_jobs *jobs)
{
    const ShapeKey k = shape_key(SEMB_KIND_CRS, wr, g, jobs);
    return BatchKey{wc, wr, k.traces, k.ns};
}

BatchChoice chosen_batch(int wc, int wr, const semb_gathers *g, const semb_jobs *jobs)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    const auto it = g_batch.find(batch_key(wc, wr, g, jobs));
    return it == g_batch.end() ? BatchChoice{kDefaultBatchShape, kDefaultBatchSplit} : it->second;
}

int chosen_shape(int kind, int w, const semb_gathers *g, const semb_jobs *jobs)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    const auto it = g_shapes.find(shape_key(kind, w, g, jobs));
    return it == g_shapes.end() ? default_shape(kind) : it->second;
}

const char *const kShapeNames[semb::kScanShapes] = {
    "4 waves x 4 parameters (2 for w > 15), 2048-sample stage, windows behind a branch",
    "8 waves x 2 parameters, 3072-sample stage, branch-free windows",
    "8 waves x 4 parameters (2 for w > 9), 2560-sample stage, branch-free windows",
    "4 waves x 4 parameters (2 for w > 15), 2048-sample stage, branch-free windows",
    "8 waves x 4 parameters (2 for w > 15), 2048-sample stage, windows behind a branch",
    "16 waves x 4 parameters (2 for w > 15), 2048-sample stage, windows behind a branch",
};

// Every argument of a scan except the workspace (host fields only).
semb_status check_scan(int kind, const semb_gathers *g, const semb_jobs *jobs, const float *A, int32_t nA,
                       const float *B, int32_t nB, const float *q, int32_t nq, int32_t w, const semb_outputs *out)
{
    const bool crs = kind == SEMB_KIND_CRS;
    TRY(check_gathers(g, crs));
    TRY(check_jobs(jobs, crs, g));
    TRY(check_w(w));
    if (!q || nq < 1) return fail(SEMB_EINVAL, "q must be non-NULL with nq >= 1");
    if (crs && (!A || nA < 1 || !B || nB < 1)) return fail(SEMB_EINVAL, "CRS needs A, B with nA, nB >= 1");
    const long long npar = crs ? (long long)nA * nB * nq : nq;
    if (npar > 0x7fffffffLL) return fail(SEMB_EINVAL, "too many parameters");
    if (g->ns_max > kScanCap)
        return fail(SEMB_EINVAL, "the scan supports ns_max <= %d (got %d)", kScanCap, g->ns_max);
    if (jobs->njobs == 0) return SEMB_OK;  // nothing to compute, nothing is read or written
    if (!out || !out->best || !out->s_best || !out->stack)
        return fail(SEMB_EINVAL, "outputs best, s_best and stack are required");
    return SEMB_OK;
}

// shape < 0: the tuned (or default) shape for this call's key
semb_status scan_common(int kind, const semb_gathers *g, const semb_jobs *jobs, const float *A, int32_t nA,
                        const float *B, int32_t nB, const float *q, int32_t nq, int32_t w,
                        const semb_outputs *out, void *ws, size_t ws_bytes, hipStream_t stream, int shape = -1)
{
    const bool crs = kind == SEMB_KIND_CRS;
    TRY(check_scan(kind, g, jobs, A, nA, B, nB, q, nq, w, out));
    if (jobs->njobs == 0) return SEMB_OK;
    const long long npar = crs ? (long long)nA * nB * nq : nq;
    const size_t need = semb_workspace_bytes(g->nsamples);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0)
        return fail(SEMB_EWORKSPACE, "workspace must be %zu bytes, 256-byte aligned (got %zu at %p)", need,
                    ws_bytes, ws);

    const size_t plane = round_up((size_t)g->nsamples * sizeof(float));
    float *u0 = static_cast<float *>(ws);
    float *u1 = reinterpret_cast<float *>(static_cast<char *>(ws) + plane);
    float *u2sq = reinterpret_cast<float *>(static_cast<char *>(ws) + 2 * plane);
    TRY(hip_status(semb::launch_window_energy(g->samples, g->sample_off, g->trace_ptr, g->ns, g->ngathers,
                                              g->ntraces, w, u0, u1, u2sq, stream),
                   "window energy launch"));

    semb::ScanArgs a{};
    a.g = gather_view(g);
    a.j = job_view(jobs, g, crs);
    a.p.A = A;
    a.p.B = B;
    a.p.q = q;
    a.p.nA = crs ? nA : 1;
    a.p.nB = crs ? nB : 1;
    a.p.nq = nq;
    a.p.npar = (int32_t)npar;
    a.p.w = w;
    a.p.u0 = u0;
    a.p.u1 = u1;
    a.p.u2sq = u2sq;
    a.best = out->best;
    a.s_best = out->s_best;
    a.stack = out->stack;
    a.panel = out->panel;
    a.panel16 = out->panel_f16;
    const int sid = shape >= 0 ? shape : chosen_shape(kind, w, g, jobs);
    return hip_status(timed(stream, [&] { return semb::launch_scan(kind, a, sid, stream); }),
                      crs ? "crs_scan launch" : "cmp_scan launch");
}

semb_status point_common(bool grad, const semb_gathers *g, const semb_jobs *jobs, int32_t kind,
                         const float *theta, const float *g_s, int32_t w, float *s_out, float *stack_out,
                         float *g_theta, float *g_samples, hipStream_t stream)
{
    if (kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) return fail(SEMB_EINVAL, "kind must be CMP or CRS");
    const bool crs = kind == SEMB_KIND_CRS;
    TRY(check_gathers(g, crs));
    TRY(check_jobs(jobs, crs, g));
    TRY(check_w(w));
    if (jobs->njobs == 0) return SEMB_OK;
    if (!theta) return fail(SEMB_EINVAL, "theta is NULL");
    if (!grad && (!s_out || !stack_out)) return fail(SEMB_EINVAL, "s_out and stack_out are required");
    if (grad && (!g_s || !g_theta)) return fail(SEMB_EINVAL, "g_s and g_theta are required");

    semb::PointArgs a{};
    a.samples = g->samples;
    a.sample_off = g->sample_off;
    a.trace_ptr = g->trace_ptr;
    a.ns = g->ns;
    a.half_offset = g->half_offset;
    a.midpoint = g->midpoint;
    a.central_x = g->central_x;
    a.dt = g->dt;
    a.central = jobs->central;
    a.apert_ptr = crs ? jobs->apert_ptr : nullptr;
    a.apert_gather = crs ? jobs->apert_gather : nullptr;
    a.out_off = jobs->out_off;
    a.njobs = jobs->njobs;
    a.n_sblk = (g->ns_max + 63) / 64;
    a.max_apert = jobs->max_apert;
    a.theta = theta;
    a.g_s = g_s;
    a.s_out = s_out;
    a.stack_out = stack_out;
    a.g_theta = g_theta;
    a.g_samples = g_samples;
    a.w = w;
    if (grad) return hip_status(timed(stream, [&] { return semb::launch_grad(kind, a, stream); }), "semblance_grad launch");
    return hip_status(timed(stream, [&] { return semb::launch_point(kind, a, stream); }), "stack launch");
}

constexpr int kBatchBlock = 32;  // parameters per CRS block of the batch kernel (8 waves x 4 for w <= 9)

bool batch_w_ok(int w) { return w == 9 || w == 11 || w == 15; }

struct BatchLayout {
    size_t plane_c, plane_r, counters, partials, total;
};

BatchLayout batch_layout(int64_t nsamples, int32_t w_cmp, int32_t w_crs, int32_t ngroups, int32_t nparts)
{
    BatchLayout L{};
    const size_t plane = round_up((size_t)(nsamples > 0 ? nsamples : 0) * sizeof(float));
    L.plane_c = 0;
    L.plane_r = (w_cmp == w_crs) ? 0 : 3 * plane;
    L.counters = (w_cmp == w_crs ? 3 : 6) * plane;
    L.partials = L.counters + round_up((size_t)(1 + (ngroups > 0 ? ngroups : 0)) * sizeof(unsigned));
    L.total = L.partials + round_up((size_t)(nparts > 0 ? nparts : 0) * 64 * sizeof(semb::Partial));
    return L;
}

// ---- the allocation-free scan's scratch --------------------------------------
// The window-energy planes of semb_scan_noalloc live in this file-scope device
// array (each GPU the library runs on holds its own copy until the process
// ends).  In host code `scratch` names a host-side stand-in, not the device
// copy: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is ever passed to a kernel.
__device__ __align__(256) unsigned char scratch[SEMB_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_at;  // device ordinal -> address of its `scratch`

semb_status scratch_address(void **at)
{
    int dev = 0;
    TRY(hip_status(hipGetDevice(&dev), "semb_scan_noalloc: hipGetDevice"));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    const auto it = g_scratch_at.find(dev);
    if (it != g_scratch_at.end()) {
        *at = it->second;
        return SEMB_OK;
    }
    void *p = nullptr;
    TRY(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "semb_scan_noalloc: hipGetSymbolAddress"));
    if (!p) return fail(SEMB_EHIP, "semb_scan_noalloc: no device address for the scratch array");
    g_scratch_at[dev] = p;
    *at = p;
    return SEMB_OK;
}

}  // namespace

void semb::set_last_error(const char *msg) { g_last_error = msg; }

extern "C" {

int64_t semb_batch_plan(const semb_batch_host *h, int32_t split_params, semb_tile *tiles, int64_t max_tiles,
                        int32_t *ngroups, int32_t *nparts)
{
    if (!h || !h->kind || !h->central || !h->apert_ptr || !h->apert_gather || !h->ns || !h->trace_ptr) {
        fail(SEMB_EINVAL, "semb_batch_plan: a required host array is NULL");
        return -1;
    }
    if (h->njobs < 0 || h->ngathers < 1 || h->npar_cmp < 1 || h->npar_crs < 1 || split_params < 1) {
        fail(SEMB_EINVAL, "semb_batch_plan: invalid sizes");
        return -1;
    }
    // whole blocks, in 64-bit so that a split of INT32_MAX ("never split") cannot overflow
    const int64_t split64 = ((int64_t)split_params + kBatchBlock - 1) / kBatchBlock * kBatchBlock;
    const int32_t split = (int32_t)std::min<int64_t>(split64, 0x7fffffffLL);
    struct Item {
        double cost;
        semb_tile t;
    };
    std::vector<Item> items;
    int64_t ng = 0, np = 0;
    for (int32_t j = 0; j < h->njobs; ++j) {
        const int32_t c = h->central[j];
        if (c < 0 || c >= h->ngathers) {
            fail(SEMB_EINVAL, "semb_batch_plan: job %d has central gather %d out of range", j, c);
            return -1;
        }
        const bool crs = h->kind[j] == SEMB_KIND_CRS;
        if (!crs && h->kind[j] != SEMB_KIND_CMP) {
            fail(SEMB_EINVAL, "semb_batch_plan: job %d has an unknown kind", j);
            return -1;
        }
        int64_t ntr = 0;
        if (crs && (h->apert_ptr[j + 1] - h->apert_ptr[j] < 0 ||
                    h->apert_ptr[j + 1] - h->apert_ptr[j] > SEMB_APERT_LIMIT)) {
            fail(SEMB_EINVAL, "semb_batch_plan: job %d lists %d aperture gathers (1..%d allowed)", j,
                 h->apert_ptr[j + 1] - h->apert_ptr[j], SEMB_APERT_LIMIT);
            return -1;
        }
        if (crs) {
            for (int32_t k = h->apert_ptr[j]; k < h->apert_ptr[j + 1]; ++k) {
                const int32_t gg = h->apert_gather[k];
                if (gg < 0 || gg >= h->ngathers) {
                    fail(SEMB_EINVAL, "semb_batch_plan: job %d has an aperture gather out of range", j);
                    return -1;
                }
                ntr += h->trace_ptr[gg + 1] - h->trace_ptr[gg];
            }
        } else {
            ntr = h->trace_ptr[c + 1] - h->trace_ptr[c];
        }
        const int32_t npar = crs ? h->npar_crs : h->npar_cmp;
        const int32_t nsplit = (int32_t)(((int64_t)npar + split - 1) / split);
        const int32_t nsb = (h->ns[c] + 63) / 64;
        for (int32_t b = 0; b < nsb; ++b) {
            const int32_t nrow = std::min(64, h->ns[c] - 64 * b);
            const int32_t grp = nsplit > 1 ? (int32_t)ng++ : -1;
            const int32_t base = nsplit > 1 ? (int32_t)np : 0;
            if (nsplit > 1) np += nsplit;
            // groups and partial slots index 32-bit fields and a workspace of np * 64 partials
            if (ng > 0x7fffffffLL || np > 0x7fffffffLL / 64) {
                fail(SEMB_EINVAL, "semb_batch_plan: too many split tiles; use a larger split_params");
                return -1;
            }
            for (int32_t sp = 0; sp < nsplit; ++sp) {
                Item it;
                it.t.job = j;
                it.t.sblk = b;
                it.t.p_begin = sp * split;
                it.t.p_end = std::min(npar, (sp + 1) * split);
                it.t.group = grp;
                it.t.split = sp;
                it.t.nsplit = nsplit;
                it.t.part_base = base;
                // work estimate: rows x parameters x traces (+ a fixed cost per tile)
                it.cost = (double)nrow * (it.t.p_end - it.t.p_begin) * (double)(ntr + 4) + 4096.0;
                items.push_back(it);
            }
        }
    }
    // longest first; ties keep job order
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
    if (ngroups) *ngroups = (int32_t)ng;
    if (nparts) *nparts = (int32_t)np;
    if (tiles) {
        if ((int64_t)items.size() > max_tiles) {
            fail(SEMB_EINVAL, "semb_batch_plan: %zu tiles do not fit in max_tiles = %lld", items.size(),
                 (long long)max_tiles);
            return -1;
        }
        for (size_t i = 0; i < items.size(); ++i) tiles[i] = items[i].t;
    }
    return (int64_t)items.size();
}

size_t semb_batch_workspace_bytes(int64_t nsamples, int32_t w_cmp, int32_t w_crs, int32_t ngroups,
                                  int32_t nparts)
{
    return batch_layout(nsamples, w_cmp, w_crs, ngroups, nparts).total;
}

}  // extern "C"

namespace {
semb_status batch_common(const semb_gathers *g, const semb_jobs *jobs, const semb_batch *b, const semb_tile *tiles,
                         int64_t ntiles, int32_t ngroups, int32_t nparts, const semb_outputs *out, void *ws,
                         size_t ws_bytes, hipStream_t stream, int shape);
}  // namespace

extern "C" semb_status scan_batch(const semb_gathers *g, const semb_jobs *jobs, const semb_batch *b,
                                  const semb_tile *tiles, int64_t ntiles, int32_t ngroups, int32_t nparts,
                                  const semb_outputs *out, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return batch_common(g, jobs, b, tiles, ntiles, ngroups, nparts, out, ws, ws_bytes, stream, -1);
}

namespace {

// shape < 0: the tuned (or default) batch shape for this call's key
semb_status batch_common(const semb_gathers *g, const semb_jobs *jobs, const semb_batch *b, const semb_tile *tiles,
                         int64_t ntiles, int32_t ngroups, int32_t nparts, const semb_outputs *out, void *ws,
                         size_t ws_bytes, hipStream_t stream, int shape)
{
    TRY(check_gathers(g, true));
    TRY(check_jobs(jobs, true, g));
    if (!b || !b->kind || !b->q_cmp || b->nq_cmp < 1 || !b->A || b->nA < 1 || !b->B || b->nB < 1 || !b->q_crs ||
        b->nq_crs < 1)
        return fail(SEMB_EINVAL, "scan_batch: incomplete batch parameters");
    if (!batch_w_ok(b->w_cmp) || !batch_w_ok(b->w_crs))
        return fail(SEMB_EINVAL, "scan_batch supports windows 9, 11 and 15 (got %d, %d)", b->w_cmp, b->w_crs);
    if ((long long)b->nA * b->nB * b->nq_crs > 0x7fffffffLL) return fail(SEMB_EINVAL, "too many CRS parameters");
    if (g->ns_max > kScanCap) return fail(SEMB_EINVAL, "the scan supports ns_max <= %d", kScanCap);
    if (ntiles < 0 || ngroups < 0 || nparts < 0) return fail(SEMB_EINVAL, "negative plan sizes");
    if (ntiles > 0 && !tiles) return fail(SEMB_EINVAL, "tiles is NULL");
    if (!out || !out->best || !out->s_best || !out->stack) return fail(SEMB_EINVAL, "outputs are required");
    if (out->panel || out->panel_f16)
        return fail(SEMB_EINVAL, "scan_batch writes no panel (panel and panel_f16 must be NULL)");
    const BatchLayout lay = batch_layout(g->nsamples, b->w_cmp, b->w_crs, ngroups, nparts);
    if (!ws || ws_bytes < lay.total || ((uintptr_t)ws % kAlign) != 0)
        return fail(SEMB_EWORKSPACE, "workspace must be %zu bytes, 256-byte aligned (got %zu at %p)", lay.total,
                    ws_bytes, ws);
    char *base = static_cast<char *>(ws);
    const size_t plane = round_up((size_t)g->nsamples * sizeof(float));
    float *uc = reinterpret_cast<float *>(base + lay.plane_c);
    float *ur = reinterpret_cast<float *>(base + lay.plane_r);
    TRY(hip_status(semb::launch_window_energy(g->samples, g->sample_off, g->trace_ptr, g->ns, g->ngathers,
                                              g->ntraces, b->w_cmp, uc, uc + plane / 4, uc + 2 * (plane / 4),
                                              stream),
                   "window energy launch"));
    if (b->w_crs != b->w_cmp)
        TRY(hip_status(semb::launch_window_energy(g->samples, g->sample_off, g->trace_ptr, g->ns, g->ngathers,
                                                  g->ntraces, b->w_crs, ur, ur + plane / 4, ur + 2 * (plane / 4),
                                                  stream),
                       "window energy launch"));
    semb::BatchArgs a{};
    a.g = gather_view(g);
    a.j = job_view(jobs, g, true);
    a.kind = b->kind;
    a.pc.A = nullptr;
    a.pc.B = nullptr;
    a.pc.q = b->q_cmp;
    a.pc.nA = a.pc.nB = 1;
    a.pc.nq = b->nq_cmp;
    a.pc.npar = b->nq_cmp;
    a.pc.w = b->w_cmp;
    a.pc.u0 = uc;
    a.pc.u1 = uc + plane / 4;
    a.pc.u2sq = uc + 2 * (plane / 4);
    a.pr.A = b->A;
    a.pr.B = b->B;
    a.pr.q = b->q_crs;
    a.pr.nA = b->nA;
    a.pr.nB = b->nB;
    a.pr.nq = b->nq_crs;
    a.pr.npar = b->nA * b->nB * b->nq_crs;
    a.pr.w = b->w_crs;
    a.pr.u0 = ur;
    a.pr.u1 = ur + plane / 4;
    a.pr.u2sq = ur + 2 * (plane / 4);
    a.tiles = tiles;
    a.ntiles = ntiles;
    a.counters = reinterpret_cast<unsigned int *>(base + lay.counters);
    a.partials = reinterpret_cast<semb::Partial *>(base + lay.partials);
    a.ngroups = ngroups;
    a.nparts = nparts;
    a.best = out->best;
    a.s_best = out->s_best;
    a.stack = out->stack;
    const int bs = shape >= 0 ? shape : chosen_batch(b->w_cmp, b->w_crs, g, jobs).shape;
    return hip_status(timed(stream, [&] { return semb::launch_batch(a, ngroups, bs, stream); }), "scan_batch launch");
}

}  // namespace

extern "C" {


size_t semb_workspace_bytes(int64_t nsamples)
{
    if (nsamples <= 0) return kAlign;
    return 3 * round_up((size_t)nsamples * sizeof(float));
}

semb_status cmp_scan(const semb_gathers *g, const semb_jobs *jobs, const float *q, int32_t nq, int32_t w,
                     const semb_outputs *out, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return scan_common(SEMB_KIND_CMP, g, jobs, nullptr, 1, nullptr, 1, q, nq, w, out, ws, ws_bytes, stream);
}

semb_status crs_scan(const semb_gathers *g, const semb_jobs *jobs, const float *A, int32_t nA, const float *B,
                     int32_t nB, const float *q, int32_t nq, int32_t w, const semb_outputs *out, void *ws,
                     size_t ws_bytes, hipStream_t stream)
{
    return scan_common(SEMB_KIND_CRS, g, jobs, A, nA, B, nB, q, nq, w, out, ws, ws_bytes, stream);
}

semb_status semb_scan_noalloc(int32_t kind, const semb_gathers *g, const semb_jobs *jobs, const float *A, int32_t nA,
                              const float *B, int32_t nB, const float *q, int32_t nq, int32_t w,
                              const semb_outputs *out, hipStream_t stream)
{
    if (kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) return fail(SEMB_EINVAL, "kind must be CMP or CRS");
    if (!g || !jobs) return fail(SEMB_EINVAL, "gathers and jobs are required");
    const size_t need = semb_workspace_bytes(g->nsamples);
    if (need > (size_t)SEMB_NOALLOC_SCRATCH_BYTES)
        return fail(SEMB_EINVAL,
                    "semb_scan_noalloc: %lld samples need %zu bytes of window-energy scratch; the static "
                    "scratch holds %zu (use cmp_scan / crs_scan with a workspace)",
                    (long long)g->nsamples, need, (size_t)SEMB_NOALLOC_SCRATCH_BYTES);
    TRY(check_scan(kind, g, jobs, A, nA, B, nB, q, nq, w, out));
    if (jobs->njobs == 0) return SEMB_OK;
    // the lookup below touches no device memory and allocates nothing
    void *ws = nullptr;
    TRY(scratch_address(&ws));
    return scan_common(kind, g, jobs, A, nA, B, nB, q, nq, w, out, ws, (size_t)SEMB_NOALLOC_SCRATCH_BYTES, stream);
}

semb_status stack(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, const float *theta, int32_t w,
                  float *s_out, float *stack_out, hipStream_t stream)
{
    return point_common(false, g, jobs, kind, theta, nullptr, w, s_out, stack_out, nullptr, nullptr, stream);
}

semb_status semblance_grad(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, const float *theta,
                           const float *g_s, int32_t w, float *g_theta, float *g_samples, hipStream_t stream)
{
    return point_common(true, g, jobs, kind, theta, g_s, w, nullptr, nullptr, g_theta, g_samples, stream);
}

semb_status semb_refine(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, float *theta,
                        const semb_refine_opts *o, int32_t w, float *s_out, float *stack_out, hipStream_t stream)
{
    if (kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) return fail(SEMB_EINVAL, "kind must be CMP or CRS");
    const bool crs = kind == SEMB_KIND_CRS;
    TRY(check_gathers(g, crs));
    TRY(check_jobs(jobs, crs, g));
    TRY(check_w(w));
    if (!o) return fail(SEMB_EINVAL, "refine options are NULL");
    if (o->steps < 0 || !(o->eta0 >= 0.f) || !isfinite(o->eta0) || !(o->grow >= 1.f) || !isfinite(o->grow))
        return fail(SEMB_EINVAL, "steps must be >= 0, eta0 finite and >= 0, grow finite and >= 1");
    for (int k = 0; k < 3; ++k)
        if (!isfinite(o->scale[k]) || !(o->lo[k] <= o->hi[k]))
            return fail(SEMB_EINVAL, "scale must be finite and lo <= hi for every component");
    if (jobs->njobs == 0) return SEMB_OK;
    if (!theta || !s_out || !stack_out) return fail(SEMB_EINVAL, "theta, s_out and stack_out are required");
    semb::PointArgs a{};
    a.samples = g->samples;
    a.sample_off = g->sample_off;
    a.trace_ptr = g->trace_ptr;
    a.ns = g->ns;
    a.half_offset = g->half_offset;
    a.midpoint = g->midpoint;
    a.central_x = g->central_x;
    a.dt = g->dt;
    a.central = jobs->central;
    a.apert_ptr = crs ? jobs->apert_ptr : nullptr;
    a.apert_gather = crs ? jobs->apert_gather : nullptr;
    a.out_off = jobs->out_off;
    a.njobs = jobs->njobs;
    a.n_sblk = (g->ns_max + 63) / 64;
    a.max_apert = jobs->max_apert;
    a.theta = theta;
    a.s_out = s_out;
    a.stack_out = stack_out;
    a.w = w;
    semb::RefineArgs r{};
    r.theta = theta;
    r.steps = o->steps;
    r.eta0 = o->eta0;
    r.grow = o->grow;
    for (int k = 0; k < 3; ++k) {
        r.scale[k] = o->scale[k];
        r.lo[k] = o->lo[k];
        r.hi[k] = o->hi[k];
    }
    return hip_status(timed(stream, [&] { return semb::launch_refine(kind, a, r, stream); }), "semb_refine launch");
}

semb_status semb_theta_from_best(const int32_t *best, int64_t n_out, const float *A, int32_t nA, const float *B,
                                 int32_t nB, const float *q, int32_t nq, float *theta, hipStream_t stream)
{
    if (n_out < 0) return fail(SEMB_EINVAL, "n_out must be >= 0");
    if (n_out == 0) return SEMB_OK;
    if (!best || !q || nq < 1 || !theta) return fail(SEMB_EINVAL, "best, q and theta are required, nq >= 1");
    if ((A && nA < 1) || (B && nB < 1)) return fail(SEMB_EINVAL, "nA and nB must be >= 1");
    if ((long long)(A ? nA : 1) * (B ? nB : 1) * nq > 0x7fffffffLL)
        return fail(SEMB_EINVAL, "too many parameters");
    return hip_status(semb::launch_theta_from_best(best, n_out, A, A ? nA : 1, B, B ? nB : 1, q, nq, theta, stream),
                      "semb_theta_from_best launch");
}

semb_status semb_theta_shift(float *theta, int64_t n, const float *d, const float *lo, const float *hi,
                             hipStream_t stream)
{
    if (n < 0) return fail(SEMB_EINVAL, "semb_theta_shift: n must be >= 0");
    if (n == 0) return SEMB_OK;
    if (!theta || !d || !lo || !hi) return fail(SEMB_EINVAL, "semb_theta_shift: theta, d, lo and hi are required");
    for (int k = 0; k < 3; ++k)
        if (!(lo[k] <= hi[k]) || !isfinite(d[k])) return fail(SEMB_EINVAL, "semb_theta_shift: need lo <= hi, finite d");
    return hip_status(semb::launch_theta_shift(theta, n, d, lo, hi, stream), "semb_theta_shift launch");
}

semb_status semb_kernel_timer_start(int32_t capacity)
{
    if (capacity < 1 || capacity > 65536) return fail(SEMB_EINVAL, "timer capacity must be in 1..65536");
    KernelTimer &t = g_timer;
    t.release();
    t.start.assign(capacity, nullptr);
    t.stop.assign(capacity, nullptr);
    for (int32_t i = 0; i < capacity; ++i) {
        hipError_t e = hipEventCreate(&t.start[i]);
        if (e == hipSuccess) e = hipEventCreate(&t.stop[i]);
        if (e != hipSuccess) {
            t.release();
            return hip_status(e, "semb_kernel_timer_start: hipEventCreate");
        }
    }
    t.on = true;
    return SEMB_OK;
}

semb_status semb_kernel_timer_stop(int32_t *count, float *ms, int32_t ms_len)
{
    KernelTimer &t = g_timer;
    t.on = false;
    const int n = t.used;
    if (count) *count = n;
    semb_status st = SEMB_OK;
    for (int i = 0; i < n && i < ms_len && ms; ++i) {
        hipError_t e = hipEventSynchronize(t.stop[i]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], t.start[i], t.stop[i]);
        if (e != hipSuccess) {
            st = hip_status(e, "semb_kernel_timer_stop");
            break;
        }
    }
    t.release();
    return st;
}

semb_status semb_probe(int32_t probe, int32_t reps, double *rate, double *ms)
{
    if (probe < SEMB_PROBE_FMA_F32 || probe > SEMB_PROBE_LDS_READ2) return fail(SEMB_EINVAL, "unknown probe");
    if (reps < 1 || reps > 100) return fail(SEMB_EINVAL, "reps must be in 1..100");
    if (!rate || !ms) return fail(SEMB_EINVAL, "rate and ms are required");
    return hip_status((hipError_t)semb::run_probe(probe, reps, rate, ms), "semb_probe");
}

semb_status semb_corrected_gathers(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, const float *theta,
                                   const int64_t *corr_off, float *out, hipStream_t stream)
{
    if (kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) return fail(SEMB_EINVAL, "kind must be CMP or CRS");
    const bool crs = kind == SEMB_KIND_CRS;
    TRY(check_gathers(g, crs));
    TRY(check_jobs(jobs, crs, g));
    if (jobs->njobs == 0) return SEMB_OK;
    if (!theta || !corr_off || !out) return fail(SEMB_EINVAL, "theta, corr_off and out are required");
    semb::PointArgs a{};
    a.samples = g->samples;
    a.sample_off = g->sample_off;
    a.trace_ptr = g->trace_ptr;
    a.ns = g->ns;
    a.half_offset = g->half_offset;
    a.midpoint = g->midpoint;
    a.central_x = g->central_x;
    a.dt = g->dt;
    a.central = jobs->central;
    a.apert_ptr = crs ? jobs->apert_ptr : nullptr;
    a.apert_gather = crs ? jobs->apert_gather : nullptr;
    a.out_off = jobs->out_off;
    a.njobs = jobs->njobs;
    a.n_sblk = (g->ns_max + 63) / 64;
    a.max_apert = jobs->max_apert;
    a.theta = theta;
    a.w = 1;
    return hip_status(semb::launch_corrected(kind, a, corr_off, out, stream), "semb_corrected_gathers launch");
}

semb_status semb_panel_peaks(const float *panel, int64_t n_rows, int32_t nA, int32_t nB, int32_t nq, int32_t K,
                             int32_t *best_k, float *s_k, hipStream_t stream)
{
    if (n_rows < 0 || nA < 1 || nB < 1 || nq < 1 || K < 1 || K > 8)
        return fail(SEMB_EINVAL, "semb_panel_peaks: n_rows >= 0, nA, nB, nq >= 1 and 1 <= K <= 8 are required");
    if ((long long)nA * nB * nq > 0x7fffffffLL) return fail(SEMB_EINVAL, "semb_panel_peaks: grid too large");
    if (n_rows == 0) return SEMB_OK;
    if (!panel || !best_k || !s_k) return fail(SEMB_EINVAL, "semb_panel_peaks: panel, best_k and s_k are required");
    return hip_status(semb::launch_panel_peaks(panel, n_rows, nA, nB, nq, K, best_k, s_k, stream),
                      "semb_panel_peaks launch");
}

semb_status semb_best_of(int32_t K, int64_t n, const float *s_k, const float *stack_k, const float *theta_k,
                         float *s_out, float *stack_out, float *theta_out, hipStream_t stream)
{
    if (K < 1 || n < 0) return fail(SEMB_EINVAL, "semb_best_of: K >= 1 and n >= 0 are required");
    if (n == 0) return SEMB_OK;
    if (!s_k || !stack_k || !theta_k || !s_out || !stack_out || !theta_out)
        return fail(SEMB_EINVAL, "semb_best_of: every array is required");
    return hip_status(semb::launch_best_of(K, n, s_k, stack_k, theta_k, s_out, stack_out, theta_out, stream),
                      "semb_best_of launch");
}

const char *semb_shape_name(int32_t shape)
{
    return (shape >= 0 && shape < semb::kScanShapes) ? kShapeNames[shape] : nullptr;
}

semb_status semb_set_scan_shape(int32_t kind, int32_t w, const semb_gathers *g, const semb_jobs *jobs,
                                int32_t shape)
{
    if ((kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) || !g || !jobs)
        return fail(SEMB_EINVAL, "semb_set_scan_shape: kind must be CMP or CRS, g and jobs non-NULL");
    if (shape < -1 || shape >= semb::kScanShapes)
        return fail(SEMB_EINVAL, "semb_set_scan_shape: shape must be -1 .. %d", semb::kScanShapes - 1);
    std::lock_guard<std::mutex> lk(g_shape_mu);
    const ShapeKey key = shape_key(kind, w, g, jobs);
    if (shape < 0)
        g_shapes.erase(key);
    else
        g_shapes[key] = shape;
    return SEMB_OK;
}

int32_t semb_scan_shape(int32_t kind, int32_t w, const semb_gathers *g, const semb_jobs *jobs)
{
    if ((kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) || !g || !jobs) return -1;
    return chosen_shape(kind, w, g, jobs);
}

void semb_clear_tuning(void)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shapes.clear();
    g_batch.clear();
}

semb_status semb_tune_scan(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, const float *A, int32_t nA,
                           const float *B, int32_t nB, const float *q, int32_t nq, int32_t w, int32_t sample_jobs,
                           int32_t reps, const semb_outputs *out, void *ws, size_t ws_bytes, int32_t *shape,
                           float *ms, hipStream_t stream)
{
    if (kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) return fail(SEMB_EINVAL, "kind must be CMP or CRS");
    if (!shape || sample_jobs < 1 || reps < 1)
        return fail(SEMB_EINVAL, "semb_tune_scan: shape must be non-NULL, sample_jobs and reps >= 1");
    const bool crs = kind == SEMB_KIND_CRS;
    TRY(check_gathers(g, crs));
    TRY(check_jobs(jobs, crs, g));
    // at least four rounds of workgroups at two per CU, or tail effects decide
    int dev = 0, cus = 0;
    TRY(hip_status(hipGetDevice(&dev), "hipGetDevice"));
    TRY(hip_status(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute"));
    const int n_sblk = std::max(1, (g->ns_max + 63) / 64);
    const long long min_jobs = (8LL * std::max(cus, 1) + n_sblk - 1) / n_sblk;
    semb_jobs sub = *jobs;
    sub.njobs = (int32_t)std::min<long long>(std::max<long long>(sample_jobs, min_jobs), jobs->njobs);
    for (int s = 0; s < semb::kScanShapes && ms; ++s) ms[s] = -1.f;
    *shape = chosen_shape(kind, w, g, jobs);
    if (sub.njobs == 0) return SEMB_OK;
    // a first call validates every argument the same way the scans do
    TRY(scan_common(kind, g, &sub, A, nA, B, nB, q, nq, w, out, ws, ws_bytes, stream, default_shape(kind)));

    // the sampled jobs' output rows, on the host
    std::vector<int64_t> off(sub.njobs);
    std::vector<int32_t> cen(sub.njobs), nsv(g->ngathers);
    TRY(hip_status(hipMemcpyAsync(off.data(), jobs->out_off, sizeof(int64_t) * sub.njobs, hipMemcpyDeviceToHost,
                                  stream), "semb_tune_scan: copy"));
    TRY(hip_status(hipMemcpyAsync(cen.data(), jobs->central, sizeof(int32_t) * sub.njobs, hipMemcpyDeviceToHost,
                                  stream), "semb_tune_scan: copy"));
    TRY(hip_status(hipMemcpyAsync(nsv.data(), g->ns, sizeof(int32_t) * g->ngathers, hipMemcpyDeviceToHost, stream),
                   "semb_tune_scan: copy"));
    TRY(hip_status(hipStreamSynchronize(stream), "semb_tune_scan: synchronize"));
    for (int j = 0; j < sub.njobs; ++j)
        if (cen[j] < 0 || cen[j] >= g->ngathers)
            return fail(SEMB_EINVAL, "semb_tune_scan: job %d has central gather %d out of range", j, cen[j]);
    size_t nrows = 0;
    for (int j = 0; j < sub.njobs; ++j) nrows += (size_t)std::max(0, nsv[cen[j]]);
    // one copy per array when the sampled rows are (nearly) contiguous
    int64_t rlo = INT64_MAX, rhi = 0;
    for (int j = 0; j < sub.njobs; ++j) {
        const int64_t n = std::max(0, nsv[cen[j]]);
        if (n == 0) continue;
        rlo = std::min(rlo, off[j]);
        rhi = std::max(rhi, off[j] + n);
    }
    const bool span = rhi > rlo && (size_t)(rhi - rlo) <= 2 * nrows;
    auto fetch = [&](std::vector<int32_t> &b, std::vector<float> &sb, std::vector<float> &st) -> semb_status {
        if (span) {
            const size_t n = (size_t)(rhi - rlo);
            b.resize(n);
            sb.resize(n);
            st.resize(n);
            TRY(hip_status(hipMemcpyAsync(b.data(), out->best + rlo, 4 * n, hipMemcpyDeviceToHost, stream), "copy"));
            TRY(hip_status(hipMemcpyAsync(sb.data(), out->s_best + rlo, 4 * n, hipMemcpyDeviceToHost, stream),
                           "copy"));
            TRY(hip_status(hipMemcpyAsync(st.data(), out->stack + rlo, 4 * n, hipMemcpyDeviceToHost, stream),
                           "copy"));
            TRY(hip_status(hipStreamSynchronize(stream), "semb_tune_scan: synchronize"));
            // keep only the sampled rows (rows between jobs may hold anything)
            std::vector<char> keep(n, 0);
            for (int j = 0; j < sub.njobs; ++j)
                for (int64_t r = off[j]; r < off[j] + std::max(0, nsv[cen[j]]); ++r) keep[(size_t)(r - rlo)] = 1;
            size_t k = 0;
            for (size_t i = 0; i < n; ++i)
                if (keep[i]) {
                    b[k] = b[i];
                    sb[k] = sb[i];
                    st[k] = st[i];
                    ++k;
                }
            b.resize(k);
            sb.resize(k);
            st.resize(k);
            return SEMB_OK;
        }
        b.resize(nrows);
        sb.resize(nrows);
        st.resize(nrows);
        size_t at = 0;
        for (int j = 0; j < sub.njobs; ++j) {
            const size_t n = (size_t)std::max(0, nsv[cen[j]]);
            if (n == 0) continue;
            TRY(hip_status(hipMemcpyAsync(&b[at], out->best + off[j], 4 * n, hipMemcpyDeviceToHost, stream), "copy"));
            TRY(hip_status(hipMemcpyAsync(&sb[at], out->s_best + off[j], 4 * n, hipMemcpyDeviceToHost, stream),
                           "copy"));
            TRY(hip_status(hipMemcpyAsync(&st[at], out->stack + off[j], 4 * n, hipMemcpyDeviceToHost, stream),
                           "copy"));
            at += n;
        }
        return hip_status(hipStreamSynchronize(stream), "semb_tune_scan: synchronize");
    };

    hipEvent_t e0 = nullptr, e1 = nullptr;
    TRY(hip_status(hipEventCreate(&e0), "hipEventCreate"));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SEMB_EHIP, "hipEventCreate failed");
    }
    semb_status st = SEMB_OK;
    std::vector<int32_t> rb, cb;
    std::vector<float> rs, rt, cs, ct;
    int best_shape = default_shape(kind);
    float best_ms = 0.f;
    const int d = default_shape(kind);
    for (int k = 0; k < semb::kScanShapes && st == SEMB_OK; ++k) {
        const int sid = k == 0 ? d : (k <= d ? k - 1 : k);  // the default first
        st = scan_common(kind, g, &sub, A, nA, B, nB, q, nq, w, out, ws, ws_bytes, stream, sid);  // warm-up
        if (st == SEMB_OK) st = hip_status(hipEventRecord(e0, stream), "hipEventRecord");
        for (int r = 0; r < reps && st == SEMB_OK; ++r)
            st = scan_common(kind, g, &sub, A, nA, B, nB, q, nq, w, out, ws, ws_bytes, stream, sid);
        if (st == SEMB_OK) st = hip_status(hipEventRecord(e1, stream), "hipEventRecord");
        if (st == SEMB_OK) st = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
        float t = 0.f;
        if (st == SEMB_OK) st = hip_status(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
        if (st != SEMB_OK) break;
        t /= (float)reps;
        bool same = true;
        if (k == 0) {
            st = fetch(rb, rs, rt);
        } else {
            st = fetch(cb, cs, ct);
            same = cb == rb && cs.size() == rs.size() && memcmp(cs.data(), rs.data(), 4 * rs.size()) == 0 &&
                   memcmp(ct.data(), rt.data(), 4 * rt.size()) == 0;
        }
        if (st != SEMB_OK) break;
        if (ms) ms[sid] = same ? t : -1.f;
        // another shape must beat the default by 2% (timing noise does not flip the choice)
        if (same && (k == 0 || t < (best_shape == d ? 0.98f : 1.f) * best_ms)) {
            best_ms = t;
            best_shape = sid;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SEMB_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        g_shapes[shape_key(kind, w, g, jobs)] = best_shape;
    }
    *shape = best_shape;
    return SEMB_OK;
}

const char *semb_batch_shape_name(int32_t shape)
{
    static const char *const names[semb::kBatchShapes] = {
        "CRS tiles 8 waves x 4 parameters (2 for w > 9), windows behind a branch, 2048-sample stage",
        "CRS tiles 8 waves x 4 parameters (2 for w > 9), branch-free windows, 2560-sample stage",
        "CRS tiles 8 waves x 4 parameters (2 for w > 9), branch-free windows, 2048-sample stage",
    };
    return (shape >= 0 && shape < semb::kBatchShapes) ? names[shape] : nullptr;
}

semb_status semb_set_batch_choice(int32_t w_cmp, int32_t w_crs, const semb_gathers *g, const semb_jobs *jobs,
                                  int32_t shape, int32_t split_params)
{
    if (!g || !jobs) return fail(SEMB_EINVAL, "semb_set_batch_choice: g and jobs are required");
    if (shape < -1 || shape >= semb::kBatchShapes || (shape >= 0 && split_params < 1))
        return fail(SEMB_EINVAL, "semb_set_batch_choice: shape must be -1 .. %d and split_params >= 1",
                    semb::kBatchShapes - 1);
    std::lock_guard<std::mutex> lk(g_shape_mu);
    const BatchKey key = batch_key(w_cmp, w_crs, g, jobs);
    if (shape < 0)
        g_batch.erase(key);
    else
        g_batch[key] = BatchChoice{shape, split_params};
    return SEMB_OK;
}

void semb_batch_choice(int32_t w_cmp, int32_t w_crs, const semb_gathers *g, const semb_jobs *jobs, int32_t *shape,
                       int32_t *split_params)
{
    BatchChoice c{kDefaultBatchShape, kDefaultBatchSplit};
    if (g && jobs) c = chosen_batch(w_cmp, w_crs, g, jobs);
    if (shape) *shape = c.shape;
    if (split_params) *split_params = c.split;
}

semb_status semb_tune_batch(const semb_gathers *g, const semb_jobs *jobs, const semb_batch *b, const semb_tile *tiles,
                            int64_t ntiles, int32_t ngroups, int32_t nparts, int32_t split_params, int32_t reps,
                            const semb_outputs *out, void *ws, size_t ws_bytes, int32_t *shape, float *ms,
                            hipStream_t stream)
{
    if (!shape || reps < 1 || split_params < 1)
        return fail(SEMB_EINVAL, "semb_tune_batch: shape must be non-NULL, reps and split_params >= 1");
    // a first call validates every argument the same way scan_batch does
    TRY(batch_common(g, jobs, b, tiles, ntiles, ngroups, nparts, out, ws, ws_bytes, stream, kDefaultBatchShape));
    for (int k = 0; k < semb::kBatchShapes && ms; ++k) ms[k] = -1.f;
    const size_t n = (size_t)std::max<int64_t>(jobs->n_out, 0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TRY(hip_status(hipEventCreate(&e0), "hipEventCreate"));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SEMB_EHIP, "hipEventCreate failed");
    }
    std::vector<int32_t> rb(n), cb(n);
    std::vector<float> rs(n), rt(n), cs(n), ct(n);
    auto fetch = [&](std::vector<int32_t> &bb, std::vector<float> &ss, std::vector<float> &tt) -> semb_status {
        if (n == 0) return SEMB_OK;
        TRY(hip_status(hipMemcpyAsync(bb.data(), out->best, 4 * n, hipMemcpyDeviceToHost, stream), "copy"));
        TRY(hip_status(hipMemcpyAsync(ss.data(), out->s_best, 4 * n, hipMemcpyDeviceToHost, stream), "copy"));
        TRY(hip_status(hipMemcpyAsync(tt.data(), out->stack, 4 * n, hipMemcpyDeviceToHost, stream), "copy"));
        return hip_status(hipStreamSynchronize(stream), "semb_tune_batch: synchronize");
    };
    semb_status st = SEMB_OK;
    int best_shape = kDefaultBatchShape;
    float best_ms = 0.f;
    for (int k = 0; k < semb::kBatchShapes && st == SEMB_OK; ++k) {
        const int sid = k == 0 ? kDefaultBatchShape : (k <= kDefaultBatchShape ? k - 1 : k);  // the default first
        st = batch_common(g, jobs, b, tiles, ntiles, ngroups, nparts, out, ws, ws_bytes, stream, sid);  // warm-up
        if (st == SEMB_OK) st = hip_status(hipEventRecord(e0, stream), "hipEventRecord");
        for (int r = 0; r < reps && st == SEMB_OK; ++r)
            st = batch_common(g, jobs, b, tiles, ntiles, ngroups, nparts, out, ws, ws_bytes, stream, sid);
        if (st == SEMB_OK) st = hip_status(hipEventRecord(e1, stream), "hipEventRecord");
        if (st == SEMB_OK) st = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
        float t = 0.f;
        if (st == SEMB_OK) st = hip_status(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
        if (st != SEMB_OK) break;
        t /= (float)reps;
        bool same = true;
        if (k == 0) {
            st = fetch(rb, rs, rt);
        } else {
            st = fetch(cb, cs, ct);
            same = cb == rb && memcmp(cs.data(), rs.data(), 4 * n) == 0 && memcmp(ct.data(), rt.data(), 4 * n) == 0;
        }
        if (st != SEMB_OK) break;
        if (ms) ms[sid] = same ? t : -1.f;
        // another shape must beat the default by 2% (timing noise does not flip the choice)
        if (same && (k == 0 || t < (best_shape == kDefaultBatchShape ? 0.98f : 1.f) * best_ms)) {
            best_ms = t;
            best_shape = sid;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SEMB_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        g_batch[batch_key(b->w_cmp, b->w_crs, g, jobs)] = BatchChoice{best_shape, split_params};
    }
    *shape = best_shape;
    return SEMB_OK;
}

int32_t semb_tuning_save(const char *path)
{
    if (!path) {
        fail(SEMB_EINVAL, "semb_tuning_save: path is NULL");
        return -1;
    }
    std::lock_guard<std::mutex> lk(g_shape_mu);
    FILE *f = fopen(path, "w");
    if (!f) {
        fail(SEMB_EINVAL, "semb_tuning_save: cannot open %s", path);
        return -1;
    }
    int32_t n = 0;
    fprintf(f, "# semb tuning table v1 (%s)\n", semb_version());
    fprintf(f, "# scan  kind w traces_bucket ns_bucket shape\n");
    fprintf(f, "# batch w_cmp w_crs traces_bucket ns_bucket shape split_params\n");
    for (const auto &kv : g_shapes) {
        fprintf(f, "scan %d %d %d %d %d\n", kv.first.kind, kv.first.w, kv.first.traces, kv.first.ns, kv.second);
        ++n;
    }
    for (const auto &kv : g_batch) {
        fprintf(f, "batch %d %d %d %d %d %d\n", kv.first.wc, kv.first.wr, kv.first.traces, kv.first.ns,
                kv.second.shape, kv.second.split);
        ++n;
    }
    if (fclose(f) != 0) {
        fail(SEMB_EINVAL, "semb_tuning_save: writing %s failed", path);
        return -1;
    }
    return n;
}

int32_t semb_tuning_load(const char *path)
{
    if (!path) {
        fail(SEMB_EINVAL, "semb_tuning_load: path is NULL");
        return -1;
    }
    FILE *f = fopen(path, "r");
    if (!f) {
        fail(SEMB_EINVAL, "semb_tuning_load: cannot open %s", path);
        return -1;
    }
    std::map<ShapeKey, int> scans;
    std::map<BatchKey, BatchChoice> batches;
    char line[256];
    int lineno = 0;
    bool bad = false;
    // a window the scans accept, and a power-of-two bucket index
    auto ok_w = [](int w) { return w >= 1 && w <= SEMB_W_MAX && (w & 1); };
    auto ok_bucket = [](int b) { return b >= 0 && b <= 40; };  // log2_bucket's range
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        const size_t len = strlen(line);
        if (len == sizeof line - 1 && line[len - 1] != '\n') {  // longer than any entry
            bad = true;
            break;
        }
        const char *p = line;
        while (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n') ++p;
        if (*p == '#' || *p == '\0') continue;
        int a[6], end = -1;
        if (sscanf(p, "scan %d %d %d %d %d %n", &a[0], &a[1], &a[2], &a[3], &a[4], &end) == 5 && end > 0 &&
            p[end] == '\0') {
            if ((a[0] != SEMB_KIND_CMP && a[0] != SEMB_KIND_CRS) || !ok_w(a[1]) || !ok_bucket(a[2]) ||
                !ok_bucket(a[3]) || a[4] < 0 || a[4] >= semb::kScanShapes) {
                bad = true;
                break;
            }
            scans[ShapeKey{a[0], a[1], a[2], a[3]}] = a[4];
        } else if (sscanf(p, "batch %d %d %d %d %d %d %n", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5], &end) == 6 &&
                   end > 0 && p[end] == '\0') {
            if (!ok_w(a[0]) || !ok_w(a[1]) || !ok_bucket(a[2]) || !ok_bucket(a[3]) || a[4] < 0 ||
                a[4] >= semb::kBatchShapes || a[5] < 1) {
                bad = true;
                break;
            }
            batches[BatchKey{a[0], a[1], a[2], a[3]}] = BatchChoice{a[4], a[5]};
        } else {
            bad = true;
            break;
        }
    }
    fclose(f);
    if (bad) {
        fail(SEMB_EINVAL, "semb_tuning_load: %s line %d is not a tuning entry", path, lineno);
        return -1;
    }
    std::lock_guard<std::mutex> lk(g_shape_mu);
    for (const auto &kv : scans) g_shapes[kv.first] = kv.second;
    for (const auto &kv : batches) g_batch[kv.first] = kv.second;
    return (int32_t)(scans.size() + batches.size());
}

const char *semb_last_error(void) { return g_last_error.c_str(); }

const char *semb_version(void) { return "semb-mi355x 0.1 (gfx950)"; }

}  // extern "C"
