// api.cpp -- host side of the C ABI declared in include/semb.h: argument
// validation, workspace carving, launch configuration and error reporting.
// Nothing here allocates device memory or synchronises a stream.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>

#include "internal.h"

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

semb_status scan_common(int kind, const semb_gathers *g, const semb_jobs *jobs, const float *A, int32_t nA,
                        const float *B, int32_t nB, const float *q, int32_t nq, int32_t w,
                        const semb_outputs *out, void *ws, size_t ws_bytes, hipStream_t stream)
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
    a.A = A;
    a.B = B;
    a.q = q;
    a.nA = crs ? nA : 1;
    a.nB = crs ? nB : 1;
    a.nq = nq;
    a.npar = (int32_t)npar;
    a.best = out->best;
    a.s_best = out->s_best;
    a.stack = out->stack;
    a.panel = out->panel;
    a.u0 = u0;
    a.u1 = u1;
    a.u2sq = u2sq;
    a.w = w;
    return hip_status(semb::launch_scan(kind, a, stream), crs ? "crs_scan launch" : "cmp_scan launch");
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
    a.theta = theta;
    a.g_s = g_s;
    a.s_out = s_out;
    a.stack_out = stack_out;
    a.g_theta = g_theta;
    a.g_samples = g_samples;
    a.w = w;
    if (grad) return hip_status(semb::launch_grad(kind, a, stream), "semblance_grad launch");
    return hip_status(semb::launch_point(kind, a, stream), "stack launch");
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

const char *semb_last_error(void) { return g_last_error.c_str(); }

const char *semb_version(void) { return "semb-mi355x 0.1 (gfx950)"; }

}  // extern "C"
