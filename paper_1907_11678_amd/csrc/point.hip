// point.hip -- gfx950 kernels that evaluate the semblance at one given
// parameter per output sample (`stack`) and its gradient (`semblance_grad`).
//
// Same sums as the scan (Eq. (1) over the interpolated window of
// Algorithm 1, CMP traveltime of section 2.1 / CRS surface of section 2.2),
// but with a single parameter per output sample there is nothing to share
// across parameters, so each lane owns one output sample and reads the trace
// windows straight from global memory (neighbouring lanes read neighbouring
// windows, which the L1/L2 caches coalesce).  The intersection arithmetic
// (FP64, traveltime.h) is the scan's, so a point evaluation at a grid
// parameter reproduces the scan's value.
//
// Gradient (the ABI header states the formulas): pass 1 recomputes U, D, M
// and S; pass 2 revisits every contributing trace, forms dS/dv for each
// window sample, accumulates dS/dtau and scatters dS/dsample with float
// atomics (every output sample's windows overlap those of its neighbours).

#include <limits.h>
#include <math.h>

#include "internal.h"
#include "traveltime.h"

namespace semb {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int xcd_tile(int bid, int nblk)
{
    const int per = nblk >> 3, rem = nblk & 7;
    const int x = bid & 7, local = bid >> 3;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + local;
}

// One (sample, trace) intersection in the scan's arithmetic (traveltime.h).
struct Isect {
    bool valid;
    float x;      // fraction of the intersection
    int a;        // window start
    float tau;    // intersection, samples
};

template <int KIND, int W>
__device__ __forceinline__ Isect intersect(int s, double A, double B, double q, double h, double dm,
                                           double inv_dt, int nsg)
{
    constexpr int HW = (W - 1) / 2;
    const double cc = h * h * inv_dt * inv_dt;
    const double sd = (double)s;
    double num;
    if (KIND == SEMB_KIND_CMP) {
        num = q * cc;
    } else {
        const double al = A * 2.0 * dm * inv_dt;
        const double be = B * 2.0 * dm * dm * inv_dt;
        num = fma(sd, 2.0 * al + be, fma(al, al, q * cc));
    }
    const double T = sd * sd + num;
    const Hit hit = hit_from_tau(sqrt_refined(T), HW);
    Isect r;
    r.valid = on_trace(hit.a, nsg - 1 - W) && T >= 0.0;
    r.x = hit.x;
    r.a = r.valid ? hit.a : 0;
    r.tau = (float)hit.tau;
    return r;
}

// The rows of a job: its central gather, aperture and output row offset.
struct RowCtx {
    int c, k0, k1;
    const int32_t *ag;  // aperture gathers, or NULL for the central alone
    double xc, inv_dt;
};

template <int KIND>
__device__ __forceinline__ RowCtx row_ctx(const PointArgs &a, int job)
{
    RowCtx r;
    r.c = a.central[job];
    r.k0 = 0;
    r.k1 = 1;
    r.ag = nullptr;
    if (KIND == SEMB_KIND_CRS && a.apert_ptr != nullptr) {
        r.k0 = a.apert_ptr[job];
        r.k1 = a.apert_ptr[job + 1];
        r.ag = a.apert_gather;
    }
    r.xc = (KIND == SEMB_KIND_CRS) ? (double)a.central_x[r.c] : 0.0;
    r.inv_dt = 1.0 / (double)a.dt;
    return r;
}

// Semblance sums at one parameter: U[W], D, M (pass 1 of Eq. (1)).
template <int W>
struct Sums {
    float U[W];
    float D, M;
    __device__ float S() const
    {
        float N = 0.f;
#pragma unroll
        for (int j = 0; j < W; ++j) N = fmaf(U[j], U[j], N);
        return (M > 0.f && D > 0.f) ? N / (M * D) : 0.f;
    }
    __device__ float stack() const
    {
        float L = 0.f;
#pragma unroll
        for (int j = 0; j < W; ++j) L += U[j];
        return (M > 0.f) ? L / (M * (float)W) : 0.f;
    }
};

template <int KIND, int W>
__device__ __forceinline__ Sums<W> sums_at(const PointArgs &a, const RowCtx &r, int s, double A, double B,
                                           double q)
{
    Sums<W> t;
#pragma unroll
    for (int j = 0; j < W; ++j) t.U[j] = 0.f;
    t.D = 0.f;
    t.M = 0.f;
    for (int k = r.k0; k < r.k1; ++k) {
        const int g = r.ag ? r.ag[k] : r.c;
        const int nsg = a.ns[g];
        const int tb = a.trace_ptr[g], te = a.trace_ptr[g + 1];
        for (int i = tb; i < te; ++i) {
            // displacement rounded to FP32 as the scan's trace table holds it
            const float dmf = (KIND == SEMB_KIND_CRS) ? (float)((double)a.midpoint[i] - r.xc) : 0.f;
            const Isect hit = intersect<KIND, W>(s, A, B, q, a.half_offset[i], dmf, r.inv_dt, nsg);
            if (!hit.valid) continue;
            const float *f = a.samples + a.sample_off[g] + (int64_t)(i - tb) * nsg + hit.a;
            float prev = f[0];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const float nxt = f[j + 1];
                const float v = fmaf(hit.x, nxt - prev, prev);
                t.U[j] += v;
                t.D = fmaf(v, v, t.D);
                prev = nxt;
            }
            t.M += 1.f;
        }
    }
    return t;
}

// Pass 2: gs * dS/d(A, B, q) at the parameter whose sums are t (S > 0 needs
// M > 0 and D > 0), scattering gs * dS/dsample into g_samples if not NULL.
template <int KIND, int W>
__device__ __forceinline__ void grad_at(const PointArgs &a, const RowCtx &r, int s, double A, double B, double q,
                                        const Sums<W> &t, float gs, float *g_samples, float &gA, float &gB,
                                        float &gq)
{
    gA = gB = gq = 0.f;
    if (!(t.M > 0.f && t.D > 0.f) || gs == 0.f) return;
    const float S = t.S();
    const float inv_MD = 1.f / (t.M * t.D);
    const float SM = S * t.M;
    const float dtf = a.dt;
    const float t0 = (float)s * dtf;
    for (int k = r.k0; k < r.k1; ++k) {
        const int g = r.ag ? r.ag[k] : r.c;
        const int nsg = a.ns[g];
        const int tb = a.trace_ptr[g], te = a.trace_ptr[g + 1];
        for (int i = tb; i < te; ++i) {
            const float dmf = (KIND == SEMB_KIND_CRS) ? (float)((double)a.midpoint[i] - r.xc) : 0.f;
            const Isect hit = intersect<KIND, W>(s, A, B, q, a.half_offset[i], dmf, r.inv_dt, nsg);
            if (!hit.valid) continue;
            const int64_t base = a.sample_off[g] + (int64_t)(i - tb) * nsg + hit.a;
            const float *f = a.samples + base;
            float dS_dtau = 0.f;
            float carry = 0.f;  // x * dS/dv of the previous window sample
            float prev = f[0];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const float nxt = f[j + 1];
                const float slope = nxt - prev;
                const float v = fmaf(hit.x, slope, prev);
                const float dSdv = 2.f * (t.U[j] - SM * v) * inv_MD;
                dS_dtau = fmaf(dSdv, slope, dS_dtau);
                if (g_samples) atomicAdd(g_samples + base + j, gs * ((1.f - hit.x) * dSdv + carry));
                carry = hit.x * dSdv;
                prev = nxt;
            }
            if (g_samples) atomicAdd(g_samples + base + W, gs * carry);
            if (hit.tau > 0.f) {
                // dtau/dT = 1 / (2 dt sqrt(T)) with sqrt(T) = tau * dt
                const float k_t = dS_dtau / (2.f * hit.tau * dtf * dtf);
                const float h = a.half_offset[i];
                if (KIND == SEMB_KIND_CRS) {
                    gA = fmaf(k_t, 4.f * dmf * (t0 + 2.f * (float)A * dmf), gA);
                    gB = fmaf(k_t, 2.f * t0 * dmf * dmf, gB);
                }
                gq = fmaf(k_t, h * h, gq);
            }
        }
    }
    gA *= gs;
    gB *= gs;
    gq *= gs;
}

// One lane per output sample: the row of lane l of the workgroup, or -1.
template <int KIND>
__device__ __forceinline__ int64_t my_row(const PointArgs &a, int &job, int &s)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    job = tile / a.n_sblk;
    const int sblk = tile - job * a.n_sblk;
    if (job >= a.njobs) return -1;
    s = sblk * WAVE + (int)threadIdx.x;
    if (s >= a.ns[a.central[job]]) return -1;
    return a.out_off[job] + s;
}

template <int KIND, int W, bool GRAD>
__global__ void __launch_bounds__(WAVE)
point_kernel(PointArgs a)
{
    int job, s;
    const int64_t row = my_row<KIND>(a, job, s);
    if (row < 0) return;
    if (KIND == SEMB_KIND_CRS && apert_over(a.apert_ptr, a.max_apert, job)) {  // the documented marker
        if (!GRAD) {
            a.s_out[row] = -1.f;
            a.stack_out[row] = 0.f;
        } else {
            a.g_theta[3 * row + 0] = a.g_theta[3 * row + 1] = a.g_theta[3 * row + 2] = 0.f;
        }
        return;
    }
    const RowCtx r = row_ctx<KIND>(a, job);
    const double A = (KIND == SEMB_KIND_CRS) ? (double)a.theta[3 * row + 0] : 0.0;
    const double B = (KIND == SEMB_KIND_CRS) ? (double)a.theta[3 * row + 1] : 0.0;
    const double q = (double)a.theta[3 * row + 2];
    const Sums<W> t = sums_at<KIND, W>(a, r, s, A, B, q);
    if (!GRAD) {
        a.s_out[row] = t.S();
        a.stack_out[row] = t.stack();
        return;
    }
    float gA, gB, gq;
    grad_at<KIND, W>(a, r, s, A, B, q, t, a.g_s[row], a.g_samples, gA, gB, gq);
    a.g_theta[3 * row + 0] = gA;
    a.g_theta[3 * row + 1] = gB;
    a.g_theta[3 * row + 2] = gq;
}

// Gradient-ascent refinement of every output sample's parameter, all steps in
// one kernel (rows are independent).  In coordinates normalised by the grid
// spacing (u = theta / scale) every component takes its own step: it moves
// u_k by eta_k in the direction of the sign of dS/du_k, clamped to [lo, hi];
// eta_k grows by `grow` while the sign of its derivative repeats from the
// last accepted step and halves when it flips.  A step is kept only if S
// increases; otherwise every eta_k halves and the sign memory is cleared.
// (Per-component step lengths follow the anisotropy of S in (A, B, q), and
// sign steps are not thrown off by the jumps of the gradient where an
// intersection crosses a sample.)  Writes the refined theta, its S and stack.
template <int KIND, int W>
__global__ void __launch_bounds__(WAVE)
refine_kernel(PointArgs a, RefineArgs o)
{
    int job, s;
    const int64_t row = my_row<KIND>(a, job, s);
    if (row < 0) return;
    if (KIND == SEMB_KIND_CRS && apert_over(a.apert_ptr, a.max_apert, job)) {  // theta left as given
        a.s_out[row] = -1.f;
        a.stack_out[row] = 0.f;
        return;
    }
    const RowCtx r = row_ctx<KIND>(a, job);
    float th[3] = {o.theta[3 * row + 0], o.theta[3 * row + 1], o.theta[3 * row + 2]};
    if (KIND == SEMB_KIND_CMP) th[0] = th[1] = 0.f;
    Sums<W> cur = sums_at<KIND, W>(a, r, s, th[0], th[1], th[2]);
    float S = cur.S();
    float eta[3] = {o.eta0, o.eta0, o.eta0};
    float last[3] = {0.f, 0.f, 0.f};  // signs of the last accepted step (0: none)
    constexpr int K0 = KIND == SEMB_KIND_CMP ? 2 : 0;  // CMP moves q only
    for (int it = 0; it < o.steps; ++it) {
        float g[3];
        grad_at<KIND, W>(a, r, s, th[0], th[1], th[2], cur, 1.f, nullptr, g[0], g[1], g[2]);
        float tr[3] = {th[0], th[1], th[2]};
        float sg[3] = {0.f, 0.f, 0.f};
        bool any = false;
#pragma unroll
        for (int k = K0; k < 3; ++k) {
            sg[k] = g[k] > 0.f ? 1.f : (g[k] < 0.f ? -1.f : 0.f);
            const float same = sg[k] * last[k];
            eta[k] *= same > 0.f ? o.grow : (same < 0.f ? 0.5f : 1.f);
            tr[k] = fminf(fmaxf(fmaf(sg[k] * eta[k], o.scale[k], th[k]), o.lo[k]), o.hi[k]);
            any |= sg[k] != 0.f;
        }
        if (!any) break;  // flat (or S = 0): nothing to climb
        const Sums<W> nxt = sums_at<KIND, W>(a, r, s, tr[0], tr[1], tr[2]);
        const float Sn = nxt.S();
        if (Sn > S) {
            S = Sn;
            cur = nxt;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                th[k] = tr[k];
                last[k] = sg[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                eta[k] *= 0.5f;
                last[k] = 0.f;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) o.theta[3 * row + k] = th[k];
    a.s_out[row] = S;
    a.stack_out[row] = cur.stack();
}

// theta[row] = (A, B, q) of the flat index best[row] ((iA * nB + iB) * nq + iq).
__global__ void theta_from_best_kernel(const int32_t *best, int64_t n, const float *A, int nA, const float *B, int nB,
                                       const float *q, int nq, float *theta)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int b = best[i];
        const int npar = nA * nB * nq;
        b = b < 0 ? 0 : (b >= npar ? npar - 1 : b);
        const int iq = b % nq, rest = b / nq;
        theta[3 * i + 0] = A ? A[rest / nB] : 0.f;
        theta[3 * i + 1] = B ? B[rest % nB] : 0.f;
        theta[3 * i + 2] = q[iq];
    }
}

// theta[i] = clamp(theta[i] + d, lo, hi) per component: a further start of a
// multi-start refinement beside a coarse peak.
__global__ void theta_shift_kernel(float *theta, int64_t n, float3 d, float3 lo, float3 hi)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        theta[3 * i + 0] = fminf(fmaxf(theta[3 * i + 0] + d.x, lo.x), hi.x);
        theta[3 * i + 1] = fminf(fmaxf(theta[3 * i + 1] + d.y, lo.y), hi.y);
        theta[3 * i + 2] = fminf(fmaxf(theta[3 * i + 2] + d.z, lo.z), hi.z);
    }
}

// Gathers corrected along each output sample's parameter (quality control):
// lane l reads every aperture trace at the intersection of its row, with the
// interpolation of a one-sample window, and writes it to the job's corrected
// trace (coalesced across lanes); 0 where the trace does not contribute.
template <int KIND>
__global__ void __launch_bounds__(WAVE)
corrected_kernel(PointArgs a, const int64_t *__restrict__ corr_off, float *__restrict__ out)
{
    int job, s;
    const int64_t row = my_row<KIND>(a, job, s);
    if (row < 0) return;
    const RowCtx r = row_ctx<KIND>(a, job);
    const int nsc = a.ns[r.c];
    const double A = (KIND == SEMB_KIND_CRS) ? (double)a.theta[3 * row + 0] : 0.0;
    const double B = (KIND == SEMB_KIND_CRS) ? (double)a.theta[3 * row + 1] : 0.0;
    const double q = (double)a.theta[3 * row + 2];
    // an aperture longer than the caller declared: every corrected value is 0
    const bool over = KIND == SEMB_KIND_CRS && apert_over(a.apert_ptr, a.max_apert, job);
    float *o = out + corr_off[job] + s;
    for (int k = r.k0; k < r.k1; ++k) {
        const int g = r.ag ? r.ag[k] : r.c;
        const int nsg = a.ns[g];
        const int tb = a.trace_ptr[g], te = a.trace_ptr[g + 1];
        for (int i = tb; i < te; ++i, o += nsc) {
            if (over) {
                *o = 0.f;
                continue;
            }
            const float dmf = (KIND == SEMB_KIND_CRS) ? (float)((double)a.midpoint[i] - r.xc) : 0.f;
            const Isect hit = intersect<KIND, 1>(s, A, B, q, a.half_offset[i], dmf, r.inv_dt, nsg);
            float v = 0.f;
            if (hit.valid) {
                const float *f = a.samples + a.sample_off[g] + (int64_t)(i - tb) * nsg + hit.a;
                v = fmaf(hit.x, f[1] - f[0], f[0]);
            }
            *o = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Starting points for a multi-start refinement: the K best local maxima of
// each row of a semblance panel over its nA x nB x nq grid.  A cell is a
// local maximum when every neighbour (diagonals included) is smaller, or
// equal with a larger flat index, so a plateau yields one peak.  One wave per
// row; lanes take cells lane, lane + 64, ...; each lane keeps its 8 best
// peaks, then K rounds of a wave-wide argmax pick the row's K best (largest S,
// then smallest index).  A row with fewer than K peaks repeats its best.
// ---------------------------------------------------------------------------
constexpr int PEAKS_KMAX = 8;

__device__ __forceinline__ bool peak_better(float v, int c, float w, int d)
{
    return v > w || (v == w && c < d);
}

__global__ void __launch_bounds__(256)
panel_peaks_kernel(const float *__restrict__ panel, int64_t n_rows, int nA, int nB, int nq, int K,
                   int32_t *__restrict__ best_k, float *__restrict__ s_k)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    if (row >= n_rows) return;  // uniform per wave; no barrier below
    const int npar = nA * nB * nq;
    const float *S = panel + row * (int64_t)npar;
    float ts[PEAKS_KMAX];
    int ti[PEAKS_KMAX];
#pragma unroll
    for (int k = 0; k < PEAKS_KMAX; ++k) {
        ts[k] = -INFINITY;
        ti[k] = INT_MAX;
    }
    for (int c = lane; c < npar; c += WAVE) {
        const float v = S[c];
        const int iq = c % nq, r = c / nq, iB = r % nB, iA = r / nB;
        bool peak = true;
        for (int da = -1; da <= 1; ++da) {
            const int a = iA + da;
            if (a < 0 || a >= nA) continue;
            for (int db = -1; db <= 1; ++db) {
                const int b = iB + db;
                if (b < 0 || b >= nB) continue;
                for (int dq = -1; dq <= 1; ++dq) {
                    const int qq = iq + dq;
                    if (qq < 0 || qq >= nq || (da == 0 && db == 0 && dq == 0)) continue;
                    const int n = (a * nB + b) * nq + qq;
                    if (peak_better(S[n], n, v, c)) peak = false;
                }
            }
        }
        if (peak && peak_better(v, c, ts[PEAKS_KMAX - 1], ti[PEAKS_KMAX - 1])) {
            ts[PEAKS_KMAX - 1] = v;
            ti[PEAKS_KMAX - 1] = c;
#pragma unroll
            for (int k = PEAKS_KMAX - 1; k > 0; --k) {
                if (peak_better(ts[k], ti[k], ts[k - 1], ti[k - 1])) {
                    const float tv = ts[k];
                    const int tc = ti[k];
                    ts[k] = ts[k - 1];
                    ti[k] = ti[k - 1];
                    ts[k - 1] = tv;
                    ti[k - 1] = tc;
                }
            }
        }
    }
    int first = 0;
    float first_s = 0.f;
    for (int k = 0; k < K; ++k) {
        float bv = ts[0];
        int bi = ti[0];
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv, o, WAVE);
            const int oi = __shfl_xor(bi, o, WAVE);
            if (peak_better(ov, oi, bv, bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (ti[0] == bi && bi != INT_MAX) {  // the lane holding the winner drops it
#pragma unroll
            for (int j = 0; j < PEAKS_KMAX - 1; ++j) {
                ts[j] = ts[j + 1];
                ti[j] = ti[j + 1];
            }
            ts[PEAKS_KMAX - 1] = -INFINITY;
            ti[PEAKS_KMAX - 1] = INT_MAX;
        }
        if (k == 0) {
            first = bi;
            first_s = bv;
        }
        if (lane == 0) {
            const bool have = bi != INT_MAX;
            best_k[(int64_t)k * n_rows + row] = have ? bi : first;
            s_k[(int64_t)k * n_rows + row] = have ? bv : first_s;
        }
    }
}

// For each row, the candidate k with the largest s_k[k][row] (first on ties):
// its S, stack and theta.
__global__ void best_of_kernel(int K, int64_t n, const float *__restrict__ s_k, const float *__restrict__ stack_k,
                               const float *__restrict__ theta_k, float *__restrict__ s_out,
                               float *__restrict__ stack_out, float *__restrict__ theta_out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int kb = 0;
        float sb = s_k[i];
        for (int k = 1; k < K; ++k) {
            const float v = s_k[(int64_t)k * n + i];
            if (v > sb) {
                sb = v;
                kb = k;
            }
        }
        const int64_t src = (int64_t)kb * n + i;
        s_out[i] = sb;
        stack_out[i] = stack_k[src];
        theta_out[3 * i + 0] = theta_k[3 * src + 0];
        theta_out[3 * i + 1] = theta_k[3 * src + 1];
        theta_out[3 * i + 2] = theta_k[3 * src + 2];
    }
}

template <int KIND, bool GRAD, int W>
hipError_t launch_pw(const PointArgs &a, hipStream_t stream)
{
    const long long nblk = (long long)a.njobs * a.n_sblk;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL((point_kernel<KIND, W, GRAD>), dim3((unsigned)nblk), dim3(WAVE), 0, stream, a);
    return hipGetLastError();
}

template <int KIND, bool GRAD>
hipError_t launch_p(const PointArgs &a, hipStream_t stream)
{
    switch (a.w) {
    case 1: return launch_pw<KIND, GRAD, 1>(a, stream);
    case 3: return launch_pw<KIND, GRAD, 3>(a, stream);
    case 5: return launch_pw<KIND, GRAD, 5>(a, stream);
    case 7: return launch_pw<KIND, GRAD, 7>(a, stream);
    case 9: return launch_pw<KIND, GRAD, 9>(a, stream);
    case 11: return launch_pw<KIND, GRAD, 11>(a, stream);
    case 13: return launch_pw<KIND, GRAD, 13>(a, stream);
    case 15: return launch_pw<KIND, GRAD, 15>(a, stream);
    case 17: return launch_pw<KIND, GRAD, 17>(a, stream);
    case 19: return launch_pw<KIND, GRAD, 19>(a, stream);
    case 21: return launch_pw<KIND, GRAD, 21>(a, stream);
    case 23: return launch_pw<KIND, GRAD, 23>(a, stream);
    case 25: return launch_pw<KIND, GRAD, 25>(a, stream);
    case 27: return launch_pw<KIND, GRAD, 27>(a, stream);
    case 29: return launch_pw<KIND, GRAD, 29>(a, stream);
    case 31: return launch_pw<KIND, GRAD, 31>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int KIND, int W>
hipError_t launch_rw(const PointArgs &a, const RefineArgs &o, hipStream_t stream)
{
    const long long nblk = (long long)a.njobs * a.n_sblk;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL((refine_kernel<KIND, W>), dim3((unsigned)nblk), dim3(WAVE), 0, stream, a, o);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_r(const PointArgs &a, const RefineArgs &o, hipStream_t stream)
{
    switch (a.w) {
    case 1: return launch_rw<KIND, 1>(a, o, stream);
    case 3: return launch_rw<KIND, 3>(a, o, stream);
    case 5: return launch_rw<KIND, 5>(a, o, stream);
    case 7: return launch_rw<KIND, 7>(a, o, stream);
    case 9: return launch_rw<KIND, 9>(a, o, stream);
    case 11: return launch_rw<KIND, 11>(a, o, stream);
    case 13: return launch_rw<KIND, 13>(a, o, stream);
    case 15: return launch_rw<KIND, 15>(a, o, stream);
    case 17: return launch_rw<KIND, 17>(a, o, stream);
    case 19: return launch_rw<KIND, 19>(a, o, stream);
    case 21: return launch_rw<KIND, 21>(a, o, stream);
    case 23: return launch_rw<KIND, 23>(a, o, stream);
    case 25: return launch_rw<KIND, 25>(a, o, stream);
    case 27: return launch_rw<KIND, 27>(a, o, stream);
    case 29: return launch_rw<KIND, 29>(a, o, stream);
    case 31: return launch_rw<KIND, 31>(a, o, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_refine(int kind, const PointArgs &a, const RefineArgs &o, hipStream_t stream)
{
    return kind == SEMB_KIND_CMP ? launch_r<SEMB_KIND_CMP>(a, o, stream) : launch_r<SEMB_KIND_CRS>(a, o, stream);
}

hipError_t launch_theta_from_best(const int32_t *best, int64_t n, const float *A, int nA, const float *B, int nB,
                                  const float *q, int nq, float *theta, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    hipLaunchKernelGGL(theta_from_best_kernel, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, stream, best,
                       n, A, nA, B, nB, q, nq, theta);
    return hipGetLastError();
}

hipError_t launch_theta_shift(float *theta, int64_t n, const float *d, const float *lo, const float *hi,
                              hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    hipLaunchKernelGGL(theta_shift_kernel, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, stream, theta, n,
                       make_float3(d[0], d[1], d[2]), make_float3(lo[0], lo[1], lo[2]),
                       make_float3(hi[0], hi[1], hi[2]));
    return hipGetLastError();
}

hipError_t launch_corrected(int kind, const PointArgs &a, const int64_t *corr_off, float *out, hipStream_t stream)
{
    const long long nblk = (long long)a.njobs * a.n_sblk;
    if (nblk == 0) return hipSuccess;
    if (kind == SEMB_KIND_CMP)
        hipLaunchKernelGGL((corrected_kernel<SEMB_KIND_CMP>), dim3((unsigned)nblk), dim3(WAVE), 0, stream, a,
                           corr_off, out);
    else
        hipLaunchKernelGGL((corrected_kernel<SEMB_KIND_CRS>), dim3((unsigned)nblk), dim3(WAVE), 0, stream, a,
                           corr_off, out);
    return hipGetLastError();
}

hipError_t launch_panel_peaks(const float *panel, int64_t n_rows, int nA, int nB, int nq, int K, int32_t *best_k,
                              float *s_k, hipStream_t stream)
{
    if (n_rows <= 0) return hipSuccess;
    const int64_t nb = (n_rows + 3) / 4;  // 4 waves (rows) per block
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(panel_peaks_kernel, dim3((unsigned)nb), dim3(4 * WAVE), 0, stream, panel, n_rows, nA, nB,
                       nq, K, best_k, s_k);
    return hipGetLastError();
}

hipError_t launch_best_of(int K, int64_t n, const float *s_k, const float *stack_k, const float *theta_k,
                          float *s_out, float *stack_out, float *theta_out, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    hipLaunchKernelGGL(best_of_kernel, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, stream, K, n, s_k,
                       stack_k, theta_k, s_out, stack_out, theta_out);
    return hipGetLastError();
}

hipError_t launch_point(int kind, const PointArgs &a, hipStream_t stream)
{
    return kind == SEMB_KIND_CMP ? launch_p<SEMB_KIND_CMP, false>(a, stream)
                                 : launch_p<SEMB_KIND_CRS, false>(a, stream);
}

hipError_t launch_grad(int kind, const PointArgs &a, hipStream_t stream)
{
    return kind == SEMB_KIND_CMP ? launch_p<SEMB_KIND_CMP, true>(a, stream)
                                 : launch_p<SEMB_KIND_CRS, true>(a, stream);
}

}  // namespace semb
