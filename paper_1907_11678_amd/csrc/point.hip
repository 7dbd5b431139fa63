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

template <int KIND, int W, bool GRAD>
__global__ void __launch_bounds__(WAVE)
point_kernel(PointArgs a)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int job = tile / a.n_sblk;
    const int sblk = tile - job * a.n_sblk;
    if (job >= a.njobs) return;
    const int c = a.central[job];
    const int nsc = a.ns[c];
    const int s = sblk * WAVE + (int)threadIdx.x;
    if (s >= nsc) return;

    const int64_t row = a.out_off[job] + s;
    const double inv_dt = 1.0 / (double)a.dt;
    const double A = (KIND == SEMB_KIND_CRS) ? (double)a.theta[3 * row + 0] : 0.0;
    const double B = (KIND == SEMB_KIND_CRS) ? (double)a.theta[3 * row + 1] : 0.0;
    const double q = (double)a.theta[3 * row + 2];
    const double xc = (KIND == SEMB_KIND_CRS) ? (double)a.central_x[c] : 0.0;

    int k0 = 0, k1 = 1;
    if (KIND == SEMB_KIND_CRS && a.apert_ptr != nullptr) {
        k0 = a.apert_ptr[job];
        k1 = a.apert_ptr[job + 1];
    }

    float U[W];
#pragma unroll
    for (int j = 0; j < W; ++j) U[j] = 0.f;
    float D = 0.f, M = 0.f;

    // ---- pass 1: U, D, M ---------------------------------------------------
    for (int k = k0; k < k1; ++k) {
        const int g = (KIND == SEMB_KIND_CRS && a.apert_ptr != nullptr) ? a.apert_gather[k] : c;
        const int nsg = a.ns[g];
        const int tb = a.trace_ptr[g], te = a.trace_ptr[g + 1];
        for (int i = tb; i < te; ++i) {
            // displacement rounded to FP32 as the scan's trace table holds it
            const float dmf = (KIND == SEMB_KIND_CRS) ? (float)((double)a.midpoint[i] - xc) : 0.f;
            const Isect hit = intersect<KIND, W>(s, A, B, q, a.half_offset[i], dmf, inv_dt, nsg);
            if (!hit.valid) continue;
            const float *f = a.samples + a.sample_off[g] + (int64_t)(i - tb) * nsg + hit.a;
            float prev = f[0];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const float nxt = f[j + 1];
                const float v = fmaf(hit.x, nxt - prev, prev);
                U[j] += v;
                D = fmaf(v, v, D);
                prev = nxt;
            }
            M += 1.f;
        }
    }
    float N = 0.f, L = 0.f;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        N = fmaf(U[j], U[j], N);
        L += U[j];
    }
    const bool live = (M > 0.f && D > 0.f);
    const float S = live ? N / (M * D) : 0.f;

    if (!GRAD) {
        a.s_out[row] = S;
        a.stack_out[row] = (M > 0.f) ? L / (M * (float)W) : 0.f;
        return;
    }

    // ---- pass 2: dS/dtau per trace, dS/dsample scattered -------------------
    const float gs = a.g_s[row];
    float gA = 0.f, gB = 0.f, gq = 0.f;
    if (live && gs != 0.f) {
        const float inv_MD = 1.f / (M * D);
        const float SM = S * M;
        const float dtf = a.dt;
        const float t0 = (float)s * dtf;
        for (int k = k0; k < k1; ++k) {
            const int g = (KIND == SEMB_KIND_CRS && a.apert_ptr != nullptr) ? a.apert_gather[k] : c;
            const int nsg = a.ns[g];
            const int tb = a.trace_ptr[g], te = a.trace_ptr[g + 1];
            for (int i = tb; i < te; ++i) {
                const float dmf = (KIND == SEMB_KIND_CRS) ? (float)((double)a.midpoint[i] - xc) : 0.f;
                const Isect hit = intersect<KIND, W>(s, A, B, q, a.half_offset[i], dmf, inv_dt, nsg);
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
                    const float dSdv = 2.f * (U[j] - SM * v) * inv_MD;
                    dS_dtau = fmaf(dSdv, slope, dS_dtau);
                    if (a.g_samples) atomicAdd(a.g_samples + base + j, gs * ((1.f - hit.x) * dSdv + carry));
                    carry = hit.x * dSdv;
                    prev = nxt;
                }
                if (a.g_samples) atomicAdd(a.g_samples + base + W, gs * carry);
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
    }
    a.g_theta[3 * row + 0] = gs * gA;
    a.g_theta[3 * row + 1] = gs * gB;
    a.g_theta[3 * row + 2] = gs * gq;
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

}  // namespace

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
