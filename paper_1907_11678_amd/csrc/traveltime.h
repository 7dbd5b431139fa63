// traveltime.h -- the intersection of a traveltime curve (CMP, section 2.1)
// or surface (CRS, section 2.2) with one trace, in the arithmetic every
// kernel of the library shares.
//
// In samples: tau^2 = s^2 + num with
//   CMP  num = q h^2/dt^2,
//   CRS  num = s (2 alpha + beta) + alpha^2 + q h^2/dt^2,
//        alpha = 2 A dm / dt,  beta = 2 B dm^2 / dt,
// which is T/dt^2 for T = t0^2 + q h^2, resp. T = (t0 + 2 A dm)^2 + 2 t0 B dm^2
// + q h^2, t0 = s dt.  The square root is taken in FP64 from the hardware
// reciprocal square root (accurate to about 2^-23) plus one Newton step, so
// tau, k = floor(tau) and the fraction x = tau - k are exact to ~1e-12
// samples: the set of contributing traces and the interpolation weights are
// those of an exact evaluation, whatever the size of tau.
#pragma once

#include <hip/hip_runtime.h>

namespace semb {

// tau = sqrt(max(T, 1e-300)): the square root for T > 0 and ~1e-150 (floor 0,
// fraction 0 in FP32) for T <= 0; callers reject T < 0 themselves.
__device__ __forceinline__ double sqrt_refined(double T)
{
    const double Tm = fmax(T, 1e-300);
    const double y = __builtin_amdgcn_rsq(Tm);  // ~1/sqrt(T), rel. err ~2^-23
    const double t0 = Tm * y;
    const double r = fma(-t0, t0, Tm);
    return fma(r, 0.5 * y, t0);
}

// The scan's form: sqrt(T) for T > 0 by the same reciprocal square root and
// Newton step, without the clamp.  For T <= 0 the result is NaN or infinite;
// the scan rejects those T itself and clamps the result before converting it.
__device__ __forceinline__ double sqrt_newton(double T)
{
    const double y = __builtin_amdgcn_rsq(T);
    const double t0 = T * y;
    const double r = fma(-t0, t0, T);
    return fma(r, 0.5 * y, t0);
}

// Window start a = floor(tau) - hw and fraction x of one intersection, tau >= 0.
struct Hit {
    int a;
    float x;
    double tau;
};

__device__ __forceinline__ Hit hit_from_tau(double tau, int hw)
{
    // a tau of 2^30 or more cannot start a window on any trace the ABI accepts;
    // the clamp keeps the conversion in range, where truncation is floor
    const double tc = fmin(tau, 1073741824.0);
    const int k = (int)tc;
    Hit h;
    h.a = k - hw;
    h.x = (float)(tc - (double)k);
    h.tau = tau;
    return h;
}

// Does a window starting at a (w samples plus the one after) lie on a trace
// whose last valid window start is lim = ns - 1 - w?
__device__ __forceinline__ bool on_trace(int a, int lim)
{
    return (unsigned)a <= (unsigned)lim && lim >= 0;
}

}  // namespace semb
